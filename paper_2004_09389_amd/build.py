"""Build the HIP library for gfx950 in-tree.

    python -m paper_2004_09389_amd.build

compiles every source under csrc/ with hipcc (in parallel, objects under
_build/) and links them into paper_2004_09389_amd/libhdg.so.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhdg.so")
OBJ = os.path.join(HERE, "_build")
SOURCES = ["csrc/hdg_host.cpp", "csrc/hdg_rt0_host.cpp", "csrc/hdg_kernels.hip", "csrc/hdg_mlp.hip",
           "csrc/hdg_rt0.hip", "csrc/hdg_imex.hip", "csrc/hdg_dgs.hip", "csrc/hdg_stream.hip",
           "csrc/hdg_small.hip", "csrc/hdg_api.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
    # packed FP32 instructions stay off: plain scalar FP32 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)
    return res


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include")]
    jobs = []
    for s in SOURCES:
        obj = os.path.join(OBJ, os.path.basename(s) + ".o")
        jobs.append((obj, [hipcc, *FLAGS, *inc, "-x", "hip", "-c", os.path.join(HERE, s), "-o", obj]))
    workers = min(len(jobs), max(1, min(8, os.cpu_count() or 1)))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(lambda j: _run(j[1], verbose), jobs))
    for (obj, cmd), res in zip(jobs, results):
        if res.returncode != 0:
            sys.stderr.write(res.stdout + res.stderr)
            raise RuntimeError(f"hipcc failed on {cmd[-3]}")
    out_tmp = LIB + ".tmp"
    res = _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *[o for o, _ in jobs], "-o", out_tmp], verbose)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed linking libhdg.so")
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
