"""Build the HIP library for gfx950 in-tree.

    python -m paper_2004_09389_amd.build

compiles every source under csrc/ with hipcc into paper_2004_09389_amd/libhdg.so.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhdg.so")
SOURCES = ["csrc/hdg_host.cpp", "csrc/hdg_rt0_host.cpp", "csrc/hdg_kernels.hip", "csrc/hdg_mlp.hip",
           "csrc/hdg_rt0.hip", "csrc/hdg_imex.hip", "csrc/hdg_dgs.hip", "csrc/hdg_stream.hip",
           "csrc/hdg_api.hip"]

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off: plain scalar FP32 code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable",
]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out_tmp = LIB + ".tmp"
    srcs = []
    for s in SOURCES:
        path = os.path.join(HERE, s)
        if s.endswith(".cpp"):
            srcs += ["-x", "hip", path]
        else:
            srcs += ["-x", "hip", path]
    cmd = [hipcc, *FLAGS, "-I", os.path.join(ROOT, "include"), *srcs, "-o", out_tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed building libhdg.so")
    if verbose and res.stderr.strip():
        sys.stderr.write(res.stderr)
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
