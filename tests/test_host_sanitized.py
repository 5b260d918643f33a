"""Host builders (topology, reference tables, P1 and RT0 levels) built with the
host compiler alone under AddressSanitizer, UndefinedBehaviorSanitizer and
libstdc++'s bounds-checked containers, and run on the sphere hierarchy
(levels 0-2), the 1 x 1 torus and the torus hierarchy 4 -> 8 -> 16.

The driver (tests/host/check_builders.cpp) checks what the mathematics fixes:
Euler characteristic and facet/cell incidence, partition of unity and
quadrature of the reference tables, symmetry, positive definiteness and the
constant-mode mass of the P1 form, Galerkin coarsening against a dense
P^T A P (and against the rediscretised coarse form on the flat nested torus),
the V-cycle matrix (the exact inverse on one level; symmetric and convergent
on several), RT0 patch inverses, P^T S_fine P = S_coarse for the nested RT0
spaces, reproduction of constant fields by the Lax-Friedrichs prolongation,
and that malformed meshes are rejected with HDG_EINVAL.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from hdg_inputs.mesh import Hierarchy, icosphere_hierarchy, torus, torus_hierarchy

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2004_09389_amd", "csrc")


def _write(path, H):
    with open(path, "wb") as f:
        np.array([len(H.meshes)], np.int32).tofile(f)
        for m in H.meshes:
            np.array([1 if m.kind == "sphere" else 0, m.n_vert, m.n_cell], np.int32).tofile(f)
            np.array([m.period], np.float64).tofile(f)
            np.ascontiguousarray(m.vert_xyz, np.float64).tofile(f)
            np.ascontiguousarray(m.cell_vert, np.int32).tofile(f)
            np.ascontiguousarray(m.cell_shift, np.int32).tofile(f)
        for p in H.parents:
            np.ascontiguousarray(p, np.int32).tofile(f)


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_host_builders_under_sanitizers(tmp_path):
    exe = str(tmp_path / "check_builders")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-D_GLIBCXX_ASSERTIONS",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "host", "check_builders.cpp"),
           os.path.join(CSRC, "hdg_host.cpp"), os.path.join(CSRC, "hdg_rt0_host.cpp"), "-o", exe]
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stderr
    files = {"sphere": icosphere_hierarchy(2), "torus1": Hierarchy([torus(1)], []),
             "torus": torus_hierarchy(16, 4)}
    paths = []
    for name, H in files.items():
        paths.append(str(tmp_path / name))
        _write(paths[-1], H)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe, *paths], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0 and run.stdout.rstrip().endswith("ALL OK"), run.stdout[-2000:] + run.stderr[-4000:]
    assert "runtime error" not in run.stderr and "Sanitizer" not in run.stderr, run.stderr[-4000:]
    for tag in ("sphere level 2 topology", "torus1 RT0 levels", "torus RT0 levels", "sphere P1 levels",
                "open mesh rejected"):
        assert f"ok {tag}" in run.stdout
