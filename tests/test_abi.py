"""The C-ABI library loads and exports every symbol include/hdg.h declares
(no GPU needed: no compute call is made)."""
import ctypes
import os
import re

import pytest

from paper_2004_09389_amd import hdg

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "hdg.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hdg_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_entry_points():
    syms = declared_symbols()
    for name in ("hdg_setup", "hdg_condense", "hdg_trace_apply", "hdg_mg_vcycle", "hdg_solve",
                 "hdg_recover", "hdg_destroy", "hdg_last_error"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    lib = hdg.load_library()
    for name in declared_symbols():
        assert hasattr(lib, name), name
        assert getattr(lib, name) is not None


def test_binding_signatures_cover_header():
    assert set(declared_symbols()) == set(hdg._SIGS)


def test_default_options_and_errors_without_gpu():
    o = hdg.default_options()
    assert (o.nu_pre, o.nu_post, o.p1_nu, o.restart, o.max_rhs) == (2, 2, 2, 30, 1)
    assert o.omega == 0.7 and abs(o.p1_omega - 2 / 3) < 1e-15 and o.rtol == 1e-8
    lib = hdg.load_library()
    assert lib.hdg_default_options(None) == hdg.HDG_EINVAL
    # a NULL context is rejected before any device work
    assert lib.hdg_condense(None, 1, None, None, None) == hdg.HDG_EINVAL
    assert lib.hdg_get_sizes(None, None) == hdg.HDG_EINVAL
    assert isinstance(lib.hdg_last_error(), bytes)


def test_struct_layouts_match_header():
    # the ctypes mirrors must have the C struct sizes (natural alignment)
    assert ctypes.sizeof(hdg.HdgMesh) == 4 * 3 + 4 + 8 + 3 * 8
    assert ctypes.sizeof(hdg.HdgParams) == 8 + 6 * 8 + 8
    assert ctypes.sizeof(hdg.HdgSolveInfo) == 4 * 4 + 8
    # ... + ir_inner_rtol (8) + persistent (4, padded to 8)
    assert ctypes.sizeof(hdg.HdgOptions) == 4 * 6 + 8 + 4 + 4 + 8 + 8 + 4 * 4 + 8 + 4 + 4 + 4 + 4 + 8 + 8 + 8
    assert ctypes.sizeof(hdg.HdgTuning) == 12
    assert ctypes.sizeof(hdg.HdgSizes) == 8 * 4 + 8 + 2 * 8 + 8


def test_struct_offsets_match_c_compiler(tmp_path):
    """Every field offset of the ctypes mirrors equals the C compiler's offsetof
    for the structs of include/hdg.h (compiled here with gcc)."""
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    structs = {"hdg_mesh": hdg.HdgMesh, "hdg_params": hdg.HdgParams, "hdg_options": hdg.HdgOptions,
               "hdg_solve_info": hdg.HdgSolveInfo, "hdg_sizes": hdg.HdgSizes, "hdg_tuning": hdg.HdgTuning,
               "hdg_imex_tableau": hdg.HdgImexTableau, "hdg_imex_info": hdg.HdgImexInfo}
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


@pytest.mark.parametrize("method", ["theta", "ars232", "ssp322", "ars443"])
def test_library_tableaux_equal_the_oracles(method):
    """The library's tableaux (host code, no GPU) against the oracle's, both
    typed from the IMEX methods section; the oracle's are pinned by the order
    conditions."""
    import numpy as np
    from oracle.imex import tableau
    for theta in ((0.5, 0.55) if method == "theta" else (0.5,)):
        t = hdg.imex_tableau(method, theta)
        a, at, b, bt = tableau(method, theta)
        s = len(b)
        assert t.stages == s
        lib_a = np.array([[t.a[i][j] for j in range(5)] for i in range(5)])
        lib_at = np.array([[t.at[i][j] for j in range(5)] for i in range(5)])
        assert np.abs(lib_a[:s, :s] - a).max() < 1e-15 and np.abs(lib_at[:s, :s] - at).max() < 1e-15
        assert np.abs(np.array(t.b[:s]) - b).max() < 1e-15 and np.abs(np.array(t.bt[:s]) - bt).max() < 1e-15
        assert not lib_a[s:].any() and not lib_at[s:].any()


def test_imex_entry_points_reject_bad_arguments_without_gpu():
    lib = hdg.load_library()
    t = hdg.HdgImexTableau()
    assert lib.hdg_imex_tableau_get(7, 0.5, ctypes.byref(t)) == hdg.HDG_EINVAL
    assert lib.hdg_imex_tableau_get(hdg.HDG_IMEX_THETA, 0.0, ctypes.byref(t)) == hdg.HDG_EINVAL
    n = ctypes.c_int64()
    assert lib.hdg_imex_work_size(None, ctypes.byref(t), 1, ctypes.byref(n)) == hdg.HDG_EINVAL
    assert lib.hdg_imex_run(None, ctypes.byref(t), 0.1, 0.0, 1, 1, None, None, None, None) == hdg.HDG_EINVAL
    assert lib.hdg_dg_tendency(None, 1, 0.1, None, None, None) == hdg.HDG_EINVAL
    assert lib.hdg_dgs_setup(None, None, 0, None) == hdg.HDG_EINVAL
    assert lib.hdg_dgs_solve(None, 1, None, None, None, None) == hdg.HDG_EINVAL


def test_bandwidth_probes_check_arguments_before_any_launch():
    """Every rejected call fails its host-side check, so no pointer here is used."""
    lib = hdg.load_library()
    P = ctypes.c_void_p
    assert [lib.hdg_stream_read_blocks(n) for n in (0, 1, 2048, 2049, -3)] == [0, 1, 1, 2, 0]
    E = hdg.HDG_EINVAL
    assert lib.hdg_stream_triad(None, None, 1.0, None, 4, None) == E
    assert lib.hdg_stream_triad(P(4096), P(8192), 1.0, P(65536), -1, None) == E
    assert lib.hdg_stream_triad(P(4096 + 8), P(1 << 20), 1.0, P(1 << 21), 4, None) == E  # misaligned
    assert lib.hdg_stream_triad(P(4096), P(8192), 1.0, P(4096 + 16), 4, None) == E  # a overlaps b
    assert lib.hdg_stream_read(None, 4, P(4096), 1, None) == E
    assert lib.hdg_stream_read(P(4096), 4097, P(1 << 20), 2, None) == E  # partial too short
    assert lib.hdg_stream_read(P(4096 + 8), 4, P(1 << 20), 1, None) == E  # misaligned
    assert lib.hdg_stream_read(P(4096), 4096, P(4096 + 64), 2, None) == E  # partial overlaps src
    assert lib.hdg_stream_triad(None, None, 1.0, None, 0, None) == hdg.HDG_OK  # empty: nothing launched
    assert lib.hdg_stream_read(None, 0, None, 0, None) == hdg.HDG_OK
