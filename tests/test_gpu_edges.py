"""Edge cases of the C ABI on the GPU: argument errors caught on the host
before any launch, zero right-hand sides (alone and inside a batch), the
largest batch (64 right-hand sides), the smallest mesh, and a clockwise cell
reported by the setup's per-cell condensation."""
import numpy as np
import pytest

import hdg_inputs as hi

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def make(n=6, p=2, **opts):
    from paper_2004_09389_amd.hdg import HdgSolver
    return HdgSolver(hi.torus_hierarchy(n, n // 2 if n > 2 else 1), p, 0.4, 1.0, 1.0, 0.5, 0.0, **opts)


def test_argument_errors_are_reported():
    import torch
    from paper_2004_09389_amd.hdg import HDG_EINVAL, HdgError, HdgSolver
    with pytest.raises(HdgError) as e:
        HdgSolver(hi.torus_hierarchy(4, 2), 4, 0.4)
    assert e.value.code == HDG_EINVAL and "degree" in str(e.value)
    with pytest.raises(HdgError):
        HdgSolver(hi.torus_hierarchy(4, 2), 2, -1.0)
    s = make(max_rhs=2)
    x = s.trace_zeros(3)
    with pytest.raises(ValueError) as e:
        s.trace_apply(x)                       # nrhs above max_rhs: the binding rejects it ...
    assert "max_rhs" in str(e.value)
    import ctypes
    y = s.trace_zeros(3)                       # ... and so does the C ABI when called directly
    rc = s.lib.hdg_trace_apply(s.ctx, 3, 0, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), None)
    assert rc == HDG_EINVAL and "max_rhs" in s.lib.hdg_last_error().decode()
    # an empty batch (nrhs = 0) is an argument error at every entry point, not a no-op launch
    px, py = ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())
    assert s.lib.hdg_trace_apply(s.ctx, 0, 0, px, py, None) == HDG_EINVAL
    assert s.lib.hdg_mg_vcycle(s.ctx, 0, 0, px, py, None) == HDG_EINVAL
    assert s.lib.hdg_solve(s.ctx, 0, px, py, None, None) == HDG_EINVAL
    q = s.cell_zeros(1)
    assert s.lib.hdg_condense(s.ctx, 0, ctypes.c_void_p(q.data_ptr()), py, None) == HDG_EINVAL
    assert s.lib.hdg_stage_solve(s.ctx, 0, ctypes.c_void_p(q.data_ptr()), py, ctypes.c_void_p(q.data_ptr()),
                                 None, None) == HDG_EINVAL
    assert "nrhs" in s.lib.hdg_last_error().decode()
    # a trace buffer that is not 16-byte aligned
    flat = torch.zeros(s.n_facet * s.m + 1, dtype=torch.float64, device="cuda")
    mis = flat[1:].view(s.n_facet, s.m, 1)
    with pytest.raises(HdgError) as e:
        s.trace_apply(mis)
    assert "aligned" in str(e.value)
    with pytest.raises(HdgError):
        s.set_tuning(rhs_block=3)
    with pytest.raises(HdgError):
        s.set_tuning(mlp_samples_per_lane=5)
    # the context still works after the rejected calls
    y = host(s.trace_apply(to_dev(np.ones((s.n_facet, s.m, 1)))))
    assert np.all(np.isfinite(y))


def test_zero_right_hand_sides():
    """A zero right-hand side converges at once to lam = 0, alone and as one
    column of a batch whose other columns iterate."""
    from oracle.hdg import HdgOracle
    s = make(max_rhs=3, krylov=2, rtol=1e-11)
    lam, info = s.solve(s.trace_zeros(1))
    assert info[0].iters == 0 and info[0].status == 0 and np.all(host(lam) == 0)
    hier = hi.torus_hierarchy(6, 3)
    o = HdgOracle(hier.fine, 2, 0.4, 1.0, 1.0, 0.5, 0.0)
    r = hi.iid_rhs(hier.fine, 2, 5, nrhs=3)
    r[..., 1] = 0.0
    rhat = s.condense(to_dev(r))
    lam, info = s.solve(rhat)
    lam = host(lam)
    assert np.all(lam[..., 1] == 0) and all(i.status == 0 for i in info)
    for k in (0, 2):
        assert rel(lam[..., k].ravel(), o.solve(r[..., k])[1]) < 1e-8


def test_largest_batch():
    """64 right-hand sides (the maximum) through condense, solve and recover;
    every column against the oracle."""
    from oracle.hdg import HdgOracle
    hier = hi.torus_hierarchy(6, 3)
    s = make(max_rhs=64, rtol=1e-11)
    o = HdgOracle(hier.fine, 2, 0.4, 1.0, 1.0, 0.5, 0.0)
    r = hi.iid_rhs(hier.fine, 2, 9, nrhs=64)
    q, lam, info = s.step(to_dev(r))
    q, lam = host(q), host(lam)
    assert all(i.status == 0 for i in info)
    for k in (0, 17, 63):
        q_ref, lam_ref = o.solve(r[..., k])
        assert rel(lam[..., k].ravel(), lam_ref) < 1e-9
        for fld in range(3):
            assert rel(q[:, fld, :, k], q_ref[:, fld]) < 1e-9


def _exact_cases():
    import sys
    import os
    sys.path.insert(0, os.path.dirname(__file__))
    from test_oracle_exact import CASES
    return CASES


@pytest.mark.parametrize("c", _exact_cases(), ids=lambda c: f"p{c['p']}-f{c['f']}-tau{c['tau']}")
@pytest.mark.parametrize("precision", ["fp64", "fp64-multi-launch", "mixed"])
def test_two_cell_mesh_equals_exact_solution(c, precision):
    """The smallest periodic mesh (one square, two cells, three facets): the
    library's condense / solve / recover against the stage's exact solution
    computed over Q(sqrt 2) (tests/golden/exact_torus1.txt): FP64 to 1e-10,
    the mixed-precision path to 1e-8, every field separately."""
    from paper_2004_09389_amd.hdg import HDG_FP64, HDG_MIXED, HdgSolver
    hier = hi.torus_hierarchy(1, 1)
    prec = HDG_MIXED if precision == "mixed" else HDG_FP64
    s = HdgSolver(hier, c["p"], float(c["dt"]), float(c["g"]), float(c["H"]), float(c["f"]), 0.0,
                  float(c["tau"]), rtol=1e-11 if precision == "mixed" else 1e-13, precision=prec,
                  persistent=0 if precision == "fp64-multi-launch" else 1)
    q, lam, info = s.step(to_dev(c["r"][..., None]))
    assert info[0].status == 0
    tol = 1e-8 if precision == "mixed" else 1e-10
    assert rel(host(lam)[..., 0].ravel(), c["lam"]) < tol
    for fld in range(3):
        assert rel(host(q)[:, fld, :, 0], c["q"][:, fld]) < tol
    s.close()


def test_not_converged_and_breakdown_are_reported():
    """maxit reached: HDG_ENOTCONV with the info filled; a non-finite
    right-hand side: HDG_EBREAKDOWN, the context still usable afterwards."""
    import torch
    from paper_2004_09389_amd.hdg import HDG_EBREAKDOWN, HDG_ENOTCONV, HdgError
    hier = hi.torus_hierarchy(6, 3)
    s = make(maxit=2, rtol=1e-12, krylov=2)
    r = to_dev(hi.iid_rhs(hier.fine, 2, 3))
    rhat = s.condense(r)
    lam, info = s.solve(rhat, allow_notconv=True)
    assert info[0].status == HDG_ENOTCONV and info[0].iters == 2 and info[0].rel_res > 1e-12
    bad = rhat.clone()
    bad[0, 0, 0] = float("nan")
    with pytest.raises(HdgError) as e:
        s.solve(bad)
    assert e.value.code == HDG_EBREAKDOWN
    lam, info = s.solve(rhat, allow_notconv=True)
    assert info[0].status == HDG_ENOTCONV and np.all(np.isfinite(host(lam)))


def test_mixed_breakdown_leaves_the_context_in_fp64():
    """A non-finite right-hand side in the FP32 inner solve of HDG_MIXED_IR and in
    the mixed solve reports HDG_EBREAKDOWN; afterwards the FP64 entry points
    (apply, V-cycle, solve) still read and write FP64 vectors."""
    from oracle.hdg import HdgOracle
    from paper_2004_09389_amd.hdg import HDG_EBREAKDOWN, HDG_MIXED, HDG_MIXED_IR, HdgError
    hier = hi.torus_hierarchy(6, 3)
    o = HdgOracle(hier.fine, 2, 0.4, 1.0, 1.0, 0.5, 0.0)
    for prec in (HDG_MIXED_IR, HDG_MIXED):
        s = make(precision=prec, krylov=2, rtol=1e-10)
        r = hi.iid_rhs(hier.fine, 2, 7)
        rhat = s.condense(to_dev(r))
        bad = rhat.clone()
        bad[1, 0, 0] = float("inf")
        with pytest.raises(HdgError) as e:
            s.solve(bad)
        assert e.value.code == HDG_EBREAKDOWN
        x = np.random.default_rng(2).standard_normal((s.n_facet, s.m, 1))
        assert rel(host(s.trace_apply(to_dev(x)))[..., 0].ravel(), o.apply(x[..., 0].ravel())) < 1e-12
        lam, info = s.solve(rhat)
        assert info[0].status == 0
        assert rel(host(lam)[..., 0].ravel(), o.solve(r[..., 0])[1]) < 1e-8
        s.close()


def test_ir_inner_rtol_is_validated():
    from paper_2004_09389_amd.hdg import HdgError
    with pytest.raises(HdgError) as e:
        make(ir_inner_rtol=1.5)
    assert "ir_inner_rtol" in str(e.value)


@pytest.mark.parametrize("p", [1, 3])
def test_inverted_cell_is_reported(p):
    """A clockwise cell (one vertex of the 4 x 4 torus moved across the
    opposite edge of a neighbouring cell): the per-cell condensation flags the
    non-positive area and setup fails with that message; a valid mesh set up
    afterwards still solves."""
    from paper_2004_09389_amd.hdg import HdgError, HdgSolver
    hier = hi.torus_hierarchy(4, 4)
    m = hier.fine
    m.vert_xyz = m.vert_xyz.copy()
    # vertex (1, 1) to x = -h/2: the cell (0, 0), (1, 1), (0, 1) of the first square turns clockwise
    m.vert_xyz[1 * 4 + 1, 0] = -0.5 * m.period / 4
    with pytest.raises(HdgError, match="non-positive area"):
        HdgSolver(hier, p, 0.4, 1.0, 1.0, 0.5, 0.0)
    s = make(4, p)
    r = np.random.default_rng(3).standard_normal((s.n_cell, 3, s.n_loc, 1))
    q, lam, info = s.step(to_dev(r))
    assert info[0].status == 0
    s.close()
