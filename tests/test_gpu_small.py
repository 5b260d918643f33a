"""The persistent single-launch solve of small trace systems (one workgroup per
right-hand side, every trace and P1 vector in LDS): hdg_stage_solve (Steps
1-3 in one launch) and hdg_solve on small contexts, against the oracle's
direct solves and the exact two-cell solution, and against the multi-launch
solve of the same context (opt.persistent = 0)."""
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


def solver(hier, p, dt, f0=0.0, omega=0.0, g=1.0, H=1.0, **opts):
    from paper_2004_09389_amd.hdg import HdgSolver
    return HdgSolver(hier, p, dt, g, H, f0, omega, **opts)


def check_vs_oracle(q, lam, r, mesh, p, dt, f0=0.0, omega=0.0, g=1.0, H=1.0, tol=1e-10):
    from oracle.hdg import HdgOracle
    o = HdgOracle(mesh, p, dt, g, H, f0, omega)
    for k in range(r.shape[-1]):
        q_ref, lam_ref = o.solve(r[..., k])
        assert rel(lam[..., k].ravel(), lam_ref) < tol, k
        for fld in range(3):
            assert rel(q[:, fld, :, k], q_ref[:, fld]) < tol, (k, fld)


def test_torus8_p1_qualifies_and_matches_the_oracle():
    """8x8 torus (128 cells), p = 1, f = 0, Courant 4: the context qualifies
    for the persistent solve; Steps 1-3 in one launch equal the oracle's direct
    solve (PCG, rtol 1e-12)."""
    hier = hi.torus_hierarchy(8, 4)
    s = solver(hier, 1, 0.5, rtol=1e-12)
    assert s.sizes.persistent == 1
    r = hi.iid_rhs(hier.fine, 1, 0, nrhs=1)
    q, lam, info = s.stage_solve(to_dev(r))
    assert info[0].status == 0 and info[0].rel_res <= 1e-12 and 5 <= info[0].iters <= 20
    check_vs_oracle(host(q), host(lam), r, hier.fine, 1, 0.5)


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("f0", [0.0, 1.0])
def test_stage_solve_every_degree(p, f0):
    """PCG (f = 0) and flexible GMRES (f != 0) inside the launch, p = 1..3,
    three right-hand sides (one workgroup each)."""
    hier = hi.torus_hierarchy(8, 4)
    s = solver(hier, p, 0.5, f0=f0, rtol=1e-12, max_rhs=3)
    assert s.sizes.persistent == 1
    r = hi.iid_rhs(hier.fine, p, 10 + p, nrhs=3)
    q, lam, info = s.stage_solve(to_dev(r))
    assert all(i.status == 0 and i.rel_res <= 1e-12 for i in info)
    check_vs_oracle(host(q), host(lam), r, hier.fine, p, 0.5, f0=f0)


@pytest.mark.parametrize("f0", [0.0, 0.7])
def test_solve_equals_multi_launch_solve(f0):
    """hdg_solve through the persistent kernel and through the multi-launch
    solve (opt.persistent = 0) of the same problem agree to 1e-11, and the
    persistent solve keeps a nonzero initial guess."""
    hier = hi.torus_hierarchy(8, 4)
    p = 2
    a = solver(hier, p, 0.5, f0=f0, rtol=1e-12, max_rhs=2)
    b = solver(hier, p, 0.5, f0=f0, rtol=1e-12, max_rhs=2, persistent=0)
    assert a.sizes.persistent == 1 and b.sizes.persistent == 0
    r = to_dev(hi.iid_rhs(hier.fine, p, 21, nrhs=2))
    rhat = a.condense(r)
    guess = to_dev(0.1 * hi.iid_trace(a.n_facet, p, 5, nrhs=2))
    la, ia = a.solve(rhat, guess.clone())
    lb, ib = b.solve(rhat, guess.clone())
    assert all(i.status == 0 for i in ia + ib)
    assert rel(host(la), host(lb)) < 1e-11
    # the same preconditioner: at a tolerance far from round-off (no true-residual
    # restarts) the iteration counts agree, up to the one iteration the multi-launch
    # solve runs past convergence because it checks convergence one iteration late
    a8 = solver(hier, p, 0.5, f0=f0, rtol=1e-8, max_rhs=2)
    b8 = solver(hier, p, 0.5, f0=f0, rtol=1e-8, max_rhs=2, persistent=0)
    _, i8a = a8.solve(rhat)
    _, i8b = b8.solve(rhat)
    for x, y in zip(i8a, i8b):
        assert x.refinements == 1 and 0 <= y.iters - x.iters <= 1, (x.iters, y.iters)


def test_sphere_with_latitude_dependent_coriolis():
    """Icosahedral sphere, level 1 (80 cells), p = 2, f = 2 Omega sin(lat): FGMRES in the launch."""
    hier = hi.icosphere_hierarchy(1, 6.371e6)
    s = solver(hier, 2, 1800.0, omega=7.292e-5, g=9.81, H=5960.0, rtol=1e-12, max_rhs=2)
    assert s.sizes.persistent == 1
    r = hi.iid_rhs(hier.fine, 2, 31, nrhs=2)
    q, lam, info = s.stage_solve(to_dev(r))
    assert all(i.status == 0 for i in info)
    check_vs_oracle(host(q), host(lam), r, hier.fine, 2, 1800.0, omega=7.292e-5, g=9.81, H=5960.0)


def test_large_batch_and_repeatability():
    """16 right-hand sides in one launch; a second call gives identical bits."""
    hier = hi.torus_hierarchy(8, 4)
    s = solver(hier, 1, 0.5, rtol=1e-10, max_rhs=16)
    r = hi.iid_rhs(hier.fine, 1, 40, nrhs=16)
    q1, l1, info = s.stage_solve(to_dev(r))
    q2, l2, _ = s.stage_solve(to_dev(r))
    assert all(i.status == 0 and i.rel_res <= 1e-10 for i in info)
    assert np.array_equal(host(q1), host(q2)) and np.array_equal(host(l1), host(l2))
    check_vs_oracle(host(q1)[..., ::5], host(l1)[..., ::5], r[..., ::5], hier.fine, 1, 0.5, tol=1e-8)


def test_not_converged_and_breakdown():
    """maxit reached: HDG_ENOTCONV with the info filled; a NaN right-hand side:
    HDG_EBREAKDOWN; the context works afterwards."""
    from paper_2004_09389_amd.hdg import HDG_EBREAKDOWN, HDG_ENOTCONV, HdgError
    hier = hi.torus_hierarchy(8, 4)
    s = solver(hier, 1, 0.5, rtol=1e-14, maxit=2, max_rhs=2)
    r = hi.iid_rhs(hier.fine, 1, 50, nrhs=2)
    q, lam, info = s.stage_solve(to_dev(r), allow_notconv=True)
    assert all(i.status == HDG_ENOTCONV and i.iters == 2 and i.rel_res > 1e-14 for i in info)
    bad = r.copy()
    bad[3, 0, 0, 1] = np.nan
    with pytest.raises(HdgError) as e:
        s.stage_solve(to_dev(bad))
    assert e.value.code == HDG_EBREAKDOWN
    s2 = solver(hier, 1, 0.5, rtol=1e-12)
    q, lam, info = s2.stage_solve(to_dev(r[..., :1]))
    assert info[0].status == 0
    check_vs_oracle(host(q), host(lam), r[..., :1], hier.fine, 1, 0.5)


def test_multi_launch_stage_solve():
    """A context too large for one workgroup (32x32 torus, p = 3) runs
    hdg_stage_solve as condense / solve / recover with the same result."""
    hier = hi.torus_hierarchy(32, 8)
    s = solver(hier, 3, 0.1, f0=0.5, rtol=1e-12)
    assert s.sizes.persistent == 0
    r = hi.iid_rhs(hier.fine, 3, 60)
    q, lam, info = s.stage_solve(to_dev(r))
    q2, lam2, _ = s.step(to_dev(r))
    assert info[0].status == 0
    assert rel(host(lam), host(lam2)) < 1e-10 and rel(host(q), host(q2)) < 1e-10
