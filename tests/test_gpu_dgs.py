"""GPU parity of the non-hybridised DG baseline (native DG section) against the
oracle: the stage operator, the three-step approximate Schur-complement
preconditioner, and solves against the direct DG solution and the HDG path."""
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


CASES = {
    "torus8_p1": (lambda: hi.torus_hierarchy(8, 4), 1, 0.5, 1.3, 0.8, 1.0, 0.0),
    "torus8_p2": (lambda: hi.torus_hierarchy(8, 4), 2, 0.5, 1.3, 0.8, 1.0, 0.0),
    "torus8_p3": (lambda: hi.torus_hierarchy(8, 4), 3, 0.5, 1.3, 0.8, 0.0, 0.0),
    "sphere2_p2": (lambda: hi.icosphere_hierarchy(2), 2, 0.3, 1.0, 1.0, 0.5, 0.3),
}


def build(case, nb=1):
    from oracle.dgschur import DgApproxSchur
    from paper_2004_09389_amd.hdg import HdgSolver
    mk, p, dt, g, H, f0, om = CASES[case]
    hier = mk()
    print(f"[dgs] {case} nb={nb}", flush=True)
    s = HdgSolver(hier, p, dt, g, H, f0, om, rtol=1e-11, maxit=300, max_rhs=nb)
    s.dgs_setup()
    o = DgApproxSchur(hier, p, dt, g, H, f0, om)
    return s, o, hier


@pytest.mark.parametrize("case", list(CASES))
def test_operator_and_preconditioner_match_oracle(case):
    nb = 2
    s, o, hier = build(case, nb)
    x = np.random.default_rng(5).standard_normal((hier.fine.n_cell, 3, s.n_loc, nb))
    y = host(s.dgs_apply(to_dev(x)))
    z = host(s.dgs_precondition(to_dev(x)))
    for k in range(nb):
        xv = x[..., k].ravel()
        assert rel(y[..., k].ravel(), o.A @ xv) < 1e-12
        assert rel(z[..., k].ravel(), o.precondition(xv)) < 1e-10
    s.close()


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("nb", [1, 3])
def test_solve_matches_the_direct_dg_solution(case, nb):
    s, o, hier = build(case, nb)
    r = hi.iid_rhs(hier.fine, s.p, 8, nrhs=nb)
    q, info = s.dgs_solve(to_dev(r))
    q = host(q)
    for k in range(nb):
        ref = o.to_cell(o.direct(o.rhs(r[..., k])))
        assert rel(q[..., k], ref) < 1e-9
        assert info[k].status == 0 and info[k].rel_res <= 1e-11
    _, its = o.gmres(o.rhs(r[..., 0]), rtol=1e-11)
    assert abs(info[0].iters - its) <= max(2, its // 10)
    s.close()


def test_baseline_and_hdg_give_the_same_stage_solution():
    """The two solvers of the same implicit stage (HDG == DG, Eq. linear_hybridized)."""
    s, o, hier = build("torus8_p2")
    r = to_dev(hi.iid_rhs(hier.fine, 2, 9))
    q_dg, _ = s.dgs_solve(r)
    q_hdg, _, _ = s.step(r)
    assert rel(host(q_dg), host(q_hdg)) < 1e-9
    s.close()


def _paper_iterations():
    import os
    rows = []
    for line in open(os.path.join(os.path.dirname(__file__), "golden", "iterations_linear.txt")):
        if line.startswith("#") or not line.strip():
            continue
        rows.append([None if t == "-" else float(t) for t in line.split()])
    return rows


@pytest.mark.parametrize("p", [1, 3])
def test_iterations_at_the_papers_courant_number(p):
    """Like-for-like with the paper's iteration table for the linear problem
    (DG column: 12-14 at p = 1, 13-15.5 at p = 3, HDG 7-8): flat bathymetry,
    f = 0, rtol 1e-8, the implicit stage of its ARS2(2,3,2) stepper
    (kappa = c gamma dt, dt = (2 / (2p + 1)) h, gamma = 1 - 1/sqrt 2) on the
    32^2 ... 128^2 tori.  The sub-solves differ (cell-block inverses and a
    Galerkin two-level cycle instead of ILU and GAMG) and the stop is on the
    true residual, so the counts are bounded, not matched."""
    import torch
    from paper_2004_09389_amd.hdg import HdgSolver
    table = _paper_iterations()
    col = 1 if p == 1 else 3
    lo = min(r[col] for r in table)
    hi_ = max(r[col] for r in table)
    gamma = 1.0 - 1.0 / np.sqrt(2.0)
    its, hdg_its = [], []
    for n in (32, 64, 128):
        hier = hi.torus_hierarchy(n, min(32, n))
        s = HdgSolver(hier, p, gamma * (2.0 / (2 * p + 1)) / n, 1.0, 1.0, 0.0, 0.0, maxit=400, p1_tail_max=0)
        s.dgs_setup()
        r = torch.from_numpy(hi.fourier_rhs_torus(hier.fine, p, 100)).cuda()
        _, info = s.dgs_solve(r)
        assert info[0].status == 0
        its.append(info[0].iters)
        hdg_its.append(s.step(r)[2][0].iters)
        s.close()
    print(f"p={p}: DG iterations {its} (paper {lo}-{hi_}), HDG {hdg_its}")
    assert lo - 3 <= min(its) and max(its) <= hi_ + 3 and max(its) - min(its) <= 3
    assert min(its) > max(hdg_its)


def test_solve_is_deterministic_and_reports_non_convergence():
    """Two solves of the same input give identical bits; a maxit too small for
    rtol returns HDG_ENOTCONV with the final true residual in info."""
    from paper_2004_09389_amd.hdg import HDG_ENOTCONV, HdgError, HdgSolver
    hier = hi.torus_hierarchy(8, 4)
    s = HdgSolver(hier, 2, 0.5, 1.3, 0.8, 1.0, 0.0, rtol=1e-10, maxit=300)
    s.dgs_setup()
    r = to_dev(hi.iid_rhs(hier.fine, 2, 12))
    q1, _ = s.dgs_solve(r)
    q2, _ = s.dgs_solve(r)
    assert np.array_equal(host(q1), host(q2))
    s.close()
    s = HdgSolver(hier, 2, 0.5, 1.3, 0.8, 1.0, 0.0, rtol=1e-12, maxit=3)
    s.dgs_setup()
    with pytest.raises(HdgError):
        s.dgs_solve(r)
    q, info = s.dgs_solve(r, allow_notconv=True)
    assert info[0].status == HDG_ENOTCONV and 1e-12 < info[0].rel_res < 1.0
    s.close()
