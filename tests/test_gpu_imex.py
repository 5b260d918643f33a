"""GPU parity of IMEX time stepping (time discretisation and IMEX methods
sections) against the oracle: the explicit flux evaluation, every tableau
(Theta at 1/2 and 0.55, ARS2(2,3,2), SSP2(3,2,2), ARS3(4,4,3)) with both
fluxes, batches, and the stationary vortex's Delta_2 convergence through the
HIP path.

The oracle evaluates every flux term explicitly with its own assembled DG
operator and solves each stage directly; the library takes the flux terms of
implicit stages from the stage equations and solves them iteratively, so the
two agree to the stage solver's tolerance (rtol 1e-12 here)."""
import math

import numpy as np
import pytest

import hdg_inputs as hi

pytestmark = pytest.mark.gpu

G, H = 1.3, 0.8


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def solver(hier, p, dt_stage, flux="upwind", f0=0.0, g=G, h=H, **opts):
    from paper_2004_09389_amd.hdg import HDG_FLUX_LF, HDG_FLUX_UPWIND, HdgSolver
    print(f"[imex] solver n={hier.fine.n_cell} p={p} dt={dt_stage:.4g} flux={flux} f0={f0} {opts}", flush=True)
    fl = HDG_FLUX_LF if flux == "lf" else HDG_FLUX_UPWIND
    opts.setdefault("rtol", 1e-12)
    opts.setdefault("maxit", 400)
    return HdgSolver(hier, p, dt_stage, g, h, f0, 0.0, flux=fl, **opts)


@pytest.mark.parametrize("flux", ["upwind", "lf"])
@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("f0", [0.0, 1.5])
def test_dg_tendency_matches_oracle(flux, p, f0):
    """dt M^-1 (L + N_c) q against the oracle's assembled DG operator, at two
    right-hand sides; the context's own Coriolis term is included."""
    from oracle.imex import LinearSwe
    n, nb, dt = 8, 2, 0.07
    m = hi.torus(n)
    s = solver(hi.torus_hierarchy(n, 4), p, 0.3, flux, f0=f0, max_rhs=nb)
    swe = LinearSwe(m, p, g=G, H=H, f=f0, flux=flux)
    q = hi.iid_rhs(m, p, 31, nrhs=nb)
    got = host(s.dg_tendency(to_dev(q), dt))
    x = swe.to_vec(q)
    ref = swe.from_vec(dt * swe._mass.solve((swe.L + swe.N) @ x), m.n_cell)
    for k in range(nb):
        assert rel(got[..., k], ref[..., k]) < 1e-11
    s.close()


def test_dg_tendency_on_the_sphere():
    """The trace uses each cell's own frame normal on the piecewise-flat sphere."""
    from oracle.imex import LinearSwe
    hier = hi.icosphere_hierarchy(2)
    m = hier.fine
    s = solver(hier, 2, 0.2, g=1.0, h=1.0)
    swe = LinearSwe(m, 2, g=1.0, H=1.0, f=0.0)
    q = hi.iid_rhs(m, 2, 5)
    got = host(s.dg_tendency(to_dev(q), 0.2))
    ref = swe.tendency(q, 0.2)
    assert rel(got, ref) < 1e-11
    s.close()


CASES = [("theta", 0.5), ("theta", 0.55), ("ars232", None), ("ssp322", None), ("ars443", None)]


@pytest.mark.parametrize("flux", ["upwind", "lf"])
@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("method,theta", CASES)
def test_imex_steps_match_oracle(method, theta, p, flux):
    """Three steps from random coefficients with explicit Coriolis (f = 2)."""
    from oracle.imex import LinearSwe, tableau
    from paper_2004_09389_amd.hdg import imex_gamma, imex_tableau
    n, dt, f, steps = 8, 0.04, 2.0, 3
    m = hi.torus(n)
    tab = imex_tableau(method, theta if theta is not None else 0.5)
    s = solver(hi.torus_hierarchy(n, 4), p, imex_gamma(tab) * dt, flux)
    q0 = hi.iid_rhs(m, p, 11)
    q = to_dev(q0)
    info = s.imex_run(tab, dt, f, q, steps)
    assert info.steps == steps and info.status == 0
    assert info.solves == steps * sum(tab.at[i][i] != 0 for i in range(tab.stages))
    swe = LinearSwe(m, p, g=G, H=H, f=f, flux=flux)
    ref = swe.run(tableau(method, theta) if theta is not None else tableau(method), dt, steps, q0)
    assert rel(host(q), ref) < 1e-9
    s.close()


@pytest.mark.parametrize("method", ["theta", "ars232"])
def test_imex_batch_matches_oracle_per_column(method):
    """Four right-hand sides in one run, each against its own oracle run; the
    run split into two calls (the carried flux term re-evaluated) agrees."""
    from oracle.imex import LinearSwe, tableau
    from paper_2004_09389_amd.hdg import imex_gamma, imex_tableau
    n, p, dt, f, nb = 8, 2, 0.05, 1.0, 4
    m = hi.torus(n)
    tab = imex_tableau(method, 0.5)
    s = solver(hi.torus_hierarchy(n, 4), p, imex_gamma(tab) * dt, max_rhs=nb)
    q0 = hi.iid_rhs(m, p, 40, nrhs=nb)
    q = to_dev(q0)
    s.imex_run(tab, dt, f, q, 4)
    q2 = to_dev(q0)
    s.imex_run(tab, dt, f, q2, 2)
    s.imex_run(tab, dt, f, q2, 2)
    swe = LinearSwe(m, p, g=G, H=H, f=f)
    for k in range(nb):
        ref = swe.run(tableau(method, 0.5), dt, 4, q0[..., k:k + 1])[..., 0]
        assert rel(host(q)[..., k], ref) < 1e-9
        assert rel(host(q2)[..., k], ref) < 1e-9
    s.close()


def test_imex_rejects_a_mismatched_context():
    """The context must be set up for gamma dt and without implicit Coriolis."""
    from paper_2004_09389_amd.hdg import HdgError, imex_tableau
    n, p = 4, 1
    tab = imex_tableau("ars232")
    s = solver(hi.torus_hierarchy(n, 4), p, 0.1)
    q = to_dev(hi.iid_rhs(hi.torus(n), p, 1))
    with pytest.raises(HdgError):
        s.imex_run(tab, 0.1, 0.0, q, 1)          # context dt is not gamma * 0.1
    s.close()
    s = solver(hi.torus_hierarchy(n, 4), p, tab.at[1][1] * 0.1, f0=1.0)
    with pytest.raises(HdgError):
        s.imex_run(tab, 0.1, 0.0, q, 1)          # implicit Coriolis in the context
    s.close()


def test_vortex_converges_at_the_papers_rate_through_the_gpu():
    """The stationary vortex (p = 1, n = 16 and 32, ARS2(2,3,2), the paper's
    time step, T = 1/2): Delta_2 equals the oracle's and drops at least as
    h^(3/2); the stage solves take a handful of iterations."""
    from oracle.imex import LinearSwe, l2_error, tableau
    from paper_2004_09389_amd.hdg import imex_gamma, imex_tableau
    v = hi.Vortex()
    tab = imex_tableau("ars232")
    errs = []
    for n in (16, 32):
        m = hi.torus(n)
        dt, steps = hi.paper_time_step(n, 1)
        s = solver(hi.torus_hierarchy(n, 4), 1, imex_gamma(tab) * dt, g=v.c_g, h=v.c_g, rtol=1e-10)
        q0 = hi.vortex_coefficients(m, 1, v)
        q = to_dev(q0)
        info = s.imex_run(tab, dt, v.f, q, steps)
        assert info.iters_max <= 20
        swe = LinearSwe(m, 1, g=v.c_g, H=v.c_g, f=v.f)
        e = l2_error(swe, host(q)[..., 0], lambda xy: v.state(xy))
        e_ref = l2_error(swe, swe.run(tableau("ars232"), dt, steps, q0)[..., 0], lambda xy: v.state(xy))
        assert abs(e - e_ref) < 1e-6 * e_ref
        errs.append(e)
        s.close()
    assert math.log2(errs[0] / errs[1]) >= 1.5


@pytest.mark.parametrize("precision", ["mixed", "mixed_ir"])
@pytest.mark.parametrize("method", ["theta", "ars443"])
def test_imex_with_mixed_precision_stage_solves(method, precision):
    """Stage solves in HDG_MIXED / HDG_MIXED_IR (FP64 true residual to rtol
    1e-11): the steps agree with the oracle to 1e-8."""
    from oracle.imex import LinearSwe, tableau
    from paper_2004_09389_amd.hdg import HDG_MIXED, HDG_MIXED_IR, imex_gamma, imex_tableau
    n, p, dt, f, steps = 16, 3, 0.03, 2.0, 2
    m = hi.torus(n)
    tab = imex_tableau(method, 0.5)
    prec = HDG_MIXED if precision == "mixed" else HDG_MIXED_IR
    s = solver(hi.torus_hierarchy(n, 4), p, imex_gamma(tab) * dt, precision=prec, rtol=1e-11, krylov=2)
    q0 = hi.iid_rhs(m, p, 17)
    q = to_dev(q0)
    info = s.imex_run(tab, dt, f, q, steps)
    assert info.status == 0 and info.rel_res_max <= 1e-11
    ref = LinearSwe(m, p, g=G, H=H, f=f).run(tableau(method, 0.5), dt, steps, q0)
    assert rel(host(q), ref) < 1e-8
    s.close()


def test_imex_on_the_sphere_with_an_f_plane():
    """Icosahedral sphere (level 2, p = 2), ARS2(2,3,2), constant explicit f in
    every cell's frame, against the oracle."""
    from oracle.imex import LinearSwe, tableau
    from paper_2004_09389_amd.hdg import imex_gamma, imex_tableau
    hier = hi.icosphere_hierarchy(2)
    m = hier.fine
    dt, f, steps = 0.05, 1.5, 3
    tab = imex_tableau("ars232")
    s = solver(hier, 2, imex_gamma(tab) * dt, g=1.0, h=1.0)
    q0 = hi.iid_rhs(m, 2, 23)
    q = to_dev(q0)
    info = s.imex_run(tab, dt, f, q, steps)
    assert info.status == 0
    ref = LinearSwe(m, 2, g=1.0, H=1.0, f=f).run(tableau("ars232"), dt, steps, q0)
    assert rel(host(q), ref) < 1e-9
    s.close()


def test_imex_lax_friedrichs_batch():
    """Lax-Friedrichs flux, three right-hand sides, ARS3(4,4,3)."""
    from oracle.imex import LinearSwe, tableau
    from paper_2004_09389_amd.hdg import imex_gamma, imex_tableau
    n, p, dt, f, nb = 8, 2, 0.04, 1.0, 3
    m = hi.torus(n)
    tab = imex_tableau("ars443")
    s = solver(hi.torus_hierarchy(n, 4), p, imex_gamma(tab) * dt, "lf", max_rhs=nb)
    q0 = hi.iid_rhs(m, p, 29, nrhs=nb)
    q = to_dev(q0)
    s.imex_run(tab, dt, f, q, 2)
    swe = LinearSwe(m, p, g=G, H=H, f=f, flux="lf")
    for k in range(nb):
        assert rel(host(q)[..., k], swe.run(tableau("ars443"), dt, 2, q0[..., k:k + 1])[..., 0]) < 1e-9
    s.close()


@pytest.mark.parametrize("p", [2, 3])
def test_vortex_rate_at_higher_degree_through_the_gpu(p):
    """The stationary vortex at p = 2, 3 (n = 16, 32; ARS2(2,3,2), the paper's
    time step, T = 1/2): Delta_2 drops at least as h^(p + 1/2) between the two
    meshes and equals the oracle's on the coarser one."""
    from oracle.imex import LinearSwe, l2_error, tableau
    from paper_2004_09389_amd.hdg import imex_gamma, imex_tableau
    v = hi.Vortex()
    tab = imex_tableau("ars232")
    errs = []
    for n in (16, 32):
        m = hi.torus(n)
        dt, steps = hi.paper_time_step(n, p)
        s = solver(hi.torus_hierarchy(n, 4), p, imex_gamma(tab) * dt, g=v.c_g, h=v.c_g, rtol=1e-10)
        q0 = hi.vortex_coefficients(m, p, v)
        q = to_dev(q0)
        info = s.imex_run(tab, dt, v.f, q, steps)
        assert info.status == 0
        swe = LinearSwe(m, p, g=v.c_g, H=v.c_g, f=v.f)
        e = l2_error(swe, host(q)[..., 0], lambda xy: v.state(xy))
        if n == 16:
            e_ref = l2_error(swe, swe.run(tableau("ars232"), dt, steps, q0)[..., 0], lambda xy: v.state(xy))
            assert abs(e - e_ref) < 1e-6 * e_ref
        errs.append(e)
        s.close()
    print(f"p={p}: Delta_2 {errs}, rate {math.log2(errs[0] / errs[1]):.2f}")
    assert math.log2(errs[0] / errs[1]) >= p + 0.5


def test_imex_is_deterministic_and_reports_non_convergence():
    """Repeated runs give identical bits; a stage solve stopped at maxit makes the
    run return HDG_ENOTCONV (steps still completed, status in info)."""
    from paper_2004_09389_amd.hdg import HDG_ENOTCONV, HdgError, imex_gamma, imex_tableau
    n, p, dt = 8, 2, 0.05
    tab = imex_tableau("theta", 0.5)
    q0 = hi.iid_rhs(hi.torus(n), p, 3)
    s = solver(hi.torus_hierarchy(n, 4), p, imex_gamma(tab) * dt)
    a, b = to_dev(q0), to_dev(q0)
    s.imex_run(tab, dt, 1.0, a, 3)
    s.imex_run(tab, dt, 1.0, b, 3)
    assert np.array_equal(host(a), host(b))
    s.close()
    s = solver(hi.torus_hierarchy(n, 4), p, imex_gamma(tab) * dt, rtol=1e-14, maxit=1)
    with pytest.raises(HdgError):
        s.imex_run(tab, dt, 1.0, to_dev(q0), 1)
    info = s.imex_run(tab, dt, 1.0, to_dev(q0), 2, allow_notconv=True)
    assert info.status == HDG_ENOTCONV and info.steps == 2 and info.solves == 2
    s.close()
