"""GPU parity: every C-ABI entry point against the FP64 CPU oracle on the
same seeded inputs.

Tolerances: the FP64 path to 1e-10 relative L2 (per field), operator-level
entry points to 1e-12; the mixed-precision solve to 1e-8.  Integer topology
is compared bit-exactly.
"""
import numpy as np
import pytest

import hdg_inputs as hi

pytestmark = pytest.mark.gpu

HMS = 6.371e6


def _cases():
    return {
        # name: (hierarchy factory, p, dt, g, H, f0, omega)
        "torus8_p1_courant4": (lambda: hi.torus_hierarchy(8, 4), 1, 0.5, 1.0, 1.0, 0.0, 0.0),
        "torus12_p2_coriolis": (lambda: hi.torus_hierarchy(12, 3), 2, 0.3, 2.0, 0.5, 0.7, 0.0),
        "torus16_p3_f1": (lambda: hi.torus_hierarchy(16, 4), 3, 0.5, 1.0, 1.0, 1.0, 0.0),
        "torus1_twocell_p1": (lambda: hi.torus_hierarchy(1, 1), 1, 0.5, 1.0, 1.0, 0.0, 0.0),
        "sphere_L2_p2": (lambda: hi.icosphere_hierarchy(2, HMS), 2, 1800.0, 9.81, 5960.0, 0.0, 7.292e-5),
        # six P1 levels; only the finest (9216 vertices) is above the tail-kernel bound
        "torus96_p1_deep": (lambda: hi.torus_hierarchy(96, 3), 1, 8.0 / 96, 1.0, 1.0, 1.0, 0.0),
    }


CASES = _cases()
_CACHE = {}


def setup_case(name, **opts):
    import torch
    from oracle.hdg import HdgOracle
    from oracle.p1 import TraceMultigrid
    from paper_2004_09389_amd.hdg import HdgSolver

    key = (name, tuple(sorted(opts.items())))
    if key in _CACHE:
        return _CACHE[key]
    mk, p, dt, g, H, f0, om = CASES[name]
    hier = mk()
    print(f"[case] {name} opts={opts}", flush=True)
    solver = HdgSolver(hier, p, dt, g, H, f0, om, **opts)
    oracle = HdgOracle(hier.fine, p, dt, g, H, f0, om)
    mg = TraceMultigrid(oracle, hier)
    _CACHE[key] = (hier, solver, oracle, mg)
    torch.cuda.synchronize()
    return _CACHE[key]


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def trace_np(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_topology_bit_exact(name):
    hier, solver, oracle, _ = setup_case(name)
    fc, fl, fv = solver.topology()
    t = oracle.topo
    assert np.array_equal(fc, t.facet_cell) and np.array_equal(fl, t.facet_loc)
    assert np.array_equal(fv, t.facet_vert)


@pytest.mark.parametrize("name", list(CASES))
def test_condense(name):
    hier, solver, oracle, _ = setup_case(name)
    r = hi.iid_rhs(hier.fine, solver.p, 11, nrhs=2)
    rhat = trace_np(solver.condense(to_dev(r))) if solver.options.max_rhs >= 2 else None
    if rhat is None:
        rhat = np.stack([trace_np(solver.condense(to_dev(r[..., k:k + 1])))[..., 0] for k in range(2)], -1)
    for k in range(2):
        ref = oracle.rhat(r[..., k])
        assert rel(rhat[..., k].ravel(), ref) < 1e-12


@pytest.mark.parametrize("name", list(CASES))
def test_trace_apply(name):
    from paper_2004_09389_amd.hdg import HDG_MIXED
    hier, solver, oracle, _ = setup_case(name)
    x = np.random.default_rng(3).standard_normal((solver.n_facet, solver.m, 1))
    ref = oracle.apply(x[..., 0].ravel())
    y = trace_np(solver.trace_apply(to_dev(x)))[..., 0].ravel()
    assert rel(y, ref) < 1e-12
    y32 = trace_np(solver.trace_apply(to_dev(x), HDG_MIXED))[..., 0].ravel()
    assert rel(y32, ref) < 1e-5


@pytest.mark.parametrize("name", list(CASES))
def test_vcycle(name):
    from paper_2004_09389_amd.hdg import HDG_MIXED
    hier, solver, oracle, mg = setup_case(name)
    r = np.random.default_rng(5).standard_normal((solver.n_facet, solver.m, 1))
    ref = mg.vcycle(r[..., 0].ravel())
    z = trace_np(solver.mg_vcycle(to_dev(r)))[..., 0].ravel()
    assert rel(z, ref) < 1e-11
    z16 = trace_np(solver.mg_vcycle(to_dev(r), HDG_MIXED))[..., 0].ravel()
    assert rel(z16, ref) < 3e-2


@pytest.mark.parametrize("name", ["torus16_p3_f1", "sphere_L2_p2", "torus96_p1_deep"])
def test_one_rhs_p1_kernels_match_the_batched_path(name):
    """At one right-hand side the P1 residual is fused into the restriction (its
    children summed by shuffles instead of in list order) and the prolongation
    into the first post-sweep; the one-column V-cycle agrees with column 0 of the
    four-column one (one thread per (vertex, rhs), separate kernels) to rounding:
    1e-13 in FP64, 1e-5 with FP32 P1 vectors; both against the oracle (P1 tail
    off, so every level runs its kernels)."""
    from paper_2004_09389_amd.hdg import HDG_MIXED
    hier, s, oracle, mg = setup_case(name, p1_tail_max=0, max_rhs=4)
    s.set_tuning(rhs_block=1)
    x = np.random.default_rng(61).standard_normal((s.n_facet, s.m, 4))
    ref = mg.vcycle(x[..., 0].ravel())
    for prec, tol, otol in ((0, 1e-13, 1e-11), (HDG_MIXED, 1e-5, 3e-2)):
        z4 = trace_np(s.mg_vcycle(to_dev(x), prec))
        z1 = trace_np(s.mg_vcycle(to_dev(np.ascontiguousarray(x[..., :1])), prec))
        assert rel(z1[..., 0].ravel(), z4[..., 0].ravel()) < tol, prec
        assert rel(z1[..., 0].ravel(), ref) < otol, prec
    s.set_tuning(rhs_block=4)


@pytest.mark.parametrize("damping", [0.55, 0.9])
def test_vcycle_damping_option(damping):
    """The block-Jacobi damping set through the binding (damping=, the options
    field omega) reaches the kernels: V-cycle against the oracle's at that damping."""
    from oracle.p1 import TraceMultigrid
    hier, solver, oracle, _ = setup_case("torus16_p3_f1", damping=damping)
    mg = TraceMultigrid(oracle, hier, omega=damping)
    r = np.random.default_rng(6).standard_normal((solver.n_facet, solver.m, 1))
    ref = mg.vcycle(r[..., 0].ravel())
    assert rel(trace_np(solver.mg_vcycle(to_dev(r)))[..., 0].ravel(), ref) < 1e-11
    assert rel(ref, TraceMultigrid(oracle, hier).vcycle(r[..., 0].ravel())) > 1e-3   # the damping matters


@pytest.mark.parametrize("name", ["torus8_p1_courant4", "torus96_p1_deep", "sphere_L2_p2"])
def test_vcycle_without_tail_kernel(name):
    """Every P1 level as separate kernels (and the dense coarsest solve as a
    multi-block mat-vec) gives the same V-cycle as the single-workgroup tail."""
    hier, solver, oracle, mg = setup_case(name, p1_tail_max=0)
    r = np.random.default_rng(6).standard_normal((solver.n_facet, solver.m, 2))
    ref = mg.vcycle(r[..., 0].ravel())
    z = trace_np(solver.mg_vcycle(to_dev(r[..., :1].copy())))[..., 0].ravel()
    assert rel(z, ref) < 1e-11


@pytest.mark.parametrize("name", list(CASES))
def test_solve_and_recover_fp64(name):
    hier, solver, oracle, _ = setup_case(name, rtol=1e-12)
    r = hi.iid_rhs(hier.fine, solver.p, 21)
    q_ref, lam_ref = oracle.solve(r[..., 0])
    rd = to_dev(r)
    rhat = solver.condense(rd)
    lam, info = solver.solve(rhat)
    assert info[0].status == 0 and info[0].rel_res <= 1e-12
    q = trace_np(solver.recover(rd, lam))[..., 0]
    assert rel(trace_np(lam)[..., 0].ravel(), lam_ref) < 1e-10
    for fld in range(3):
        assert rel(q[:, fld], q_ref[:, fld]) < 1e-10


@pytest.mark.parametrize("name", ["torus8_p1_courant4", "torus16_p3_f1", "sphere_L2_p2"])
def test_solve_mixed(name):
    from paper_2004_09389_amd.hdg import HDG_MIXED, HDG_KRYLOV_FGMRES
    hier, solver, oracle, _ = setup_case(name, rtol=1e-10, precision=HDG_MIXED, krylov=HDG_KRYLOV_FGMRES)
    r = hi.iid_rhs(hier.fine, solver.p, 31)
    q_ref, lam_ref = oracle.solve(r[..., 0])
    rd = to_dev(r)
    q, lam, info = solver.step(rd)
    assert info[0].status == 0
    assert rel(trace_np(lam)[..., 0].ravel(), lam_ref) < 1e-8
    q = trace_np(q)[..., 0]
    for fld in range(3):
        assert rel(q[:, fld], q_ref[:, fld]) < 1e-8


@pytest.mark.parametrize("name", ["torus8_p1_courant4", "torus16_p3_f1", "sphere_L2_p2"])
@pytest.mark.parametrize("nb", [1, 3, 4])
def test_solve_mixed_ir(name, nb):
    """HDG_MIXED_IR: FP64 refinement around an inner FGMRES whose basis and
    V-cycle vectors are FP32 (one thread per (facet, rhs) at nb = 1, 3 and the
    RHS-blocked kernels at nb = 4); every column against the oracle."""
    from paper_2004_09389_amd.hdg import HDG_KRYLOV_FGMRES, HDG_MIXED_IR
    hier, solver, oracle, _ = setup_case(name, rtol=1e-10, precision=HDG_MIXED_IR, krylov=HDG_KRYLOV_FGMRES,
                                         max_rhs=nb)
    r = hi.iid_rhs(hier.fine, solver.p, 33, nrhs=nb)
    q, lam, info = solver.step(to_dev(r))
    q, lam = trace_np(q), trace_np(lam)
    for k in range(nb):
        q_ref, lam_ref = oracle.solve(r[..., k])
        assert info[k].status == 0 and info[k].rel_res <= 1e-10 and info[k].refinements >= 2
        assert rel(lam[..., k].ravel(), lam_ref) < 1e-8
        for fld in range(3):
            assert rel(q[:, fld, :, k], q_ref[:, fld]) < 1e-8
    print(f"{name} nb={nb}: {info[0]}")


@pytest.mark.parametrize("name", ["torus8_p1_courant4", "torus12_p2_coriolis"])
def test_batched_matches_single(name):
    hier, solver, oracle, _ = setup_case(name, rtol=1e-12, max_rhs=3)
    r = hi.iid_rhs(hier.fine, solver.p, 41, nrhs=3)
    qb, lamb, infob = solver.step(to_dev(r))
    qb, lamb = trace_np(qb), trace_np(lamb)
    for k in range(3):
        q_ref, lam_ref = oracle.solve(r[..., k])
        assert rel(lamb[..., k].ravel(), lam_ref) < 1e-10
        for fld in range(3):
            assert rel(qb[:, fld, :, k], q_ref[:, fld]) < 1e-10


@pytest.mark.parametrize("name,prec", [("torus8_p1_courant4", 0), ("torus16_p3_f1", 0), ("torus16_p3_f1", 1),
                                       ("torus16_p3_f1", 2)])
def test_graph_replay_matches_eager(name, prec):
    """Captured Krylov iterations replayed several times, with eager work and
    synchronisations between the replays, give bitwise the eager result."""
    import torch
    hier, sg, oracle, _ = setup_case(name, rtol=1e-10, precision=prec, use_graph=1)
    _, se, _, _ = setup_case(name, rtol=1e-10, precision=prec, use_graph=0)
    for seed in (51, 52, 53):
        r = to_dev(hi.iid_rhs(hier.fine, sg.p, seed))
        qg, lg, ig = sg.step(r)
        junk = torch.randn(1000, device="cuda").sum()    # eager work between replays
        torch.cuda.synchronize()
        qe, le, ie = se.step(r)
        torch.cuda.synchronize()
        assert ig[0].iters == ie[0].iters and ig[0].status == 0
        assert torch.equal(lg, le) and torch.equal(qg, qe), (seed, float(junk))


@pytest.mark.parametrize("name", ["torus8_p1_courant4", "torus12_p2_coriolis", "torus16_p3_f1"])
@pytest.mark.parametrize("nb", [4, 8, 16])
def test_rhs_blocked_rows_bitwise(name, nb):
    """Four right-hand sides per thread with LDS-staged rows accumulate in the
    same order as one thread per (facet, rhs): bitwise-equal apply, residual
    and V-cycles, each column matching the oracle."""
    _rhs_blocked_bitwise(name, nb)


@pytest.mark.parametrize("name,nb", [("torus16_p3_f1", 32), ("torus16_p3_f1", 64), ("sphere_L2_p2", 8)])
def test_rhs_blocked_rows_bitwise_wide_blocks(name, nb):
    """The same at 512- and 1024-thread blocks (32 and 64 right-hand sides,
    where the row staging covers the block in one partial batch) and on a
    sphere whose facet count leaves a ragged last block."""
    _rhs_blocked_bitwise(name, nb)


def _rhs_blocked_bitwise(name, nb):
    from paper_2004_09389_amd.hdg import HDG_MIXED
    print(f"[rb] {name} nb={nb}", flush=True)
    hier, s, oracle, mg = setup_case(name, max_rhs=max(16, nb))
    x = np.random.default_rng(60 + nb).standard_normal((s.n_facet, s.m, nb))
    xd = to_dev(x)
    outs = {}
    for rb in (1, 4):
        s.set_tuning(rhs_block=rb)
        outs[rb] = [trace_np(s.trace_apply(xd)), trace_np(s.trace_apply(xd, HDG_MIXED)),
                    trace_np(s.mg_vcycle(xd)), trace_np(s.mg_vcycle(xd, HDG_MIXED))]
    s.set_tuning(rhs_block=4)
    for a, b in zip(outs[1], outs[4]):
        assert np.array_equal(a, b)
    for k in (0, nb - 1):
        assert rel(outs[4][0][..., k].ravel(), oracle.apply(x[..., k].ravel())) < 1e-12
        assert rel(outs[4][2][..., k].ravel(), mg.vcycle(x[..., k].ravel())) < 1e-11


@pytest.mark.parametrize("name", ["torus8_p1_courant4", "torus12_p2_coriolis", "torus16_p3_f1", "sphere_L2_p2"])
def test_batched_cell_kernels_bitwise(name):
    """Condense and recover with 8 right-hand sides equal the one-column calls
    bit for bit and the oracle to 1e-12."""
    hier, s, oracle, _ = setup_case(name, max_rhs=16)
    nb = 8
    r = hi.iid_rhs(hier.fine, s.p, 70, nrhs=nb)
    lam = np.random.default_rng(71).standard_normal((s.n_facet, s.m, nb))
    rhat_b = trace_np(s.condense(to_dev(r)))
    q_b = trace_np(s.recover(to_dev(r), to_dev(lam)))
    for k in (0, 3, nb - 1):
        rk = np.ascontiguousarray(r[..., k:k + 1])
        lk = np.ascontiguousarray(lam[..., k:k + 1])
        assert np.array_equal(trace_np(s.condense(to_dev(rk)))[..., 0], rhat_b[..., k])
        assert np.array_equal(trace_np(s.recover(to_dev(rk), to_dev(lk)))[..., 0], q_b[..., k])
        assert rel(rhat_b[..., k].ravel(), oracle.rhat(r[..., k])) < 1e-12
        q_ref = oracle.recover(r[..., k], lam[..., k].ravel())
        for fld in range(3):
            assert rel(q_b[:, fld, :, k], q_ref[:, fld]) < 1e-12


@pytest.mark.parametrize("name", ["torus16_p3_f1", "sphere_L2_p2"])
def test_cells_per_block_tuning_bitwise(name, tmp_path):
    """The cells per block of the batched condensation and recovery kernels
    (tuning field cell_cells) changes no bit, at 4 and at 32 right-hand sides
    (the latter with the prefetched staging of condensation); hdg_autotune
    picks one of its candidates, and a tuning cache file returns the same
    choice."""
    hier, s, _, _ = setup_case(name, max_rhs=32)
    for nb in (4, 32):
        r = hi.iid_rhs(hier.fine, s.p, 80 + nb, nrhs=nb)
        lam = np.random.default_rng(81 + nb).standard_normal((s.n_facet, s.m, nb))
        ref = None
        for cc in (0, 1, 3, 8, 32):
            s.set_tuning(cell_cells=cc)
            got = (trace_np(s.condense(to_dev(r))), trace_np(s.recover(to_dev(r), to_dev(lam))))
            if ref is None:
                ref = got
            else:
                assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (nb, cc)
        chosen = s.autotune(nb, cache=str(tmp_path / "tuning.json"))
        assert chosen["cell_cells"] in (0, 1, 2, 4, 8, 16), chosen
        assert s.get_tuning() == chosen
        assert s.autotune(nb, cache=str(tmp_path / "tuning.json")) == chosen
        assert np.array_equal(trace_np(s.condense(to_dev(r))), ref[0])
    s.set_tuning(cell_cells=0)


CHEB_CASES = ["torus8_p1_courant4", "torus12_p2_coriolis", "torus16_p3_f1", "sphere_L2_p2"]


@pytest.mark.parametrize("name", CHEB_CASES)
@pytest.mark.parametrize("nu", [(2, 2), (1, 1), (3, 2), (1, 3)])
def test_chebyshev_vcycle(name, nu):
    """Chebyshev smoothing: the eigenvalue estimate and the V-cycle against the
    oracle's textbook Chebyshev iteration (FP64 1e-11, mixed 3e-2)."""
    from oracle.p1 import TraceMultigrid
    from paper_2004_09389_amd.hdg import HDG_MIXED, HDG_SMOOTH_CHEBYSHEV
    hier, s, oracle, _ = setup_case(name, smoother=HDG_SMOOTH_CHEBYSHEV, nu_pre=nu[0], nu_post=nu[1])
    mg = TraceMultigrid(oracle, hier, smoother="chebyshev", nu_pre=nu[0], nu_post=nu[1])
    assert abs(s.sizes.lambda_max - mg.lambda_max) <= 1e-10 * mg.lambda_max
    r = np.random.default_rng(8).standard_normal((s.n_facet, s.m, 1))
    ref = mg.vcycle(r[..., 0].ravel())
    assert rel(trace_np(s.mg_vcycle(to_dev(r)))[..., 0].ravel(), ref) < 1e-11
    assert rel(trace_np(s.mg_vcycle(to_dev(r), HDG_MIXED))[..., 0].ravel(), ref) < 3e-2


@pytest.mark.parametrize("name", ["torus12_p2_coriolis", "torus16_p3_f1"])
def test_chebyshev_rhs_blocked_bitwise(name):
    from paper_2004_09389_amd.hdg import HDG_MIXED, HDG_SMOOTH_CHEBYSHEV
    hier, s, oracle, _ = setup_case(name, smoother=HDG_SMOOTH_CHEBYSHEV, max_rhs=8, nu_pre=3, nu_post=3)
    x = to_dev(np.random.default_rng(9).standard_normal((s.n_facet, s.m, 8)))
    outs = []
    for rb in (1, 4):
        s.set_tuning(rhs_block=rb)
        outs.append([trace_np(s.mg_vcycle(x)), trace_np(s.mg_vcycle(x, HDG_MIXED))])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("name,prec", [("torus8_p1_courant4", 0), ("torus16_p3_f1", 0), ("torus16_p3_f1", 1),
                                       ("sphere_L2_p2", 1)])
def test_chebyshev_solve(name, prec):
    """Solves with the Chebyshev smoother (PCG when symmetric, else FGMRES)."""
    from paper_2004_09389_amd.hdg import HDG_SMOOTH_CHEBYSHEV
    hier, s, oracle, _ = setup_case(name, smoother=HDG_SMOOTH_CHEBYSHEV, precision=prec, rtol=1e-12)
    r = hi.iid_rhs(hier.fine, s.p, 23)
    q, lam, info = s.step(to_dev(r))
    q_ref, lam_ref = oracle.solve(r[..., 0])
    print(name, prec, info[0])
    assert info[0].status == 0
    assert rel(trace_np(lam)[..., 0].ravel(), lam_ref) < 1e-9
    for fld in range(3):
        assert rel(trace_np(q)[:, fld, :, 0], q_ref[:, fld]) < 1e-9


@pytest.mark.parametrize("name", ["torus8_p1_courant4", "torus12_p2_coriolis", "torus16_p3_f1", "sphere_L2_p2",
                                  "torus96_p1_deep"])
def test_galerkin_coarse_form(name):
    """Galerkin P1 hierarchy (S_c = pi^T S pi, then P^T A P) against the oracle's:
    V-cycle to 1e-11 (tail kernel on and off), solve to the oracle's direct solution."""
    from oracle.p1 import TraceMultigrid
    hier, s, oracle, _ = setup_case(name, p1_galerkin=1, rtol=1e-12)
    _, s0, _, _ = setup_case(name, p1_galerkin=1, p1_tail_max=0)
    mg = TraceMultigrid(oracle, hier, galerkin=True)
    r = np.random.default_rng(12).standard_normal((s.n_facet, s.m, 1))
    ref = mg.vcycle(r[..., 0].ravel())
    assert rel(trace_np(s.mg_vcycle(to_dev(r)))[..., 0].ravel(), ref) < 1e-11
    assert rel(trace_np(s0.mg_vcycle(to_dev(r)))[..., 0].ravel(), ref) < 1e-11
    rr = hi.iid_rhs(hier.fine, s.p, 24)
    q, lam, info = s.step(to_dev(rr))
    print(name, "galerkin", info[0])
    assert info[0].status == 0
    assert rel(trace_np(lam)[..., 0].ravel(), oracle.solve(rr[..., 0])[1]) < 1e-9
