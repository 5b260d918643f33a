"""GPU tests of the learned smoother against the FP64 oracle.

Tolerances: data generation (FP64 arithmetic) 1e-11 relative; BF16 network
arithmetic (loss, gradient, learned V-cycle) 2e-2 relative, the bound for
BF16 operands with FP32 accumulation (unit roundoff 2^-9 per rounded
operand, a few roundings deep).  The oracle receives the weights rounded to
BF16 (round to nearest even), the values the library multiplies with.
"""
import numpy as np
import pytest

import hdg_inputs as hi

pytestmark = pytest.mark.gpu

HMS = 6.371e6
CASES = {
    "torus8_p1": (lambda: hi.torus_hierarchy(8, 4), 1, 0.5, 1.0, 1.0, 0.0, 0.0),
    "torus12_p2_coriolis": (lambda: hi.torus_hierarchy(12, 3), 2, 0.3, 2.0, 0.5, 0.7, 0.0),
    "torus16_p3_f1": (lambda: hi.torus_hierarchy(16, 4), 3, 0.5, 1.0, 1.0, 1.0, 0.0),
    "sphere_L2_p2": (lambda: hi.icosphere_hierarchy(2, HMS), 2, 1800.0, 9.81, 5960.0, 0.0, 7.292e-5),
}
_CACHE = {}


def setup(name, **opts):
    import torch
    from oracle.hdg import HdgOracle
    from oracle.p1 import TraceMultigrid
    from paper_2004_09389_amd.hdg import HDG_SMOOTH_MLP, HdgSolver

    opts.setdefault("smoother", HDG_SMOOTH_MLP)
    key = (name, tuple(sorted(opts.items())))
    if key not in _CACHE:
        mk, p, dt, g, H, f0, om = CASES[name]
        hier = mk()
        print(f"[case] {name} opts={opts}", flush=True)
        solver = HdgSolver(hier, p, dt, g, H, f0, om, **opts)
        oracle = HdgOracle(hier.fine, p, dt, g, H, f0, om)
        _CACHE[key] = (hier, solver, oracle, TraceMultigrid(oracle, hier))
        torch.cuda.synchronize()
    return _CACHE[key]


def bf16_round(a):
    """Round FP32 values to the nearest BF16 (ties to even), returned as float64."""
    b = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def weights(m, seed, scale=0.05):
    W1, _ = hi.mlp_init(m, 64, seed)
    W2 = np.random.default_rng(seed + 1).standard_normal((m, 64)) * scale
    return W1.astype(np.float32), W2.astype(np.float32)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name", list(CASES))
def test_untrained_learned_vcycle_is_block_jacobi(name):
    hier, solver, oracle, mg = setup(name)
    W1, _ = weights(solver.m, 3)
    solver.mlp_set_weights(W1, np.zeros((solver.m, 64), np.float32))
    r = np.random.default_rng(5).standard_normal((solver.n_facet, solver.m, 1))
    z = host(solver.mg_vcycle(to_dev(r)))[..., 0].ravel()
    assert rel(z, mg.vcycle(r[..., 0].ravel())) < 1e-11


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("coarse_its", [0, 1, 3])
def test_make_data(name, coarse_its):
    from oracle.mlp import training_pair
    hier, solver, oracle, mg = setup(name)
    e = np.random.default_rng(21).standard_normal((solver.n_facet, solver.m, 1))
    u, t = solver.mlp_make_data(to_dev(e), coarse_its)
    u_ref, t_ref = training_pair(mg, e[..., 0].ravel(), coarse_its)
    assert rel(host(u)[..., 0].ravel(), u_ref) < 1e-11
    assert rel(host(t)[..., 0].ravel(), t_ref) < 1e-11


@pytest.mark.parametrize("name", list(CASES))
def test_loss_and_gradient(name):
    from oracle.mlp import features, loss_and_grad, patch_table, training_pair
    hier, solver, oracle, mg = setup(name)
    W1, W2 = weights(solver.m, 4, scale=0.2)
    solver.mlp_set_weights(W1, W2)
    e = np.random.default_rng(22).standard_normal(solver.n_facet * solver.m)
    u, t = training_pair(mg, e, 1)
    ids, rev = patch_table(oracle.topo)
    m = solver.m
    loss_ref, g1_ref, g2_ref = loss_and_grad(bf16_round(W1), bf16_round(W2),
                                             features(u.reshape(-1, m), ids, rev), t.reshape(-1, m))
    loss, g1, g2 = solver.mlp_loss_grad(to_dev(u.reshape(-1, m, 1)), to_dev(t.reshape(-1, m, 1)))
    print(f"loss {loss:.6e} ref {loss_ref:.6e}  dW1 {rel(g1, g1_ref):.2e}  dW2 {rel(g2, g2_ref):.2e}")
    assert abs(loss - loss_ref) <= 2e-2 * loss_ref
    assert rel(g1, g1_ref) < 2e-2
    assert rel(g2, g2_ref) < 2e-2


@pytest.mark.parametrize("name", list(CASES))
def test_learned_vcycle(name):
    from oracle.mlp import LearnedTraceMultigrid
    hier, solver, oracle, mg = setup(name)
    W1, W2 = weights(solver.m, 6, scale=0.1)
    solver.mlp_set_weights(W1, W2)
    lmg = LearnedTraceMultigrid(oracle, hier, bf16_round(W1), bf16_round(W2))
    r = np.random.default_rng(7).standard_normal((solver.n_facet, solver.m, 1))
    ref = lmg.vcycle(r[..., 0].ravel())
    z = host(solver.mg_vcycle(to_dev(r)))[..., 0].ravel()
    err = rel(z, ref)
    print(f"learned V-cycle rel {err:.2e} (vs block-Jacobi cycle {rel(ref, mg.vcycle(r[..., 0].ravel())):.2e})")
    assert err < 2e-2


def test_weights_round_trip():
    hier, solver, oracle, mg = setup("torus12_p2_coriolis")
    W1, W2 = weights(solver.m, 8)
    solver.mlp_set_weights(W1, W2)
    A, B = solver.mlp_get_weights()
    assert np.array_equal(A, W1) and np.array_equal(B, W2)


def test_training_lowers_held_out_loss():
    """Adam on first-cycle pairs of random initial errors lowers the loss on
    an error it never saw."""
    from oracle.mlp import features, loss_and_grad, patch_table, training_pair
    from paper_2004_09389_amd.learned import train
    hier, solver, oracle, mg = setup("torus16_p3_f1", max_rhs=4)
    m = solver.m
    W1, _ = hi.mlp_init(m, 64, 0)
    solver.mlp_set_weights(W1.astype(np.float32), np.zeros((m, 64), np.float32))
    e_test = hi.iid_trace(solver.n_facet, solver.p, 99)[..., 0].ravel()
    u, t = training_pair(mg, e_test, 2)
    ids, rev = patch_table(oracle.topo)
    f = features(u.reshape(-1, m), ids, rev)
    l0 = loss_and_grad(W1, np.zeros((m, 64)), f, t.reshape(-1, m))[0]
    hist, _ = train(solver, batches=16, epochs=8, lr=3e-3)
    A, B = solver.mlp_get_weights()
    l1 = loss_and_grad(A.astype(np.float64), B.astype(np.float64), f, t.reshape(-1, m))[0]
    print(f"held-out loss {l0:.4e} -> {l1:.4e}; training loss {hist[0]:.4e} -> {hist[-1]:.4e}")
    assert np.all(np.isfinite(hist))
    assert abs(hist[0] - l0) < 0.2 * l0      # same data distribution before training
    assert l1 < 0.75 * l0


def test_trained_smoother_gain_on_unseen_seeds():
    """Train on random initial errors (seeds 1000+), then solve unseen
    right-hand sides (seeds 2000-2009, iid and smooth Fourier) to 1e-8 with
    FGMRES: the learned cycle contracts the error more than block-Jacobi
    and needs no more iterations on any seed, fewer on average."""
    import torch
    from paper_2004_09389_amd.hdg import HDG_SMOOTH_BJACOBI
    from paper_2004_09389_amd.learned import train
    hier, learned, oracle, mg = setup("torus16_p3_f1", max_rhs=4)
    _, plain, _, _ = setup("torus16_p3_f1", max_rhs=4, smoother=HDG_SMOOTH_BJACOBI, krylov=2)
    W1, _ = hi.mlp_init(learned.m, 64, 0)
    learned.mlp_set_weights(W1.astype(np.float32), np.zeros((learned.m, 64), np.float32))
    train(learned, batches=32, epochs=8, lr=3e-3)
    its = []
    for sd in range(2000, 2010):
        r = (hi.iid_rhs if sd % 2 == 0 else hi.fourier_rhs_torus)(hier.fine, 3, sd)
        row = []
        for s in (plain, learned):
            rhat = s.condense(to_dev(r))
            lam, info = s.solve(rhat)
            assert info[0].status == 0 and info[0].fallbacks == 0
            assert rel(host(lam)[..., 0].ravel(), oracle.solve(r[..., 0])[1]) < 1e-6
            row.append(info[0].iters)
        its.append(row)
    its = np.array(its)
    print("iterations (block-Jacobi, learned) per seed:", its.tolist())
    # contraction of the stationary iteration e <- e - V(S e) on an unseen error
    e = to_dev(hi.iid_trace(learned.n_facet, 3, 2100))
    ratios = []
    for s in (plain, learned):
        x = e.clone()
        nrm = []
        for k in range(8):
            r = s.trace_apply(x)
            nrm.append(float(torch.linalg.norm(r)))
            x = x - s.mg_vcycle(r)
        ratios.append((nrm[-1] / nrm[2]) ** (1 / 5))
    print(f"stationary contraction block-Jacobi {ratios[0]:.3f} learned {ratios[1]:.3f}")
    assert ratios[1] < ratios[0]
    assert np.all(its[:, 1] <= its[:, 0]) and its[:, 1].mean() < its[:, 0].mean()


def _solve_case(name, **opts):
    hier, solver, oracle, mg = setup(name, **opts)
    r = hi.iid_rhs(hier.fine, solver.p, 31, nrhs=1)
    rhat = solver.condense(to_dev(r))
    lam, info = solver.solve(rhat)
    ref = oracle.solve(r[..., 0])[1]
    return solver, host(lam)[..., 0].ravel(), ref, info[0]


def test_solve_with_learned_smoother_matches_oracle():
    solver, lam, ref, info = _solve_case("torus16_p3_f1", rtol=1e-12)
    W1, W2 = weights(solver.m, 10, scale=0.02)
    solver.mlp_set_weights(W1, W2)
    _, lam, ref, info = _solve_case("torus16_p3_f1", rtol=1e-12)
    print(info)
    assert info.status == 0 and info.rel_res <= 1e-12
    assert rel(lam, ref) < 1e-9


@pytest.mark.parametrize("nb", [1, 4])
def test_solve_learned_mixed_ir_matches_oracle(nb):
    """The learned smoother inside the FP32 inner solve of HDG_MIXED_IR (FP32
    basis and V-cycle vectors, FP64 refinement): every column to 1e-8."""
    from paper_2004_09389_amd.hdg import HDG_MIXED_IR
    hier, solver, oracle, _ = setup("torus16_p3_f1", rtol=1e-10, precision=HDG_MIXED_IR, max_rhs=nb)
    W1, W2 = weights(solver.m, 10, scale=0.02)
    solver.mlp_set_weights(W1, W2)
    r = hi.iid_rhs(hier.fine, solver.p, 35, nrhs=nb)
    lam, info = solver.solve(solver.condense(to_dev(r)))
    lam = host(lam)
    for k in range(nb):
        assert info[k].status == 0 and info[k].rel_res <= 1e-10
        assert rel(lam[..., k].ravel(), oracle.solve(r[..., k])[1]) < 1e-8
    print(info[0])


def test_fallback_on_garbage_weights():
    """Weights that wreck the cycle trip the fallback; the solve still converges."""
    hier, solver, oracle, mg = setup("torus12_p2_coriolis", rtol=1e-10)
    rng = np.random.default_rng(11)
    solver.mlp_set_weights((rng.standard_normal((64, 5 * solver.m)) * 10).astype(np.float32),
                           (rng.standard_normal((solver.m, 64)) * 10).astype(np.float32))
    _, lam, ref, info = _solve_case("torus12_p2_coriolis", rtol=1e-10)
    print(info)
    assert info.fallbacks == 1 and info.status == 0
    assert rel(lam, ref) < 1e-8


def test_fallback_threshold_forces_block_jacobi():
    """A threshold no iteration can meet reverts to block-Jacobi after the
    first measured step, and the iteration count matches the plain solve's
    within the two learned iterations."""
    from paper_2004_09389_amd.hdg import HDG_SMOOTH_BJACOBI
    _, _, _, plain = _solve_case("torus8_p1", rtol=1e-10, smoother=HDG_SMOOTH_BJACOBI, krylov=2)
    _, lam, ref, info = _solve_case("torus8_p1", rtol=1e-10, fallback_ratio=1e-9)
    print(plain, info)
    assert info.fallbacks == 1 and info.status == 0
    assert abs(info.iters - plain.iters) <= 2
    assert rel(lam, ref) < 1e-8


def test_tuning_does_not_change_results():
    """Samples per lane change the launch shape only: bitwise-equal V-cycles."""
    hier, solver, oracle, mg = setup("torus12_p2_coriolis")
    W1, W2 = weights(solver.m, 12, scale=0.1)
    solver.mlp_set_weights(W1, W2)
    r = to_dev(np.random.default_rng(13).standard_normal((solver.n_facet, solver.m, 1)))
    outs = []
    for tpw in (1, 2, 1):
        solver.set_tuning(mlp_samples_per_lane=tpw)
        outs.append(host(solver.mg_vcycle(r)))
    chosen = solver.autotune(1)
    assert chosen["mlp_samples_per_lane"] in (1, 2) and solver.get_tuning() == chosen
    outs.append(host(solver.mg_vcycle(r)))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])


@pytest.mark.parametrize("nb", [4, 8])
def test_four_rhs_per_lane_bitwise(nb):
    """Four consecutive right-hand sides per lane in the learned smoothing kernel
    (16-byte gathers) give the same bits as one and two samples per lane, in the
    V-cycle (FP64 vectors) and in a mixed solve (FP32 vectors)."""
    from paper_2004_09389_amd.hdg import HDG_MIXED
    hier, solver, oracle, mg = setup("torus12_p2_coriolis", max_rhs=8, precision=HDG_MIXED, rtol=1e-10)
    W1, W2 = weights(solver.m, 12, scale=0.1)
    solver.mlp_set_weights(W1, W2)
    r = to_dev(np.random.default_rng(17).standard_normal((solver.n_facet, solver.m, nb)))
    rc = to_dev(hi.iid_rhs(hier.fine, solver.p, 19, nrhs=nb))
    outs, sols = [], []
    for tpw in (1, 2, 4):
        solver.set_tuning(mlp_samples_per_lane=tpw)
        outs.append(host(solver.mg_vcycle(r)))
        lam, info = solver.solve(solver.condense(rc))
        sols.append((host(lam), [i.iters for i in info]))
    for o in outs[1:]:
        assert np.array_equal(o, outs[0])
    for lam, its in sols[1:]:
        assert np.array_equal(lam, sols[0][0]) and its == sols[0][1]
    chosen = solver.autotune(nb)
    assert chosen["mlp_samples_per_lane"] in (1, 2, 4)


def _gain(hier, p, dt, f0, kind, rtol, seeds=range(2000, 2010)):
    """Train on random initial errors (seeds 1000+), then solve unseen right-hand
    sides with block-Jacobi and with the learned smoother (mixed precision,
    FGMRES, the same sweeps) one at a time: iterations and HIP-event time per
    solve (after one untimed solve of each right-hand side)."""
    import torch
    from paper_2004_09389_amd.hdg import HDG_MIXED, HDG_SMOOTH_BJACOBI, HDG_SMOOTH_MLP, HdgSolver
    from paper_2004_09389_amd.learned import train
    common = dict(rtol=rtol, precision=HDG_MIXED, krylov=2, p1_tail_max=0 if hier.fine.n > 8 else 4096)
    learned = HdgSolver(hier, p, dt, 1.0, 1.0, f0, 0.0, smoother=HDG_SMOOTH_MLP, max_rhs=8, **common)
    plain = HdgSolver(hier, p, dt, 1.0, 1.0, f0, 0.0, smoother=HDG_SMOOTH_BJACOBI, max_rhs=8, **common)
    W1, _ = hi.mlp_init(p + 1, 64, 0)
    learned.mlp_set_weights(W1.astype(np.float32), np.zeros((p + 1, 64), np.float32))
    hist, _ = train(learned, batches=32, epochs=8, lr=3e-3)
    its, ms = [], []
    for sd in seeds:
        r = hi.iid_rhs(hier.fine, p, sd) if kind == "iid" else hi.fourier_rhs_torus(hier.fine, p, sd)
        rd = to_dev(r)
        row_i, row_t = [], []
        for s in (plain, learned):
            rhat = s.condense(rd)
            s.solve(rhat)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            lam, info = s.solve(rhat)
            b.record()
            torch.cuda.synchronize()
            assert info[0].status == 0
            row_i.append(info[0].iters)
            row_t.append(a.elapsed_time(b))
        its.append(row_i)
        ms.append(row_t)
    plain.close()
    learned.close()
    return hist, np.array(its), np.array(ms)


def test_torus8_p1_training_and_gain():
    """The 8 x 8 torus (p = 1, f = 0, Courant 4, iid right-hand sides):
    on unseen seeds 2000-2009 the trained network needs fewer FGMRES
    iterations to 1e-8 than block-Jacobi on average and never more on a seed;
    the time per solve of both is reported (at 384 unknowns each iteration is
    a chain of launches, so the learned step's extra launch costs time)."""
    hier = hi.torus_hierarchy(8, 4)
    hist, its, ms = _gain(hier, 1, 0.5, 0.0, "iid", 1e-8)
    print(f"8x8 torus loss {hist[0]:.3f} -> {hist[-1]:.3f}; iterations (block-Jacobi, learned): {its.tolist()}; "
          f"mean ms per solve {ms.mean(0).round(4).tolist()}")
    assert hist[-1] < hist[0]
    assert its[:, 1].mean() < its[:, 0].mean() and np.all(its[:, 1] <= its[:, 0])


def test_torus256_p3_gain_iterations_and_time():
    """The 256 x 256 torus (p = 3, f = 1, Courant 8, Fourier right-hand
    sides): on unseen seeds 2000-2009, iterations and time to 1e-8 of the
    learned smoother against block-Jacobi.  The network must gain in at least
    one of the two (it gains iterations: about one per solve); both are printed."""
    hier = hi.torus_hierarchy(256, 32)
    hist, its, ms = _gain(hier, 3, 8.0 / 256, 1.0, "fourier", 1e-8)
    gain_its = its[:, 0].mean() - its[:, 1].mean()
    gain_time = ms[:, 0].mean() - ms[:, 1].mean()
    print(f"256x256 torus loss {hist[0]:.3f} -> {hist[-1]:.3f}; iterations (block-Jacobi, learned): {its.tolist()}; "
          f"mean ms per solve {ms.mean(0).round(4).tolist()} (gain {gain_its:.2f} iterations, {gain_time:.4f} ms)")
    assert gain_its > 0 or gain_time > 0
    assert np.all(its[:, 1] <= its[:, 0] + 1)
