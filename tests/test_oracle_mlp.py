"""Pins of the learned-smoother reference (CPU)."""
import numpy as np
import pytest

import hdg_inputs as hi
from oracle.fem import topology
from oracle.hdg import HdgOracle
from oracle.mlp import features, forward, init_weights, loss_and_grad, patch_table


@pytest.mark.parametrize("m", [2, 3, 4])
def test_gradient_finite_difference(m):
    """Backward pass against central finite differences (relative 1e-7)."""
    rng = np.random.default_rng(1)
    W1, _ = init_weights(m, 64, seed=2)
    W2 = rng.standard_normal((m, 64)) * 0.1
    feats = rng.standard_normal((50, 5 * m))
    tgt = rng.standard_normal((50, m))
    loss, dW1, dW2 = loss_and_grad(W1, W2, feats, tgt)
    eps = 1e-6
    for W, dW in ((W1, dW1), (W2, dW2)):
        for idx in [(0, 0), (min(3, W.shape[0] - 1), 1), (W.shape[0] - 1, W.shape[1] - 1), (W.shape[0] // 2, 2)]:
            old = W[idx]
            W[idx] = old + eps
            lp = loss_and_grad(W1, W2, feats, tgt)[0]
            W[idx] = old - eps
            lm = loss_and_grad(W1, W2, feats, tgt)[0]
            W[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - dW[idx]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9


def test_positive_homogeneity():
    """No biases and ReLU: the correction scales with the residual (c(a r) = a c(r), a > 0)."""
    m = 3
    W1, _ = init_weights(m, 64, seed=3)
    W2 = np.random.default_rng(4).standard_normal((m, 64))
    f = np.random.default_rng(5).standard_normal((20, 5 * m))
    c1, _ = forward(W1, W2, f)
    c2, _ = forward(W1, W2, 7.5 * f)
    assert np.abs(c2 - 7.5 * c1).max() < 1e-12 * np.abs(c2).max()


def test_untrained_network_is_zero_correction():
    W1, W2 = init_weights(4, 64, seed=0)
    c, _ = forward(W1, W2, np.random.default_rng(0).standard_normal((10, 20)))
    assert np.all(c == 0.0)


def test_patch_orientation_follows_the_source_cell():
    """Slot 0 is in the facet's own direction; slots 1-4 list the facet's
    nodes counter-clockwise around the cell they are taken from.  Checked with
    a periodic field evaluated at each cell's own unwrapped corners."""
    n, p = 5, 3
    mesh = hi.torus(n)
    topo = topology(mesh)
    ids, rev = patch_table(topo)
    m = p + 1
    X = mesh.cell_coords()[..., :2]
    s = np.arange(m) / p
    field = lambda q: np.sin(2 * np.pi * q[..., 0]) * np.cos(2 * np.pi * q[..., 1]) + 0.3 * np.sin(2 * np.pi * q[..., 1])

    def ccw_nodes(K, i):
        a = X[K, (i + 1) % 3]
        b = X[K, (i + 2) % 3]
        return a[:, None, :] + s[None, :, None] * (b - a)[:, None, :]

    K0, i0 = topo.facet_cell[:, 0], topo.facet_loc[:, 0]
    u = field(ccw_nodes(K0, i0))                       # global direction = owner's CCW
    f = features(u, ids, rev).reshape(-1, 5, m)
    assert np.abs(f[:, 0] - u).max() < 1e-12
    for side in (0, 1):
        K, i = topo.facet_cell[:, side], topo.facet_loc[:, side]
        for jj in (1, 2):
            slot = 1 + 2 * side + (jj - 1)
            want = field(ccw_nodes(K, (i + jj) % 3))
            assert np.abs(f[:, slot] - want).max() < 1e-12


def _small_problem(p=2, n=4):
    from oracle.p1 import TraceMultigrid
    hier = hi.torus_hierarchy(n, 2)
    hdg = HdgOracle(hier.fine, p, dt=0.05, f0=1.0)
    return hier, hdg, TraceMultigrid(hdg, hier)


def test_training_pair_limits():
    """coarse_its = 0 gives t = e - omega D^-1 S e; many P1 V-cycles converge to
    the exact coarse complement (I - pi S_c^-1 pi^T S) e, computed here with a
    dense solve of S_c."""
    from oracle.mlp import training_pair
    hier, hdg, tmg = _small_problem()
    e = np.random.default_rng(7).standard_normal(hdg.S.shape[0])
    u0, t0 = training_pair(tmg, e, 0)
    Dfull = np.zeros((tmg.ne * tmg.m, tmg.ne * tmg.m))
    for k in range(tmg.ne):
        Dfull[k * tmg.m:(k + 1) * tmg.m, k * tmg.m:(k + 1) * tmg.m] = tmg.D[k]
    S = hdg.S.toarray()
    u_ref = tmg.omega * np.linalg.solve(Dfull, S @ e)
    assert np.abs(u0 - u_ref).max() < 1e-12 * np.abs(u_ref).max()
    assert np.abs(t0 - (e - u_ref)).max() < 1e-12 * np.abs(e).max()
    _, t50 = training_pair(tmg, e, 50)
    Pi = tmg.pi.toarray()
    Sc = tmg.Sc.toarray()
    exact = e - Pi @ np.linalg.solve(Sc, Pi.T @ (S @ e)) - u_ref
    assert np.abs(t50 - exact).max() < 1e-9 * np.abs(exact).max()


def test_learned_vcycle_reduces_to_block_jacobi():
    """W2 = 0: the learned step is the block-Jacobi step, so the two V-cycles agree."""
    from oracle.mlp import LearnedTraceMultigrid
    hier, hdg, tmg = _small_problem()
    W1, W2 = init_weights(hdg.m, 64, seed=1)
    lmg = LearnedTraceMultigrid(hdg, hier, W1, W2)
    b = np.random.default_rng(8).standard_normal(hdg.S.shape[0])
    assert np.abs(lmg.vcycle(b) - tmg.vcycle(b)).max() < 1e-12 * np.abs(tmg.vcycle(b)).max()


def test_learned_vcycle_is_positively_homogeneous():
    """With nonzero weights the cycle is nonlinear but V(a b) = a V(b) for a > 0."""
    from oracle.mlp import LearnedTraceMultigrid
    hier, hdg, _ = _small_problem()
    W1, _ = init_weights(hdg.m, 64, seed=1)
    W2 = np.random.default_rng(2).standard_normal((hdg.m, 64)) * 0.05
    lmg = LearnedTraceMultigrid(hdg, hier, W1, W2)
    b = np.random.default_rng(9).standard_normal(hdg.S.shape[0])
    v1, v2 = lmg.vcycle(b), lmg.vcycle(3.0 * b)
    assert np.abs(v2 - 3.0 * v1).max() < 1e-11 * np.abs(v2).max()
    assert np.abs(lmg.vcycle(-b) + v1).max() > 1e-6 * np.abs(v1).max()   # not odd: ReLU


def test_weight_file_round_trip(tmp_path):
    from paper_2004_09389_amd.learned import load_weights, save_weights
    W1, _ = init_weights(3, 64, seed=5)
    W2 = np.random.default_rng(6).standard_normal((3, 64))
    path = str(tmp_path / "w.bin")
    save_weights(path, 2, W1, W2)
    p, A, B = load_weights(path)
    assert p == 2 and np.array_equal(A, W1.astype(np.float32)) and np.array_equal(B, W2.astype(np.float32))
    with open(path, "r+b") as f:
        f.write(b"XXXX")
    with pytest.raises(ValueError):
        load_weights(path)
