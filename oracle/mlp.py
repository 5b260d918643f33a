"""Learned facet-patch smoother: FP64 reference (oracle).

Not in the paper: a small network stands in for the block-Jacobi smoother of
the non-nested V-cycle (the block-Jacobi smoother itself is the future-work
smoother of the conclusion).  Definitions, shared with the library by
convention and implemented here independently:

* patch of facet e: e, then the other two facets of its owner cell (local
  order (i+1)%3, (i+2)%3), then those of its second cell -- the five facets
  of e's block row of S;
* features: u = omega D^-1 r on every patch facet (block-Jacobi corrections of
  the current residual r), slot 0 in the facet's own direction, slots 1-4 in
  the counter-clockwise direction of the cell they are taken from; 5(p+1)
  values per facet and right-hand side, in slot-major order;
* normalisation: s = RMS of the features; network input z = features / s;
* network: h = ReLU(W1 z) (64 hidden units, no biases), y = W2 h ((p+1)
  outputs); correction c = s y on facet e (positively homogeneous in r);
* smoother step: x <- x + u_e + c_e;
* training target for an error e (r = S e): the part of e the coarse grid
  cannot remove, minus the block-Jacobi step: t = [(I - P_c) e]_e - u_e,
  P_c = pi S_c^-1 pi^T S with S_c^-1 applied as a fixed number of P1 V-cycles;
  loss = mean over (facet, rhs) of sum_o (y_o - t_o / s)^2.

Parity unpinned for the learned smoother's benefit (no reference exists);
the forward/backward arithmetic is pinned by a finite-difference check.
"""
from __future__ import annotations

import numpy as np

from .p1 import TraceMultigrid


def patch_table(topo):
    """Patch facet ids (ne, 5) and reversal flags (ne, 5) (slot 0 never reversed)."""
    ne = topo.n_facet
    ids = np.zeros((ne, 5), dtype=np.int64)
    rev = np.zeros((ne, 5), dtype=bool)
    ids[:, 0] = np.arange(ne)
    for side in (0, 1):
        K = topo.facet_cell[:, side]
        i = topo.facet_loc[:, side]
        for jj in (1, 2):
            i2 = (i + jj) % 3
            slot = 1 + 2 * side + (jj - 1)
            ids[:, slot] = topo.cell_facet[K, i2]
            rev[:, slot] = topo.cell_rev[K, i2]
    return ids, rev


def features(u, ids, rev):
    """u: (ne, m) block-Jacobi corrections -> (ne, 5m) patch features."""
    ne, m = u.shape
    f = u[ids]                                  # (ne, 5, m)
    f = np.where(rev[:, :, None], f[:, :, ::-1], f)
    return f.reshape(ne, ids.shape[1] * m)


def forward(W1, W2, feats):
    """Returns correction c (n, m) and the intermediates."""
    n, k = feats.shape
    s = np.sqrt(np.mean(feats ** 2, axis=1))
    safe = np.where(s > 0, s, 1.0)
    z = feats / safe[:, None]
    a = z @ W1.T                                # pre-activation (n, 64)
    h = np.maximum(a, 0.0)
    y = h @ W2.T                                # (n, m)
    c = np.where(s[:, None] > 0, y * s[:, None], 0.0)
    return c, dict(s=s, z=z, a=a, h=h, y=y)


def loss_and_grad(W1, W2, feats, targets):
    """Mean-squared loss on normalised targets and its gradient (dW1, dW2)."""
    _, st = forward(W1, W2, feats)
    s = st["s"]
    safe = np.where(s > 0, s, 1.0)
    tau = targets / safe[:, None]
    d = st["y"] - tau
    n = feats.shape[0]
    loss = float(np.sum(d ** 2) / n)
    dy = 2.0 * d / n                            # (n, m)
    dW2 = dy.T @ st["h"]                        # (m, 64)
    dh = (dy @ W2) * (st["a"] > 0)              # (n, 64)
    dW1 = dh.T @ st["z"]                        # (64, 5m)
    return loss, dW1, dW2


def smoother_step(x, r, Dinv_w, ids, rev, W1, W2):
    """x <- x + u_e + c_e with u = omega D^-1 r (trace vectors as (ne, m))."""
    u = np.einsum("eab,eb->ea", Dinv_w, r)
    c, _ = forward(W1, W2, features(u, ids, rev))
    return x + u + c


def training_pair(tmg, e, coarse_its):
    """(u, t) for the trace error e (flat, facet-major): r = S e,
    u = omega D^-1 r, x_c = coarse_its stationary P1 V-cycles on S_c x_c = pi^T r
    from zero, t = e - pi x_c - u."""
    r = tmg.S @ e
    u = tmg.omega * tmg.block_jacobi(r)
    bc = tmg.pi.T @ r
    xc = np.zeros_like(bc)
    for _ in range(coarse_its):
        xc = xc + tmg.mg.vcycle(bc - tmg.Sc @ xc)
    return u, e - tmg.pi @ xc - u


class LearnedTraceMultigrid(TraceMultigrid):
    """The non-nested V-cycle with every smoothing step replaced by the
    learned step (W2 = 0 gives back the block-Jacobi V-cycle)."""

    def __init__(self, hdg, hier, W1, W2, **kw):
        super().__init__(hdg, hier, **kw)
        self.W1, self.W2 = np.asarray(W1, dtype=np.float64), np.asarray(W2, dtype=np.float64)
        self.ids, self.rev = patch_table(hdg.topo)

    def smooth(self, b, x, nu):
        for _ in range(nu):
            r = (b - self.S @ x).reshape(self.ne, self.m)
            x = smoother_step(x.reshape(self.ne, self.m), r, self.omega * self.Dinv, self.ids, self.rev,
                              self.W1, self.W2).ravel()
        return x


def init_weights(m, hidden=64, seed=0):
    """The seeded initial weights (an input, drawn by hdg_inputs.mlp_init)."""
    from hdg_inputs import mlp_init
    return mlp_init(m, hidden, seed)
