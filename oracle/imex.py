"""IMEX Runge-Kutta time stepping of the linearised SWE (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Time discretisation section.  Written in the weak form, the semi-discrete
linear SWE is  d/dt M(q) = N_0(q) + L(q)  (Eq. linear_non_hybridized): M the
mass form, L the linear flux terms (here the standard upwind DG operator; the
HDG solution of each stage coincides with it, Eq. linear_hybridized), and N_0
the source, which for flat bathymetry is the Coriolis term -f u_perp.  The
fast terms L are integrated implicitly and N_0 explicitly.  An s-stage IMEX
method with Butcher tableaux (a, at, b, bt) builds the stages

    M Q_i = M q_n + dt sum_{j<i} a_ij N_0(Q_j) + dt sum_{j<=i} at_ij L(Q_j)

(Eq. IMEX_HDG_I; the j = i term is moved to the left, giving the system
M - at_ii dt L, i.e. the implicit stage solved by the HDG method with
kappa = c at_ii dt) and then

    M q_{n+1} = M q_n + dt sum_i b_i N_0(Q_i) + dt sum_i bt_i L(Q_i)

(Eq. IMEX_HDG_II), one mass solve.  The Theta(theta) method (Eq.
theta_method) is the two-stage tableau whose first stage is q_n.

Tableaux (IMEX methods section): Theta(theta); ARS2(2,3,2) with
gamma = 1 - 1/sqrt 2, delta = -2 sqrt(2) / 3; SSP2(3,2,2); ARS3(4,4,3).
Pinned by the order conditions of the stated orders and by the observed
order of convergence against the matrix exponential of the semi-discrete
system.

Variables: the library's (h, u) with g, H; internally the symmetric
phi = h sqrt(g/H), c = sqrt(g H), as in the hdg module.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse.linalg as spla

from .fem import to_3d, volume_points
from .hdg import DgOracle
from .lf import DgLfOracle

METHODS = ("theta", "ars232", "ssp322", "ars443")


def tableau(method: str, theta: float = 0.5):
    """(a, at, b, bt) as float arrays for one of METHODS."""
    if method == "theta":
        a = [[0, 0], [1, 0]]
        at = [[0, 0], [1 - theta, theta]]
        b = [1, 0]
        bt = [1 - theta, theta]
    elif method == "ars232":
        g = 1.0 - 1.0 / math.sqrt(2.0)
        d = -2.0 * math.sqrt(2.0) / 3.0
        a = [[0, 0, 0], [g, 0, 0], [d, 1 - d, 0]]
        at = [[0, 0, 0], [0, g, 0], [0, 1 - g, g]]
        b = [0, 1 - g, g]
        bt = [0, 1 - g, g]
    elif method == "ssp322":
        a = [[0, 0, 0], [0, 0, 0], [0, 1, 0]]
        at = [[0.5, 0, 0], [-0.5, 0.5, 0], [0, 0.5, 0.5]]
        b = [0, 0.5, 0.5]
        bt = [0, 0.5, 0.5]
    elif method == "ars443":
        a = [[0, 0, 0, 0, 0],
             [1 / 2, 0, 0, 0, 0],
             [11 / 18, 1 / 18, 0, 0, 0],
             [5 / 6, -5 / 6, 1 / 2, 0, 0],
             [1 / 4, 7 / 4, 3 / 4, -7 / 4, 0]]
        b = [1 / 4, 7 / 4, 3 / 4, -7 / 4, 0]
        at = [[0, 0, 0, 0, 0],
              [0, 1 / 2, 0, 0, 0],
              [0, 1 / 6, 1 / 2, 0, 0],
              [0, -1 / 2, 1 / 2, 1 / 2, 0],
              [0, 3 / 2, -3 / 2, 1 / 2, 1 / 2]]
        bt = [0, 3 / 2, -3 / 2, 1 / 2, 1 / 2]
    else:
        raise ValueError(f"unknown IMEX method {method!r}")
    return tuple(np.array(x, dtype=np.float64) for x in (a, at, b, bt))


class LinearSwe:
    """Semi-discrete linear SWE  M q' = L q + N q  in symmetric variables, with
    L = -c K (DG flux terms, upwind or Lax-Friedrichs) and N = -F (Coriolis
    source)."""

    def __init__(self, mesh, p, g=1.0, H=1.0, f=0.0, tau=1.0, flux="upwind"):
        if flux == "upwind":
            self.dg = DgOracle(mesh, p, dt=1.0, g=g, H=H, f0=f, tau=tau)
        elif flux == "lf":
            self.dg = DgLfOracle(mesh, p, dt=1.0, g=g, H=H, f0=f, tau=tau)
        else:
            raise ValueError(f"unknown flux {flux!r}")
        self.c, self.hscale, self.n = self.dg.c, self.dg.hscale, self.dg.n
        M, K, F = self.dg.parts()
        self.M = M.tocsc()
        self.L = (-self.c) * K
        self.N = -F
        self._mass = spla.splu(self.M)
        self._stage = {}

    # -- (n_cell, 3, n_loc, nrhs) coefficients of (h, u1, u2) <-> (N, nrhs) symmetric vectors
    def to_vec(self, q):
        q = np.array(q, dtype=np.float64)
        q[:, 0] *= self.hscale
        return q.reshape(-1, q.shape[-1])

    def from_vec(self, x, nk):
        q = x.reshape(nk, 3, self.n, -1).copy()
        q[:, 0] /= self.hscale
        return q

    def _stage_solver(self, coef):
        if coef not in self._stage:
            self._stage[coef] = spla.splu((self.M - coef * self.L).tocsc())
        return self._stage[coef]

    def step(self, tab, dt, x):
        """One IMEX step from the symmetric vector x (N, nrhs)."""
        a, at, b, bt = tab
        s = len(b)
        Mx = self.M @ x
        NQ, LQ = [], []
        for i in range(s):
            rhs = Mx.copy()
            for j in range(i):
                rhs += dt * a[i, j] * NQ[j] + dt * at[i, j] * LQ[j]
            if at[i, i] == 0.0:
                Q = self._mass.solve(rhs)
            else:
                Q = self._stage_solver(dt * at[i, i]).solve(rhs)
            NQ.append(self.N @ Q)
            LQ.append(self.L @ Q)
        rhs = Mx.copy()
        for i in range(s):
            rhs += dt * b[i] * NQ[i] + dt * bt[i] * LQ[i]
        return self._mass.solve(rhs)

    def run(self, tab, dt, steps, q):
        """`steps` IMEX steps from (n_cell, 3, n_loc, nrhs) coefficients q."""
        x = self.to_vec(q)
        for _ in range(steps):
            x = self.step(tab, dt, x)
        return self.from_vec(x, q.shape[0])

    def tendency(self, q, dt):
        """dt M^-1 L q in (h, u) coefficients: the implicit term of the Theta
        method's first stage (the explicit flux evaluation)."""
        x = self.to_vec(q)
        return self.from_vec(dt * self._mass.solve(self.L @ x), q.shape[0])

    def generator(self):
        """Dense M^-1 (L + N), for the matrix-exponential reference on tiny meshes."""
        A = (self.L + self.N).toarray()
        return np.linalg.solve(self.M.toarray(), A)


def l2_error(swe: LinearSwe, q, exact, period=1.0, degree=None):
    """Delta_2 of Eq. L2_error: the L2 norm over the domain of
    (phi - phi_exact, u - u_exact), with phi = hscale h, by a collapsed Gauss
    rule of the given degree (default 2p + 6) on every cell.
    q: (n_cell, 3, n_loc) coefficients of (h, u1, u2); exact(xy) -> (phi, u1, u2)."""
    dg = swe.dg
    deg = 2 * dg.p + 6 if degree is None else degree
    Z, w = volume_points(dg.geo, deg)
    V = dg.basis.values(Z)                                   # (nk, Q, n)
    xy = to_3d(dg.geo, Z)[..., :2]
    ex = exact(xy)
    err2 = 0.0
    for fld in range(3):
        val = np.einsum("cqi,ci->cq", V, q[:, fld])
        if fld == 0:
            val = val * swe.hscale
        err2 += np.sum(w * (val - ex[fld]) ** 2)
    return math.sqrt(err2)
