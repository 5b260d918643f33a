"""The stationary vortex of the linearised SWE on the periodic unit square.

Test-case definition (stationary vortex section): radially symmetric
height perturbation phi(r) with compact support on r < r_+ and a purely
tangential velocity u(r) e_theta in geostrophic balance, so that the state
does not change in time.  Paper values (non-dimensional): c_g = 1.89,
f = 4 pi, delta = 0.1, r_- = 0.05, r_+ = 0.45, sigma = 0.25, flat
bathymetry phi_B = 1 for the linear equations.

For the linearised equations (Eq. SWE_continuum_linear with phi_B = 1) the
balance c_g grad phi = -f u_perp of a tangential field gives
u(r) = (c_g / f) phi'(r) = L_R phi'(r), and div u = 0 holds for any u(r)
e_theta.  (The vortex section writes the linear velocity with a factor
(phi + phi_B); with that factor the state would not be steady for the
linearised equations, so the balanced form L_R phi_B phi' is used.)

The paper's domain [-1/2, 1/2]^2 is the periodic unit square here, with the
vortex centred at (period / 2, period / 2); r_+ < 1/2 keeps the support
inside one period.  In the library's variables (h, u) with g = H = c_g the
symmetric variable is phi = h and c = sqrt(g H) = c_g.

Nothing here is part of the method: it evaluates the closed-form state at
given points, and samples it at the DG nodes as an initial condition.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .mesh import Mesh
from .rhs import n_loc, node_coords


@dataclass(frozen=True)
class Vortex:
    c_g: float = 1.89
    f: float = 4.0 * math.pi
    delta: float = 0.1
    r_minus: float = 0.05
    r_plus: float = 0.45
    sigma: float = 0.25
    centre: float = 0.5          # both coordinates, in units of the period

    @property
    def L_R(self) -> float:
        return self.c_g / self.f

    def _s(self, r):
        """The tanh argument and its derivative on r_- < r < r_+ (elsewhere 0)."""
        inside = (r > self.r_minus) & (r < self.r_plus)
        ri = np.where(inside, r, 0.5 * (self.r_minus + self.r_plus))
        a, b = ri - self.r_minus, ri - self.r_plus
        s = self.sigma / a + self.sigma / b
        ds = -self.sigma / a ** 2 - self.sigma / b ** 2
        return inside, s, ds

    def phi(self, r):
        r = np.asarray(r, dtype=np.float64)
        inside, s, _ = self._s(r)
        val = 0.5 * (1.0 + np.tanh(s))
        val = np.where(inside, val, np.where(r <= self.r_minus, 1.0, 0.0))
        return -self.delta * val

    def dphi(self, r):
        r = np.asarray(r, dtype=np.float64)
        inside, s, ds = self._s(r)
        sech2 = 1.0 / np.cosh(np.clip(s, -350.0, 350.0)) ** 2
        return np.where(inside, -0.5 * self.delta * sech2 * ds, 0.0)

    def state(self, xy, period: float = 1.0):
        """(phi, u_x, u_y) at points xy (..., 2), each of shape xy.shape[:-1]."""
        d = np.asarray(xy, dtype=np.float64) - self.centre * period
        d = d - period * np.round(d / period)          # nearest periodic image
        r = np.hypot(d[..., 0], d[..., 1])
        ut = self.L_R * self.dphi(r)
        rs = np.where(r > 0.0, r, 1.0)
        return self.phi(r), -ut * d[..., 1] / rs, ut * d[..., 0] / rs


def vortex_coefficients(mesh: Mesh, p: int, vortex: Vortex = Vortex()) -> np.ndarray:
    """The vortex sampled at the DG nodes: (n_cell, 3, n_loc, 1) values of (h, u_x, u_y)."""
    if mesh.kind != "torus":
        raise ValueError("the stationary vortex is defined on the periodic square")
    xy = node_coords(mesh, p)[..., :2]
    phi, ux, uy = vortex.state(xy, mesh.period)
    out = np.zeros((mesh.n_cell, 3, n_loc(p), 1))
    out[:, 0, :, 0], out[:, 1, :, 0], out[:, 2, :, 0] = phi, ux, uy
    return out


def paper_time_step(n: int, p: int, c_g: float = 1.89, rho: float = 0.2, gamma: float = 10.0,
                    t_final: float = 0.5):
    """Time step of the time-step-size section: the explicit step
    c_g dt_expl / h = rho / (2p + 1) with h = 1/n, times gamma; the final time
    t_final is reached in a whole number of equal steps (dt rounded down).
    Returns (dt, n_steps)."""
    dt0 = gamma * rho / ((2 * p + 1) * c_g * n)
    steps = int(math.ceil(t_final / dt0 - 1e-12))
    return t_final / steps, steps
