"""The non-hybridised DG solver with the approximate Schur-complement
preconditioner (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Native DG section (Eqs. native_dg_system, native_matrix_representation,
S_approx_diag): GMRES on the standard DG system A q = R of one implicit stage,
split by field as [[A_pp, A_pu], [A_up, A_uu]], preconditioned by three steps:

  1. V   ~ A_uu^-1 R_u
  2. Phi ~ S^-1 (R_p - A_pu V),   S = A_pp - A_pu diag(A_uu)^-1 A_up
  3. U   ~ A_uu^-1 (R_u - A_up Phi)

Readings (the paper runs PETSc's fieldsplit with ILU for A_uu and one GAMG
V-cycle with Chebyshev smoothing for S):
* A_uu^-1 ~ cell-block Jacobi: the exact inverse of each cell's 2n x 2n
  diagonal block of A_uu (ILU's parallel counterpart on the DG block
  structure);
* S^-1 ~ one two-level cycle on the DG phi space: Chebyshev(nu) smoothing
  preconditioned by the inverse of each cell's own block
  A_pp,KK - A_pu,KK D_K^-1 A_up,KK (the paths through neighbouring cells left
  out), on [0.1, 1.1] lambda_max (20 power steps from the fixed start vector
  of p1.power_start), then the coarse correction on conforming P1 with the
  Galerkin operator P^T S P (P: nodal interpolation of P1 into the DG phi
  space), solved by one P1 geometric-multigrid V-cycle with Galerkin
  coarsening, then Chebyshev(nu) again.

All vectors are in the symmetric variables of the hdg module, ordered
(cell, field, node) as DgOracle.matrix().
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .hdg import DgOracle
from .p1 import P1Multigrid, chebyshev, power_estimate


def interpolation(mesh, p):
    """P: P1 vertex values -> DG phi nodal values, (n_cell * n_loc, n_vert):
    the value at lattice node (i, j) / p of cell K is the barycentric
    combination (1 - (i+j)/p, i/p, j/p) of its three corner values."""
    lat = [(i, j) for j in range(p + 1) for i in range(p + 1 - j)]
    n = len(lat)
    nk = mesh.n_cell
    w = np.array([[1.0 - (i + j) / p, i / p, j / p] for i, j in lat])        # (n, 3)
    rows = np.repeat(np.arange(nk * n), 3)
    cols = np.repeat(mesh.cell_vert[:, None, :], n, axis=1).reshape(-1)
    vals = np.tile(w.reshape(-1), nk)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nk * n, mesh.n_vert))


class DgApproxSchur:
    """The DG system, its field blocks and the three-step preconditioner."""

    def __init__(self, hier, p, dt, g=1.0, H=1.0, f0=0.0, omega=0.0, tau=1.0, nu=2, p1_nu=2,
                 p1_omega=2.0 / 3.0):
        mesh = hier.fine
        self.dg = DgOracle(mesh, p, dt, g, H, f0, omega, tau)
        self.hier, self.p, self.nu = hier, p, nu
        n, nk = self.dg.n, mesh.n_cell
        self.n, self.nk = n, nk
        A = self.dg.matrix().tocsr()
        self.A = A
        cell = np.arange(nk)[:, None] * 3 * n
        self.ip = (cell + np.arange(n)[None, :]).ravel()
        self.iu = (cell + n + np.arange(2 * n)[None, :]).ravel()
        self.App = A[self.ip][:, self.ip].tocsr()
        self.Apu = A[self.ip][:, self.iu].tocsr()
        self.Aup = A[self.iu][:, self.ip].tocsr()
        self.Auu = A[self.iu][:, self.iu].tocsr()
        self.D = self.Auu.diagonal()
        self.S = (self.App - self.Apu @ sp.diags(1.0 / self.D) @ self.Aup).tocsr()
        # cell-diagonal blocks
        self.Auu_inv = np.linalg.inv(self._cell_blocks(self.Auu, 2 * n, 2 * n))
        Spp = self._cell_blocks(self.App, n, n)
        Spu = self._cell_blocks(self.Apu, n, 2 * n)
        Sup = self._cell_blocks(self.Aup, 2 * n, n)
        Dk = self.D.reshape(nk, 2 * n)
        self.S_own = Spp - np.einsum("kab,kb,kbc->kac", Spu, 1.0 / Dk, Sup)
        self.S_own_inv = np.linalg.inv(self.S_own)
        self.lmax = power_estimate(self.S, self.own_prec)
        self.P = interpolation(mesh, p)
        self.Sc = (self.P.T @ self.S @ self.P).tocsr()
        self.mg = P1Multigrid(hier, None, omega=p1_omega, nu=p1_nu, fine_operator=self.Sc)

    def _cell_blocks(self, M, r, c):
        """(nk, r, c) diagonal cell blocks of a field block ordered by cell."""
        out = np.zeros((self.nk, r, c))
        Mc = M.tocoo()
        K = Mc.row // r
        keep = (Mc.col // c) == K
        out[K[keep], Mc.row[keep] % r, Mc.col[keep] % c] = Mc.data[keep]
        return out

    def own_prec(self, x):
        return np.einsum("kab,kb->ka", self.S_own_inv, x.reshape(self.nk, self.n)).ravel()

    def auu_solve(self, x):
        return np.einsum("kab,kb->ka", self.Auu_inv, x.reshape(self.nk, 2 * self.n)).ravel()

    def s_cycle(self, b):
        """One two-level cycle for S x = b from x = 0."""
        a, bnd = 0.1 * self.lmax, 1.1 * self.lmax
        x = chebyshev(self.S, self.own_prec, b, np.zeros_like(b), self.nu, a, bnd)
        r = b - self.S @ x
        x = x + self.P @ self.mg.vcycle(self.P.T @ r)
        return chebyshev(self.S, self.own_prec, b, x, self.nu, a, bnd)

    def precondition(self, R, auu_solve=None, s_solve=None):
        """The three steps for R (N,); the sub-solves default to the readings
        above and may be replaced (e.g. by exact solves)."""
        auu_solve = auu_solve or self.auu_solve
        s_solve = s_solve or self.s_cycle
        Rp, Ru = R[self.ip], R[self.iu]
        V = auu_solve(Ru)
        Phi = s_solve(Rp - self.Apu @ V)
        U = auu_solve(Ru - self.Aup @ Phi)
        out = np.zeros_like(R)
        out[self.ip], out[self.iu] = Phi, U
        return out

    def rhs(self, r_cell):
        """R = mass-weighted (r, v)_K in symmetric variables, (N,)."""
        return self.dg.load(r_cell).ravel()

    def to_cell(self, x):
        q = x.reshape(self.nk, 3, self.n).copy()
        q[:, 0] /= self.dg.hscale
        return q

    def gmres(self, R, rtol=1e-10, restart=30, maxit=300):
        """Right-preconditioned restarted GMRES on A q = R (true residual);
        returns (q, iterations)."""
        N = R.shape[0]
        x = np.zeros(N)
        bn = np.linalg.norm(R)
        its = 0
        while its < maxit:
            r = R - self.A @ x
            beta = np.linalg.norm(r)
            if beta <= rtol * bn:
                break
            V = [r / beta]
            Z = []
            Hm = np.zeros((restart + 1, restart))
            k = 0
            for k in range(restart):
                z = self.precondition(V[k])
                Z.append(z)
                w = self.A @ z
                for j in range(k + 1):
                    Hm[j, k] = w @ V[j]
                    w = w - Hm[j, k] * V[j]
                Hm[k + 1, k] = np.linalg.norm(w)
                its += 1
                e1 = np.zeros(k + 2)
                e1[0] = beta
                y = np.linalg.lstsq(Hm[:k + 2, :k + 1], e1, rcond=None)[0]
                res = np.linalg.norm(Hm[:k + 2, :k + 1] @ y - e1)
                if res <= rtol * bn or Hm[k + 1, k] == 0.0 or its >= maxit:
                    break
                V.append(w / Hm[k + 1, k])
            x = x + np.column_stack(Z) @ y
        return x, its

    def direct(self, R):
        return spla.splu(self.A.tocsc()).solve(R)
