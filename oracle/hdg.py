"""HDG and standard-DG systems for one implicit stage of the linearised SWE (oracle).

Equations.  The caller's problem  u + dt (f k x u + g grad h) = r_u,
h + dt H div u = r_h  is rewritten in the symmetric variables of the paper's
linearised SWE (Eq. SWE_continuum_linear with flat bathymetry phi_B = 1):
c = sqrt(g H), phi = h sqrt(g/H), kappa = c dt (the paper's c_g alpha dt with
alpha = 1), giving

    phi + kappa div u = r_phi,     u + dt f k x u + kappa grad phi = r_u,

with r_phi = sqrt(g/H) r_h.  Inputs are the DG coefficients of (r_h, r_u);
the right-hand side functional is R(v) = (r, v) (Eq. ABCMform, f the Riesz
representer).

HDG form (Eq. bilinear_HDG_upwind with phi_B = 1 and the stabilisation
2 sqrt(phi_B) {{.}} written per side as tau): for every cell K

  (phi,psi)_K - kappa (u, grad psi)_K + kappa <u.n + tau (phi - lam), psi>_dK
  (u,w)_K + dt (f k x u, w)_K - kappa (phi, div w)_K + kappa <lam, w.n>_dK

and on every facet  sum_K <u.n + tau (phi - lam), mu>_e = 0  (flux
condition, Eq. flux_condition).  Split as A q + B lam = f,  C q - M lam = 0
(Eq. ABCMform); Schur complement S = M + C A^-1 B, rhat = C A^-1 f,
q = A^-1 (f - B lam) (Steps 1-3, Eqs. schur_system, reconstruct_solution).

Standard DG (Appendix A, Eq. bilinear_standardDG_upwind): on straight facets
the trace condition holds pointwise, so lam = {{phi}} + [[u]] / (2 tau); the
mass flux on side K is (u_K.n_K - u_o.n_o)/2 + tau (phi_K - phi_o)/2 and the
momentum flux is lam n_K.  Written with each side's own normal it also holds
on the piecewise-flat sphere (no curvature term is needed).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import (CellBasis, facet_points, facet_rule, geometry, lagrange1d,
                  to_3d, topology, volume_points)


def n_loc(p):
    return (p + 1) * (p + 2) // 2


class LocalOperators:
    """Per-cell matrices of the HDG form (oracle).

    Ordering of cell unknowns: [phi (n), u_1 (n), u_2 (n)]; of local trace
    unknowns: local facet 0, 1, 2, each with p+1 nodes in the cell's
    counter-clockwise direction.
    """

    def __init__(self, mesh, p, dt, g=1.0, H=1.0, f0=0.0, omega=0.0, tau=1.0):
        self.mesh, self.p, self.dt, self.g, self.H = mesh, p, dt, g, H
        self.f0, self.omega, self.tau = f0, omega, tau
        self.c = np.sqrt(g * H)
        self.kappa = self.c * dt
        self.hscale = np.sqrt(g / H)           # phi = hscale * h
        self.geo = geometry(mesh)
        self.topo = topology(mesh)
        self.basis = CellBasis(self.geo, p)
        self.n = n_loc(p)
        self.m = p + 1
        self._volume()
        self._facets()

    # -- Coriolis parameter: constant on the torus, 2 Omega sin(latitude) on the sphere
    def coriolis(self, X3):
        f = np.full(X3.shape[:-1], self.f0)
        if self.mesh.kind == "sphere" and self.omega != 0.0:
            f = f + 2.0 * self.omega * X3[..., 2] / np.linalg.norm(X3, axis=-1)
        return f

    def _volume(self):
        Z, w = volume_points(self.geo, 2 * self.p + 2)
        Phi = self.basis.values(Z)
        G = self.basis.grads(Z)
        fq = self.coriolis(to_3d(self.geo, Z))
        self.M = np.einsum("cq,cqi,cqj->cij", w, Phi, Phi)
        self.Mf = np.einsum("cq,cq,cqi,cqj->cij", w, fq, Phi, Phi)
        # Q[d][c, i, j] = (phi_j, d_d phi_i)_K
        self.Q = [np.einsum("cq,cqi,cqj->cij", w, G[..., d], Phi) for d in range(2)]

    def _facets(self):
        p, m = self.p, self.m
        s, ws = facet_rule(p)
        mu = lagrange1d(p, s)
        self.fvals, self.fw = [], []
        self.E, self.T, self.F = [], [], []
        for i in range(3):
            Zf = facet_points(self.geo, i, s)
            V = self.basis.values(Zf)                       # (nk, nq, n)
            wt = ws[None, :] * self.geo.flen[:, i:i + 1]    # (nk, nq)
            self.fvals.append(V)
            self.fw.append(wt)
            self.E.append(np.einsum("cq,cqi,cqj->cij", wt, V, V))
            self.T.append(np.einsum("cq,cqi,qk->cik", wt, V, mu))
            self.F.append(np.einsum("cq,qk,ql->ckl", wt, mu, mu))

    def hdg_blocks(self):
        """A (nk, 3n, 3n), B (nk, 3n, 3m), C (nk, 3m, 3n), Mt (nk, 3m, 3m)."""
        n, m, kap, tau, dt = self.n, self.m, self.kappa, self.tau, self.dt
        nk = self.M.shape[0]
        nrm = self.geo.fnormal
        A = np.zeros((nk, 3 * n, 3 * n))
        B = np.zeros((nk, 3 * n, 3 * m))
        C = np.zeros((nk, 3 * m, 3 * n))
        Mt = np.zeros((nk, 3 * m, 3 * m))
        P, U = slice(0, n), [slice(n, 2 * n), slice(2 * n, 3 * n)]
        A[:, P, P] = self.M
        for d in range(2):
            A[:, P, U[d]] = -kap * self.Q[d]
            A[:, U[d], P] = -kap * self.Q[d]
            A[:, U[d], U[d]] = self.M
        A[:, U[0], U[1]] = -dt * self.Mf
        A[:, U[1], U[0]] = dt * self.Mf
        for i in range(3):
            L = slice(i * m, (i + 1) * m)
            nd = [nrm[:, i, 0][:, None, None], nrm[:, i, 1][:, None, None]]
            A[:, P, P] += kap * tau * self.E[i]
            for d in range(2):
                A[:, P, U[d]] += kap * nd[d] * self.E[i]
            B[:, P, L] = -kap * tau * self.T[i]
            C[:, L, P] = tau * np.transpose(self.T[i], (0, 2, 1))
            for d in range(2):
                B[:, U[d], L] = kap * nd[d] * self.T[i]
                C[:, L, U[d]] = nd[d] * np.transpose(self.T[i], (0, 2, 1))
            Mt[:, L, L] = tau * self.F[i]
        return A, B, C, Mt

    def trace_index(self):
        """Global trace dof of each local trace dof, (nk, 3m)."""
        p, m = self.p, self.m
        t = self.topo
        k = np.arange(m)
        g = np.zeros((t.cell_facet.shape[0], 3 * m), dtype=np.int64)
        for i in range(3):
            kk = np.where(t.cell_rev[:, i:i + 1], p - k[None, :], k[None, :])
            g[:, i * m:(i + 1) * m] = t.cell_facet[:, i:i + 1] * m + kk
        return g

    def load(self, r_cell):
        """Mass-weighted right-hand side f = (r, v)_K in symmetric variables.

        r_cell: (nk, 3, n) DG coefficients of (r_h, r_u1, r_u2) -> (nk, 3n).
        """
        r = np.array(r_cell, dtype=np.float64)
        r[:, 0] *= self.hscale
        return np.einsum("cij,cfj->cfi", self.M, r).reshape(r.shape[0], -1)


class HdgOracle(LocalOperators):
    """Hybridised system, Schur complement and three-step solve (oracle)."""

    def __init__(self, *args, **kw):
        super().__init__(*args, **kw)
        A, B, C, Mt = self.hdg_blocks()
        self.A, self.B, self.C, self.Mt = A, B, C, Mt
        Ainv = np.linalg.inv(A)
        self.Ainv = Ainv
        self.Sloc = Mt + C @ Ainv @ B
        self.gidx = self.trace_index()
        nt = 3 * self.m
        rows = np.repeat(self.gidx[:, :, None], nt, axis=2)
        cols = np.repeat(self.gidx[:, None, :], nt, axis=1)
        N = self.topo.n_facet * self.m
        self.S = sp.csr_matrix((self.Sloc.ravel(), (rows.ravel(), cols.ravel())), shape=(N, N))
        self.n_trace = N

    def rhat(self, r_cell):
        """Step 1: rhat = C A^-1 f, scattered to facets.  (n_facet * m,)"""
        f = self.load(r_cell)
        loc = np.einsum("cij,cj->ci", self.C, np.einsum("cij,cj->ci", self.Ainv, f))
        out = np.zeros(self.n_trace)
        np.add.at(out, self.gidx.ravel(), loc.ravel())
        return out

    def recover(self, r_cell, lam):
        """Step 3: q = A^-1 (f - B lam); returned as (nk, 3, n) in (h, u1, u2)."""
        f = self.load(r_cell)
        lk = lam[self.gidx]
        q = np.einsum("cij,cj->ci", self.Ainv, f - np.einsum("cij,cj->ci", self.B, lk))
        q = q.reshape(-1, 3, self.n)
        q[:, 0] /= self.hscale
        return q

    def apply(self, x):
        return self.S @ x

    def solve(self, r_cell):
        """Direct solve of the trace system (SuperLU), then recovery."""
        rh = self.rhat(r_cell)
        lam = spla.splu(self.S.tocsc()).solve(rh)
        return self.recover(r_cell, lam), lam


class DgOracle(LocalOperators):
    """Standard (non-hybridised) upwind DG system, assembled and solved directly."""

    def matrix(self):
        """The implicit-stage system  M + kappa K + dt F  (CSR)."""
        return self._assemble(1.0, self.kappa, self.dt)

    def parts(self):
        """The semi-discrete pieces in symmetric variables, each CSR:
        mass M, the kappa-term K (volume and upwind facet terms at kappa = 1)
        and the Coriolis term F (at dt = 1), so that the stage system is
        M + kappa K + dt F and the time derivative is M q' = -c K q - F q."""
        out = [self._assemble(1.0, 0.0, 0.0), self._assemble(0.0, 1.0, 0.0), self._assemble(0.0, 0.0, 1.0)]
        for a in out:
            a.eliminate_zeros()
        return tuple(out)

    def _assemble(self, cm, kap, dt):
        n, tau = self.n, self.tau
        nk = self.M.shape[0]
        topo, nrm = self.topo, self.geo.fnormal
        rows, cols, vals = [], [], []

        def add(cellr, fr, cellc, fc, blk):
            # blk: (len(cellr), n, n) block at (field fr of cellr, field fc of cellc)
            r = (cellr[:, None] * 3 + fr) * n + np.arange(n)[None, :]
            c = (cellc[:, None] * 3 + fc) * n + np.arange(n)[None, :]
            rows.append(np.repeat(r[:, :, None], n, 2).ravel())
            cols.append(np.repeat(c[:, None, :], n, 1).ravel())
            vals.append(blk.ravel())

        allc = np.arange(nk)
        # cell terms: (phi,psi) + (u,w) + dt (f k x u, w) - kappa (u, grad psi) - kappa (phi, div w)
        add(allc, 0, allc, 0, cm * self.M)
        for d in range(2):
            add(allc, 1 + d, allc, 1 + d, cm * self.M)
            add(allc, 0, allc, 1 + d, -kap * self.Q[d])
            add(allc, 1 + d, allc, 0, -kap * self.Q[d])
        add(allc, 1, allc, 2, -dt * self.Mf)
        add(allc, 2, allc, 1, dt * self.Mf)

        # facet terms, from each side a with partner b
        fc, fl = topo.facet_cell, topo.facet_loc
        FV = np.stack(self.fvals, axis=1)     # (nk, 3, nq, n)
        FW = np.stack(self.fw, axis=1)        # (nk, 3, nq)
        for a_side, b_side in ((0, 1), (1, 0)):
            Ka, Kb = fc[:, a_side], fc[:, b_side]
            ia, ib = fl[:, a_side], fl[:, b_side]
            Va = FV[Ka, ia]                        # (ne, nq, n)
            # the partner runs the facet backwards: reverse its points (symmetric rule)
            Vb = FV[Kb, ib][:, ::-1]
            w = FW[Ka, ia]
            na = nrm[Ka, ia]          # (ne, 2)
            nb = nrm[Kb, ib]
            Eaa = np.einsum("eq,eqi,eqj->eij", w, Va, Va)
            Eab = np.einsum("eq,eqi,eqj->eij", w, Va, Vb)
            # mass flux (u_a.n_a - u_b.n_b)/2 + tau (phi_a - phi_b)/2 tested with psi_a
            add(Ka, 0, Ka, 0, 0.5 * kap * tau * Eaa)
            add(Ka, 0, Kb, 0, -0.5 * kap * tau * Eab)
            for d in range(2):
                add(Ka, 0, Ka, 1 + d, 0.5 * kap * na[:, d, None, None] * Eaa)
                add(Ka, 0, Kb, 1 + d, -0.5 * kap * nb[:, d, None, None] * Eab)
            # momentum flux lam n_a, lam = (phi_a + phi_b)/2 + (u_a.n_a + u_b.n_b)/(2 tau)
            for d in range(2):
                add(Ka, 1 + d, Ka, 0, 0.5 * kap * na[:, d, None, None] * Eaa)
                add(Ka, 1 + d, Kb, 0, 0.5 * kap * na[:, d, None, None] * Eab)
                for d2 in range(2):
                    add(Ka, 1 + d, Ka, 1 + d2, kap / (2 * tau) * (na[:, d] * na[:, d2])[:, None, None] * Eaa)
                    add(Ka, 1 + d, Kb, 1 + d2, kap / (2 * tau) * (na[:, d] * nb[:, d2])[:, None, None] * Eab)
        N = nk * 3 * n
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(N, N))

    def solve(self, r_cell):
        """Returns q (nk, 3, n) in (h, u1, u2) and the facet values
        lam = {{phi}} + [[u]]/(2 tau) at the trace nodes, (n_facet * m,)."""
        Amat = self.matrix()
        f = self.load(r_cell).ravel()
        x = spla.splu(Amat.tocsc()).solve(f)
        q = x.reshape(-1, 3, self.n)
        lam = self.trace_values(q)
        q = q.copy()
        q[:, 0] /= self.hscale
        return q, lam

    def trace_values(self, q):
        """lam at the trace nodes from a DG field q (symmetric variables)."""
        p, m, tau = self.p, self.m, self.tau
        topo, nrm = self.topo, self.geo.fnormal
        sn = np.arange(m) / p
        lam = np.zeros((topo.n_facet, m))
        vals = np.stack([self.basis.values(facet_points(self.geo, i, sn)) for i in range(3)], 1)
        for side in (0, 1):
            K = topo.facet_cell[:, side]
            i = topo.facet_loc[:, side]
            V = vals[K, i]
            if side == 1:
                V = V[:, ::-1]
            phi = np.einsum("eqi,ei->eq", V, q[K, 0])
            un = (np.einsum("eqi,ei->eq", V, q[K, 1]) * nrm[K, i, 0][:, None]
                  + np.einsum("eqi,ei->eq", V, q[K, 2]) * nrm[K, i, 1][:, None])
            lam += 0.5 * phi + un / (2 * tau)
        return lam.ravel()
