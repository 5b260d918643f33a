"""Lax-Friedrichs flux: hybridised system with a vector trace and the
lowest-order Raviart-Thomas coarse space (oracle).

HDG form (Eq. bilinear_HDG_lax with phi_B = 1, the stabilisation written per
side as tau; tau = 1 is the paper's flux).  The trace is a vector uhat in
Lambda_h x Lambda_h and the form does not involve a scalar trace.  For every
cell K

  (phi,psi)_K - kappa (u, grad psi)_K + kappa <uhat.n, psi>_dK
  (u,w)_K + dt (f k x u, w)_K - kappa (phi, div w)_K
        + kappa <phi n + tau (u - uhat), w>_dK

and on every facet  sum_K <phi_K n_K + tau (u_K - uhat), what>_e = 0.  The
split A q + B uhat = f, C q - M uhat = 0 and the Schur complement
S = M + C A^-1 B are those of the upwind case (Eq. ABCMform, Steps 1-3).

Standard DG with the same flux (the plain definition of the result): the
trace condition holds pointwise on straight facets, so
uhat = {{u}} + [[phi]]/(2 tau) with [[phi]] = phi_a n_a + phi_b n_b; the mass
flux on side a is uhat.n_a and the momentum flux is
(phi_a n_a - phi_b n_b)/2 + tau (u_a - u_b)/2 -- on flat facets the local
Lax-Friedrichs (Rusanov) flux of the linear system, penalising the jump of
every velocity component.

Trace layout: facet e, Cartesian component d, node k -> e*2m + d*m + k (node
k in the facet's direction).  Torus only: on the piecewise-flat sphere the
two cells of a facet have different tangent planes, and a vector trace
needs a convention the paper handles only through the curvature term of its
non-hybridised scheme.

Coarse space (non-nested multigrid section, Lax-Friedrichs case): lowest-
order Raviart-Thomas on the same mesh.  DOF of facet e: the flux
int_e u.n_e ds, n_e the owner cell's outward normal.  Basis on cell K:
sigma_i (x - v_i) / (2|K|) for the local facet i opposite local vertex i,
sigma_i = +1 in the owner and -1 in the other cell.  Prolongation pi: the
L2 projection of {{u_c}} onto the trace space; u_c is linear along a facet,
so for p >= 1 this is the nodal value of the two cells' average.
Restriction: pi^T.  Coarse form S_c = (1/kappa) [(u, w) + kappa^2 (div u,
div w)] (Eq. coarse_problem_LF with the scale of the upwind case: the trace
equation is not multiplied by kappa); the scale is pinned by the Galerkin
ratio test.

The RT0 problem is solved approximately by one geometric-multigrid V-cycle
over the nested torus hierarchy (the paper uses AMG here and names patch
smoothers as the geometric alternative): RT0 spaces of nested meshes are
nested, so the transfer is the inclusion (the coarse field's exact flux
through each fine facet) and the rediscretised S_c equals P^T A P; the
smoother is additive Schwarz over vertex patches (all facets touching a
vertex, exact patch solve, damping omega_p), whose patches contain the
discrete-divergence-free fields that point Jacobi cannot smooth; the coarsest
level is solved with a dense inverse.

The trace cycle as a linear operator is pinned to the two-level iteration
matrix (exact RT0 coarse inverse, and the textbook RT0 V-cycle with
vertex-patch Schwarz smoothing built from explicit matrices); the other pins
fix the discretisation, the transfer and the coarse scale.  Parity unpinned
for the convergence rate the cycle reaches (no printed reference for this
configuration beyond the paper's iteration counts).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .fem import facet_points, geometry, topology
from .hdg import LocalOperators
from .quadrature import triangle_rule


# --------------------------------------------------------------------------- HDG with the LF flux

class LfLocal(LocalOperators):
    """Per-cell matrices of the Lax-Friedrichs HDG form.

    Cell unknowns [phi (n), u_1 (n), u_2 (n)]; local trace unknowns: local
    facet i, component d, node k (cell's counter-clockwise direction) at
    i*2m + d*m + k.
    """

    def __init__(self, mesh, *args, **kw):
        if mesh.kind != "torus":
            raise ValueError("the Lax-Friedrichs trace is built on the torus only")
        super().__init__(mesh, *args, **kw)
        self.mt = 2 * self.m          # trace unknowns per facet

    def hdg_blocks(self):
        n, m, kap, tau, dt = self.n, self.m, self.kappa, self.tau, self.dt
        nk = self.M.shape[0]
        nrm = self.geo.fnormal
        nt = 3 * 2 * m
        A = np.zeros((nk, 3 * n, 3 * n))
        B = np.zeros((nk, 3 * n, nt))
        C = np.zeros((nk, nt, 3 * n))
        Mt = np.zeros((nk, nt, nt))
        P, U = slice(0, n), [slice(n, 2 * n), slice(2 * n, 3 * n)]
        A[:, P, P] = self.M
        for d in range(2):
            A[:, P, U[d]] = -kap * self.Q[d]           # -kappa (u, grad psi)
            A[:, U[d], P] = -kap * self.Q[d]           # -kappa (phi, div w)
            A[:, U[d], U[d]] = self.M
        A[:, U[0], U[1]] = -dt * self.Mf
        A[:, U[1], U[0]] = dt * self.Mf
        for i in range(3):
            for d in range(2):
                nd = nrm[:, i, d][:, None, None]
                L = slice(i * 2 * m + d * m, i * 2 * m + (d + 1) * m)
                Tt = np.transpose(self.T[i], (0, 2, 1))
                A[:, U[d], P] += kap * nd * self.E[i]            # kappa <phi n, w>
                A[:, U[d], U[d]] += kap * tau * self.E[i]        # kappa tau <u, w>
                B[:, P, L] = kap * nd * self.T[i]                # kappa <uhat.n, psi>
                B[:, U[d], L] = -kap * tau * self.T[i]           # -kappa tau <uhat, w>
                C[:, L, P] = nd * Tt                             # <phi n, what>
                C[:, L, U[d]] = tau * Tt                         # tau <u, what>
                Mt[:, L, L] = tau * self.F[i]                    # tau <uhat, what>
        return A, B, C, Mt

    def trace_index(self):
        """Global trace dof of each local trace dof, (nk, 6m)."""
        p, m = self.p, self.m
        t = self.topo
        k = np.arange(m)
        g = np.zeros((t.cell_facet.shape[0], 6 * m), dtype=np.int64)
        for i in range(3):
            kk = np.where(t.cell_rev[:, i:i + 1], p - k[None, :], k[None, :])
            for d in range(2):
                g[:, i * 2 * m + d * m:i * 2 * m + (d + 1) * m] = t.cell_facet[:, i:i + 1] * 2 * m + d * m + kk
        return g


class HdgLfOracle(LfLocal):
    """Lax-Friedrichs hybridised system, Schur complement and three-step solve."""

    def __init__(self, *args, **kw):
        super().__init__(*args, **kw)
        A, B, C, Mt = self.hdg_blocks()
        self.A, self.B, self.C, self.Mt = A, B, C, Mt
        self.Ainv = np.linalg.inv(A)
        self.Sloc = Mt + C @ self.Ainv @ B
        self.gidx = self.trace_index()
        nt = 6 * self.m
        rows = np.repeat(self.gidx[:, :, None], nt, axis=2)
        cols = np.repeat(self.gidx[:, None, :], nt, axis=1)
        N = self.topo.n_facet * self.mt
        self.S = sp.csr_matrix((self.Sloc.ravel(), (rows.ravel(), cols.ravel())), shape=(N, N))
        self.n_trace = N

    def rhat(self, r_cell):
        f = self.load(r_cell)
        loc = np.einsum("cij,cj->ci", self.C, np.einsum("cij,cj->ci", self.Ainv, f))
        out = np.zeros(self.n_trace)
        np.add.at(out, self.gidx.ravel(), loc.ravel())
        return out

    def recover(self, r_cell, lam):
        f = self.load(r_cell)
        q = np.einsum("cij,cj->ci", self.Ainv, f - np.einsum("cij,cj->ci", self.B, lam[self.gidx]))
        q = q.reshape(-1, 3, self.n)
        q[:, 0] /= self.hscale
        return q

    def apply(self, x):
        return self.S @ x

    def solve(self, r_cell):
        rh = self.rhat(r_cell)
        lam = spla.splu(self.S.tocsc()).solve(rh)
        return self.recover(r_cell, lam), lam


class DgLfOracle(LfLocal):
    """Standard DG with the Lax-Friedrichs flux, assembled and solved directly."""

    def matrix(self):
        """The implicit-stage system  M + kappa K + dt F  (CSR)."""
        return self._assemble(1.0, self.kappa, self.dt)

    def parts(self):
        """Mass M, the kappa-term K (at kappa = 1) and the Coriolis term F (at
        dt = 1), each CSR, in symmetric variables (see DgOracle.parts)."""
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
            r = (cellr[:, None] * 3 + fr) * n + np.arange(n)[None, :]
            c = (cellc[:, None] * 3 + fc) * n + np.arange(n)[None, :]
            rows.append(np.repeat(r[:, :, None], n, 2).ravel())
            cols.append(np.repeat(c[:, None, :], n, 1).ravel())
            vals.append(blk.ravel())

        allc = np.arange(nk)
        add(allc, 0, allc, 0, cm * self.M)
        for d in range(2):
            add(allc, 1 + d, allc, 1 + d, cm * self.M)
            add(allc, 0, allc, 1 + d, -kap * self.Q[d])
            add(allc, 1 + d, allc, 0, -kap * self.Q[d])
        add(allc, 1, allc, 2, -dt * self.Mf)
        add(allc, 2, allc, 1, dt * self.Mf)

        fc, fl = topo.facet_cell, topo.facet_loc
        FV = np.stack(self.fvals, axis=1)
        FW = np.stack(self.fw, axis=1)
        for a_side, b_side in ((0, 1), (1, 0)):
            Ka, Kb = fc[:, a_side], fc[:, b_side]
            ia, ib = fl[:, a_side], fl[:, b_side]
            Va = FV[Ka, ia]
            Vb = FV[Kb, ib][:, ::-1]
            w = FW[Ka, ia]
            na, nb = nrm[Ka, ia], nrm[Kb, ib]
            Eaa = np.einsum("eq,eqi,eqj->eij", w, Va, Va)
            Eab = np.einsum("eq,eqi,eqj->eij", w, Va, Vb)
            nab = np.einsum("ed,ed->e", na, nb)[:, None, None]
            # mass flux uhat.n_a = (u_a + u_b).n_a / 2 + (phi_a + phi_b n_b.n_a) / (2 tau)
            add(Ka, 0, Ka, 0, kap / (2 * tau) * Eaa)
            add(Ka, 0, Kb, 0, kap / (2 * tau) * nab * Eab)
            for d in range(2):
                add(Ka, 0, Ka, 1 + d, 0.5 * kap * na[:, d, None, None] * Eaa)
                add(Ka, 0, Kb, 1 + d, 0.5 * kap * na[:, d, None, None] * Eab)
            # momentum flux (phi_a n_a - phi_b n_b)/2 + tau (u_a - u_b)/2
            for d in range(2):
                add(Ka, 1 + d, Ka, 0, 0.5 * kap * na[:, d, None, None] * Eaa)
                add(Ka, 1 + d, Kb, 0, -0.5 * kap * nb[:, d, None, None] * Eab)
                add(Ka, 1 + d, Ka, 1 + d, 0.5 * kap * tau * Eaa)
                add(Ka, 1 + d, Kb, 1 + d, -0.5 * kap * tau * Eab)
        N = nk * 3 * n
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(N, N))

    def solve(self, r_cell):
        """q (nk, 3, n) in (h, u1, u2) and uhat = {{u}} + [[phi]]/(2 tau) at the
        trace nodes, (n_facet * 2m,)."""
        Amat = self.matrix()
        x = spla.splu(Amat.tocsc()).solve(self.load(r_cell).ravel())
        q = x.reshape(-1, 3, self.n)
        lam = self.trace_values(q)
        q = q.copy()
        q[:, 0] /= self.hscale
        return q, lam

    def trace_values(self, q):
        p, m, tau = self.p, self.m, self.tau
        topo, nrm = self.topo, self.geo.fnormal
        sn = np.arange(m) / p
        lam = np.zeros((topo.n_facet, 2, m))
        vals = np.stack([self.basis.values(facet_points(self.geo, i, sn)) for i in range(3)], 1)
        for side in (0, 1):
            K, i = topo.facet_cell[:, side], topo.facet_loc[:, side]
            V = vals[K, i]
            if side == 1:
                V = V[:, ::-1]
            phi = np.einsum("eqi,ei->eq", V, q[K, 0])
            for d in range(2):
                ud = np.einsum("eqi,ei->eq", V, q[K, 1 + d])
                lam[:, d] += 0.5 * ud + phi * nrm[K, i, d][:, None] / (2 * tau)
        return lam.ravel()


# --------------------------------------------------------------------------- RT0 coarse space

class Rt0Space:
    """Lowest-order Raviart-Thomas space on a torus mesh (flux DOFs per facet)."""

    def __init__(self, mesh):
        if mesh.kind != "torus":
            raise ValueError("RT0 coarse space: torus only")
        self.mesh = mesh
        self.geo = geometry(mesh)
        self.topo = topology(mesh)
        self.sigma = np.where(self.topo.cell_rev, -1.0, 1.0)      # (nk, 3)

    def eval(self, K, X, F):
        """u_c at points X (len, 2) of cells K (len,) in those cells' frame
        coordinates (relative to corner 0), F the facet fluxes."""
        geo, topo = self.geo, self.topo
        out = np.zeros((len(K), 2))
        for i in range(3):
            coef = self.sigma[K, i] * F[topo.cell_facet[K, i]] / (2.0 * geo.area[K])
            out += coef[:, None] * (X - geo.P[K, i])
        return out

    def basis_at(self, K, X):
        """Values of the three local basis functions: (len, 3, 2)."""
        geo = self.geo
        return (self.sigma[K][:, :, None] * (X[:, None, :] - geo.P[K]) / (2.0 * geo.area[K])[:, None, None])

    def matrices(self):
        """RT0 mass matrix and div-div matrix, CSR (n_facet x n_facet)."""
        geo, topo = self.geo, self.topo
        nk = geo.area.shape[0]
        ref, w = triangle_rule(2)
        Z = ref[None, :, 0:1] * geo.P[:, None, 1, :] + ref[None, :, 1:2] * geo.P[:, None, 2, :]
        W = w[None, :] * (2.0 * geo.area)[:, None]
        phi = np.stack([self.sigma[:, i, None, None] * (Z - geo.P[:, None, i]) / (2.0 * geo.area)[:, None, None]
                        for i in range(3)], axis=2)                       # (nk, Q, 3, 2)
        Mloc = np.einsum("cq,cqid,cqjd->cij", W, phi, phi)
        div = self.sigma / geo.area[:, None]                              # div phi_i = sigma_i / |K|
        Dloc = geo.area[:, None, None] * div[:, :, None] * div[:, None, :]
        cf = topo.cell_facet
        rows = np.repeat(cf[:, :, None], 3, 2).ravel()
        cols = np.repeat(cf[:, None, :], 3, 1).ravel()
        N = topo.n_facet
        M = sp.csr_matrix((Mloc.ravel(), (rows, cols)), shape=(N, N))
        D = sp.csr_matrix((Dloc.ravel(), (rows, cols)), shape=(N, N))
        return M, D

    def interpolate_constant(self, a):
        """DOFs of the constant field a (2,): F_e = L_e a.n_e."""
        topo, geo = self.topo, self.geo
        K, i = topo.facet_cell[:, 0], topo.facet_loc[:, 0]
        return geo.flen[K, i] * (geo.fnormal[K, i] @ np.asarray(a, dtype=float))


def rt0_coarse_operator(mesh, kappa):
    """S_c = (1/kappa) [M_RT + kappa^2 D_RT]  (Eq. coarse_problem_LF, scaled)."""
    M, D = Rt0Space(mesh).matrices()
    return ((M + kappa ** 2 * D) / kappa).tocsr()


def lf_prolongation(hdg: LfLocal, space: Rt0Space):
    """pi: RT0 fluxes -> trace nodal values (n_facet*2m, n_facet): the average of
    the two cells' u_c at each trace node."""
    p, m = hdg.p, hdg.m
    topo, geo = hdg.topo, hdg.geo
    ne = topo.n_facet
    sn = np.arange(m) / p
    rows, cols, vals = [], [], []
    for side in (0, 1):
        K, i = topo.facet_cell[:, side], topo.facet_loc[:, side]
        for k in range(m):
            # the other cell runs the facet backwards: its parameter for global node k is 1 - k/p
            s = sn[k] if side == 0 else 1.0 - sn[k]
            X = _facet_point(geo, K, i, s)
            phi = space.basis_at(K, X)                                        # (ne, 3, 2)
            for j in range(3):
                col = topo.cell_facet[K, j]
                for d in range(2):
                    rows.append(np.arange(ne) * 2 * m + d * m + k)
                    cols.append(col)
                    vals.append(0.5 * phi[:, j, d])
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(ne * 2 * m, ne))


def _facet_point(geo, K, i, s):
    """Point at counter-clockwise parameter s of local facet i of cells K: (len, 2)."""
    a = geo.P[K, (i + 1) % 3]
    b = geo.P[K, (i + 2) % 3]
    return a + s * (b - a)


def rt0_transfer(fine_mesh, coarse_mesh, parents):
    """Inclusion of RT0(coarse) into RT0(fine) for a uniform refinement:
    fine flux = exact flux of the coarse field through the fine facet,
    L_f * u_c(midpoint) . n_f (u_c is linear in the coarse cell)."""
    fs, cs = Rt0Space(fine_mesh), Rt0Space(coarse_mesh)
    ft, fg, cg = fs.topo, fs.geo, cs.geo
    key = {}
    for Kc, tri in enumerate(coarse_mesh.cell_vert):
        k = frozenset(int(v) for v in tri)
        if len(k) != 3 or k in key:
            raise ValueError("coarse RT0 level too small: cells are not determined by their vertices")
        key[k] = Kc
    period = coarse_mesh.period
    ne = ft.n_facet
    rows, cols, vals = [], [], []
    for e in range(ne):
        Kf, i = int(ft.facet_cell[e, 0]), int(ft.facet_loc[e, 0])
        verts = set()
        for v in fine_mesh.cell_vert[Kf]:
            verts.update(int(x) for x in parents[v])
        Kc = key[frozenset(verts)]
        # midpoint in unwrapped coordinates, moved to the coarse cell's periodic image
        Xf = _cell_xy(fine_mesh, Kf)
        mid = 0.5 * (Xf[(i + 1) % 3] + Xf[(i + 2) % 3])
        Xc = _cell_xy(coarse_mesh, Kc)
        cen = Xc.mean(axis=0)
        mid = mid - period * np.round((mid - cen) / period)
        phi = cs.basis_at(np.array([Kc]), (mid - Xc[0])[None, :])[0]          # (3, 2)
        w = fg.flen[Kf, i] * (phi @ fg.fnormal[Kf, i])
        for j in range(3):
            rows.append(e)
            cols.append(int(cs.topo.cell_facet[Kc, j]))
            vals.append(w[j])
    P = sp.csr_matrix((vals, (rows, cols)), shape=(ne, cs.topo.n_facet))
    P.data[np.abs(P.data) < 1e-14] = 0.0
    P.eliminate_zeros()
    return P


def _cell_xy(mesh, K):
    x = mesh.vert_xyz[mesh.cell_vert[K], :2].copy()
    x += mesh.period * mesh.cell_shift[K]
    return x


class Rt0Multigrid:
    """One V-cycle of geometric multigrid for the RT0 coarse problem."""

    def __init__(self, hier, kappa, omega=0.5, nu=1, n_min=4):
        keep = [l for l, msh in enumerate(hier.meshes) if msh.n >= n_min]
        if not keep or keep[-1] != len(hier.meshes) - 1:
            raise ValueError("the finest mesh must have n >= n_min")
        self.meshes = [hier.meshes[l] for l in keep]
        self.P = [rt0_transfer(hier.meshes[l], hier.meshes[l - 1], hier.parents[l - 1]) for l in keep[1:]]
        self.A = [rt0_coarse_operator(msh, kappa) for msh in self.meshes]
        self.omega, self.nu = omega, nu
        self.patches = [vertex_patches(msh, self.A[l]) for l, msh in enumerate(self.meshes)]
        self.coarse_inv = np.linalg.inv(self.A[0].toarray())

    def smooth(self, level, b, x):
        A = self.A[level]
        for _ in range(self.nu):
            r = b - A @ x
            dx = np.zeros_like(x)
            for idx, inv in self.patches[level]:
                np.add.at(dx, idx, np.einsum("vij,vj->vi", inv, r[idx]))
            x = x + self.omega * dx
        return x

    def vcycle(self, b, level=None):
        if level is None:
            level = len(self.A) - 1
        if level == 0:
            return self.coarse_inv @ b
        A = self.A[level]
        x = self.smooth(level, b, np.zeros_like(b))
        P = self.P[level - 1]
        x = x + P @ self.vcycle(P.T @ (b - A @ x), level - 1)
        return self.smooth(level, b, x)


def vertex_patches(mesh, A):
    """Facets touching each vertex, grouped by patch size: [(idx (nv_s, s), inv (nv_s, s, s))]."""
    topo = topology(mesh)
    inc = [[] for _ in range(mesh.n_vert)]
    for e, (a, b) in enumerate(topo.facet_vert):
        inc[a].append(e)
        if b != a:
            inc[b].append(e)
    Ad = A.tocsr()
    out = []
    for s in sorted({len(x) for x in inc}):
        idx = np.array([x for x in inc if len(x) == s], dtype=np.int64)
        blocks = np.stack([Ad[row][:, row].toarray() for row in idx])
        out.append((idx, np.linalg.inv(blocks)))
    return out


class LfTraceMultigrid:
    """Non-nested two-level V-cycle (Alg. twolevel_vcycle) for the
    Lax-Friedrichs trace system: facet block-Jacobi (2m x 2m blocks), RT0
    coarse space, pi = L2 projection of {{u_c}}."""

    def __init__(self, hdg: HdgLfOracle, hier, omega=0.7, nu_pre=2, nu_post=2, rt_omega=0.5, rt_nu=1,
                 exact_coarse=False, smoother="jacobi"):
        if hier.fine.n_vert != hdg.mesh.n_vert or hier.fine.n_cell != hdg.mesh.n_cell:
            raise ValueError("hierarchy's finest mesh must be the HDG mesh")
        self.S = hdg.S
        mt, ne = hdg.mt, hdg.topo.n_facet
        Sd = self.S.tocsr()
        e = np.arange(ne)
        D = np.zeros((ne, mt, mt))
        for a in range(mt):
            for b in range(mt):
                D[:, a, b] = np.asarray(Sd[e * mt + a, e * mt + b]).ravel()
        self.Dinv = np.linalg.inv(D)
        self.mt, self.ne = mt, ne
        self.space = Rt0Space(hdg.mesh)
        self.pi = lf_prolongation(hdg, self.space)
        self.mg = Rt0Multigrid(hier, hdg.kappa, rt_omega, rt_nu)
        self.Sc = self.mg.A[-1]
        self.exact_coarse = exact_coarse
        if exact_coarse:
            self._lu = spla.splu(self.Sc.tocsc())
        self.omega, self.nu_pre, self.nu_post = omega, nu_pre, nu_post
        if smoother not in ("jacobi", "chebyshev"):
            raise ValueError("smoother must be 'jacobi' or 'chebyshev'")
        self.smoother = smoother
        if smoother == "chebyshev":
            # the same Chebyshev smoother as the upwind case (interval [0.1, 1.1] lambda_max)
            from .p1 import power_estimate
            self.lambda_max = power_estimate(self.S, self.block_jacobi)
            self.cheb_interval = (0.1 * self.lambda_max, 1.1 * self.lambda_max)

    def block_jacobi(self, r):
        return np.einsum("eab,eb->ea", self.Dinv, r.reshape(self.ne, self.mt)).ravel()

    def smooth(self, b, x, nu):
        if self.smoother == "chebyshev":
            from .p1 import chebyshev
            return chebyshev(self.S, self.block_jacobi, b, x, nu, *self.cheb_interval)
        for _ in range(nu):
            x = x + self.omega * self.block_jacobi(b - self.S @ x)
        return x

    def coarse_solve(self, rc):
        return self._lu.solve(rc) if self.exact_coarse else self.mg.vcycle(rc)

    def vcycle(self, b):
        x = self.smooth(b, np.zeros_like(b), self.nu_pre)
        x = x + self.pi @ self.coarse_solve(self.pi.T @ (b - self.S @ x))
        return self.smooth(b, x, self.nu_post)
