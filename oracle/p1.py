"""Non-nested multigrid preconditioner for the trace system (oracle).

* Coarse space: conforming P1 on the same mesh (upwind case of the
  non-nested multigrid section).  Prolongation pi is the natural injection of
  a P1 function onto the skeleton; restriction is its transpose acting on
  residual (dual) vectors.
* Coarse form: the weak form of phi - kappa^2 div grad phi
  (Eq. coarse_problem_upwind).  Its scale relative to the trace system
  follows from the trace equation not being multiplied by kappa: for a
  smooth P1 function, (pi phi)^T S (pi phi) ~ (1/kappa) [ (phi, phi) +
  kappa^2 (grad phi, grad phi) ], so S_c = (1/kappa) (M_1 + kappa^2 K_1).
  This reading is pinned by the Galerkin-ratio test.
* The coarse problem is solved approximately by one geometric-multigrid
  V-cycle over a nested P1 hierarchy (rediscretised S_c on every level,
  linear-interpolation transfer from the mesh's parent map, damped Jacobi,
  dense solve on the coarsest level).  Variant (galerkin=True): the Galerkin
  form S_c = pi^T S pi of the section's footnote on the finest P1 level and
  P^T A P below it.
* Two-level V-cycle (Alg. twolevel_vcycle): presmooth, residual, restrict,
  coarse solve, prolong, postsmooth; the smoother is damped facet-block
  Jacobi (the block-Jacobi smoother named as future work in the conclusion)
  or, as in the paper's solver settings, Chebyshev iteration of degree nu
  preconditioned by facet-block Jacobi.
* Chebyshev interval: [0.1, 1.1] times an estimate of the largest eigenvalue
  of D^-1 S (the PETSc default transform of an eigenvalue estimate, which the
  paper's runs inherit).  The estimate is 20 power iterations from the fixed
  start vector v_i = (((i * 2654435761) mod 2^32) / 2^32) - 1/2 (i the global
  trace index): v <- D^-1 S v / ||D^-1 S v||, estimate = ||D^-1 S v||.

The V-cycles as linear operators are pinned to the textbook iteration
matrices (two-level and recursive V-cycle forms built from the explicit level
matrices), the coarse operator to its scale, the smoother blocks to the
diagonal blocks of S.  Parity unpinned for the convergence rate the cycle
reaches: no printed reference exists for this smoother beyond the paper's
iteration counts, which the tests bound.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .fem import geometry


def p1_matrices(mesh):
    """Assembled P1 mass and stiffness matrices on the (flat-celled) mesh."""
    geo = geometry(mesh)
    P = geo.P                                          # (nk, 3, 2)
    nk = P.shape[0]
    area = geo.area
    # barycentric gradients: solve [1 x y] c = e_i at the three corners
    V = np.concatenate([np.ones((nk, 3, 1)), P], axis=2)   # (nk, 3, 3)
    Cf = np.linalg.inv(V)                                  # columns: coefficients of lambda_i
    grad = np.transpose(Cf[:, 1:3, :], (0, 2, 1))          # (nk, 3 (i), 2)
    Kloc = area[:, None, None] * np.einsum("cid,cjd->cij", grad, grad)
    Mloc = area[:, None, None] / 12.0 * (np.ones((3, 3)) + np.eye(3))[None]
    cv = mesh.cell_vert.astype(np.int64)
    rows = np.repeat(cv[:, :, None], 3, 2).ravel()
    cols = np.repeat(cv[:, None, :], 3, 1).ravel()
    N = mesh.n_vert
    M = sp.csr_matrix((Mloc.ravel(), (rows, cols)), shape=(N, N))
    K = sp.csr_matrix((Kloc.ravel(), (rows, cols)), shape=(N, N))
    return M, K


def coarse_operator(mesh, kappa):
    M, K = p1_matrices(mesh)
    return ((M + kappa ** 2 * K) / kappa).tocsr()


def injection(topo, p, n_vert):
    """pi: P1 vertex values -> trace nodal values, (n_facet*(p+1), n_vert)."""
    m = p + 1
    ne = topo.n_facet
    s = np.arange(m) / p
    rows = np.repeat(np.arange(ne * m), 2)
    v0 = np.repeat(topo.facet_vert[:, 0], m)
    v1 = np.repeat(topo.facet_vert[:, 1], m)
    cols = np.stack([v0, v1], 1).ravel()
    vals = np.stack([np.tile(1.0 - s, ne), np.tile(s, ne)], 1).ravel()
    return sp.csr_matrix((vals, (rows, cols)), shape=(ne * m, n_vert))


def transfer(parents, n_coarse):
    """Linear interpolation from level l-1 to level l given the parent map."""
    nf = parents.shape[0]
    rows = np.repeat(np.arange(nf), 2)
    cols = parents.ravel()
    vals = np.full(2 * nf, 0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, n_coarse))   # duplicates sum to 1


class P1Multigrid:
    """One V-cycle of geometric multigrid for S_c on a nested P1 hierarchy."""

    def __init__(self, hier, kappa, omega=2.0 / 3.0, nu=2, fine_operator=None):
        self.P = [transfer(par, hier.meshes[l].n_vert) for l, par in enumerate(hier.parents)]
        if fine_operator is None:
            self.A = [coarse_operator(m, kappa) for m in hier.meshes]
        else:
            # Galerkin hierarchy: the given finest operator, then A_{l-1} = P^T A_l P
            A = [sp.csr_matrix(fine_operator)]
            for P in reversed(self.P):
                A.insert(0, (P.T @ A[0] @ P).tocsr())
            self.A = A
        self.Dinv = [1.0 / a.diagonal() for a in self.A]
        self.omega, self.nu = omega, nu
        self.coarse_inv = np.linalg.inv(self.A[0].toarray())

    def vcycle(self, b, level=None):
        if level is None:
            level = len(self.A) - 1
        if level == 0:
            return self.coarse_inv @ b
        A, Di, w = self.A[level], self.Dinv[level], self.omega
        x = np.zeros_like(b)
        for _ in range(self.nu):
            x = x + w * Di * (b - A @ x)
        r = b - A @ x
        P = self.P[level - 1]
        x = x + P @ self.vcycle(P.T @ r, level - 1)
        for _ in range(self.nu):
            x = x + w * Di * (b - A @ x)
        return x


def facet_blocks(S, ne, m):
    """Diagonal m x m block of S for every facet: D_e[a, b] = S[e m + a, e m + b]."""
    Sd = S.tocsr()
    e = np.arange(ne)
    D = np.zeros((ne, m, m))
    for a in range(m):
        for b in range(m):
            D[:, a, b] = np.asarray(Sd[e * m + a, e * m + b]).ravel()
    return D


class TraceMultigrid:
    """Non-nested two-level V-cycle on the trace space (Alg. twolevel_vcycle)."""

    def __init__(self, hdg, hier, omega=None, nu_pre=2, nu_post=2, p1_omega=2.0 / 3.0, p1_nu=2,
                 exact_coarse=False, smoother="jacobi", galerkin=False):
        if hier.fine.n_vert != hdg.mesh.n_vert or hier.fine.n_cell != hdg.mesh.n_cell:
            raise ValueError("hierarchy's finest mesh must be the HDG mesh")
        self.S = hdg.S
        m = hdg.m
        ne = hdg.topo.n_facet
        self.D = facet_blocks(self.S, ne, m)
        self.Dinv = np.linalg.inv(self.D)
        self.m, self.ne = m, ne
        self.pi = injection(hdg.topo, hdg.p, hdg.mesh.n_vert)
        if galerkin:
            # the coarse form footnoted in the non-nested multigrid section: S_c(q, v) = S(pi q, pi v)
            Sc = (self.pi.T @ self.S @ self.pi).tocsr()
            self.mg = P1Multigrid(hier, hdg.kappa, p1_omega, p1_nu, fine_operator=Sc)
        else:
            self.mg = P1Multigrid(hier, hdg.kappa, p1_omega, p1_nu)
        self.Sc = self.mg.A[-1]
        self.exact_coarse = exact_coarse
        if exact_coarse:
            import scipy.sparse.linalg as spla
            self._lu = spla.splu(self.Sc.tocsc())
        self.omega = omega if omega is not None else default_omega()
        self.nu_pre, self.nu_post = nu_pre, nu_post
        if smoother not in ("jacobi", "chebyshev"):
            raise ValueError("smoother must be 'jacobi' or 'chebyshev'")
        self.smoother = smoother
        if smoother == "chebyshev":
            self.lambda_max = power_estimate(self.S, self.block_jacobi)
            self.cheb_interval = (0.1 * self.lambda_max, 1.1 * self.lambda_max)

    def block_jacobi(self, r):
        return np.einsum("eab,eb->ea", self.Dinv, r.reshape(self.ne, self.m)).ravel()

    def smooth(self, b, x, nu):
        if self.smoother == "chebyshev":
            return chebyshev(self.S, self.block_jacobi, b, x, nu, *self.cheb_interval)
        for _ in range(nu):
            x = x + self.omega * self.block_jacobi(b - self.S @ x)
        return x

    def coarse_solve(self, rc):
        return self._lu.solve(rc) if self.exact_coarse else self.mg.vcycle(rc)

    def vcycle(self, b):
        x = self.smooth(b, np.zeros_like(b), self.nu_pre)
        res = b - self.S @ x
        x = x + self.pi @ self.coarse_solve(self.pi.T @ res)
        return self.smooth(b, x, self.nu_post)


def power_start(n):
    """Fixed start vector of the eigenvalue estimate: v_i = frac(i * 2654435761 / 2^32) - 1/2."""
    i = np.arange(n, dtype=np.uint64)
    return ((i * np.uint64(2654435761)) % np.uint64(2 ** 32)).astype(np.float64) / 2.0 ** 32 - 0.5


def power_estimate(S, prec, iters=20):
    """Largest eigenvalue estimate of prec(S .): 20 normalised power steps."""
    v = power_start(S.shape[0])
    v = v / np.linalg.norm(v)
    lam = 0.0
    for _ in range(iters):
        w = prec(S @ v)
        lam = np.linalg.norm(w)
        v = w / lam
    return lam


def chebyshev(S, prec, b, x, k, a, bnd):
    """k steps of Chebyshev iteration for S x = b preconditioned by prec on the
    interval [a, bnd] (the textbook three-term form: theta the centre, delta
    the half width, sigma = theta / delta)."""
    theta, delta = 0.5 * (bnd + a), 0.5 * (bnd - a)
    sigma = theta / delta
    rho = 1.0 / sigma
    d = prec(b - S @ x) / theta
    for step in range(k):
        x = x + d
        if step == k - 1:
            break
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * prec(b - S @ x)
        rho = rho_new
    return x


def default_omega():
    """Damping of the facet block-Jacobi sweep (a stated constant, see tests)."""
    return 0.7
