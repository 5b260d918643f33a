"""Pins of the Lax-Friedrichs oracle (vector trace, RT0 coarse space) against
facts the paper and the mathematics fix: HDG == DG with the same flux (the
theorem of the hybridisation section), closed-form constant states,
conservation, symmetry / definiteness, convergence rates, exactness of the
nested RT0 transfer, the coarse-form scale (Galerkin ratio) and the
properties of the multigrid pieces.
"""
import numpy as np
import pytest

import hdg_inputs as hi
from oracle.fem import facet_points
from oracle.lf import (DgLfOracle, HdgLfOracle, LfTraceMultigrid, Rt0Multigrid, Rt0Space, lf_prolongation,
                       rt0_coarse_operator, rt0_transfer)


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("f0,tau", [(0.0, 1.0), (0.7, 1.0), (0.4, 2.0)])
def test_hdg_equals_dg(p, f0, tau):
    """Theorem (hybridisation section): the hybridised LF solution equals the
    standard DG solution with the LF flux, and uhat = {{u}} + [[phi]]/(2 tau)."""
    mesh = hi.torus(4)
    args = (mesh, p, 0.3, 1.3, 0.8, f0, 0.0)
    h, d = HdgLfOracle(*args, tau=tau), DgLfOracle(*args, tau=tau)
    r = hi.iid_rhs(mesh, p, 11)[..., 0]
    qh, lh = h.solve(r)
    qd, ld = d.solve(r)
    assert rel(qh, qd) < 1e-12 and rel(lh, ld) < 1e-12


@pytest.mark.parametrize("p", [1, 3])
def test_constant_state(p):
    """Closed form: constant (r_h, r_u) gives h = r_h, u = (I + dt f J)^-1 r_u,
    and the trace equals the constant velocity."""
    mesh = hi.torus(3)
    dt, g, H, f0 = 0.4, 2.0, 0.5, 0.9
    h = HdgLfOracle(mesh, p, dt, g, H, f0, 0.0)
    n = h.n
    h0, U0 = 0.7, np.array([0.3, -1.2])
    r = np.zeros((mesh.n_cell, 3, n))
    r[:, 0], r[:, 1], r[:, 2] = h0, U0[0], U0[1]
    q, lam = h.solve(r)
    a = dt * f0
    u = np.linalg.solve(np.array([[1.0, -a], [a, 1.0]]), U0)
    assert np.abs(q[:, 0] - h0).max() < 1e-12
    assert np.abs(q[:, 1] - u[0]).max() < 1e-12 and np.abs(q[:, 2] - u[1]).max() < 1e-12
    lam = lam.reshape(-1, 2, p + 1)
    assert np.abs(lam[:, 0] - u[0]).max() < 1e-12 and np.abs(lam[:, 1] - u[1]).max() < 1e-12


@pytest.mark.parametrize("p", [1, 2])
def test_conservation(p):
    """Testing with psi = 1 and w = e_d: the facet terms telescope (single-valued
    trace, opposite normals), so int phi = int r_phi and, with f = 0,
    int u = int r_u."""
    mesh = hi.torus(4)
    h = HdgLfOracle(mesh, p, 0.5, 1.0, 1.0, 0.0, 0.0)
    r = hi.iid_rhs(mesh, p, 3)[..., 0]
    q, _ = h.solve(r)
    one = np.ones(h.n)
    for fld in range(3):
        lhs = np.einsum("cij,ci,j->", h.M, q[:, fld], one)
        rhs = np.einsum("cij,ci,j->", h.M, r[:, fld], one)
        assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(rhs))


@pytest.mark.parametrize("p", [1, 3])
def test_single_valued_flux(p):
    """The trace equation holds pointwise: on every facet the two one-sided
    momentum fluxes phi_K n_K + tau (u_K - uhat) cancel at the trace nodes."""
    mesh = hi.torus(4)
    h = HdgLfOracle(mesh, p, 0.6, 1.0, 1.0, 0.5, 0.0)
    r = hi.iid_rhs(mesh, p, 5)[..., 0]
    q, lam = h.solve(r)
    q = q.copy()
    q[:, 0] *= h.hscale
    lam = lam.reshape(-1, 2, p + 1)
    topo, nrm = h.topo, h.geo.fnormal
    sn = np.arange(p + 1) / p
    vals = np.stack([h.basis.values(facet_points(h.geo, i, sn)) for i in range(3)], 1)
    total = np.zeros_like(lam)
    for side in (0, 1):
        K, i = topo.facet_cell[:, side], topo.facet_loc[:, side]
        V = vals[K, i]
        if side == 1:
            V = V[:, ::-1]
        phi = np.einsum("eqi,ei->eq", V, q[K, 0])
        for d in range(2):
            ud = np.einsum("eqi,ei->eq", V, q[K, 1 + d])
            total[:, d] += phi * nrm[K, i, d][:, None] + h.tau * (ud - lam[:, d])
    assert np.abs(total).max() < 1e-11 * np.abs(lam).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_symmetric_positive_definite(p):
    """f = 0: the LF trace operator is symmetric positive definite."""
    h = HdgLfOracle(hi.torus(3), p, 0.5, 1.0, 1.0, 0.0, 0.0)
    S = h.S.toarray()
    assert np.abs(S - S.T).max() < 1e-13 * np.abs(S).max()
    assert np.linalg.eigvalsh(S).min() > 0


@pytest.mark.parametrize("p", [1, 2, 3])
def test_manufactured_solution_rate(p):
    """A smooth periodic solution of the continuous problem, L2-projected
    right-hand side: the LF DG error converges at a rate > p + 1/2."""
    from oracle.fem import volume_points
    tp = 2 * np.pi
    phi = lambda x, y: np.sin(tp * x) * np.cos(tp * y)
    ux = lambda x, y: 0.5 * np.cos(tp * x) * np.sin(tp * y)
    uy = lambda x, y: np.sin(tp * (x + y))
    divu = lambda x, y: -0.5 * tp * np.sin(tp * x) * np.sin(tp * y) + tp * np.cos(tp * (x + y))
    gx = lambda x, y: tp * np.cos(tp * x) * np.cos(tp * y)
    gy = lambda x, y: -tp * np.sin(tp * x) * np.sin(tp * y)
    errs = []
    for n in (4, 8, 16):
        mesh = hi.torus(n)
        d = DgLfOracle(mesh, p, 0.05, 1.0, 1.0, 0.9, 0.0)
        kap, dt, f0 = d.kappa, d.dt, 0.9
        Z, w = volume_points(d.geo, 2 * p + 6)
        X = Z + d.geo.corners3[:, None, 0, :2]
        V = d.basis.values(Z)
        Minv = np.linalg.inv(d.M)
        proj = lambda fn: np.einsum("cij,cj->ci", Minv, np.einsum("cq,cqi,cq->ci", w, V, fn(X[..., 0], X[..., 1])))
        r = np.stack([proj(lambda x, y: phi(x, y) + kap * divu(x, y)),
                      proj(lambda x, y: ux(x, y) - dt * f0 * uy(x, y) + kap * gx(x, y)),
                      proj(lambda x, y: uy(x, y) + dt * f0 * ux(x, y) + kap * gy(x, y))], 1)
        q, _ = d.solve(r)
        err = 0.0
        for fld, fn in ((0, phi), (1, ux), (2, uy)):
            e = np.einsum("cqi,ci->cq", V, q[:, fld]) - fn(X[..., 0], X[..., 1])
            err += np.sum(w * e ** 2)
        errs.append(np.sqrt(err))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > p + 0.5, (errs, rates)


# ----------------------------------------------------------------- RT0 coarse space

def test_rt0_mass_and_divergence_of_constants():
    """Closed forms on the unit torus: a constant field a has L2 norm^2 |a|^2
    and zero divergence."""
    s = Rt0Space(hi.torus(5))
    M, D = s.matrices()
    a = np.array([0.6, -1.7])
    F = s.interpolate_constant(a)
    assert abs(F @ (M @ F) - a @ a) < 1e-13
    assert np.abs(D @ F).max() < 1e-12


def test_rt0_basis_fluxes():
    """The local basis function of facet i has unit flux through facet i
    (outward, times sigma_i) and none through the other two facets."""
    s = Rt0Space(hi.torus(3))
    geo = s.geo
    from oracle.quadrature import gauss01
    t, wt = gauss01(2)
    K = np.arange(geo.area.shape[0])
    for i in range(3):
        for j in range(3):
            a, b = geo.P[:, (j + 1) % 3], geo.P[:, (j + 2) % 3]
            flux = 0.0
            for tk, wk in zip(t, wt):
                X = a + tk * (b - a)
                phi = s.basis_at(K, X)[:, i]
                flux = flux + wk * geo.flen[:, j] * np.einsum("cd,cd->c", phi, geo.fnormal[:, j])
            want = s.sigma[:, i] if i == j else 0.0
            assert np.abs(flux - want).max() < 1e-13


def test_rt0_transfer_is_exact_inclusion():
    """Nested RT0 spaces: P reproduces constant fields and P^T A_f P equals the
    rediscretised coarse operator."""
    hier = hi.torus_hierarchy(16, 4)
    for l in range(1, len(hier.meshes)):
        P = rt0_transfer(hier.meshes[l], hier.meshes[l - 1], hier.parents[l - 1])
        cs, fs = Rt0Space(hier.meshes[l - 1]), Rt0Space(hier.meshes[l])
        a = np.array([0.3, -1.1])
        assert rel(P @ cs.interpolate_constant(a), fs.interpolate_constant(a)) < 1e-14
        Af, Ac = rt0_coarse_operator(hier.meshes[l], 0.3), rt0_coarse_operator(hier.meshes[l - 1], 0.3)
        G = (P.T @ Af @ P).toarray()
        assert np.abs(G - Ac.toarray()).max() < 1e-13 * np.abs(Ac.toarray()).max()


@pytest.mark.parametrize("p", [1, 3])
def test_prolongation_of_constant_fields(p):
    """pi of a constant RT0 field gives that constant vector at every trace node."""
    mesh = hi.torus(4)
    h = HdgLfOracle(mesh, p, 0.3, 1.0, 1.0, 0.0, 0.0)
    s = Rt0Space(mesh)
    a = np.array([-0.4, 0.9])
    v = (lf_prolongation(h, s) @ s.interpolate_constant(a)).reshape(-1, 2, p + 1)
    assert np.abs(v[:, 0] - a[0]).max() < 1e-13 and np.abs(v[:, 1] - a[1]).max() < 1e-13


@pytest.mark.parametrize("p", [1, 3])
def test_galerkin_ratio(p):
    """Scale of the coarse form: for smooth RT0 fields (one gradient-like, one
    divergence-free) (pi u)^T S (pi u) / S_c(u, u) tends to 1 as h -> 0."""
    out = []
    for n in (8, 16, 32):
        mesh = hi.torus(n)
        kap = 0.25
        h = HdgLfOracle(mesh, p, kap, 1.0, 1.0, 0.0, 0.0)
        s = Rt0Space(mesh)
        pi = lf_prolongation(h, s)
        Sc = rt0_coarse_operator(mesh, kap)
        K, i = s.topo.facet_cell[:, 0], s.topo.facet_loc[:, 0]
        X = 0.5 * (s.geo.P[K, (i + 1) % 3] + s.geo.P[K, (i + 2) % 3]) + mesh.cell_coords()[K, 0, :2]
        row = []
        for U in (np.stack([np.cos(2 * np.pi * X[:, 0]), 0 * X[:, 1]], -1),
                  np.stack([np.sin(2 * np.pi * X[:, 1]), np.cos(2 * np.pi * X[:, 0])], -1)):
            F = s.geo.flen[K, i] * np.einsum("ed,ed->e", U, s.geo.fnormal[K, i])
            v = pi @ F
            row.append((v @ (h.S @ v)) / (F @ (Sc @ F)))
        out.append(row)
    out = np.abs(np.array(out) - 1.0)
    assert np.all(out[1:] < out[:-1])          # approaches 1 monotonically
    assert out[-1].max() < (0.12 if p == 1 else 0.05)


def test_rt0_vcycle_symmetric_and_convergent():
    """The RT0 V-cycle is a symmetric operator B and I - B A contracts, with a
    rate that does not degrade as kappa^2 / h^2 grows (the vertex patches hold
    the divergence-free fields)."""
    hier = hi.torus_hierarchy(16, 4)
    rates = []
    for kappa in (0.02, 0.5, 2.0):
        mg = Rt0Multigrid(hier, kappa)
        A = mg.A[-1].toarray()
        N = A.shape[0]
        B = np.stack([mg.vcycle(np.eye(N)[:, j]) for j in range(N)], 1)
        assert np.abs(B - B.T).max() < 1e-12 * np.abs(B).max()
        rates.append(np.abs(np.linalg.eigvals(np.eye(N) - B @ A)).max())
    assert max(rates) < 0.6 and rates[2] < rates[1] + 0.02


def test_lf_vcycle_symmetric_and_iteration_count():
    """f = 0: the LF trace V-cycle is symmetric; at the paper's LF Courant number
    (rho gamma / (2p + 1) = 2/7 at p = 3) the preconditioned CG converges in a
    number of iterations close to the paper's (about 9 for its HDG solver)."""
    p, n = 3, 8
    mesh = hi.torus(n)
    h = HdgLfOracle(mesh, p, (2.0 / 7.0) / n, 1.0, 1.0, 0.0, 0.0)
    mg = LfTraceMultigrid(h, hi.torus_hierarchy(n, 4))
    N = h.n_trace
    rng = np.random.default_rng(0)
    X = rng.standard_normal((N, 3))
    VX = np.stack([mg.vcycle(X[:, j]) for j in range(3)], 1)
    G = X.T @ VX
    assert np.abs(G - G.T).max() < 1e-11 * np.abs(G).max()
    b = h.rhat(hi.fourier_rhs_torus(mesh, p, 100)[..., 0])
    x, r = np.zeros(N), b.copy()
    z = mg.vcycle(r)
    d, rz = z.copy(), r @ z
    for its in range(1, 60):
        Sd = h.S @ d
        a = rz / (d @ Sd)
        x += a * d
        r -= a * Sd
        if np.linalg.norm(r) <= 1e-8 * np.linalg.norm(b):
            break
        z = mg.vcycle(r)
        rzn = r @ z
        d = z + rzn / rz * d
        rz = rzn
    assert np.linalg.norm(b - h.S @ x) <= 1e-8 * np.linalg.norm(b)
    assert its <= 20


def _schwarz_vcycle_by_recursion(meshes, A, P, omega, nu):
    """Textbook V-cycle recursion with additive Schwarz smoothing over vertex
    patches (the facets touching each vertex, found here from the topology):
    J = I - omega sum_v R_v^T (R_v A R_v^T)^-1 R_v A, B_0 = A_0^-1,
    I - B_l A_l = J^nu (I - P B_{l-1} P^T A_l) J^nu."""
    from oracle.fem import topology
    B = np.linalg.inv(A[0])
    for l in range(1, len(A)):
        n = A[l].shape[0]
        fv = topology(meshes[l]).facet_vert
        M = np.zeros((n, n))
        for v in range(meshes[l].n_vert):
            idx = np.flatnonzero((fv[:, 0] == v) | (fv[:, 1] == v))
            M[np.ix_(idx, idx)] += np.linalg.inv(A[l][np.ix_(idx, idx)])
        I = np.eye(n)
        J = np.linalg.matrix_power(I - omega * M @ A[l], nu)
        E = J @ (I - P[l - 1] @ B @ P[l - 1].T @ A[l]) @ J
        B = (I - E) @ np.linalg.inv(A[l])
    return B


@pytest.mark.parametrize("exact", [True, False])
def test_lf_vcycle_is_the_two_level_iteration_matrix(exact):
    """The Lax-Friedrichs trace cycle (Alg. twolevel_vcycle with the RT0 coarse
    space) as a matrix: I - B S = J^2 (I - pi B_c pi^T S) J^2 with J the damped
    2m x 2m facet block-Jacobi sweep (blocks inverted here from S) and B_c the
    exact RT0 inverse or the textbook two-level RT0 V-cycle with vertex-patch
    Schwarz smoothing; f != 0."""
    hier = hi.torus_hierarchy(8, 2)
    o = HdgLfOracle(hier.fine, 1, 0.3, 1.0, 1.0, 0.5, 0.0)
    tm = LfTraceMultigrid(o, hier, exact_coarse=exact)
    n, mt = o.n_trace, o.mt
    B = np.column_stack([tm.vcycle(e) for e in np.eye(n)])
    S = o.S.toarray()
    Dinv = np.zeros_like(S)
    for e in range(n // mt):
        sl = slice(e * mt, (e + 1) * mt)
        Dinv[sl, sl] = np.linalg.inv(S[sl, sl])
    I = np.eye(n)
    J = I - tm.omega * Dinv @ S
    if exact:
        Bc = np.linalg.inv(tm.Sc.toarray())
    else:
        assert len(tm.mg.A) == 2
        Bc = _schwarz_vcycle_by_recursion(tm.mg.meshes, [a.toarray() for a in tm.mg.A],
                                          [p.toarray() for p in tm.mg.P], tm.mg.omega, tm.mg.nu)
    pi = tm.pi.toarray()
    E = np.linalg.matrix_power(J, tm.nu_post) @ (I - pi @ Bc @ pi.T @ S) @ np.linalg.matrix_power(J, tm.nu_pre)
    ref = (I - E) @ np.linalg.inv(S)
    assert np.abs(B - ref).max() < 1e-10 * np.abs(ref).max()
