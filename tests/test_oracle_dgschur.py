"""Pins of the oracle's non-hybridised DG solver with the approximate
Schur-complement preconditioner (native DG section): the three steps are an
exact block factorisation when the sub-solves are exact, the Galerkin coarse
operator has a closed cell-wise form, the preconditioned GMRES reaches the
direct DG solution, and the iteration count does not grow with the mesh."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import hdg_inputs as hi
from oracle.dgschur import DgApproxSchur, interpolation
from oracle.fem import geometry
from oracle.p1 import p1_matrices


@pytest.mark.parametrize("p", [1, 2])
def test_exact_sub_solves_give_the_exact_inverse(p):
    """With A_uu^-1 exact and S replaced by the exact Schur complement
    A_pp - A_pu A_uu^-1 A_up solved exactly, the three steps are the block-LU
    inverse: P^-1 A x = x (pins the order and signs of the steps)."""
    o = DgApproxSchur(hi.torus_hierarchy(4, 4), p, 0.3, 1.3, 0.8, 1.0)
    auu = spla.splu(o.Auu.tocsc())
    Sex = o.App.toarray() - o.Apu.toarray() @ np.linalg.solve(o.Auu.toarray(), o.Aup.toarray())
    x = np.random.default_rng(0).standard_normal(o.A.shape[0])
    y = o.precondition(o.A @ x, auu_solve=auu.solve, s_solve=lambda b: np.linalg.solve(Sex, b))
    assert np.linalg.norm(y - x) < 1e-10 * np.linalg.norm(x)


@pytest.mark.parametrize("case", ["torus", "sphere"])
def test_galerkin_coarse_operator_has_the_cellwise_form(case):
    """P^T S P = M_1 + kappa^2 sum_K sum_d beta_Kd d_d phi d_d psi with
    beta_Kd = sum_i (int_K phi_i)^2 / diag(A_uu)_(K,d,i) (P1 gradients are
    constant per cell): for continuous phi and psi the facet terms of A_pp
    and A_pu cancel and A_up P phi is kappa M grad phi."""
    if case == "torus":
        hier, p, dt, f0, om = hi.torus_hierarchy(8, 4), 2, 0.5, 1.0, 0.0
    else:
        hier, p, dt, f0, om = hi.icosphere_hierarchy(2), 3, 0.3, 0.5, 0.3
    o = DgApproxSchur(hier, p, dt, 1.0, 1.0, f0, om)
    mesh = hier.fine
    nk, n = mesh.n_cell, o.n
    rs = o.dg.M.sum(axis=2)
    beta = np.einsum("ki,kdi->kd", rs ** 2, 1.0 / o.D.reshape(nk, 2, n))
    geo = geometry(mesh)
    V = np.concatenate([np.ones((nk, 3, 1)), geo.P], axis=2)
    grad = np.transpose(np.linalg.inv(V)[:, 1:3, :], (0, 2, 1))
    Kloc = np.einsum("kd,kid,kjd->kij", beta, grad, grad)
    cv = mesh.cell_vert.astype(np.int64)
    Kb = sp.csr_matrix((Kloc.ravel(), (np.repeat(cv[:, :, None], 3, 2).ravel(),
                                       np.repeat(cv[:, None, :], 3, 1).ravel())), shape=(mesh.n_vert,) * 2)
    M1, _ = p1_matrices(mesh)
    formula = M1 + o.dg.kappa ** 2 * Kb
    assert abs(formula - o.Sc).max() < 1e-13 * abs(o.Sc).max()


def test_interpolation_reproduces_linear_fields():
    """P maps the vertex values of a linear function to its values at the DG
    nodes (checked with the periodic coordinate on a torus cell patch)."""
    m = hi.torus(4)
    P = interpolation(m, 3)
    x = m.vert_xyz[:, 0]
    xn = hi.rhs.node_coords(m, 3)[..., 0]
    cells_inside = np.all(m.cell_shift[:, :, 0] == 0, axis=1)      # no periodic wrap in x
    got = (P @ x).reshape(m.n_cell, -1)
    assert np.abs(got[cells_inside] - xn[cells_inside]).max() < 1e-14
    assert np.allclose(P @ np.ones(m.n_vert), 1.0)


@pytest.mark.parametrize("case", ["torus", "sphere"])
def test_gmres_reaches_the_direct_solution(case):
    if case == "torus":
        hier, p, dt, g, H, f0, om = hi.torus_hierarchy(8, 4), 2, 0.5, 1.3, 0.8, 1.0, 0.0
    else:
        hier, p, dt, g, H, f0, om = hi.icosphere_hierarchy(2), 3, 0.3, 1.0, 1.0, 0.5, 0.3
    o = DgApproxSchur(hier, p, dt, g, H, f0, om)
    R = o.rhs(hi.iid_rhs(hier.fine, p, 3)[..., 0])
    x, its = o.gmres(R, rtol=1e-11)
    xd = o.direct(R)
    assert np.linalg.norm(x - xd) < 1e-9 * np.linalg.norm(xd)
    assert its < 200


def test_preconditioner_is_linear_and_iterations_are_mesh_independent():
    its = []
    for n in (8, 16):
        o = DgApproxSchur(hi.torus_hierarchy(n, 4), 1, 4.0 / n)
        R = o.rhs(hi.iid_rhs(o.hier.fine, 1, 3)[..., 0])
        _, k = o.gmres(R, rtol=1e-8)
        its.append(k)
    assert abs(its[1] - its[0]) <= 0.1 * its[0]
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal((2, o.A.shape[0]))
    lhs = o.precondition(2.0 * x - 3.0 * y)
    assert np.linalg.norm(lhs - (2.0 * o.precondition(x) - 3.0 * o.precondition(y))) < 1e-12 * np.linalg.norm(lhs)


def test_s_cycle_is_the_two_level_iteration_matrix():
    """The Schur-complement cycle as a matrix: I - B S = C (I - P B_c P^T S) C
    with C the Chebyshev error propagator (the smoother from x = e with b = 0;
    its polynomial is pinned with the multigrid pins) and B_c the textbook
    P1 V-cycle recursion on the explicit Galerkin level matrices."""
    from oracle.p1 import chebyshev
    o = DgApproxSchur(hi.torus_hierarchy(4, 2), 1, 0.3, 1.3, 0.8, 1.0)
    S = o.S.toarray()
    n = S.shape[0]
    B = np.column_stack([o.s_cycle(e) for e in np.eye(n)])
    a, bnd = 0.1 * o.lmax, 1.1 * o.lmax
    C = np.column_stack([chebyshev(o.S, o.own_prec, np.zeros(n), e, o.nu, a, bnd) for e in np.eye(n)])
    A = [m.toarray() for m in o.mg.A]
    Pl = [m.toarray() for m in o.mg.P]
    Bc = np.linalg.inv(A[0])
    for l in range(1, len(A)):
        I = np.eye(A[l].shape[0])
        J = np.linalg.matrix_power(I - o.mg.omega * (A[l] / np.diag(A[l])[:, None]), o.mg.nu)
        Bc = (I - J @ (I - Pl[l - 1] @ Bc @ Pl[l - 1].T @ A[l]) @ J) @ np.linalg.inv(A[l])
    P = o.P.toarray() if sp.issparse(o.P) else np.asarray(o.P)
    I = np.eye(n)
    ref = (I - C @ (I - P @ Bc @ P.T @ S) @ C) @ np.linalg.inv(S)
    assert len(A) == 2
    assert np.abs(B - ref).max() < 1e-10 * np.abs(ref).max()
