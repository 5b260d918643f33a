"""Pins of the oracle's IMEX time stepping (time discretisation and IMEX
methods sections) against what the paper and the mathematics fix:
the order conditions of additive Runge-Kutta methods, the paper's table of
orders and per-step evaluation counts, the observed order against the matrix
exponential of the semi-discrete system, conservation of mass, the steady
vortex and the paper's spatial convergence rate."""
import itertools
import math
import os

import numpy as np
import pytest
import scipy.linalg as sl

import hdg_inputs as hi
from oracle.imex import METHODS, LinearSwe, l2_error, tableau

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _methods_table():
    rows = {}
    for line in open(os.path.join(GOLD, "imex_methods.txt")):
        if line.startswith("#") or not line.strip():
            continue
        t = line.split()
        rows[t[0]] = dict(zip(("order", "n_L", "n_N", "n_mass", "n_implicit"), map(int, t[1:])))
    return rows


def _order_conditions(tab, order):
    """Residuals of the additive Runge-Kutta order conditions up to `order`
    (every combination of the explicit / implicit weights, matrices and
    abscissae)."""
    a, at, b, bt = tab
    c, ct = a.sum(1), at.sum(1)
    res = []
    for w in (b, bt):
        res.append(w.sum() - 1.0)
        if order >= 2:
            for cc in (c, ct):
                res.append(w @ cc - 0.5)
        if order >= 3:
            for c1, c2 in itertools.product((c, ct), repeat=2):
                res.append(w @ (c1 * c2) - 1.0 / 3.0)
            for A, cc in itertools.product((a, at), (c, ct)):
                res.append(w @ (A @ cc) - 1.0 / 6.0)
        if order >= 4:
            cs, As = (c, ct), (a, at)
            for c1, c2, c3 in itertools.product(cs, repeat=3):
                res.append(w @ (c1 * c2 * c3) - 1.0 / 4.0)
            for c1, A, c2 in itertools.product(cs, As, cs):
                res.append(w @ (c1 * (A @ c2)) - 1.0 / 8.0)
            for A, c1, c2 in itertools.product(As, cs, cs):
                res.append(w @ (A @ (c1 * c2)) - 1.0 / 12.0)
            for A1, A2, c1 in itertools.product(As, As, cs):
                res.append(w @ (A1 @ (A2 @ c1)) - 1.0 / 24.0)
    return np.abs(np.array(res))


@pytest.mark.parametrize("method", METHODS)
def test_tableau_satisfies_the_order_conditions_of_its_stated_order(method):
    """Tab. timestepper_comparison gives the order; every coupling condition up
    to it holds, and one of the next order fails (the order is sharp)."""
    order = _methods_table()[method]["order"]
    for theta in ((0.5, 0.55) if method == "theta" else (None,)):
        tab = tableau(method, theta) if theta is not None else tableau(method)
        a, at, b, bt = tab
        assert np.allclose(np.triu(a), 0.0) and np.allclose(np.triu(at, 1), 0.0)
        assert _order_conditions(tab, order).max() < 1e-14
        assert _order_conditions(tab, order + 1).max() > 1e-3


def test_theta_half_is_second_order_in_its_implicit_part():
    """The asterisk of Tab. timestepper_comparison: Crank-Nicolson for the
    linear part at theta = 1/2 only."""
    for theta, ok in ((0.5, True), (0.55, False)):
        _, at, _, bt = tableau("theta", theta)
        assert (abs(bt @ at.sum(1) - 0.5) < 1e-15) == ok


@pytest.mark.parametrize("method", METHODS)
def test_evaluation_counts_match_the_papers_table(method):
    """Tab. timestepper_comparison: implicit solves = stages with a nonzero
    implicit diagonal; N evaluations = stages whose explicit column or weight
    is nonzero; L evaluations = stages whose implicit column below the
    diagonal or weight is nonzero (for Theta, whose update equals its last
    stage, Eq. theta_method, only the column below the diagonal)."""
    a, at, b, bt = tableau(method)
    s = len(b)
    row = _methods_table()[method]
    n_impl = sum(at[i, i] != 0 for i in range(s))
    n_N = sum(bool(np.any(a[j + 1:, j] != 0) or b[j] != 0) for j in range(s))
    if method == "theta":
        n_L = sum(bool(np.any(at[j + 1:, j] != 0)) for j in range(s))
    else:
        n_L = sum(bool(np.any(at[j + 1:, j] != 0) or bt[j] != 0) for j in range(s))
    assert (n_impl, n_N, n_L) == (row["n_implicit"], row["n_N"], row["n_L"])


@pytest.mark.parametrize("method,theta,f,order", [
    ("theta", 0.5, 0.0, 2), ("theta", 0.5, 1.0, 1), ("theta", 0.55, 0.0, 1),
    ("ars232", None, 1.0, 2), ("ssp322", None, 1.0, 2), ("ars443", None, 1.0, 3)])
def test_observed_order_against_the_matrix_exponential(method, theta, f, order):
    """Exact solution of the semi-discrete system M q' = (L + N) q on the 2x2
    torus (p = 1, 72 unknowns): expm(T M^-1 (L + N)) q_0.  Halving dt divides
    the error by 2^order."""
    m = hi.torus(2)
    swe = LinearSwe(m, 1, g=1.0, H=1.0, f=f)
    q0 = hi.iid_rhs(m, 1, seed=7)
    x0 = swe.to_vec(q0)
    T = 0.5
    xe = sl.expm(T * swe.generator()) @ x0
    tab = tableau(method, theta) if theta is not None else tableau(method)
    errs = []
    for k in (16, 32, 64):
        x = x0.copy()
        for _ in range(k):
            x = swe.step(tab, T / k, x)
        errs.append(np.linalg.norm(x - xe) / np.linalg.norm(xe))
    rate = math.log2(errs[1] / errs[2])
    assert abs(rate - order) < 0.15, (errs, rate)


@pytest.mark.parametrize("method,order", [("ars232", 2), ("ars443", 3)])
def test_lax_friedrichs_flux_order_against_the_matrix_exponential(method, order):
    """The same exact reference with the Lax-Friedrichs flux terms."""
    m = hi.torus(2)
    swe = LinearSwe(m, 1, g=1.0, H=1.0, f=1.0, flux="lf")
    x0 = swe.to_vec(hi.iid_rhs(m, 1, seed=7))
    xe = sl.expm(0.5 * swe.generator()) @ x0
    errs = []
    for k in (16, 32, 64):
        x = x0.copy()
        for _ in range(k):
            x = swe.step(tableau(method), 0.5 / k, x)
        errs.append(np.linalg.norm(x - xe) / np.linalg.norm(xe))
    assert abs(math.log2(errs[1] / errs[2]) - order) < 0.15, errs


@pytest.mark.parametrize("method", METHODS)
def test_mass_is_conserved(method):
    """The flux terms are conservative and the Coriolis term does not act on
    phi: the domain integral of h is unchanged by every step."""
    m = hi.torus(4)
    swe = LinearSwe(m, 2, g=1.3, H=0.8, f=2.0)
    q0 = hi.iid_rhs(m, 2, seed=3)
    q = swe.run(tableau(method), 0.05, 5, q0)
    mass = lambda qq: float(np.sum(swe.M @ swe.to_vec(qq) * _phi_mask(swe, m)))
    assert abs(mass(q) - mass(q0)) < 1e-12 * abs(mass(q0)) + 1e-14


def _phi_mask(swe, m):
    """Coefficient vector of the constant function 1 in the phi field."""
    one = np.zeros((m.n_cell, 3, swe.n, 1))
    one[:, 0] = 1.0
    return swe.to_vec(one) / swe.hscale


def test_vortex_is_a_balanced_state_of_the_linear_equations():
    """With u = L_R phi' the semi-discrete tendency M^-1 (L + N) q_0 is a
    discretisation error that shrinks under refinement, far below the size of
    either term; with the factor (phi + phi_B) printed in the vortex section
    the imbalance stays at the size of delta."""
    v = hi.Vortex()
    ratios, printed = [], []
    for n in (16, 32):
        m = hi.torus(n)
        swe = LinearSwe(m, 2, g=v.c_g, H=v.c_g, f=v.f)
        x = swe.to_vec(hi.vortex_coefficients(m, 2, v))
        tend = (swe.L + swe.N) @ x
        ratios.append(np.linalg.norm(tend) / np.linalg.norm(swe.N @ x))
        xp = swe.to_vec(hi.vortex_coefficients(m, 2, v))
        phi = xp.reshape(m.n_cell, 3, -1)[:, 0]
        xp = xp.reshape(m.n_cell, 3, -1).copy()
        xp[:, 1:] *= (1.0 + phi[:, None, :])          # the printed (phi + phi_B) factor
        xp = xp.reshape(-1, 1)
        printed.append(np.linalg.norm((swe.L + swe.N) @ xp) / np.linalg.norm(swe.N @ xp))
    assert ratios[1] < 0.3 * ratios[0]
    assert ratios[1] < 0.02
    assert min(printed) > 0.05


@pytest.mark.parametrize("p,ns", [(1, (16, 32)), (2, (8, 16))])
def test_vortex_error_converges_at_the_papers_rate(p, ns):
    """Accuracy section: Delta_2 at T = 1/2 with ARS2(2,3,2) and the time step
    of the time-step-size section decreases at least as O(h^(p + 1/2)); the
    state stays at the interpolation error of the initial condition."""
    v = hi.Vortex()
    ex = lambda xy: v.state(xy)
    errs = []
    for n in ns:
        m = hi.torus(n)
        swe = LinearSwe(m, p, g=v.c_g, H=v.c_g, f=v.f)
        q0 = hi.vortex_coefficients(m, p, v)
        dt, steps = hi.paper_time_step(n, p)
        q = swe.run(tableau("ars232"), dt, steps, q0)
        e, e0 = l2_error(swe, q[..., 0], ex), l2_error(swe, q0[..., 0], ex)
        assert e < 1.5 * e0
        errs.append(e)
    assert math.log2(errs[0] / errs[1]) >= p + 0.5


def test_tendency_of_a_smooth_field_approximates_the_derivatives():
    """dt M^-1 L q for the interpolant of a smooth field converges to
    -dt c (div u, grad phi) (symmetric variables, g = H), and vanishes for a
    constant state."""
    c = 1.7
    errs = []
    for n in (8, 16):
        m = hi.torus(n)
        swe = LinearSwe(m, 2, g=c, H=c, f=0.0)
        xy = hi.rhs.node_coords(m, 2)[..., :2]
        k = 2.0 * math.pi
        q = np.zeros((m.n_cell, 3, swe.n, 1))
        q[:, 0, :, 0] = np.sin(k * xy[..., 0]) * np.cos(k * xy[..., 1])
        q[:, 1, :, 0] = np.cos(k * xy[..., 1])
        q[:, 2, :, 0] = np.sin(k * xy[..., 0])
        t = swe.tendency(q, 0.1)[..., 0]
        exact = np.stack([np.zeros_like(xy[..., 0]),
                          -c * k * np.cos(k * xy[..., 0]) * np.cos(k * xy[..., 1]),
                          c * k * np.sin(k * xy[..., 0]) * np.sin(k * xy[..., 1])], 1) * 0.1
        errs.append(np.abs(t - exact).max() / np.abs(exact).max())
    assert errs[1] < 0.35 * errs[0] and errs[1] < 0.08
    m = hi.torus(4)
    swe = LinearSwe(m, 3, g=1.0, H=2.0, f=0.0)
    q = np.ones((m.n_cell, 3, swe.n, 1))
    assert np.abs(swe.tendency(q, 1.0)).max() < 1e-10
