"""Pin of the FP64 oracle against the exact solution of one implicit stage on
the 1x1 periodic square (2 cells, 3 facets, 1 vertex): the full HDG system of
Eq. bilinear_HDG_upwind with the flux condition (one stage of
Eq. general_linear_system) solved over Q(sqrt 2) by oracle.exact, an
assembly in exact arithmetic that shares nothing with the floating-point
oracle.  The exact values are stored in tests/golden/exact_torus1.txt
(written by tests/golden/make_exact_torus1.py)."""
from __future__ import annotations

import os
from fractions import Fraction

import numpy as np
import pytest

import hdg_inputs as hi
from oracle.hdg import DgOracle, HdgOracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "exact_torus1.txt")


def load_cases():
    cases, cur = [], None
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        key, *vals = line.split()
        if key == "case":
            p = int(vals[0])
            dt, g, H, f, tau = (Fraction(v) for v in vals[1:6])
            cur = {"p": p, "dt": dt, "g": g, "H": H, "f": f, "tau": tau, "seed": int(vals[6])}
            cases.append(cur)
        else:
            cur[key] = np.array([float(v) for v in vals])
    n = lambda c: (c["p"] + 1) * (c["p"] + 2) // 2
    for c in cases:
        c["r"] = c["r"].reshape(2, 3, n(c))
        c["q"] = c["q"].reshape(2, 3, n(c))
    return cases


CASES = load_cases()
IDS = [f"p{c['p']}-f{c['f']}-tau{c['tau']}" for c in CASES]


def rel(a, b):
    return np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b))


def oracle_args(c):
    return (hi.torus(1), c["p"], float(c["dt"]), float(c["g"]), float(c["H"]), float(c["f"]), 0.0, float(c["tau"]))


def test_golden_cases_cover_every_degree_with_and_without_coriolis():
    seen = {(c["p"], c["f"] != 0) for c in CASES}
    assert seen >= {(p, fz) for p in (1, 2, 3) for fz in (False, True)}


@pytest.mark.parametrize("c", CASES, ids=IDS)
@pytest.mark.parametrize("kind", ["hdg", "dg"])
def test_oracle_equals_exact_solution(c, kind):
    """Both oracle paths (condensed HDG trace system, monolithic standard DG)
    reproduce the exact q and lam to 1e-13, every field separately."""
    cls = HdgOracle if kind == "hdg" else DgOracle
    q, lam = cls(*oracle_args(c)).solve(c["r"])
    for fld in range(3):
        assert rel(q[:, fld], c["q"][:, fld]) < 1e-13, fld
    assert rel(lam, c["lam"]) < 1e-13


def test_golden_file_is_the_exact_solution():
    """The stored values are what oracle.exact computes (degrees 1 and 2;
    degree 3 takes tens of seconds and is covered by the oracle agreement)."""
    from oracle.exact import ExactStage, to_float, torus_cells
    for c in CASES:
        if c["p"] > 2:
            continue
        ex = ExactStage(torus_cells(1), c["p"], c["dt"], c["g"], c["H"], c["f"], c["tau"])
        q, lam = ex.solve(c["r"].tolist())
        qf = np.array([[[to_float(v) for v in fl] for fl in K] for K in q])
        lf = np.array([[to_float(v) for v in e] for e in lam]).ravel()
        assert rel(qf, c["q"]) < 1e-16 and rel(lf, c["lam"]) < 1e-16


@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("f", [Fraction(0), Fraction(3, 4)])
def test_exact_solver_constant_state(p, f):
    """The exact assembly reproduces the closed form of the stage for constant
    fields exactly: h = h0, u = (I + dt f J)^-1 U0, lam = h0 sqrt(g/H)."""
    import sympy as sp
    from oracle.exact import ExactStage, torus_cells
    n = (p + 1) * (p + 2) // 2
    h0, U0 = Fraction(3, 8), (Fraction(-5, 4), Fraction(1, 2))
    dt, g, H = Fraction(1, 2), Fraction(2), Fraction(1, 2)
    r = [[[h0] * n, [U0[0]] * n, [U0[1]] * n] for _ in range(2)]
    q, lam = ExactStage(torus_cells(1), p, dt, g, H, f).solve(r)
    a = dt * f
    det = 1 + a * a
    u1 = (U0[0] + a * U0[1]) / det
    u2 = (U0[1] - a * U0[0]) / det
    for K in range(2):
        for i in range(n):
            assert sp.simplify(q[K][0][i] - sp.Rational(h0)) == 0
            assert sp.simplify(q[K][1][i] - sp.Rational(u1)) == 0
            assert sp.simplify(q[K][2][i] - sp.Rational(u2)) == 0
    for e in lam:
        for v in e:
            assert sp.simplify(v - sp.Rational(h0) * 2) == 0   # sqrt(g/H) = 2


class _Planted(HdgOracle):
    """HdgOracle with one mistake planted in its local blocks."""
    mistake = None

    def hdg_blocks(self):
        A, B, C, Mt = super().hdg_blocks()
        n, m = self.n, self.m
        U1, U2 = slice(n, 2 * n), slice(2 * n, 3 * n)
        if self.mistake == "coriolis_sign":
            A[:, U1, U2] *= -1
            A[:, U2, U1] *= -1
        elif self.mistake == "drop_tau_in_trace_row":
            C[:, :, :n] = 0
        elif self.mistake == "transposed_gradient":
            A[:, U1, :n] = np.transpose(A[:, U1, :n], (0, 2, 1))   # (grad phi, w) for (phi, div w)
        elif self.mistake == "trace_mass_sign":
            Mt *= -1
        elif self.mistake == "reversed_facet_nodes":
            for i in range(3):
                L = slice(i * m, (i + 1) * m)
                B[:, :, L] = B[:, :, L][:, :, ::-1]
                C[:, L, :] = C[:, L, :][:, ::-1, :]
        return A, B, C, Mt


@pytest.mark.parametrize("mistake", ["coriolis_sign", "drop_tau_in_trace_row", "transposed_gradient",
                                     "trace_mass_sign", "reversed_facet_nodes"])
def test_planted_oracle_mistakes_fail_the_exact_pin(mistake, monkeypatch):
    """A plausible mistake in the oracle's assembly moves its solution far from
    the exact one (the pin discriminates)."""
    c = next(c for c in CASES if c["p"] == 2 and c["f"] != 0 and c["tau"] == 1)
    monkeypatch.setattr(_Planted, "mistake", mistake)
    q, lam = _Planted(*oracle_args(c)).solve(c["r"])
    err = max(rel(q, c["q"]), rel(lam, c["lam"]))
    assert err > 1e-6, err
