"""Write exact_torus1.txt: the exact solution of one implicit HDG stage on the
1x1 periodic square (2 cells, 3 facets, 1 vertex), computed over Q(sqrt 2) by
oracle.exact for every case listed below.

    python tests/golden/make_exact_torus1.py

Right-hand sides are seeded integer multiples of 1/8 (exact in binary
floating point, so every solver receives the same rational input).  Values
are written with 17 significant digits.
"""
from __future__ import annotations

import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.exact import ExactStage, to_float, torus_cells  # noqa: E402

# p, dt, g, H, f, tau, seed
CASES = [
    (1, "1/2", "2", "1/2", "0", "1", 11),
    (1, "1/2", "2", "1/2", "3/4", "1", 12),
    (2, "1/2", "2", "1/2", "0", "1", 21),
    (2, "1/2", "2", "1/2", "3/4", "1", 22),
    (3, "1/2", "2", "1/2", "0", "1", 31),
    (3, "1/2", "2", "1/2", "3/4", "1", 32),
    (2, "1/4", "1", "1", "-1/2", "2", 23),
]


def rhs(p, seed):
    n = (p + 1) * (p + 2) // 2
    return np.random.default_rng(seed).integers(-8, 9, size=(2, 3, n)) / 8.0


def main(path=os.path.join(HERE, "exact_torus1.txt")):
    from fractions import Fraction
    lines = ["# exact HDG stage on the 1x1 periodic square, computed over Q(sqrt 2) (oracle.exact)",
             "# case: p dt g H f tau seed; then r (h, u1, u2 coefficients per cell), q (same layout), lam (facet, node)"]
    for p, dt, g, H, f, tau, seed in CASES:
        r = rhs(p, seed)
        ex = ExactStage(torus_cells(1), p, Fraction(dt), Fraction(g), Fraction(H), Fraction(f), Fraction(tau))
        q, lam = ex.solve(r.tolist())
        lines.append(f"case {p} {dt} {g} {H} {f} {tau} {seed}")
        lines.append("r " + " ".join(repr(float(v)) for v in r.ravel()))
        lines.append("q " + " ".join(f"{to_float(v):.17e}" for K in q for fl in K for v in fl))
        lines.append("lam " + " ".join(f"{to_float(v):.17e}" for e in lam for v in e))
    with open(path, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    return path


if __name__ == "__main__":
    print(main())
