"""Quadrature rules (oracle).

Gauss-Legendre on [0, 1] from numpy, and a collapsed (Duffy) product rule on
the reference triangle {xi, eta >= 0, xi + eta <= 1}.  Pinned by the closed
form  int_T xi^a eta^b = a! b! / (a + b + 2)!.
"""
from __future__ import annotations

import numpy as np


def gauss01(n: int):
    """n-point Gauss-Legendre rule on [0, 1]: exact for degree 2n - 1."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def triangle_rule(degree: int):
    """Collapsed rule exact for polynomials of total degree <= degree.

    Points (xi, eta) = (s (1 - t), t) with s, t Gauss points on [0, 1]; the
    Jacobian (1 - t) raises the degree in t by one.
    """
    n = (degree + 2) // 2 + 1
    s, ws = gauss01(n)
    t, wt = gauss01(n)
    S, T = np.meshgrid(s, t, indexing="ij")
    W = np.outer(ws, wt) * (1.0 - T)
    pts = np.stack([(S * (1.0 - T)).ravel(), T.ravel()], axis=1)
    return pts, W.ravel()
