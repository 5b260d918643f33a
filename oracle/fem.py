"""Mesh topology, cell geometry and a physical-space Lagrange basis (oracle).

Definitions (spatial discretisation section; DG space Eq. DG_space_def, trace
space Eq. DG_trace_def):
* V_h: P^p on every cell; the basis is the Lagrange basis at the equispaced
  lattice nodes, built here directly in each cell's own 2-D coordinates by
  inverting a monomial Vandermonde matrix (no reference-element map is used
  for the basis itself).
* Lambda_h: P^p on every facet, Lagrange basis at p+1 equispaced points.
* The skeleton: every facet is the side of exactly two cells (periodic
  domain or closed sphere).

Topology conventions (also implemented, independently, by the library):
* local facet i of a cell joins local vertices (i+1)%3 -> (i+2)%3, which is
  the cell's counter-clockwise direction;
* facets are numbered in order of first appearance when cells are scanned in
  order and local facets 0, 1, 2 within a cell; the first cell is the
  facet's owner and fixes its direction; trace node k sits at parameter
  k/p along that direction;
* the second cell traverses the facet backwards, so its local node k is
  global node p - k.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .quadrature import gauss01, triangle_rule


# --------------------------------------------------------------------------- topology

@dataclass
class Topology:
    cell_facet: np.ndarray   # (n_cell, 3) facet id of local facet i
    cell_rev: np.ndarray     # (n_cell, 3) True where the cell runs against the facet direction
    facet_cell: np.ndarray   # (n_facet, 2) owner, other
    facet_loc: np.ndarray    # (n_facet, 2) local facet index in owner, other
    facet_vert: np.ndarray   # (n_facet, 2) start, end vertex (facet direction)

    @property
    def n_facet(self) -> int:
        return int(self.facet_cell.shape[0])


def _edge_key(va, sa, vb, sb):
    d = (int(sb[0] - sa[0]), int(sb[1] - sa[1]))
    if va < vb:
        return (va, vb, d)
    if va > vb:
        return (vb, va, (-d[0], -d[1]))
    return (va, va, max(d, (-d[0], -d[1])))


def topology(mesh) -> Topology:
    cv, cs = mesh.cell_vert, mesh.cell_shift
    nk = cv.shape[0]
    seen = {}
    cell_facet = np.zeros((nk, 3), dtype=np.int64)
    cell_rev = np.zeros((nk, 3), dtype=bool)
    fc, fl, fv = [], [], []
    for K in range(nk):
        for i in range(3):
            a, b = (i + 1) % 3, (i + 2) % 3
            key = _edge_key(int(cv[K, a]), cs[K, a], int(cv[K, b]), cs[K, b])
            e = seen.get(key)
            if e is None:
                e = len(fc)
                seen[key] = e
                fc.append([K, -1])
                fl.append([i, -1])
                fv.append([int(cv[K, a]), int(cv[K, b])])
            else:
                if fc[e][1] != -1:
                    raise ValueError("facet shared by more than two cells")
                fc[e][1] = K
                fl[e][1] = i
                cell_rev[K, i] = True
            cell_facet[K, i] = e
    fc = np.array(fc)
    if (fc[:, 1] < 0).any():
        raise ValueError("boundary facet found: mesh must be closed or periodic")
    return Topology(cell_facet, cell_rev, fc, np.array(fl), np.array(fv))


# --------------------------------------------------------------------------- geometry

@dataclass
class Geometry:
    corners3: np.ndarray   # (n_cell, 3, 3) unwrapped corners
    e1: np.ndarray         # (n_cell, 3) frame
    e2: np.ndarray
    P: np.ndarray          # (n_cell, 3, 2) corners in frame coordinates, relative to corner 0
    area: np.ndarray       # (n_cell,)
    fnormal: np.ndarray    # (n_cell, 3, 2) outward unit normal of local facet i (frame coords)
    flen: np.ndarray       # (n_cell, 3)


def geometry(mesh) -> Geometry:
    X = mesh.cell_coords()
    nk = X.shape[0]
    if mesh.kind == "torus":
        e1 = np.tile([1.0, 0.0, 0.0], (nk, 1))
        e2 = np.tile([0.0, 1.0, 0.0], (nk, 1))
    else:
        ab, ac = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]
        k = np.cross(ab, ac)
        k /= np.linalg.norm(k, axis=1, keepdims=True)
        e1 = ab / np.linalg.norm(ab, axis=1, keepdims=True)
        e2 = np.cross(k, e1)
    rel = X - X[:, :1, :]
    P = np.stack([np.einsum("ckd,cd->ck", rel, e1), np.einsum("ckd,cd->ck", rel, e2)], axis=-1)
    area = 0.5 * (P[:, 1, 0] * P[:, 2, 1] - P[:, 1, 1] * P[:, 2, 0])
    if (area <= 0).any():
        raise ValueError("cells must be counter-clockwise")
    fnormal = np.zeros((nk, 3, 2))
    flen = np.zeros((nk, 3))
    for i in range(3):
        t = P[:, (i + 2) % 3] - P[:, (i + 1) % 3]
        L = np.linalg.norm(t, axis=1)
        t /= L[:, None]
        fnormal[:, i, 0] = t[:, 1]     # right of the counter-clockwise traversal = outward
        fnormal[:, i, 1] = -t[:, 0]
        flen[:, i] = L
    return Geometry(X, e1, e2, P, area, fnormal, flen)


def to_3d(geo: Geometry, Z: np.ndarray) -> np.ndarray:
    """Frame coordinates (n_cell, Q, 2) -> 3-D points (n_cell, Q, 3)."""
    return (geo.corners3[:, None, 0, :] + Z[..., 0:1] * geo.e1[:, None, :]
            + Z[..., 1:2] * geo.e2[:, None, :])


# --------------------------------------------------------------------------- bases

def lattice(p: int) -> np.ndarray:
    return np.array([(i / p, j / p) for j in range(p + 1) for i in range(p + 1 - j)])


def exponents(p: int):
    return [(a, d - a) for d in range(p + 1) for a in range(d, -1, -1)]


class CellBasis:
    """Lagrange basis of P^p on each cell, in the cell's own frame coordinates."""

    def __init__(self, geo: Geometry, p: int):
        self.p = p
        self.geo = geo
        lat = lattice(p)
        self.nodes = (lat[None, :, 0:1] * geo.P[:, None, 1, :]
                      + lat[None, :, 1:2] * geo.P[:, None, 2, :])          # (nk, n, 2)
        self.center = geo.P.mean(axis=1)                                    # (nk, 2)
        self.scale = geo.flen.max(axis=1)                                   # (nk,)
        self.exps = exponents(p)
        V = self._mono(self.nodes)                                          # (nk, n, n)
        self.coef = np.linalg.inv(V)                                        # columns = basis functions

    def _mono(self, Z):
        zh = (Z - self.center[:, None, :]) / self.scale[:, None, None]
        return np.stack([zh[..., 0] ** a * zh[..., 1] ** b for a, b in self.exps], axis=-1)

    def _dmono(self, Z):
        zh = (Z - self.center[:, None, :]) / self.scale[:, None, None]
        dx = np.stack([a * zh[..., 0] ** max(a - 1, 0) * zh[..., 1] ** b for a, b in self.exps], -1)
        dy = np.stack([b * zh[..., 0] ** a * zh[..., 1] ** max(b - 1, 0) for a, b in self.exps], -1)
        s = 1.0 / self.scale[:, None, None]
        return dx * s, dy * s

    def values(self, Z):
        """Z: (nk, Q, 2) frame coords -> (nk, Q, n)."""
        return np.einsum("cqa,cai->cqi", self._mono(Z), self.coef)

    def grads(self, Z):
        """-> (nk, Q, n, 2)."""
        dx, dy = self._dmono(Z)
        gx = np.einsum("cqa,cai->cqi", dx, self.coef)
        gy = np.einsum("cqa,cai->cqi", dy, self.coef)
        return np.stack([gx, gy], axis=-1)


def lagrange1d(p: int, s: np.ndarray) -> np.ndarray:
    """Equispaced 1-D Lagrange basis on [0, 1] at points s -> (len(s), p+1)."""
    nodes = np.arange(p + 1) / p
    out = np.ones((len(s), p + 1))
    for k in range(p + 1):
        for l in range(p + 1):
            if l != k:
                out[:, k] *= (s - nodes[l]) / (nodes[k] - nodes[l])
    return out


# --------------------------------------------------------------------------- quadrature on cells

def volume_points(geo: Geometry, degree: int):
    """Quadrature points (nk, Q, 2) in frame coords and weights (nk, Q)."""
    ref, w = triangle_rule(degree)
    Z = ref[None, :, 0:1] * geo.P[:, None, 1, :] + ref[None, :, 1:2] * geo.P[:, None, 2, :]
    return Z, w[None, :] * (2.0 * geo.area)[:, None]


def facet_points(geo: Geometry, i: int, s: np.ndarray):
    """Points at counter-clockwise parameter s along local facet i -> (nk, len(s), 2)."""
    a = geo.P[:, (i + 1) % 3]
    b = geo.P[:, (i + 2) % 3]
    return a[:, None, :] + s[None, :, None] * (b - a)[:, None, :]


def facet_rule(p: int):
    return gauss01(p + 2)
