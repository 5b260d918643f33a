"""Mesh generators for the two mesh families of the paper.

* Periodic unit square split into n x n squares, each cut into two triangles
  along the (0,0)-(1,1) diagonal (grid layout section; N_cell = 2 n^2).
* Icosahedral sphere: the 20-triangle icosahedron refined r times by midpoint
  subdivision, new vertices pushed out to the sphere (spherical geometry
  section; N_cell = 20 * 4^r).  Cells are flat triangles whose vertices lie on
  the sphere.

Both families are nested under refinement; `*_hierarchy` returns the chain of
meshes from coarse to fine together with, for every vertex of a finer level,
the two coarse vertices it sits between (equal for a vertex inherited from the
coarser level).

Conventions (part of the data format, used by both the library and the
oracle):
* cells are counter-clockwise seen from outside (torus: seen from +z);
* the coordinates of local vertex k of cell K are
  vert_xyz[cell_vert[K, k]] + period * (cell_shift[K, k, 0], cell_shift[K, k, 1], 0),
  so every cell is given by its unwrapped corners.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List

import numpy as np


@dataclass
class Mesh:
    kind: str                 # "torus" or "sphere"
    vert_xyz: np.ndarray      # (n_vert, 3) float64
    cell_vert: np.ndarray     # (n_cell, 3) int32
    cell_shift: np.ndarray    # (n_cell, 3, 2) int32, periodic image offsets (zeros on the sphere)
    period: float = 1.0       # torus side length
    radius: float = 0.0       # sphere radius
    n: int = 0                # torus: squares per side; sphere: refinement level

    @property
    def n_vert(self) -> int:
        return int(self.vert_xyz.shape[0])

    @property
    def n_cell(self) -> int:
        return int(self.cell_vert.shape[0])

    def cell_coords(self) -> np.ndarray:
        """Unwrapped corner coordinates, (n_cell, 3, 3)."""
        x = self.vert_xyz[self.cell_vert].copy()
        x[:, :, 0] += self.period * self.cell_shift[:, :, 0]
        x[:, :, 1] += self.period * self.cell_shift[:, :, 1]
        return x


@dataclass
class Hierarchy:
    meshes: List[Mesh] = field(default_factory=list)     # coarse -> fine
    parents: List[np.ndarray] = field(default_factory=list)  # parents[l-1]: (n_vert_l, 2) into level l-1

    @property
    def fine(self) -> Mesh:
        return self.meshes[-1]


def torus(n: int, period: float = 1.0) -> Mesh:
    """n x n periodic squares, each split into a lower-right and an upper-left triangle."""
    if n < 1:
        raise ValueError("n must be >= 1")
    h = period / n
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    vert = np.zeros((n * n, 3))
    vert[:, 0] = (ii.ravel()) * h
    vert[:, 1] = (jj.ravel()) * h

    def vid(i, j):
        return (j % n) * n + (i % n)

    cells = np.zeros((2 * n * n, 3), dtype=np.int32)
    shifts = np.zeros((2 * n * n, 3, 2), dtype=np.int32)
    k = 0
    for j in range(n):
        for i in range(n):
            corners = {
                "00": (i, j), "10": (i + 1, j), "11": (i + 1, j + 1), "01": (i, j + 1),
            }
            for tri in (("00", "10", "11"), ("00", "11", "01")):
                for loc, name in enumerate(tri):
                    ci, cj = corners[name]
                    cells[k, loc] = vid(ci, cj)
                    shifts[k, loc, 0] = ci // n
                    shifts[k, loc, 1] = cj // n
                k += 1
    return Mesh("torus", vert, cells, shifts, period=period, n=n)


def torus_hierarchy(n: int, n_coarse: int = 4, period: float = 1.0) -> Hierarchy:
    """Chain torus(n_coarse), torus(2 n_coarse), ..., torus(n); n / n_coarse must be a power of 2."""
    sizes = [n]
    while sizes[-1] % 2 == 0 and sizes[-1] // 2 >= n_coarse:
        sizes.append(sizes[-1] // 2)
    sizes = sizes[::-1]
    meshes = [torus(s, period) for s in sizes]
    parents = []
    for nf in sizes[1:]:
        nc = nf // 2
        par = np.zeros((nf * nf, 2), dtype=np.int32)
        for j in range(nf):
            for i in range(nf):
                v = j * nf + i
                ci0, cj0 = i // 2, j // 2
                ci1, cj1 = ((i + 1) // 2) % nc, ((j + 1) // 2) % nc
                # even/even: inherited vertex; otherwise the midpoint of the coarse
                # horizontal, vertical or (0,0)-(1,1) diagonal edge
                par[v, 0] = cj0 * nc + ci0
                par[v, 1] = cj1 * nc + ci1
        parents.append(par)
    return Hierarchy(meshes, parents)


_ICO_FACES = [
    (0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
    (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
    (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
    (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1),
]


def _icosahedron(radius: float):
    g = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([
        (-1, g, 0), (1, g, 0), (-1, -g, 0), (1, -g, 0),
        (0, -1, g), (0, 1, g), (0, -1, -g), (0, 1, -g),
        (g, 0, -1), (g, 0, 1), (-g, 0, -1), (-g, 0, 1),
    ], dtype=np.float64)
    v *= radius / np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array(_ICO_FACES, dtype=np.int32)
    # orient counter-clockwise seen from outside
    a, b, c = v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]
    s = np.einsum("ij,ij->i", np.cross(b - a, c - a), a)
    flip = s < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    return v, f


def _refine_sphere(v: np.ndarray, f: np.ndarray, radius: float):
    edge_mid = {}
    newv = [row for row in v]
    par = [(i, i) for i in range(len(v))]

    def mid(a, b):
        key = (a, b) if a < b else (b, a)
        if key not in edge_mid:
            x = 0.5 * (v[a] + v[b])
            x *= radius / np.linalg.norm(x)
            edge_mid[key] = len(newv)
            newv.append(x)
            par.append(key)
        return edge_mid[key]

    out = np.zeros((4 * len(f), 3), dtype=np.int32)
    for k, (a, b, c) in enumerate(f):
        ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
        out[4 * k + 0] = (a, ab, ca)
        out[4 * k + 1] = (ab, b, bc)
        out[4 * k + 2] = (ca, bc, c)
        out[4 * k + 3] = (ab, bc, ca)
    return np.array(newv), out, np.array(par, dtype=np.int32)


def icosphere_hierarchy(level: int, radius: float = 1.0, level_coarse: int = 0) -> Hierarchy:
    v, f = _icosahedron(radius)
    meshes, parents = [], []
    for lev in range(level + 1):
        if lev > 0:
            v, f, par = _refine_sphere(v, f, radius)
            if lev > level_coarse:
                parents.append(par)
        if lev >= level_coarse:
            meshes.append(Mesh("sphere", v.copy(), f.copy(),
                               np.zeros((len(f), 3, 2), dtype=np.int32),
                               radius=radius, n=lev))
    return Hierarchy(meshes, parents)


def icosphere(level: int, radius: float = 1.0) -> Mesh:
    return icosphere_hierarchy(level, radius, level_coarse=level).fine
