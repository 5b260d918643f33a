"""Seeded right-hand sides in the DG coefficient layout.

Layout convention (shared by library and oracle, stated once here):
* a DG field on cell K is given by its values at the equispaced lattice nodes
  (i/p, j/p), i + j <= p, of the reference triangle, ordered j-major then i
  (lexicographic), mapped to x = a + xi (b - a) + eta (c - a) with (a, b, c) the
  unwrapped corners of K;
* a right-hand side array is (n_cell, 3, n_loc, nrhs): field 0 is r_h, fields
  1, 2 are the two components of r_u.  On the torus the components are along
  x and y; on the sphere they are along the cell frame e1 = (b - a)/|b - a|,
  e2 = k x e1 with k the unit normal of the flat cell.

Randomness comes only from numpy PCG64 `default_rng(seed)`.
"""
from __future__ import annotations

import numpy as np

from .mesh import Mesh


def n_loc(p: int) -> int:
    return (p + 1) * (p + 2) // 2


def ref_nodes(p: int) -> np.ndarray:
    """Equispaced lattice on the reference triangle, j-major then i, as (xi, eta)."""
    return np.array([(i / p, j / p) for j in range(p + 1) for i in range(p + 1 - j)], dtype=np.float64)


def node_coords(mesh: Mesh, p: int) -> np.ndarray:
    """Unwrapped physical coordinates of the DG nodes, (n_cell, n_loc, 3)."""
    x = mesh.cell_coords()
    xe = ref_nodes(p)
    a, b, c = x[:, 0], x[:, 1], x[:, 2]
    return a[:, None, :] + xe[None, :, 0:1] * (b - a)[:, None, :] + xe[None, :, 1:2] * (c - a)[:, None, :]


def cell_frames(mesh: Mesh):
    """Per-cell orthonormal tangent frame (e1, e2, k), each (n_cell, 3)."""
    x = mesh.cell_coords()
    if mesh.kind == "torus":
        nc = mesh.n_cell
        e1 = np.tile([1.0, 0.0, 0.0], (nc, 1))
        e2 = np.tile([0.0, 1.0, 0.0], (nc, 1))
        k = np.tile([0.0, 0.0, 1.0], (nc, 1))
        return e1, e2, k
    ab = x[:, 1] - x[:, 0]
    ac = x[:, 2] - x[:, 0]
    k = np.cross(ab, ac)
    k /= np.linalg.norm(k, axis=1, keepdims=True)
    e1 = ab / np.linalg.norm(ab, axis=1, keepdims=True)
    e2 = np.cross(k, e1)
    return e1, e2, k


def iid_rhs(mesh: Mesh, p: int, seed: int, nrhs: int = 1) -> np.ndarray:
    """iid N(0,1) coefficients, (n_cell, 3, n_loc, nrhs)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((mesh.n_cell, 3, n_loc(p), nrhs))


def _fourier_modes(rng, n_modes: int, kmax: int, dim: int):
    grid = np.stack(np.meshgrid(*([np.arange(-kmax, kmax + 1)] * dim), indexing="ij"), -1).reshape(-1, dim)
    nrm = np.linalg.norm(grid, axis=1)
    cand = grid[(nrm > 0) & (nrm <= kmax)]
    idx = rng.choice(len(cand), size=n_modes, replace=False)
    k = cand[idx].astype(np.float64)
    amp = rng.standard_normal(n_modes) * np.linalg.norm(k, axis=1) ** -2.0
    phase = rng.uniform(0.0, 2.0 * np.pi, n_modes)
    return k, amp, phase


def fourier_rhs_torus(mesh: Mesh, p: int, seed: int, nrhs: int = 1,
                      n_modes: int = 64, kmax: int = 16) -> np.ndarray:
    """Smooth periodic random field: per field, a sum of n_modes cosines with
    integer wavevectors |k| <= kmax, N(0,1) amplitudes decaying as |k|^-2 and
    uniform phases, sampled at the DG nodes.  (n_cell, 3, n_loc, nrhs)."""
    rng = np.random.default_rng(seed)
    x = node_coords(mesh, p)[..., :2] / mesh.period
    out = np.zeros((mesh.n_cell, 3, n_loc(p), nrhs))
    for r in range(nrhs):
        for fld in range(3):
            k, amp, ph = _fourier_modes(rng, n_modes, kmax, 2)
            arg = 2.0 * np.pi * np.einsum("cnd,md->cnm", x, k) + ph
            out[:, fld, :, r] = np.cos(arg) @ amp
    return out


def _cos_sum(x, modes, scale, device=None, chunk=1 << 16):
    """sum_m amp_m cos(scale k_m . x + phase_m) at the points x (..., d): with
    device (a torch device) the sums are evaluated there in float64, in chunks
    of points; the modes come from the caller's numpy generator either way."""
    k, amp, ph = modes
    if device is None:
        return np.cos(scale * np.einsum("...d,md->...m", x, k) + ph) @ amp
    import torch
    flat = x.reshape(-1, x.shape[-1])
    kt = torch.as_tensor(k, dtype=torch.float64, device=device)
    at = torch.as_tensor(amp, dtype=torch.float64, device=device)
    pt = torch.as_tensor(ph, dtype=torch.float64, device=device)
    out = np.empty(flat.shape[0])
    for i in range(0, flat.shape[0], chunk):
        xt = torch.as_tensor(flat[i:i + chunk], dtype=torch.float64, device=device)
        out[i:i + chunk] = (torch.cos(scale * (xt @ kt.T) + pt) @ at).cpu().numpy()
    return out.reshape(x.shape[:-1])


def _sin_grad_sum(x, modes, scale, device=None, chunk=1 << 16):
    """Gradient of sum_m amp_m cos(scale k_m . x + phase_m): -sum_m amp_m scale k_m sin(...)."""
    k, amp, ph = modes
    if device is None:
        s = np.sin(scale * np.einsum("...d,md->...m", x, k) + ph) * amp
        return -scale * s @ k
    import torch
    flat = x.reshape(-1, x.shape[-1])
    kt = torch.as_tensor(k, dtype=torch.float64, device=device)
    at = torch.as_tensor(amp, dtype=torch.float64, device=device)
    pt = torch.as_tensor(ph, dtype=torch.float64, device=device)
    out = np.empty(flat.shape)
    for i in range(0, flat.shape[0], chunk):
        xt = torch.as_tensor(flat[i:i + chunk], dtype=torch.float64, device=device)
        out[i:i + chunk] = (-scale * (torch.sin(scale * (xt @ kt.T) + pt) * at) @ kt).cpu().numpy()
    return out.reshape(x.shape)


def smooth_rhs_sphere(mesh: Mesh, p: int, seed: int, nrhs: int = 1,
                      n_modes: int = 64, kmax: int = 8,
                      h_scale: float = 100.0, u_scale: float = 20.0, device=None) -> np.ndarray:
    """Smooth random fields on the sphere: 3-D Fourier sums in x / radius,
    the vector one projected onto each cell's frame; height scaled to max
    |h| = h_scale, velocity to max |u| = u_scale.  (n_cell, 3, n_loc, nrhs).
    device: evaluate the sums with torch on that device (same modes)."""
    rng = np.random.default_rng(seed)
    x = node_coords(mesh, p) / mesh.radius
    e1, e2, _ = cell_frames(mesh)
    out = np.zeros((mesh.n_cell, 3, n_loc(p), nrhs))
    for r in range(nrhs):
        fields = [_cos_sum(x, _fourier_modes(rng, n_modes, kmax, 3), np.pi, device) for _ in range(4)]
        h = fields[0]
        vec = np.stack(fields[1:], -1)
        u1 = np.einsum("cnd,cd->cn", vec, e1)
        u2 = np.einsum("cnd,cd->cn", vec, e2)
        out[:, 0, :, r] = h * (h_scale / np.abs(h).max())
        umax = np.sqrt(u1 ** 2 + u2 ** 2).max()
        out[:, 1, :, r] = u1 * (u_scale / umax)
        out[:, 2, :, r] = u2 * (u_scale / umax)
    return out


def balanced_flow_sphere(mesh: Mesh, p: int, seed: int, omega: float, g: float,
                         u_max: float = 20.0, n_modes: int = 64, kmax: int = 16, device=None) -> np.ndarray:
    """A smooth random flow in linear balance on the sphere, at the DG nodes:
    streamfunction psi = a sum of n_modes random 3-D Fourier modes in x / radius
    (amplitudes N(0,1) |k|^-2, uniform phases), velocity u = n x grad_s psi
    (n the outward unit normal, grad_s the tangential gradient) scaled so that
    max |u| = u_max, height h = f psi / g with f = 2 omega z / |x| (the linear
    balance f n x u = -g grad h with f taken locally constant), the velocity
    projected onto each cell's frame.  (n_cell, 3, n_loc): (h, u1, u2)."""
    rng = np.random.default_rng(seed)
    R = mesh.radius
    X = node_coords(mesh, p)
    x = X / R
    modes = _fourier_modes(rng, n_modes, kmax, 3)
    psi = _cos_sum(x, modes, np.pi, device)
    grad = _sin_grad_sum(x, modes, np.pi, device) / R          # d psi / d X
    nrm = X / np.linalg.norm(X, axis=-1, keepdims=True)
    gs = grad - np.sum(grad * nrm, axis=-1, keepdims=True) * nrm
    u = np.cross(nrm, gs)
    scale = u_max / np.linalg.norm(u, axis=-1).max()
    psi, u = psi * scale, u * scale
    f = 2.0 * omega * nrm[..., 2]
    e1, e2, _ = cell_frames(mesh)
    out = np.zeros((mesh.n_cell, 3, n_loc(p)))
    out[:, 0] = f * psi / g
    out[:, 1] = np.einsum("cnd,cd->cn", u, e1)
    out[:, 2] = np.einsum("cnd,cd->cn", u, e2)
    return out


def iid_trace(n_facet: int, p: int, seed: int, nrhs: int = 1) -> np.ndarray:
    """iid N(0,1) trace vector (n_facet, p+1, nrhs): a random initial error."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n_facet, p + 1, nrhs))


def mlp_init(m: int, hidden: int = 64, seed: int = 0):
    """Initial weights of the learned smoother, drawn from PCG64(seed): first
    layer He-normal (std sqrt(2 / fan_in)), last layer zero.  (hidden, 5m) and
    (m, hidden), float64."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((hidden, 5 * m)) * np.sqrt(2.0 / (5 * m))
    W2 = np.zeros((m, hidden))
    return W1, W2
