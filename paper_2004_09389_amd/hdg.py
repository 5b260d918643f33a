"""ctypes binding of libhdg.so (the C ABI in include/hdg.h).

Argument marshalling only: every numerical step runs in the library's HIP
kernels.  Device buffers are torch CUDA (HIP) tensors; streams are torch's
current stream.  The library is loaded on first use (after torch, whose HIP
runtime it shares) and every call fails loudly when it has not been built.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhdg.so")

HDG_OK, HDG_EINVAL, HDG_ENOMEM, HDG_EHIP, HDG_EBREAKDOWN, HDG_ENOTCONV = 0, -1, -2, -3, -4, 1
HDG_TORUS, HDG_SPHERE = 0, 1
HDG_FLUX_UPWIND, HDG_FLUX_LF = 0, 1
HDG_FP64, HDG_MIXED, HDG_MIXED_IR = 0, 1, 2
HDG_KRYLOV_AUTO, HDG_KRYLOV_PCG, HDG_KRYLOV_FGMRES = 0, 1, 2
HDG_SMOOTH_BJACOBI, HDG_SMOOTH_MLP, HDG_SMOOTH_CHEBYSHEV = 0, 1, 2
KERNELS = {"apply": 0, "sweep": 1, "residual": 2, "condense": 3, "recover": 4, "mlp": 5}


class HdgMesh(ctypes.Structure):
    _fields_ = [("geom", ctypes.c_int32), ("n_vert", ctypes.c_int32), ("n_cell", ctypes.c_int32),
                ("period", ctypes.c_double), ("vert_xyz", ctypes.c_void_p),
                ("cell_vert", ctypes.c_void_p), ("cell_shift", ctypes.c_void_p)]


class HdgParams(ctypes.Structure):
    _fields_ = [("degree", ctypes.c_int32), ("dt", ctypes.c_double), ("g", ctypes.c_double),
                ("H", ctypes.c_double), ("f0", ctypes.c_double), ("omega", ctypes.c_double),
                ("tau", ctypes.c_double), ("flux", ctypes.c_int32)]


class HdgOptions(ctypes.Structure):
    _fields_ = [("krylov", ctypes.c_int32), ("precision", ctypes.c_int32), ("smoother", ctypes.c_int32),
                ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32), ("omega", ctypes.c_double),
                ("p1_nu", ctypes.c_int32), ("p1_omega", ctypes.c_double), ("rtol", ctypes.c_double),
                ("maxit", ctypes.c_int32), ("restart", ctypes.c_int32), ("max_rhs", ctypes.c_int32),
                ("use_graph", ctypes.c_int32), ("fallback_ratio", ctypes.c_double),
                ("p1_tail_max", ctypes.c_int32), ("p1_galerkin", ctypes.c_int32),
                ("rt_nu", ctypes.c_int32), ("rt_omega", ctypes.c_double), ("ir_inner_rtol", ctypes.c_double),
                ("persistent", ctypes.c_int32)]


class HdgSolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("refinements", ctypes.c_int32), ("fallbacks", ctypes.c_int32),
                ("status", ctypes.c_int32), ("rel_res", ctypes.c_double)]


class HdgSizes(ctypes.Structure):
    _fields_ = [("n_cell", ctypes.c_int32), ("n_facet", ctypes.c_int32), ("n_vert", ctypes.c_int32),
                ("degree", ctypes.c_int32), ("n_loc", ctypes.c_int32), ("n_levels", ctypes.c_int32),
                ("facet_dofs", ctypes.c_int32), ("flux", ctypes.c_int32), ("device_bytes", ctypes.c_int64), ("kappa", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("persistent", ctypes.c_int32)]


class HdgTuning(ctypes.Structure):
    _fields_ = [("mlp_samples_per_lane", ctypes.c_int32), ("rhs_block", ctypes.c_int32),
                ("cell_cells", ctypes.c_int32)]


HDG_IMEX_THETA, HDG_IMEX_ARS232, HDG_IMEX_SSP322, HDG_IMEX_ARS443 = 0, 1, 2, 3
IMEX_METHODS = {"theta": HDG_IMEX_THETA, "ars232": HDG_IMEX_ARS232, "ssp322": HDG_IMEX_SSP322,
                "ars443": HDG_IMEX_ARS443}


class HdgImexTableau(ctypes.Structure):
    _fields_ = [("stages", ctypes.c_int32), ("a", (ctypes.c_double * 5) * 5), ("at", (ctypes.c_double * 5) * 5),
                ("b", ctypes.c_double * 5), ("bt", ctypes.c_double * 5)]


class HdgImexInfo(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("solves", ctypes.c_int32), ("iters_total", ctypes.c_int32),
                ("iters_max", ctypes.c_int32), ("status", ctypes.c_int32), ("rel_res_max", ctypes.c_double)]


_P = ctypes.c_void_p
_I = ctypes.c_int32
_SIGS = {
    "hdg_default_options": (_I, [ctypes.POINTER(HdgOptions)]),
    "hdg_setup": (_I, [ctypes.POINTER(HdgMesh), _I, ctypes.POINTER(ctypes.c_void_p),
                       ctypes.POINTER(HdgParams), ctypes.POINTER(HdgOptions), ctypes.POINTER(_P)]),
    "hdg_get_sizes": (_I, [_P, ctypes.POINTER(HdgSizes)]),
    "hdg_get_topology": (_I, [_P, _P, _P, _P]),
    "hdg_condense": (_I, [_P, _I, _P, _P, _P]),
    "hdg_trace_apply": (_I, [_P, _I, _I, _P, _P, _P]),
    "hdg_mg_vcycle": (_I, [_P, _I, _I, _P, _P, _P]),
    "hdg_solve": (_I, [_P, _I, _P, _P, ctypes.POINTER(HdgSolveInfo), _P]),
    "hdg_recover": (_I, [_P, _I, _P, _P, _P, _P]),
    "hdg_condense_noalloc": (_I, [_P, _I, _P, _P, _P]),
    "hdg_stage_solve": (_I, [_P, _I, _P, _P, _P, ctypes.POINTER(HdgSolveInfo), _P]),
    "hdg_destroy": (None, [_P]),
    "hdg_last_error": (ctypes.c_char_p, []),
    "hdg_set_timing": (_I, [_P, _I]),
    "hdg_kernel_stats": (_I, [_P, _I, _I, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double)]),
    "hdg_copy": (_I, [_P, _P, ctypes.c_int64, _P]),
    "hdg_stream_triad": (_I, [_P, _P, ctypes.c_double, _P, ctypes.c_int64, _P]),
    "hdg_stream_read_blocks": (ctypes.c_int64, [ctypes.c_int64]),
    "hdg_stream_read": (_I, [_P, ctypes.c_int64, _P, ctypes.c_int64, _P]),
    "hdg_get_tuning": (_I, [_P, ctypes.POINTER(HdgTuning)]),
    "hdg_set_tuning": (_I, [_P, ctypes.POINTER(HdgTuning)]),
    "hdg_autotune": (_I, [_P, _I, ctypes.POINTER(HdgTuning), _P]),
    "hdg_mlp_set_weights": (_I, [_P, _P, _P]),
    "hdg_mlp_get_weights": (_I, [_P, _P, _P]),
    "hdg_mlp_make_data": (_I, [_P, _I, _P, _P, _P, _I, _P]),
    "hdg_mlp_loss_grad": (_I, [_P, _I, _P, _P, ctypes.POINTER(ctypes.c_double), _P, _P, _P]),
    "hdg_mlp_train": (_I, [_P, _I, _P, _I, _I, _I, ctypes.c_double, _P, _P]),
    "hdg_imex_tableau_get": (_I, [_I, ctypes.c_double, ctypes.POINTER(HdgImexTableau)]),
    "hdg_imex_work_size": (_I, [_P, ctypes.POINTER(HdgImexTableau), _I, ctypes.POINTER(ctypes.c_int64)]),
    "hdg_imex_run": (_I, [_P, ctypes.POINTER(HdgImexTableau), ctypes.c_double, ctypes.c_double, _I, _I, _P, _P,
                          ctypes.POINTER(HdgImexInfo), _P]),
    "hdg_dg_tendency": (_I, [_P, _I, ctypes.c_double, _P, _P, _P]),
    "hdg_dgs_setup": (_I, [_P, ctypes.POINTER(HdgMesh), _I, ctypes.POINTER(ctypes.c_void_p)]),
    "hdg_dgs_apply": (_I, [_P, _I, _P, _P, _P]),
    "hdg_dgs_precondition": (_I, [_P, _I, _P, _P, _P]),
    "hdg_dgs_solve": (_I, [_P, _I, _P, _P, ctypes.POINTER(HdgSolveInfo), _P]),
}

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libhdg.so; raises if it is missing (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run python -m paper_2004_09389_amd.build)")
    # torch first: its HIP runtime is then already in the process and the
    # library binds to the same one (loaded the other way round, torch's CUDA
    # initialisation later finds no device)
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class HdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hdg error {code}: {msg}")
        self.code = code


def _check(rc, allow=(HDG_OK,)):
    if rc not in allow:
        raise HdgError(rc, load_library().hdg_last_error().decode())
    return rc


def default_options() -> HdgOptions:
    o = HdgOptions()
    _check(load_library().hdg_default_options(ctypes.byref(o)))
    return o


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    """The current HIP stream of the current device (torch's raw-handle query when
    this torch build has it: it builds no Stream object)."""
    import torch
    raw = getattr(torch._C, "_cuda_getCurrentRawStream", None)
    if raw is not None:
        return ctypes.c_void_p(raw(torch.cuda.current_device()))
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


@dataclass
class SolveInfo:
    iters: int
    refinements: int
    fallbacks: int
    status: int
    rel_res: float


class HdgSolver:
    """One HDG context on the current GPU (see include/hdg.h for the method).

    hierarchy: hdg_inputs.Hierarchy (coarse -> fine; the finest mesh is the
    HDG mesh).  Device arrays are torch float64 tensors on cuda with the
    layouts of the C ABI: cell arrays (n_cell, 3, n_loc, nrhs), trace arrays
    (n_facet, facet_dofs, nrhs) with facet_dofs = p+1 (upwind flux) or
    2(p+1) (flux=HDG_FLUX_LF: x components at the nodes, then y).

    omega is the Earth's rotation rate (the Coriolis term); the block-Jacobi
    damping, the options field of the same name, is set with damping=.
    """

    def __init__(self, hierarchy, degree: int, dt: float, g: float = 1.0, H: float = 1.0,
                 f0: float = 0.0, omega: float = 0.0, tau: float = 1.0, flux: int = HDG_FLUX_UPWIND,
                 **options):
        import torch  # (initialises the HIP runtime through torch)
        self.lib = load_library()
        self.device = torch.cuda.current_device()
        self.hier = hierarchy
        opt = default_options()
        if "damping" in options:
            opt.omega = float(options.pop("damping"))
        for k, v in options.items():
            if not hasattr(opt, k):
                raise ValueError(f"unknown option {k}")
            setattr(opt, k, v)
        self.options = opt
        keep = []
        meshes = (HdgMesh * len(hierarchy.meshes))()
        for i, m in enumerate(hierarchy.meshes):
            vx = np.ascontiguousarray(m.vert_xyz, dtype=np.float64)
            cv = np.ascontiguousarray(m.cell_vert, dtype=np.int32)
            cs = np.ascontiguousarray(m.cell_shift, dtype=np.int32)
            keep += [vx, cv, cs]
            meshes[i] = HdgMesh(HDG_TORUS if m.kind == "torus" else HDG_SPHERE, m.n_vert, m.n_cell,
                                float(m.period), vx.ctypes.data, cv.ctypes.data, cs.ctypes.data)
        parents = (ctypes.c_void_p * len(hierarchy.meshes))()
        parents[0] = None
        for l, par in enumerate(hierarchy.parents):
            a = np.ascontiguousarray(par, dtype=np.int32)
            keep.append(a)
            parents[l + 1] = a.ctypes.data
        self._meshes, self._parents, self._keep = meshes, parents, keep
        prm = HdgParams(degree, dt, g, H, f0, omega, tau, int(flux))
        ctx = ctypes.c_void_p()
        _check(self.lib.hdg_setup(meshes, len(hierarchy.meshes), parents, ctypes.byref(prm),
                                  ctypes.byref(opt), ctypes.byref(ctx)))
        self.ctx = ctx
        sz = HdgSizes()
        _check(self.lib.hdg_get_sizes(ctx, ctypes.byref(sz)))
        self.sizes = sz
        self.p = degree
        self.flux = int(flux)
        self.m = sz.facet_dofs          # trace unknowns per facet
        self.mp = degree + 1            # trace nodes per facet (learned-smoother weight shapes)
        self.n_loc = sz.n_loc
        self.n_cell, self.n_facet, self.n_vert = sz.n_cell, sz.n_facet, sz.n_vert
        self.kappa = sz.kappa

    # ------------------------------------------------------------------ helpers
    def close(self):
        if getattr(self, "ctx", None):
            self.lib.hdg_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def trace_zeros(self, nrhs: int = 1):
        import torch
        return torch.zeros((self.n_facet, self.m, nrhs), dtype=torch.float64, device="cuda")

    def cell_zeros(self, nrhs: int = 1):
        import torch
        return torch.zeros((self.n_cell, 3, self.n_loc, nrhs), dtype=torch.float64, device="cuda")

    # Argument checks.  The C ABI receives bare device pointers and cannot see
    # buffer lengths, so every tensor is checked here against the context's
    # sizes before a pointer is passed: dtype, device, contiguity and the full
    # shape.  A mismatch raises ValueError and nothing is launched.
    def _dev_tensor(self, t, shape, name):
        import torch
        if not isinstance(t, torch.Tensor):
            raise ValueError(f"{name}: expected a torch tensor")
        if t.dtype != torch.float64:
            raise ValueError(f"{name}: expected float64, got {t.dtype}")
        if not t.is_cuda:
            raise ValueError(f"{name}: expected a CUDA tensor")
        if getattr(self, "device", None) is not None and t.device.index != self.device:
            raise ValueError(f"{name}: tensor is on cuda:{t.device.index}, the context on cuda:{self.device}")
        if not t.is_contiguous():
            raise ValueError(f"{name}: expected a contiguous tensor")
        if t.shape != tuple(shape):
            raise ValueError(f"{name}: expected shape {tuple(shape)}, got {tuple(t.shape)}")
        return t

    def _trace(self, t, name, nb=None):
        """A trace array (n_facet, facet_dofs, nrhs); returns nrhs (taken from t unless given)."""
        import torch
        if nb is None:
            if not isinstance(t, torch.Tensor) or t.dim() != 3:
                raise ValueError(f"{name}: expected a 3-d trace tensor (n_facet, facet_dofs, nrhs)")
            nb = int(t.shape[-1])
        self._nb_ok(nb, name)
        self._dev_tensor(t, (self.n_facet, self.m, nb), name)
        return nb

    def _cell(self, t, name, nb=None):
        """A cell array (n_cell, 3, n_loc, nrhs); returns nrhs (taken from t unless given)."""
        import torch
        if nb is None:
            if not isinstance(t, torch.Tensor) or t.dim() != 4:
                raise ValueError(f"{name}: expected a 4-d cell tensor (n_cell, 3, n_loc, nrhs)")
            nb = int(t.shape[-1])
        self._nb_ok(nb, name)
        self._dev_tensor(t, (self.n_cell, 3, self.n_loc, nb), name)
        return nb

    def _nb_ok(self, nb, name):
        if not 1 <= nb <= self.options.max_rhs:
            raise ValueError(f"{name}: nrhs = {nb} outside 1..max_rhs = {self.options.max_rhs}")

    @staticmethod
    def _distinct(*pairs):
        for a, b, what in pairs:
            if a.data_ptr() == b.data_ptr():
                raise ValueError(f"{what} must be distinct buffers")

    def topology(self):
        fc = np.zeros((self.n_facet, 2), dtype=np.int32)
        fl = np.zeros((self.n_facet, 2), dtype=np.int32)
        fv = np.zeros((self.n_facet, 2), dtype=np.int32)
        _check(self.lib.hdg_get_topology(self.ctx, fc.ctypes.data, fl.ctypes.data, fv.ctypes.data))
        return fc, fl, fv

    # ------------------------------------------------------------------ the ABI calls
    def condense(self, r_cell, out=None):
        nb = self._cell(r_cell, "r_cell")
        out = self.trace_zeros(nb) if out is None else out
        self._trace(out, "out", nb)
        _check(self.lib.hdg_condense(self.ctx, nb, _ptr(r_cell), _ptr(out), _stream()))
        return out

    def condense_noalloc(self, r_cell, out):
        """Step 1 with the library's static scratch (hdg_condense_noalloc): the
        caller passes the output buffer; nothing is allocated."""
        nb = self._cell(r_cell, "r_cell")
        self._trace(out, "out", nb)
        _check(self.lib.hdg_condense_noalloc(self.ctx, nb, _ptr(r_cell), _ptr(out), _stream()))
        return out

    def trace_apply(self, x, precision: int = HDG_FP64, out=None):
        nb = self._trace(x, "x")
        out = self.trace_zeros(nb) if out is None else out
        self._trace(out, "out", nb)
        self._distinct((x, out, "x and out"))
        _check(self.lib.hdg_trace_apply(self.ctx, nb, precision, _ptr(x), _ptr(out), _stream()))
        return out

    def mg_vcycle(self, r, precision: int = HDG_FP64, out=None):
        nb = self._trace(r, "r")
        out = self.trace_zeros(nb) if out is None else out
        self._trace(out, "out", nb)
        self._distinct((r, out, "r and out"))
        _check(self.lib.hdg_mg_vcycle(self.ctx, nb, precision, _ptr(r), _ptr(out), _stream()))
        return out

    def solve(self, rhat, lam=None, allow_notconv: bool = False) -> "tuple":
        nb = self._trace(rhat, "rhat")
        lam = self.trace_zeros(nb) if lam is None else lam
        self._trace(lam, "lam", nb)
        self._distinct((rhat, lam, "rhat and lam"))
        info = (HdgSolveInfo * nb)()
        allow = (HDG_OK, HDG_ENOTCONV) if allow_notconv else (HDG_OK,)
        _check(self.lib.hdg_solve(self.ctx, nb, _ptr(rhat), _ptr(lam), info, _stream()), allow)
        return lam, [SolveInfo(i.iters, i.refinements, i.fallbacks, i.status, i.rel_res) for i in info]

    def recover(self, r_cell, lam, out=None):
        nb = self._cell(r_cell, "r_cell")
        self._trace(lam, "lam", nb)
        out = self.cell_zeros(nb) if out is None else out
        self._cell(out, "out", nb)
        self._distinct((r_cell, out, "r_cell and out"))
        _check(self.lib.hdg_recover(self.ctx, nb, _ptr(r_cell), _ptr(lam), _ptr(out), _stream()))
        return out

    def step(self, r_cell):
        """Condense, solve, recover: one implicit stage.  Returns (q, lam, info)."""
        rhat = self.condense(r_cell)
        lam, info = self.solve(rhat)
        return self.recover(r_cell, lam), lam, info

    def stage_solve(self, r_cell, lam=None, q=None, allow_notconv: bool = False):
        """Steps 1-3 in one call (hdg_stage_solve: one launch when the context is
        small enough, see sizes.persistent).  Returns (q, lam, info)."""
        nb = self._cell(r_cell, "r_cell")
        lam = self.trace_zeros(nb) if lam is None else lam
        q = self.cell_zeros(nb) if q is None else q
        self._trace(lam, "lam", nb)
        self._cell(q, "q", nb)
        self._distinct((r_cell, q, "r_cell and q"))
        info = (HdgSolveInfo * nb)()
        allow = (HDG_OK, HDG_ENOTCONV) if allow_notconv else (HDG_OK,)
        _check(self.lib.hdg_stage_solve(self.ctx, nb, _ptr(r_cell), _ptr(lam), _ptr(q), info, _stream()), allow)
        return q, lam, [SolveInfo(i.iters, i.refinements, i.fallbacks, i.status, i.rel_res) for i in info]

    # ------------------------------------------------------------------ IMEX time stepping
    def dg_tendency(self, q, dt: float, out=None):
        """dt M^-1 (L(q) + N_c(q)): the explicit flux evaluation (hdg_dg_tendency)."""
        nb = self._cell(q, "q")
        out = self.cell_zeros(nb) if out is None else out
        self._cell(out, "out", nb)
        self._distinct((q, out, "q and out"))
        _check(self.lib.hdg_dg_tendency(self.ctx, nb, dt, _ptr(q), _ptr(out), _stream()))
        return out

    def imex_run(self, tableau: "HdgImexTableau", dt: float, f: float, q, steps: int, work=None,
                 allow_notconv: bool = False):
        """`steps` IMEX steps of size dt on q in place (hdg_imex_run); the context
        must have been set up with dt = gamma * dt and f0 = omega = 0.
        Returns the HdgImexInfo."""
        import torch
        nb = self._cell(q, "q")
        n = ctypes.c_int64()
        _check(self.lib.hdg_imex_work_size(self.ctx, ctypes.byref(tableau), nb, ctypes.byref(n)))
        if work is None:
            work = torch.empty(n.value, dtype=torch.float64, device="cuda")
        if not isinstance(work, torch.Tensor) or work.dim() != 1:
            raise ValueError("work: expected a 1-d tensor")
        self._dev_tensor(work, (work.numel(),), "work")
        if work.numel() < n.value:
            raise ValueError(f"work: needs at least {n.value} doubles, got {work.numel()}")
        self._distinct((q, work, "q and work"))
        info = HdgImexInfo()
        allow = (HDG_OK, HDG_ENOTCONV) if allow_notconv else (HDG_OK,)
        _check(self.lib.hdg_imex_run(self.ctx, ctypes.byref(tableau), dt, f, nb, steps, _ptr(q), _ptr(work),
                                     ctypes.byref(info), _stream()), allow)
        return info

    # ------------------------------------------------------------------ non-hybridised DG baseline
    def dgs_setup(self):
        """Build the DG + approximate Schur-complement baseline on this context."""
        _check(self.lib.hdg_dgs_setup(self.ctx, self._meshes, len(self.hier.meshes), self._parents))

    def dgs_apply(self, x, out=None):
        nb = self._cell(x, "x")
        out = self.cell_zeros(nb) if out is None else out
        self._cell(out, "out", nb)
        self._distinct((x, out, "x and out"))
        _check(self.lib.hdg_dgs_apply(self.ctx, nb, _ptr(x), _ptr(out), _stream()))
        return out

    def dgs_precondition(self, r, out=None):
        nb = self._cell(r, "r")
        out = self.cell_zeros(nb) if out is None else out
        self._cell(out, "out", nb)
        self._distinct((r, out, "r and out"))
        _check(self.lib.hdg_dgs_precondition(self.ctx, nb, _ptr(r), _ptr(out), _stream()))
        return out

    def dgs_solve(self, r_cell, out=None, allow_notconv: bool = False):
        """Solve the stage with the DG baseline; returns (q, [SolveInfo])."""
        nb = self._cell(r_cell, "r_cell")
        out = self.cell_zeros(nb) if out is None else out
        self._cell(out, "out", nb)
        self._distinct((r_cell, out, "r_cell and out"))
        info = (HdgSolveInfo * nb)()
        allow = (HDG_OK, HDG_ENOTCONV) if allow_notconv else (HDG_OK,)
        _check(self.lib.hdg_dgs_solve(self.ctx, nb, _ptr(r_cell), _ptr(out), info, _stream()), allow)
        return out, [SolveInfo(i.iters, i.refinements, i.fallbacks, i.status, i.rel_res) for i in info]

    # ------------------------------------------------------------------ learned smoother
    def mlp_set_weights(self, W1, W2):
        """W1 (64, 5(p+1)), W2 (p+1, 64); stored as FP32 (Adam state reset)."""
        W1 = np.ascontiguousarray(W1, dtype=np.float32)
        W2 = np.ascontiguousarray(W2, dtype=np.float32)
        if W1.shape != (64, 5 * self.mp) or W2.shape != (self.mp, 64):
            raise ValueError("W1 must be (64, 5(p+1)) and W2 (p+1, 64)")
        _check(self.lib.hdg_mlp_set_weights(self.ctx, W1.ctypes.data, W2.ctypes.data))

    def mlp_get_weights(self):
        W1 = np.zeros((64, 5 * self.mp), dtype=np.float32)
        W2 = np.zeros((self.mp, 64), dtype=np.float32)
        _check(self.lib.hdg_mlp_get_weights(self.ctx, W1.ctypes.data, W2.ctypes.data))
        return W1, W2

    def mlp_make_data(self, e, coarse_its: int = 1):
        """Training pair (u, t) for the trace error e."""
        nb = self._trace(e, "e")
        u, t = self.trace_zeros(nb), self.trace_zeros(nb)
        _check(self.lib.hdg_mlp_make_data(self.ctx, nb, _ptr(e), _ptr(u), _ptr(t), int(coarse_its), _stream()))
        return u, t

    def mlp_loss_grad(self, u, t):
        nb = self._trace(u, "u")
        self._trace(t, "t", nb)
        loss = ctypes.c_double()
        dW1 = np.zeros((64, 5 * self.mp), dtype=np.float32)
        dW2 = np.zeros((self.mp, 64), dtype=np.float32)
        _check(self.lib.hdg_mlp_loss_grad(self.ctx, nb, _ptr(u), _ptr(t), ctypes.byref(loss), dW1.ctypes.data,
                                          dW2.ctypes.data, _stream()))
        return float(loss.value), dW1, dW2

    def mlp_train(self, e0, cycles: int, coarse_its: int = 1, epochs: int = 1, lr: float = 1e-3):
        """Adam training in place from the error e0; returns the loss before every step."""
        nb = self._trace(e0, "e0")
        hist = np.zeros(cycles * epochs)
        _check(self.lib.hdg_mlp_train(self.ctx, nb, _ptr(e0), int(cycles), int(coarse_its), int(epochs),
                                      float(lr), hist.ctypes.data, _stream()))
        return hist

    # ------------------------------------------------------------------ launch tuning
    def get_tuning(self) -> dict:
        t = HdgTuning()
        _check(self.lib.hdg_get_tuning(self.ctx, ctypes.byref(t)))
        return _tuning_dict(t)

    def set_tuning(self, **kw):
        t = HdgTuning()
        _check(self.lib.hdg_get_tuning(self.ctx, ctypes.byref(t)))
        for k, v in kw.items():
            setattr(t, k, int(v))
        _check(self.lib.hdg_set_tuning(self.ctx, ctypes.byref(t)))

    def autotune(self, nrhs: int = 1, cache: str | None = None) -> dict:
        """hdg_autotune at nrhs right-hand sides.  With `cache` (a JSON file path)
        the choice is looked up first, under a key naming the device, the mesh,
        the degree, the flux, the precision, the smoother and nrhs, and a new
        choice is stored there."""
        key = self.tuning_key(nrhs) if cache is not None else None
        if key is not None:
            hit = tuning_cache_get(cache, key)
            if hit is not None:
                self.set_tuning(**hit)
                return self.get_tuning()
        t = HdgTuning()
        _check(self.lib.hdg_autotune(self.ctx, int(nrhs), ctypes.byref(t), _stream()))
        chosen = _tuning_dict(t)
        if key is not None:
            tuning_cache_put(cache, key, chosen)
        return chosen

    def tuning_key(self, nrhs: int) -> str:
        import torch
        o = self.options
        return "|".join(str(v) for v in (torch.cuda.get_device_name(self.device), self.hier.fine.kind,
                                          self.n_cell, self.n_facet, self.p, self.flux, o.precision,
                                          o.smoother, int(nrhs)))

    # ------------------------------------------------------------------ measurement
    def set_timing(self, repeat: int):
        """repeat = 0: off; repeat >= 1: event-time the instrumented kernels,
        each launch issued `repeat` times per event pair."""
        _check(self.lib.hdg_set_timing(self.ctx, int(repeat)))

    def kernel_stats(self, kernel: str, precision: int = HDG_FP64):
        n = ctypes.c_int64()
        ms = ctypes.c_double()
        b = ctypes.c_double()
        _check(self.lib.hdg_kernel_stats(self.ctx, KERNELS[kernel], precision, ctypes.byref(n),
                                         ctypes.byref(ms), ctypes.byref(b)))
        return int(n.value), float(ms.value), float(b.value)


def _tuning_dict(t: HdgTuning) -> dict:
    return {f: int(getattr(t, f)) for f, _ in HdgTuning._fields_}


def tuning_cache_get(path: str, key: str):
    """The tuning stored under key in the JSON file at path, or None (no file,
    no entry, or an entry that does not name every tuning field)."""
    import json
    try:
        with open(path) as f:
            entry = json.load(f).get("entries", {}).get(key)
    except (OSError, ValueError):
        return None
    fields = [f for f, _ in HdgTuning._fields_]
    if not isinstance(entry, dict) or any(not isinstance(entry.get(f), int) for f in fields):
        return None
    return {f: entry[f] for f in fields}


def tuning_cache_put(path: str, key: str, tuning: dict) -> None:
    """Store tuning under key in the JSON file at path (other entries kept;
    written to a temporary file and renamed into place)."""
    import json
    import os
    import tempfile
    data = {"version": 1, "entries": {}}
    try:
        with open(path) as f:
            old = json.load(f)
        if isinstance(old, dict) and isinstance(old.get("entries"), dict):
            data["entries"] = old["entries"]
    except (OSError, ValueError):
        pass
    data["entries"][key] = {f: int(tuning[f]) for f, _ in HdgTuning._fields_}
    d = os.path.dirname(os.path.abspath(path))
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".hdg_tuning.")
    with os.fdopen(fd, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def device_copy(src, dst):
    _dev_f64(src, dst)
    if dst.numel() < src.numel() or src.data_ptr() == dst.data_ptr():
        raise ValueError("dst must be a distinct buffer at least as long as src")
    _check(load_library().hdg_copy(_ptr(src), _ptr(dst), src.numel(), _stream()))


def _dev_f64(*ts):
    import torch
    for t in ts:
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError("expected contiguous float64 CUDA tensors")


def stream_triad(b, c, s, a):
    """a = b + s c on the current stream (hdg_stream_triad); float64 CUDA tensors."""
    _dev_f64(a, b, c)
    if not (a.numel() == b.numel() == c.numel()):
        raise ValueError("a, b and c must have the same length")
    _check(load_library().hdg_stream_triad(_ptr(b), _ptr(c), float(s), _ptr(a), a.numel(), _stream()))


def stream_read_blocks(n: int) -> int:
    return int(load_library().hdg_stream_read_blocks(int(n)))


def stream_read(src, partial):
    """Per-chunk sums of src into partial on the current stream (hdg_stream_read)."""
    _dev_f64(src, partial)
    _check(load_library().hdg_stream_read(_ptr(src), src.numel(), _ptr(partial), partial.numel(), _stream()))


def imex_tableau(method: str, theta: float = 0.5) -> HdgImexTableau:
    """The library's tableau of one of IMEX_METHODS (hdg_imex_tableau_get)."""
    t = HdgImexTableau()
    _check(load_library().hdg_imex_tableau_get(IMEX_METHODS[method], theta, ctypes.byref(t)))
    return t


def imex_gamma(t: HdgImexTableau) -> float:
    """The common nonzero diagonal entry of the implicit tableau (the stage
    operator is set up for dt_stage = gamma * dt)."""
    return next(t.at[i][i] for i in range(t.stages) if t.at[i][i] != 0.0)
