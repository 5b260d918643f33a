"""The Python binding rejects every mis-shaped, mistyped or aliased tensor
with ValueError before any library call (the C ABI takes bare device
pointers and cannot see buffer lengths).  Runs on the CPU: the tensors are
stand-ins that report CUDA residency, and the library object fails the test
if any entry point is reached."""
import ctypes

import pytest
import torch

from paper_2004_09389_amd import hdg as H


class _NoLib:
    def __getattr__(self, name):
        raise AssertionError(f"library entry {name} reached despite a bad argument")


class _Dev:
    index = 0


class FakeCuda:
    """Duck-typed stand-in for a CUDA tensor (shape, dtype, contiguity, pointer)."""
    _next = 4096

    def __init__(self, *shape, dtype=torch.float64, contiguous=True, cuda=True, ptr=None):
        self.shape = tuple(shape)
        self.dtype = dtype
        self._contig = contiguous
        self.is_cuda = cuda
        self.device = _Dev()
        FakeCuda._next += 4096
        self._ptr = FakeCuda._next if ptr is None else ptr

    def dim(self):
        return len(self.shape)

    def numel(self):
        n = 1
        for s in self.shape:
            n *= s
        return n

    def is_contiguous(self):
        return self._contig

    def data_ptr(self):
        return self._ptr


@pytest.fixture
def solver(monkeypatch):
    monkeypatch.setattr(torch, "Tensor", FakeCuda)   # isinstance checks accept the stand-ins
    s = H.HdgSolver.__new__(H.HdgSolver)
    s.lib, s.ctx, s.device = _NoLib(), ctypes.c_void_p(1), 0
    s.n_facet, s.m, s.n_cell, s.n_loc, s.mp = 12, 3, 8, 6, 3
    opt = H.HdgOptions()
    opt.max_rhs = 4
    s.options = opt
    s.trace_zeros = lambda nb=1: FakeCuda(12, 3, nb)
    s.cell_zeros = lambda nb=1: FakeCuda(8, 3, 6, nb)
    return s


def T(nb=1, **kw):
    return FakeCuda(12, 3, nb, **kw)


def C(nb=1, **kw):
    return FakeCuda(8, 3, 6, nb, **kw)


BAD_TRACE = [
    ("short", lambda: FakeCuda(11, 3, 1)),
    ("wrong dofs", lambda: FakeCuda(12, 2, 1)),
    ("2-d", lambda: FakeCuda(36, 1)),
    ("float32", lambda: T(dtype=torch.float32)),
    ("host", lambda: T(cuda=False)),
    ("strided", lambda: T(contiguous=False)),
    ("nrhs above max", lambda: T(5)),
]
BAD_CELL = [
    ("short", lambda: FakeCuda(7, 3, 6, 1)),
    ("wrong n_loc", lambda: FakeCuda(8, 3, 3, 1)),
    ("3-d", lambda: FakeCuda(8, 18, 1)),
    ("float32", lambda: C(dtype=torch.float32)),
    ("strided", lambda: C(contiguous=False)),
]


@pytest.mark.parametrize("bad", BAD_TRACE, ids=[b[0] for b in BAD_TRACE])
def test_trace_inputs(solver, bad):
    for call in (lambda x: solver.trace_apply(x), lambda x: solver.mg_vcycle(x), lambda x: solver.solve(x),
                 lambda x: solver.mlp_make_data(x), lambda x: solver.mlp_train(x, 1)):
        with pytest.raises(ValueError):
            call(bad[1]())


@pytest.mark.parametrize("bad", BAD_TRACE, ids=[b[0] for b in BAD_TRACE])
def test_trace_outputs_and_lam(solver, bad):
    with pytest.raises(ValueError):
        solver.trace_apply(T(), out=bad[1]())
    with pytest.raises(ValueError):
        solver.mg_vcycle(T(), out=bad[1]())
    with pytest.raises(ValueError):
        solver.condense(C(), out=bad[1]())
    with pytest.raises(ValueError):
        solver.solve(T(), lam=bad[1]())
    with pytest.raises(ValueError):
        solver.recover(C(), bad[1]())


def test_lam_with_fewer_rhs_than_the_solve(solver):
    with pytest.raises(ValueError):
        solver.solve(T(4), lam=T(1))
    with pytest.raises(ValueError):
        solver.recover(C(4), T(1))
    with pytest.raises(ValueError):
        solver.condense(C(2), out=T(1))


@pytest.mark.parametrize("bad", BAD_CELL, ids=[b[0] for b in BAD_CELL])
def test_cell_arrays(solver, bad):
    for call in (lambda x: solver.condense(x), lambda x: solver.recover(x, T()),
                 lambda x: solver.dg_tendency(x, 0.1), lambda x: solver.dgs_apply(x),
                 lambda x: solver.dgs_precondition(x), lambda x: solver.dgs_solve(x)):
        with pytest.raises(ValueError):
            call(bad[1]())
    for call in (lambda o: solver.recover(C(), T(), out=o), lambda o: solver.dg_tendency(C(), 0.1, out=o),
                 lambda o: solver.dgs_apply(C(), out=o), lambda o: solver.dgs_solve(C(), out=o)):
        with pytest.raises(ValueError):
            call(bad[1]())


def test_aliased_buffers(solver):
    x = T()
    with pytest.raises(ValueError):
        solver.trace_apply(x, out=x)
    with pytest.raises(ValueError):
        solver.solve(x, lam=x)
    q = C()
    with pytest.raises(ValueError):
        solver.dg_tendency(q, 0.1, out=q)


def test_imex_work_too_small(solver):
    class Lib:
        def hdg_imex_work_size(self, ctx, tab, nb, out):
            out._obj.value = 1000
            return 0

        def __getattr__(self, name):
            raise AssertionError(f"library entry {name} reached despite a bad argument")

    solver.lib = Lib()
    tab = H.HdgImexTableau()
    with pytest.raises(ValueError):
        solver.imex_run(tab, 0.1, 0.0, C(), 1, work=FakeCuda(999))
    with pytest.raises(ValueError):
        solver.imex_run(tab, 0.1, 0.0, C(), 1, work=FakeCuda(500, 2))
    with pytest.raises(ValueError):
        solver.imex_run(tab, 0.1, 0.0, C(), 1, work=FakeCuda(1000, dtype=torch.float32))


def test_learned_smoother_pair_shapes(solver):
    with pytest.raises(ValueError):
        solver.mlp_loss_grad(T(2), T(1))
