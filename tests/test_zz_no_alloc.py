"""hdg_condense_noalloc (the allocation-free condensation, static device
scratch) called through the C ABI: bit-for-bit equal to hdg_condense on two
calls in a row, the second with a smaller input, and a clear HDG_EINVAL above
the scratch size."""
import ctypes

import numpy as np
import pytest

import hdg_inputs as hi

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _both(s, r):
    """rhat from hdg_condense and from hdg_condense_noalloc (C ABI), default stream."""
    import torch
    nb = r.shape[-1]
    ref = s.trace_zeros(nb)
    out = torch.full_like(ref, float("nan"))
    assert s.lib.hdg_condense(s.ctx, nb, _ptr(r), _ptr(ref), None) == 0
    rc = s.lib.hdg_condense_noalloc(s.ctx, nb, _ptr(r), _ptr(out), None)
    assert rc == 0, s.lib.hdg_last_error().decode()
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_condense_equals_condense_then_a_smaller_input():
    import torch
    from oracle.hdg import HdgOracle
    from paper_2004_09389_amd.hdg import HdgSolver
    big = HdgSolver(hi.torus_hierarchy(16, 4), 2, 0.3, 1.0, 1.0, 0.5, 0.0, max_rhs=4)
    r1 = torch.from_numpy(hi.iid_rhs(big.hier.fine, 2, 71, nrhs=4)).to("cuda")
    ref1, out1 = _both(big, r1)
    assert np.array_equal(ref1, out1)
    o = HdgOracle(big.hier.fine, 2, 0.3, 1.0, 1.0, 0.5, 0.0)
    rh = o.rhat(r1.cpu().numpy()[..., 2])
    assert np.linalg.norm(out1[..., 2].ravel() - rh) / np.linalg.norm(rh) < 1e-12
    # second call: a smaller input on another context (8x8 torus, p = 1, one right-hand side)
    small = HdgSolver(hi.torus_hierarchy(8, 4), 1, 0.5, max_rhs=1)
    r2 = torch.from_numpy(hi.iid_rhs(small.hier.fine, 1, 72, nrhs=1)).to("cuda")
    ref2, out2 = _both(small, r2)
    assert np.array_equal(ref2, out2)
    # and the first context again with fewer right-hand sides
    ref3, out3 = _both(big, r1[..., :1].contiguous())
    assert np.array_equal(ref3, out3) and np.array_equal(out3[..., 0], out1[..., 0])
    big.close()
    small.close()


def test_noalloc_condense_rejects_inputs_beyond_the_scratch():
    import torch
    from paper_2004_09389_amd.hdg import HDG_EINVAL, HdgSolver
    s = HdgSolver(hi.torus_hierarchy(128, 32), 3, 0.05, max_rhs=11)
    r = torch.from_numpy(hi.iid_rhs(s.hier.fine, 3, 73, nrhs=11)).to("cuda")
    out = s.trace_zeros(11)
    # 3 * 4 * 32768 * 11 doubles > 4194304
    assert s.lib.hdg_condense_noalloc(s.ctx, 11, _ptr(r), _ptr(out), None) == HDG_EINVAL
    assert "use hdg_condense" in s.lib.hdg_last_error().decode()
    r10 = r[..., :10].contiguous()
    ref, got = _both(s, r10)     # 3932160 doubles: fits
    assert np.array_equal(ref, got)
    s.close()
