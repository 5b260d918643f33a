"""Training driver and weight files of the learned smoother.

The arithmetic (data generation, forward and backward passes, Adam) runs in
the library's kernels (hdg_mlp_train); this module only feeds it seeded
random initial errors and stores the result.

Training data: the first cycle of plain-multigrid runs started from random
initial guesses.  For the error e of such a guess (iid N(0,1) trace values)
the pair is (u, t) with u = omega D^-1 S e and t = (I - pi S_c^-1 pi^T S) e - u
(see include/hdg.h).  Errors left after further plain cycles are not used:
they are smooth, and their coarse-complement part is set by the coarse space
rather than by anything a facet patch can see.
"""
from __future__ import annotations

import struct
import time

import numpy as np

MAGIC = b"HDGMLP01"


def train(solver, batches: int = 32, nrhs: int | None = None, epochs: int = 8, lr: float = 1e-3,
          coarse_its: int = 2, seed0: int = 1000, verbose: bool = False):
    """Train solver's network in place on `batches` batches of random initial
    errors (seeds seed0, seed0 + 1, ...), `epochs` Adam steps per batch.
    Returns (loss history, seconds)."""
    import torch
    import hdg_inputs as hi

    nb = nrhs or solver.options.max_rhs
    hist = []
    t0 = time.perf_counter()
    for b in range(batches):
        e0 = torch.from_numpy(hi.iid_trace(solver.n_facet, solver.p, seed0 + b, nb)).to("cuda")
        h = solver.mlp_train(e0, cycles=1, coarse_its=coarse_its, epochs=epochs, lr=lr)
        hist.extend(h.tolist())
        if verbose and (b % 8 == 0 or b == batches - 1):
            print(f"[train] batch {b} loss {h[0]:.4f} -> {h[-1]:.4f}", flush=True)
    torch.cuda.synchronize()
    return np.asarray(hist), time.perf_counter() - t0


def save_weights(path: str, degree: int, W1, W2) -> None:
    """Versioned binary: magic, int32 degree, int32 hidden, FP32 W1 then W2 (row-major)."""
    W1 = np.ascontiguousarray(W1, dtype="<f4")
    W2 = np.ascontiguousarray(W2, dtype="<f4")
    m = degree + 1
    if W1.shape != (W1.shape[0], 5 * m) or W2.shape != (m, W1.shape[0]):
        raise ValueError("weight shapes do not match the degree")
    with open(path, "wb") as f:
        f.write(MAGIC)
        f.write(struct.pack("<ii", degree, W1.shape[0]))
        f.write(W1.tobytes())
        f.write(W2.tobytes())


def load_weights(path: str):
    """Returns (degree, W1, W2)."""
    with open(path, "rb") as f:
        if f.read(8) != MAGIC:
            raise ValueError(f"{path}: not a learned-smoother weight file")
        degree, hidden = struct.unpack("<ii", f.read(8))
        m = degree + 1
        W1 = np.frombuffer(f.read(4 * hidden * 5 * m), dtype="<f4").reshape(hidden, 5 * m).copy()
        W2 = np.frombuffer(f.read(4 * m * hidden), dtype="<f4").reshape(m, hidden).copy()
    return degree, W1, W2
