"""MI355X-native HDG trace-multigrid solver for one implicit stage of the
linearised rotating shallow-water equations (arXiv:2004.09389 hot path).

The numerics live in libhdg.so (HIP, gfx950) behind the C ABI of
include/hdg.h; `paper_2004_09389_amd.hdg` is its ctypes binding.

One implicit stage (condense, trace solve, recover) on the 256 x 256 torus,
p = 3, mixed precision::

    import torch
    import hdg_inputs as hi
    from paper_2004_09389_amd.hdg import HDG_MIXED, HdgSolver

    hier = hi.torus_hierarchy(256, 32)
    s = HdgSolver(hier, 3, 8.0 / 256, 1.0, 1.0, 1.0, precision=HDG_MIXED)
    r = torch.from_numpy(hi.fourier_rhs_torus(hier.fine, 3, 100)).cuda()
    q, lam, info = s.step(r)

IMEX time stepping around the stage (Coriolis explicit, so the stage context
has f0 = 0 and is set up for gamma * dt)::

    from paper_2004_09389_amd.hdg import imex_gamma, imex_tableau
    tab = imex_tableau("ars232")
    s = HdgSolver(hier, 3, imex_gamma(tab) * dt, g, H)
    info = s.imex_run(tab, dt, f, q, steps)        # q updated in place

The non-hybridised DG solver the paper compares against, on the same
context: ``s.dgs_setup(); q, info = s.dgs_solve(r)``.
"""
