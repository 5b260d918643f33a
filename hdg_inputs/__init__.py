"""Seeded synthetic inputs shared by the HIP path and the CPU oracle.

This package holds mesh generators (vertex coordinates, cell->vertex lists,
periodic image shifts, nested-refinement parent maps) and right-hand-side
generators (random DG coefficients) and the closed-form stationary vortex
used as an initial condition.  It contains none of the method's
arithmetic: no quadrature, no basis, no operator, no topology beyond the
cell->vertex lists that define a mesh.
"""
from .mesh import Mesh, Hierarchy, torus, torus_hierarchy, icosphere, icosphere_hierarchy
from .rhs import (n_loc, ref_nodes, iid_rhs, fourier_rhs_torus, smooth_rhs_sphere, balanced_flow_sphere, cell_frames,
                  mlp_init, iid_trace)
from .vortex import Vortex, vortex_coefficients, paper_time_step

__all__ = [
    "Mesh", "Hierarchy", "torus", "torus_hierarchy", "icosphere", "icosphere_hierarchy",
    "n_loc", "ref_nodes", "iid_rhs", "fourier_rhs_torus", "smooth_rhs_sphere", "balanced_flow_sphere", "cell_frames",
    "mlp_init", "iid_trace",
    "Vortex", "vortex_coefficients", "paper_time_step",
]
