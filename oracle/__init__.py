"""FP64 CPU oracle for the HDG linearised shallow-water solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
executes this package; only the tests, the smoke check and the CPU-baseline
leg of the benchmark do.  It shares no code with the HIP library: its basis,
quadrature, topology, assembly, condensation and solvers are written here
from the paper, in plain numpy / scipy, for a reader to check by eye.

What it computes (paper section / equation):
* the standard upwind DG system of the linearised SWE, one implicit stage
  (Appendix A, Eq. bilinear_standardDG_upwind; general linear system), solved
  directly with SuperLU -- the plain definition of the result;
* the HDG system (Eq. bilinear_HDG_upwind), its operator split
  (Eq. ABCMform) and the three-step Schur solve (Steps 1-3, Eqs.
  schur_system, reconstruct_solution);
* the non-nested two-level V-cycle (Alg. twolevel_vcycle) with the P1 coarse
  space, injection prolongation and coarse form (Eq. coarse_problem_upwind);
* the learned-smoother MLP forward / backward in fp64;
* the Lax-Friedrichs flux (Eq. bilinear_HDG_lax): standard DG and HDG with
  a vector trace, the lowest-order Raviart-Thomas coarse space with the
  L2-projection prolongation and the grad-div coarse form
  (Eq. coarse_problem_LF), and its geometric multigrid (module lf);
* IMEX Runge-Kutta time stepping around the implicit stage (Eqs.
  IMEX_HDG_I, IMEX_HDG_II, theta_method) with the Theta, ARS2(2,3,2),
  SSP2(3,2,2) and ARS3(4,4,3) tableaux, explicit Coriolis, and the Delta_2
  error of Eq. L2_error (module imex);
* the non-hybridised DG solver of the native DG section: GMRES with the
  three-step approximate Schur-complement preconditioner (Eqs.
  native_matrix_representation, S_approx_diag), its sub-solves read as
  cell-block Jacobi and a two-level cycle with the Galerkin P1 operator
  (module dgschur).

Functions without an independent pin say "parity unpinned" in their
docstring.
"""
