/*
 * hdg.h -- C ABI of the MI355X (gfx950) HDG trace-multigrid solver for one
 * implicit stage of the linearised rotating shallow-water equations.
 *
 * Method (Betteridge, Gibson, Graham, Mueller, arXiv:2004.09389):
 *   - hybridised DG with the upwind flux and a scalar facet trace
 *     (Eq. bilinear_HDG_upwind), one implicit stage of the general linear
 *     system (Eq. general_linear_system, alpha = 1);
 *   - static condensation onto the trace: S lam = rhat with
 *     S = M + C A^-1 B, rhat = C A^-1 f  (Eq. ABCMform; Steps 1-2,
 *     Eq. schur_system), recovery q = A^-1 (f - B lam) (Step 3,
 *     Eq. reconstruct_solution);
 *   - Krylov on the trace system preconditioned by the non-nested two-level
 *     V-cycle (Alg. twolevel_vcycle) with the P1 coarse space, injection
 *     prolongation and the coarse form of Eq. coarse_problem_upwind, the
 *     coarse problem solved by one P1 geometric-multigrid V-cycle;
 *   - alternatively (prm.flux = HDG_FLUX_LF, torus only) the Lax-Friedrichs
 *     flux with a vector trace (Eq. bilinear_HDG_lax), the lowest-order
 *     Raviart-Thomas coarse space, the L2-projection prolongation of the
 *     cells' average and the grad-div coarse form of Eq. coarse_problem_LF,
 *     solved by one geometric-multigrid V-cycle over the nested RT0 spaces
 *     with vertex-patch smoothing.
 *
 * Equations solved (in the caller's variables), with c = sqrt(g H):
 *     u + dt (f k x u + g grad h) = r_u,     h + dt H div u = r_h.
 * Internally phi = h sqrt(g/H) and kappa = c dt (symmetric form, linearised
 * SWE with flat bathymetry); the upwind trace unknown lam lives in phi
 * units, the Lax-Friedrichs trace is the velocity uhat.
 *
 * Discretisation conventions (shared with any independent checker):
 *   - DG basis: Lagrange at the equispaced lattice (i/p, j/p), i+j <= p, of
 *     the reference triangle, ordered j-major then i, mapped affinely onto the
 *     cell's unwrapped corners (a, b, c);
 *   - local facet i of a cell runs from local vertex (i+1)%3 to (i+2)%3
 *     (counter-clockwise); facets are numbered by first appearance scanning
 *     cells in order and local facets 0,1,2; the first cell owns the facet and
 *     fixes its direction; trace node k is at parameter k/p along it;
 *   - velocity components: x, y on the torus; on the sphere the flat cell's
 *     frame e1 = (b-a)/|b-a|, e2 = k x e1, k the unit cell normal;
 *   - Lax-Friedrichs trace: per facet the x components at the p+1 nodes,
 *     then the y components (facet_dofs = 2(p+1));
 *   - RT0 coarse unknown of a facet: the flux of the field through it along
 *     the owner cell's outward normal;
 *   - Coriolis f = f0 (torus) or f0 + 2 Omega z/|x| (sphere), integrated with
 *     the collapsed Gauss-Legendre rule of (p+3)^2 points.
 *
 * Array layouts (all row-major, RHS index innermost):
 *   cell arrays   [n_cell][3][n_loc][nrhs]   fields (h, u1, u2), n_loc = (p+1)(p+2)/2
 *   trace arrays  [n_facet][facet_dofs][nrhs]   facet_dofs = p+1 (upwind) or 2(p+1) (LF)
 * Device pointers are HIP device memory owned by the caller; the library
 * never frees them.  Trace arrays must be 16-byte aligned (every hipMalloc
 * and torch allocation is; HDG_EINVAL otherwise).  Host pointers are read
 * during the call only.
 *
 * Errors: every int-returning entry returns HDG_OK (0) on success, a
 * negative code on failure (message in hdg_last_error(), thread-local), and
 * HDG_ENOTCONV (> 0) when a solve stopped at maxit (info still filled).
 * Calls are asynchronous on the given stream unless stated otherwise; one
 * context must not be used from two threads or streams at once.
 */
#ifndef HDG_H
#define HDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
#define HDG_OK          0
#define HDG_EINVAL     -1   /* bad argument or shape */
#define HDG_ENOMEM     -2   /* device or host allocation failed */
#define HDG_EHIP       -3   /* HIP runtime error */
#define HDG_EBREAKDOWN -4   /* NaN / Inf or Krylov breakdown */
#define HDG_ENOTCONV    1   /* maxit reached before rtol */

#define HDG_TORUS  0
#define HDG_SPHERE 1

#define HDG_FLUX_UPWIND 0   /* scalar trace, P1 coarse space (Eq. bilinear_HDG_upwind) */
#define HDG_FLUX_LF     1   /* vector trace, RT0 coarse space (Eq. bilinear_HDG_lax); torus only */

#define HDG_FP64     0      /* everything in FP64 */
#define HDG_MIXED    1      /* FP64 Krylov with the FP64 operator; the V-cycle uses the FP32
                               operator rows, BF16 smoother rows and FP32 block inverses with FP32
                               accumulation; P1 coarse solve in FP64.  Inside hdg_solve the
                               V-cycle's work vectors and the FGMRES Z basis are FP32 (the V basis,
                               lam and the true residual FP64); hdg_mg_vcycle keeps FP64 vectors */
#define HDG_MIXED_IR 2      /* hdg_solve only: FP64 iterative refinement (true residual with the
                               FP64 operator at every restart) around an inner flexible GMRES
                               that applies the FP32 operator and the mixed V-cycle, its basis
                               vectors held in FP32; each inner solve reduces the residual by
                               ir_inner_rtol */

#define HDG_KRYLOV_AUTO   0 /* PCG when the trace operator and the V-cycle are symmetric (f = 0, FP64,
                               nu_pre = nu_post, a linear smoother), else FGMRES */
#define HDG_KRYLOV_PCG    1
#define HDG_KRYLOV_FGMRES 2

#define HDG_SMOOTH_BJACOBI   0 /* damped facet block-Jacobi sweeps */
#define HDG_SMOOTH_MLP       1 /* learned smoother (see below; upwind flux only) */
#define HDG_SMOOTH_CHEBYSHEV 2 /* Chebyshev iteration of degree nu_pre / nu_post preconditioned by facet
                                  block-Jacobi on [0.1, 1.1] lambda_max(D^-1 S), lambda_max from 20
                                  power steps at setup (the smoother of the paper's solver settings) */

/* ------------------------------------------------------------------ types */
typedef struct hdg_ctx hdg_ctx;

/* One triangle mesh.  Corner k of cell K sits at
 * vert_xyz[cell_vert[K][k]] + period * (cell_shift[K][k][0], cell_shift[K][k][1], 0).
 * Cells are counter-clockwise seen from outside (+z on the torus). */
typedef struct {
    int32_t geom;               /* HDG_TORUS or HDG_SPHERE */
    int32_t n_vert, n_cell;
    double period;              /* torus side length (ignored on the sphere) */
    const double  *vert_xyz;    /* (host) [n_vert][3] */
    const int32_t *cell_vert;   /* (host) [n_cell][3] */
    const int32_t *cell_shift;  /* (host) [n_cell][3][2], NULL means all zero */
} hdg_mesh;

typedef struct {
    int32_t degree;             /* p in 1..3: DG degree, also the trace degree */
    double dt, g, H;            /* time step, gravity, mean depth (g, H > 0, dt > 0) */
    double f0, omega;           /* Coriolis: f0 + 2 omega z/|x| on the sphere, f0 on the torus */
    double tau;                 /* HDG stabilisation (> 0); 1 is the paper's flux (either kind) */
    int32_t flux;               /* HDG_FLUX_UPWIND (0) or HDG_FLUX_LF */
} hdg_params;

typedef struct {
    int32_t krylov;             /* HDG_KRYLOV_* */
    int32_t precision;          /* solve path: HDG_FP64, HDG_MIXED or HDG_MIXED_IR */
    int32_t smoother;           /* HDG_SMOOTH_BJACOBI, HDG_SMOOTH_MLP or HDG_SMOOTH_CHEBYSHEV */
    int32_t nu_pre, nu_post;    /* smoothing sweeps (Chebyshev degree) before / after the coarse
                                   correction (default 2, 2) */
    double  omega;              /* block-Jacobi damping (default 0.7) */
    int32_t p1_nu;              /* P1 damped-Jacobi sweeps per level, pre and post (default 2) */
    double  p1_omega;           /* P1 Jacobi damping (default 2/3) */
    double  rtol;               /* stop when ||rhat - S lam||_2 <= rtol ||rhat||_2 (default 1e-8) */
    int32_t maxit;              /* max Krylov iterations in total (default 200) */
    int32_t restart;            /* FGMRES restart length (default 30, max 64) */
    int32_t max_rhs;            /* largest nrhs any call will use (default 1, max 64) */
    int32_t use_graph;          /* replay each Krylov iteration as a captured HIP graph (default 1);
                                   off while kernel timing is enabled */
    double  fallback_ratio;     /* learned smoother: revert to block-Jacobi when the relative
                                   residual shrinks by less than this factor per iteration, as a
                                   geometric mean over the current restart cycle, checked from
                                   its second iteration on (default 0.5) */
    int32_t p1_tail_max;        /* P1 levels with at most this many vertices run inside one
                                   single-workgroup kernel (default 4096, max 4096, 0 = never);
                                   only when the coarsest level has at most 256 vertices, and
                                   per call only when nrhs x the top tail level's vertices <= 4096 */
    int32_t p1_galerkin;        /* (upwind flux only) 0: the rediscretised coarse form (1/kappa)(M_1 + kappa^2 K_1) on
                                   every P1 level (default); 1: the Galerkin form S_c = pi^T S pi on
                                   the finest P1 level (the footnoted alternative of the non-nested
                                   multigrid section) and P^T A P below it */
    int32_t rt_nu;              /* LF flux: vertex-patch smoothing steps per RT0 level, pre and post
                                   (default 1) */
    double  rt_omega;           /* LF flux: damping of the additive vertex-patch smoother (default 0.5) */
    double  ir_inner_rtol;      /* HDG_MIXED_IR: relative reduction of each inner solve (default 1e-4) */
    int32_t persistent;         /* 1 (default): when the trace system is small enough for one workgroup's
                                   LDS (see hdg_sizes.persistent), hdg_solve and hdg_stage_solve run the
                                   whole solve as one launch with one workgroup per right-hand side
                                   (FP64, block-Jacobi smoother, upwind flux, restart <= 32);
                                   0: always the multi-launch solve */
} hdg_options;

typedef struct {
    int32_t iters;              /* Krylov iterations (inner iterations in mixed mode) */
    int32_t refinements;        /* outer FP64 refinement steps (mixed mode) */
    int32_t fallbacks;          /* learned-smoother fallbacks */
    int32_t status;             /* HDG_OK or HDG_ENOTCONV or HDG_EBREAKDOWN */
    double  rel_res;            /* final true relative residual ||rhat - S lam|| / ||rhat|| */
} hdg_solve_info;

typedef struct {
    int32_t n_cell, n_facet, n_vert, degree, n_loc, n_levels;
    int32_t facet_dofs;         /* trace unknowns per facet: p+1 (upwind) or 2(p+1) (LF) */
    int32_t flux;               /* HDG_FLUX_UPWIND or HDG_FLUX_LF */
    int64_t device_bytes;       /* device memory held by the context */
    double  kappa;              /* c dt */
    double  lambda_max;         /* eigenvalue estimate of D^-1 S (Chebyshev smoother), else 0 */
    int32_t persistent;         /* 1 when the context qualifies for the single-launch solve: upwind
                                   flux, at most 8 P1 levels and the LDS footprint of one workgroup
                                   (10 trace vectors, 3 vectors per P1 level and 12.6 KiB of Krylov
                                   scalars) within the device's LDS per workgroup less 2 KiB
                                   (160 KiB on gfx950): up to about 1800 trace unknowns, e.g. the
                                   8x8 torus at p = 1..3 and the 16x16 torus at p = 1 */
} hdg_sizes;

/* ------------------------------------------------------------------ entry points */

/* Fill *opt with the defaults listed above. */
int hdg_default_options(hdg_options *opt);

/* hdg_setup: build a context on the current HIP device.
 *   levels[0..n_levels-1]: multigrid hierarchy (P1, or RT0 for the LF flux), coarse to
 *     fine; levels[n_levels-1] is the HDG mesh itself (n_levels >= 1).  Each level must
 *     be the uniform refinement of the previous one.  LF flux: the RT0 hierarchy uses
 *     the finest level and every coarser level whose cells are determined by their
 *     three vertex ids (at least 16 vertices); the coarsest of them (at most 8192
 *     facets) is solved with a dense inverse.
 *   parents[l] for l = 1..n_levels-1: (host) [levels[l].n_vert][2] vertex ids in
 *     level l-1 between which vertex v of level l lies (equal ids for an
 *     inherited vertex); parents[0] is ignored (may be NULL).
 * Work (all on the device except topology and the tiny P1 level assembly):
 * topology (cell->facet maps, orientations), local assembly of A, B, C, M per
 * cell, per-cell LU-based condensation (S_K = M_K + C_K A_K^-1 B_K, A_K^-1 B_K,
 * A_K^-1 and C_K A_K^-1 with the mass weighting folded in), assembly of the
 * facet block rows of S, facet-block inverses, P1 level operators
 * (1/kappa)(M + kappa^2 K) and transfers, dense inverse on the coarsest level.
 * Synchronous.  On success *out owns all of it; free with hdg_destroy. */
int hdg_setup(const hdg_mesh *levels, int32_t n_levels, const int32_t *const *parents,
              const hdg_params *prm, const hdg_options *opt, hdg_ctx **out);

int hdg_get_sizes(const hdg_ctx *ctx, hdg_sizes *out);

/* Topology as built by the library (host output arrays, synchronous):
 * facet_cell [n_facet][2] (owner, other), facet_loc [n_facet][2],
 * facet_vert [n_facet][2] (start, end vertex). Any pointer may be NULL. */
int hdg_get_topology(const hdg_ctx *ctx, int32_t *facet_cell, int32_t *facet_loc, int32_t *facet_vert);

/* Step 1 (Eq. schur_system right-hand side): rhat = sum_K R_K^T C_K A_K^-1 (r, v)_K.
 * r_cell: (device) [n_cell][3][n_loc][nrhs] DG coefficients of (r_h, r_u);
 * rhat:   (device) [n_facet][facet_dofs][nrhs].  1 <= nrhs <= max_rhs. */
int hdg_condense(hdg_ctx *ctx, int32_t nrhs, const double *r_cell, double *rhat, void *stream);

/* hdg_condense without allocation, for callers that cannot allocate device
 * memory during the call (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and results (bit for bit)
 * as hdg_condense, with the per-cell staging in a fixed scratch array that
 * every GPU the library runs on holds for the life of the process (32 MiB;
 * resolved by hdg_setup) instead of the context's buffer.  Needs
 * 3 facet_dofs * n_cell * nrhs <= 4194304 doubles, else HDG_EINVAL (use
 * hdg_condense).  Calls no allocating routine.  The array is shared by every
 * call on that GPU and keeps the last call's contents (nothing in it needs to
 * start at zero): calls that overlap on one GPU -- from two streams, threads
 * or contexts -- race on it and must be serialised by the caller. */
int hdg_condense_noalloc(hdg_ctx *ctx, int32_t nrhs, const double *r_cell, double *rhat, void *stream);

/* y = S x, matrix-free over facet block rows (Eq. schur_system operator).
 * precision HDG_FP64 uses the FP64 rows, HDG_MIXED the FP32 rows with FP32 accumulation.
 * x, y: (device) [n_facet][facet_dofs][nrhs], must not alias. */
int hdg_trace_apply(hdg_ctx *ctx, int32_t nrhs, int32_t precision, const double *x, double *y, void *stream);

/* z = V(r): one non-nested V-cycle (Alg. twolevel_vcycle) from a zero initial guess:
 * nu_pre block-Jacobi sweeps, residual, restriction pi^T, one P1 GMG V-cycle on
 * S_c = (1/kappa)(M_1 + kappa^2 K_1) (Eq. coarse_problem_upwind), prolongation pi,
 * nu_post sweeps.  precision selects the storage of the trace-level matrices.
 * LF flux: the coarse problem is S_c = (1/kappa)(M_RT + kappa^2 D_RT) on RT0
 * (Eq. coarse_problem_LF), pi^T / pi the transpose / the nodal average of the two
 * cells' RT0 fields on each facet, solved by one RT0 GMG V-cycle: rt_nu additive
 * vertex-patch steps (damping rt_omega) before and after the correction from the
 * next coarser level (exact flux transfer between the nested levels), dense
 * inverse on the coarsest level.
 * r, z: (device) [n_facet][facet_dofs][nrhs], must not alias. */
int hdg_mg_vcycle(hdg_ctx *ctx, int32_t nrhs, int32_t precision, const double *r, double *z, void *stream);

/* Step 2: solve S lam = rhat to ||rhat - S lam|| <= rtol ||rhat|| per RHS.
 * lam is the initial guess on entry (device, [n_facet][facet_dofs][nrhs]) and the
 * solution on exit.  info: (host) [nrhs], may be NULL.  Returns when lam and info
 * are complete (as hdg_stage_solve). */
int hdg_solve(hdg_ctx *ctx, int32_t nrhs, const double *rhat, double *lam,
              hdg_solve_info *info, void *stream);

/* Step 3 (Eq. reconstruct_solution): q = A^-1 ((r, v)_K - B lam), returned as
 * (h, u1, u2) coefficients in q_cell (device, [n_cell][3][n_loc][nrhs]). */
int hdg_recover(hdg_ctx *ctx, int32_t nrhs, const double *r_cell, const double *lam,
                double *q_cell, void *stream);

/* Steps 1-3 of one implicit stage (Eqs. schur_system, reconstruct_solution):
 * condense r_cell, solve S lam = rhat from a zero initial guess to rtol, recover
 * q_cell.  When the context qualifies (hdg_sizes.persistent, opt.persistent,
 * FP64, block-Jacobi) the three steps run in ONE launch, one workgroup per
 * right-hand side holding every trace and P1 vector of its solve in LDS;
 * otherwise as hdg_condense, hdg_solve and hdg_recover.  r_cell, q_cell:
 * (device) [n_cell][3][n_loc][nrhs]; lam: (device, output)
 * [n_facet][facet_dofs][nrhs]; info: (host) [nrhs], may be NULL.  Returns as
 * hdg_solve (HDG_ENOTCONV / HDG_EBREAKDOWN with lam and q_cell still written).
 * Returns when lam, q_cell and info are complete: the stream is synchronised,
 * or, on the single-launch path, every workgroup has published its record
 * (written after its outputs, behind a system-scope fence). */
int hdg_stage_solve(hdg_ctx *ctx, int32_t nrhs, const double *r_cell, double *lam, double *q_cell,
                    hdg_solve_info *info, void *stream);

void hdg_destroy(hdg_ctx *ctx);
const char *hdg_last_error(void);

/* ------------------------------------------------------------------ IMEX time stepping
 *
 * Time discretisation section (Eqs. IMEX_HDG_I, IMEX_HDG_II, theta_method):
 * the semi-discrete linear SWE  d/dt M(q) = N_0(q) + L(q)  advanced by an
 * additive (IMEX) Runge-Kutta method, the flux terms L implicitly through
 * this context's HDG solve and the Coriolis source N_0(q) = -f k x u
 * explicitly (the paper's splitting; f is a constant, an f-plane).  Stage i
 * solves
 *     M Q_i - at_ii dt L(Q_i) = M q_n + dt sum_{j<i} (a_ij N_0(Q_j) + at_ij L(Q_j))
 * by condense / solve / recover (zero initial trace), and the step ends with
 *     M q_{n+1} = M q_n + dt sum_i (b_i N_0(Q_i) + bt_i L(Q_i)).
 * Everything runs on DG coefficients: M^-1 N_0 rotates the velocity
 * coefficients, and dt M^-1 L(Q_j) of an implicit stage is (Q_j - R_j) / at_jj,
 * R_j the stage's right-hand side in coefficients -- exact for the computed
 * Q_j and its trace, whatever the solver residual.  A first stage that is
 * explicit (Q_1 = q_n) and whose flux term is used (Theta) needs
 * dt M^-1 L(q_n): evaluated once per call (hdg_dg_tendency) and carried to the
 * next step from the last stage when the tableau is stiffly accurate.
 *
 * The context must be set up for this splitting: prm.dt = gamma dt, gamma the
 * common value of the nonzero entries on the diagonal of at, and
 * prm.f0 = prm.omega = 0 (HDG_EINVAL otherwise).  Any flux, mesh and
 * precision; the stage solves use the context's options (rtol, smoother). */
#define HDG_IMEX_THETA  0   /* Theta(theta): a = [[0,0],[1,0]], at = [[0,0],[1-theta,theta]],
                               b = [1,0], bt = [1-theta,theta] */
#define HDG_IMEX_ARS232 1   /* ARS2(2,3,2): gamma = 1 - 1/sqrt 2, delta = -2 sqrt(2)/3 */
#define HDG_IMEX_SSP322 2   /* SSP2(3,2,2) */
#define HDG_IMEX_ARS443 3   /* ARS3(4,4,3) */
#define HDG_IMEX_MAX_STAGES 5
typedef struct {
    int32_t stages;             /* s, 1..HDG_IMEX_MAX_STAGES */
    double a[5][5];             /* explicit part, strictly lower triangular */
    double at[5][5];            /* implicit part, lower triangular */
    double b[5], bt[5];         /* weights */
} hdg_imex_tableau;
typedef struct {
    int32_t steps, solves;      /* completed steps, implicit stage solves */
    int32_t iters_total;        /* Krylov iterations summed over solves (max over right-hand sides) */
    int32_t iters_max;          /* most iterations of one solve */
    int32_t status;             /* HDG_OK, or HDG_ENOTCONV when a solve stopped at maxit */
    double rel_res_max;         /* largest final relative trace residual */
} hdg_imex_info;

/* The tableaux of the IMEX methods section (theta used by HDG_IMEX_THETA only). */
int hdg_imex_tableau_get(int32_t method, double theta, hdg_imex_tableau *out);

/* Device workspace of hdg_imex_run, in doubles: two cell arrays per stage, one
 * more for the carried flux term and two trace arrays. */
int hdg_imex_work_size(const hdg_ctx *ctx, const hdg_imex_tableau *tab, int32_t nrhs, int64_t *doubles);

/* `steps` IMEX steps of size dt from q (device, [n_cell][3][n_loc][nrhs], (h, u1, u2)
 * coefficients), in place.  f: the explicit Coriolis parameter.  work: device, at
 * least hdg_imex_work_size doubles, 16-byte aligned.  info (host) may be NULL.
 * Returns HDG_ENOTCONV (steps still completed) when a stage solve stopped at maxit.
 * Synchronises the stream (every stage solve does). */
int hdg_imex_run(hdg_ctx *ctx, const hdg_imex_tableau *tab, double dt, double f, int32_t nrhs, int32_t steps,
                 double *q, double *work, hdg_imex_info *info, void *stream);

/* Explicit flux evaluation  out = dt M^-1 (L(q) + N_c(q)),  N_c the context's own
 * (implicit) Coriolis term: with lam(q) the DG trace of q -- {{phi}} + [[u]]/(2 tau)
 * for the upwind flux, {{u}} + [[phi]]/(2 tau) for Lax-Friedrichs, the values for
 * which the hybridised and the standard DG forms coincide -- the context's stage
 * equations with trace lam(q) hold for q and a right-hand side r; then
 * out = (dt / prm.dt) (q - r) (Eq. linear_hybridized; L as in Eq. L_definitions).
 * q, out: device, [n_cell][3][n_loc][nrhs], must not alias. */
int hdg_dg_tendency(hdg_ctx *ctx, int32_t nrhs, double dt, const double *q, double *out, void *stream);

/* ------------------------------------------------------------------ non-hybridised DG baseline
 *
 * Native DG section (Eqs. native_dg_system, native_matrix_representation,
 * S_approx_diag): the same implicit stage solved without hybridisation, as the
 * comparison the paper makes.  GMRES (restarted, flexible, true-residual
 * restarts) on the standard upwind DG system  A q = R  (A: the stage matrix
 * split by fields into [[A_pp, A_pu], [A_up, A_uu]], R the mass-weighted
 * right-hand side), preconditioned by three steps:
 *     V = A_uu~^-1 R_u;   Phi = S~^-1 (R_p - A_pu V);   U = A_uu~^-1 (R_u - A_up Phi),
 *     S = A_pp - A_pu diag(A_uu)^-1 A_up.
 * A_uu~^-1: the exact inverse of each cell's diagonal block of A_uu (in place of
 * the paper's ILU).  S~^-1: one two-level cycle (in place of one GAMG V-cycle):
 * Chebyshev smoothing of degree nu_pre / nu_post preconditioned by the inverse
 * of each cell's own block of S on [0.1, 1.1] lambda_max (20 power steps at
 * setup), and the coarse correction on conforming P1 with the Galerkin operator
 * P^T S P (P: nodal interpolation of P1 into the DG phi space) solved by one P1
 * multigrid V-cycle with Galerkin coarsening (p1_nu, p1_omega).  Upwind flux
 * only; uses the context's rtol, maxit and restart.
 *
 * Vectors of hdg_dgs_apply / hdg_dgs_precondition are DG coefficient vectors in
 * the symmetric variables (phi = h sqrt(g/H), u), device, [n_cell][3][n_loc][nrhs];
 * A acts on them as the mass-weighted stage equations. */
/* Build the baseline's operators on this context (levels / parents as for
 * hdg_setup, the finest level the context's mesh).  Synchronous; idempotent. */
int hdg_dgs_setup(hdg_ctx *ctx, const hdg_mesh *levels, int32_t n_levels, const int32_t *const *parents);
/* y = A x (stage matrix of the standard DG form).  x, y must not alias. */
int hdg_dgs_apply(hdg_ctx *ctx, int32_t nrhs, const double *x, double *y, void *stream);
/* z = the three-step preconditioner applied to r.  r, z must not alias. */
int hdg_dgs_precondition(hdg_ctx *ctx, int32_t nrhs, const double *r, double *z, void *stream);
/* Solve the stage for the DG coefficients r_cell of (r_h, r_u) (as hdg_condense) and
 * return q_cell = (h, u1, u2) (as hdg_recover); stops when ||R - A q|| <= rtol ||R||
 * per right-hand side.  info (host) [nrhs] may be NULL.  Returns HDG_ENOTCONV at maxit.
 * Synchronises the stream. */
int hdg_dgs_solve(hdg_ctx *ctx, int32_t nrhs, const double *r_cell, double *q_cell, hdg_solve_info *info,
                  void *stream);

/* ------------------------------------------------------------------ learned smoother
 *
 * An extension beyond the paper (whose conclusion names better smoothers as
 * future work): a small network replaces the block-Jacobi sweep of the
 * V-cycle.  For facet e the patch is e and the four other facets of its two
 * cells (the facets of e's block row of S); the features are the
 * block-Jacobi corrections u = omega D^-1 r on the patch, each slot in the
 * counter-clockwise direction of the cell it is taken from (slot 0 in e's own
 * direction), 5(p+1) values, normalised by their RMS s.  Network: h =
 * ReLU(W1 z), 64 hidden units, y = W2 h, p+1 outputs, no biases; a smoothing
 * step is x <- x + u_e + s y_e.  Inference and training run in BF16 on the
 * matrix cores with FP32 accumulation; FP32 master weights, Adam
 * (beta 0.9, 0.999, eps 1e-8).  The weights start at zero, where the
 * learned step is the block-Jacobi step.  Selected by opt.smoother =
 * HDG_SMOOTH_MLP in hdg_setup (FGMRES only; hdg_solve reverts to block-Jacobi
 * for the rest of a solve, counting info.fallbacks, once the mean residual
 * reduction per iteration is weaker than fallback_ratio, see hdg_options).
 *
 * Weight layout (host, row-major FP32): W1 [64][5(p+1)], W2 [p+1][64]. */
int hdg_mlp_set_weights(hdg_ctx *ctx, const float *W1, const float *W2);   /* resets Adam; synchronous */
int hdg_mlp_get_weights(hdg_ctx *ctx, float *W1, float *W2);               /* either may be NULL; synchronous */

/* Training pair for the trace error e (device [n_facet][p+1][nrhs]):
 * u = omega D^-1 S e (the features' source) and the target
 * t = e - pi x_c - u, x_c = coarse_its stationary P1 multigrid V-cycles on
 * S_c x_c = pi^T S e from zero (what the coarse correction leaves of e,
 * minus the block-Jacobi step).  u, t: device, same layout; synchronous. */
int hdg_mlp_make_data(hdg_ctx *ctx, int32_t nrhs, const double *e, double *u, double *t,
                      int32_t coarse_its, void *stream);

/* Loss mean over (facet, rhs) of sum_o (y_o - t_o / s)^2 and its gradient
 * (host outputs, layouts as the weights; any may be NULL).  Synchronous. */
int hdg_mlp_loss_grad(hdg_ctx *ctx, int32_t nrhs, const double *u, const double *t, double *loss,
                      float *dW1, float *dW2, void *stream);

/* Train in place: starting from the error e0 (device), for each of `cycles`
 * errors (e0, then e <- e - V(S e) with the block-Jacobi V-cycle in FP64)
 * build the training pair and take `epochs` Adam steps with learning rate lr
 * on it.  loss_hist (host, may be NULL) receives the loss before every step,
 * cycles * epochs <= 4096 values.  Synchronous. */
int hdg_mlp_train(hdg_ctx *ctx, int32_t nrhs, const double *e0, int32_t cycles, int32_t coarse_its,
                  int32_t epochs, double lr, double *loss_hist, void *stream);

/* ------------------------------------------------------------------ launch tuning
 * Launch shapes that do not change results.  hdg_autotune times each
 * candidate on the context's own mesh at nrhs right-hand sides (HIP events,
 * a few launches each, on the stream) and keeps the fastest; hdg_set_tuning
 * imposes values.  Both drop the captured graphs.  Synchronous.  At nrhs >= 2
 * hdg_autotune allocates two cell arrays of nrhs columns for its timing and
 * frees them before it returns (HDG_EHIP if the allocation fails). */
typedef struct {
    int32_t mlp_samples_per_lane; /* samples (facet, rhs) each lane gathers in the learned
                                     smoothing kernel: 1 or 2 (default 1), or 4 = four consecutive
                                     right-hand sides of one facet with 16-byte loads (applies when
                                     nrhs is a multiple of 4, else 1 is used) */
    int32_t rhs_block;          /* facet-row kernels (apply, residual, sweep) at nrhs = 4, 8, ..., 64:
                                   1 = one thread per (facet, rhs); 4 = four right-hand sides per
                                   thread with the block's rows staged in LDS (default 4) */
    int32_t cell_cells;         /* cells per block of the batched condensation and recovery
                                   kernels (nrhs >= 2; a block is cells x nrhs threads): 0 = the
                                   most that fit in 256 threads and 64 KiB of staged rows (default),
                                   1..32 = at most that many (larger values are clamped) */
} hdg_tuning;
int hdg_get_tuning(const hdg_ctx *ctx, hdg_tuning *out);
int hdg_set_tuning(hdg_ctx *ctx, const hdg_tuning *tuning);
int hdg_autotune(hdg_ctx *ctx, int32_t nrhs, hdg_tuning *chosen, void *stream);

/* ------------------------------------------------------------------ measurement helpers */

/* Per-kernel-class timing with HIP events on the launch stream.
 * hdg_set_timing(ctx, R): R = 0 switches timing off; R >= 1 brackets every
 * launch of the instrumented kernel classes with a pair of events, issuing
 * the (idempotent) launch R times back to back in between and counting the
 * elapsed time divided by R (R > 1 spreads the cost of the event records).
 * While timing is on, Krylov iterations run eagerly (no graph replay).
 * hdg_kernel_stats returns, for kernel class id and precision, the launch
 * count and the summed per-launch duration (ms) since the last
 * hdg_set_timing call, and the algorithmic bytes one launch moves at the
 * nrhs and vector entry sizes of the timed launches (every stored matrix
 * entry once, every vector entry read or written once at its stored size --
 * 4 bytes for the FP32 vectors inside mixed solves -- indices once).  For
 * the sweep class it is the average over the timed launches of each
 * launch's own operands (an input that is the same vector as another counts
 * once; the prolongation and previous-iterate terms count when present).
 * Both calls synchronise. */
#define HDG_KERNEL_APPLY    0   /* y = S x  (facet block rows) */
#define HDG_KERNEL_SWEEP    1   /* block-Jacobi sweep with the off-diagonal rows */
#define HDG_KERNEL_RESIDUAL 2   /* r - S x */
#define HDG_KERNEL_CONDENSE 3
#define HDG_KERNEL_RECOVER  4
#define HDG_KERNEL_MLP      5   /* learned smoothing step after a sweep (patch gather + network) */
#define HDG_KERNEL_COUNT    6
int hdg_set_timing(hdg_ctx *ctx, int32_t enable);
int hdg_kernel_stats(hdg_ctx *ctx, int32_t kernel, int32_t precision, int64_t *launches,
                     double *total_ms, double *bytes_per_launch);

/* Plain device copy dst[i] = src[i], i < n doubles, on the stream: the reference
 * kernel whose HBM counters calibrate the profiler's byte counts. */
int hdg_copy(const double *src, double *dst, int64_t n, void *stream);

/* Bandwidth probes (measurement only, not part of a solve): the measured HBM
 * bandwidth that the roofline reports beside the datasheet peak.  Both are
 * asynchronous on the stream and take device arrays of doubles; a block
 * covers a chunk of 2048 doubles with 16-byte loads.
 *
 * hdg_stream_triad: a[i] = b[i] + s * c[i] for 0 <= i < n (STREAM's triad).
 *   a, b and c are 16-byte aligned; a overlaps neither b nor c (b may equal c).
 * hdg_stream_read: partial[k] = the sum of src[2048 k ... 2048 k + 2047]
 *   (clipped to n) for k < hdg_stream_read_blocks(n), which is ceil(n / 2048);
 *   src is 16-byte aligned and the caller-owned partial holds at least
 *   n_partial >= hdg_stream_read_blocks(n) doubles and does not overlap src.
 * n = 0 launches nothing and accepts NULL pointers.  Otherwise HDG_EINVAL for
 * NULL, misaligned or overlapping arrays, n < 0 or a short partial. */
int hdg_stream_triad(const double *b, const double *c, double s, double *a, int64_t n, void *stream);
int64_t hdg_stream_read_blocks(int64_t n);
int hdg_stream_read(const double *src, int64_t n, double *partial, int64_t n_partial, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* HDG_H */
