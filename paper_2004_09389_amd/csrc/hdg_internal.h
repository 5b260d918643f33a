// Internal declarations of the HDG trace-multigrid library (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>

#include <cstdint>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "../../include/hdg.h"
#include "hdg_host.h"

namespace hdg {

#define HDG_HIP_CHECK(expr)                                                          \
    do {                                                                             \
        hipError_t _e = (expr);                                                      \
        if (_e != hipSuccess)                                                        \
            throw ::hdg::Error{HDG_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e)}; \
    } while (0)

// The classical Gram-Schmidt step of a Krylov basis vector left to its first
// reader (one pass over the basis per iteration): the vector r becomes
// r - sum_{d < nd} h[d][rhs] V_d, V_d of r's element type, vstride elements apart.
struct GsLag {
    const void *V = nullptr;
    int64_t vstride = 0;
    int nd = 0;
    const double *h = nullptr;   // [nd][nb]
    const int *done = nullptr;   // (device) nonzero: the step was already made explicitly
};

// ------------------------------------------------------------------ context
struct P1LevelDev {
    int n = 0, w = 0;                              // vertices, ELL width (max off-diagonals per row)
    int32_t *col = nullptr;                        // ELL [w][n]
    double *val = nullptr, *diag = nullptr, *dinv = nullptr;
    int32_t *parents = nullptr;                    // [n][2] into the coarser level (level > 0)
    int32_t *crow = nullptr, *ccol = nullptr;      // children CSR of the coarser level (restriction)
    double *cw = nullptr;
    double *b = nullptr, *x = nullptr, *y = nullptr;  // [n][max_rhs] work vectors
};

constexpr int P1_TAIL_MAX = 4096;   // levels up to this many vertices run in the tail kernel
constexpr int P1_TAIL_DENSE_MAX = 256;   // the tail also takes the dense coarsest product: only this small
constexpr int P1_TAIL_LEVELS = 8;

struct P1Lev {
    int n, w;
    const int *col;
    const double *val, *diag, *dinv;
    const int *parents;                      // into level - 1
    const int *crow, *ccol;                  // children of the level - 1 vertices
    const double *cw;
    double *b, *x, *y;
};

struct P1Tail {
    int top, nu;
    double omega;
    const double *Ainv;                      // dense inverse of level 0
    P1Lev lev[P1_TAIL_LEVELS];
};

// RT0 level on the device (Lax-Friedrichs coarse space), arrays as in Rt0Host
struct Rt0LevelDev {
    int ne = 0, nv = 0;
    int32_t *nbr = nullptr;
    double *val = nullptr;
    int32_t *pf = nullptr, *fs = nullptr;
    double *pinv = nullptr;
    int32_t *pc = nullptr;          // transfer from the next coarser level (null on the coarsest)
    double *pw = nullptr;
    int32_t *crow = nullptr, *ccol = nullptr;
    double *cw = nullptr;
    double *b = nullptr, *x = nullptr, *y = nullptr;   // [ne][max_rhs]
};

// run fn, turning an Error (or allocation failure) into its code and hdg_last_error message
int guarded(const std::function<void()> &fn);
// throw HDG_EHIP when the last kernel launch failed
void check_kernel_launch();
// throw the code of a failed C-ABI call (negative return) with its message
void check_abi(int rc);

// upload P1 operators (coarse to fine) with transfers and the coarsest dense inverse (hdg_api.hip)
void build_p1_levels(hdg_ctx *c, const hdg_mesh *levels, const int32_t *const *parents,
                     const std::vector<P1Host> &ops, std::vector<P1LevelDev> &lev, double **coarse_inv);
// device allocation owned by the context (freed by hdg_destroy)
void *ctx_alloc(hdg_ctx *c, size_t bytes);
// each side's share of the DG trace of the cell field q at its facet nodes (hdg_imex.hip):
// half [n_facet][2][facet_dofs][nrhs]; phi = hscale * field 0
void launch_dg_half(const hdg_ctx *c, int nb, double hscale, const double *q, double *half, hipStream_t s);

}  // namespace hdg

struct hdg_ctx {
    int device = 0;
    int p = 0, m = 0, n = 0, nc = 0, nt = 0;   // m: trace unknowns per facet (nu (p + 1))
    int nu = 1, flux = HDG_FLUX_UPWIND;        // trace components per node
    int n_cell = 0, n_facet = 0, n_vert = 0, geom = 0;
    double kappa = 0, hscale = 0, tau = 0, dt = 0;
    hdg_params prm{};
    hdg_options opt{};
    bool symmetric = false;
    double cheb_lmax = 0.0;               // eigenvalue estimate of D^-1 S (Chebyshev smoother)
    hdg::Topology topo;
    int64_t device_bytes = 0;
    std::vector<void *> allocations;

    // per-cell matrices, component-major [row][col][n_cell]
    double *Zr = nullptr;      // [nt][nc, padded even]  C A^-1 Mtilde  (condense), 16-byte pairs
    double *Ar = nullptr;      // [nc][nc]  A^-1 Mtilde, phi rows / hscale  (recover)
    double *Wr = nullptr;      // [nc][nt]  A^-1 B, phi rows / hscale       (recover)
    int32_t *cell_facet = nullptr;  // [3][n_cell]
    int8_t *cell_rev = nullptr;     // [3][n_cell]
    double *corners = nullptr;      // [n_cell][3][3] unwrapped corner coordinates
    double *dg_half = nullptr;      // explicit flux evaluation: trace shares [n_facet][2][m][max_rhs]
    int *dg_err = nullptr;          // its singular-matrix flag
    double *ref = nullptr;          // reference-element tables of the cell assembly

    // non-hybridised DG baseline (hdg_dgs_setup): stage matrix as A q + B lam(q) per cell
    bool dgs_ready = false;
    double *dgs_A = nullptr;        // [nc][nc][n_cell]  A_K (symmetric variables)
    double *dgs_Bn = nullptr;       // [nc][nt][n_cell]  -B_K
    double *dgs_Auu_inv = nullptr;  // [2n][2n][n_cell] inverse of the cell's diagonal block of A_uu
    double *dgs_Sown_inv = nullptr; // [n][n][n_cell]   inverse of the cell's own block of S
    double *dgs_Dinv = nullptr;     // [n_cell][2n]      1 / diag(A_uu)
    double dgs_lmax = 0.0;          // eigenvalue estimate of S_own^-1 S
    std::vector<hdg::P1LevelDev> dgs_lev;   // Galerkin P1 hierarchy of S (level 0 coarsest)
    double *dgs_coarse_inv = nullptr;
    int32_t *dgs_cvert = nullptr;   // [n_cell][3] vertex ids
    int32_t *dgs_vrow = nullptr, *dgs_vcol = nullptr;  // vertex -> 3 * cell + corner CSR
    double *dgs_half = nullptr, *dgs_lam = nullptr;    // trace shares and trace of the apply
    std::vector<double *> dgs_tmp;  // cell work vectors [n_cell][3][n_loc][max_rhs]
    double *dgs_V = nullptr, *dgs_Z = nullptr;         // FGMRES bases
    double *dgs_red = nullptr, *dgs_out = nullptr;     // reduction partials and results
    double *dgs_coef = nullptr;                        // Krylov coefficients uploaded per step

    // facet block rows, component-major [slot][a][b][n_facet]
    int32_t *nbr = nullptr;     // [4][n_facet]
    int8_t *prev = nullptr;     // [4][n_facet] learned-smoother patch orientation flags
    double *S64 = nullptr;      // [5][m][m]  slot 0 = diagonal block
    double *T64 = nullptr;      // [4][m][m]  omega D^-1 S_j (off-diagonal slots)
    double *Dw64 = nullptr;     // [m][m]     omega D^-1
    float *S32 = nullptr;
    __hip_bfloat16 *T16 = nullptr;
    float *Dw32 = nullptr;
    int32_t *facet_vert = nullptr;  // [n_facet][2]
    int32_t *d_fcell = nullptr;     // [n_facet][2] owner, other cell
    int32_t *d_floc = nullptr;      // [n_facet][2] local facet index in each
    int32_t *vf_row = nullptr, *vf_col = nullptr;  // vertex -> (facet, end) CSR, col = 2 e + end

    // P1 hierarchy, level 0 coarsest
    std::vector<hdg::P1LevelDev> lev;
    double *coarse_inv = nullptr;   // dense inverse of the coarsest level
    int tail_top = -1;              // levels 0..tail_top run in the single-workgroup tail kernel
    hdg::P1Tail tail{};

    // Lax-Friedrichs coarse space: RT0 levels (level 0 coarsest), dense inverse of level 0,
    // prolongation weights onto the trace [5][m][n_facet] and the CSR of its transpose
    std::vector<hdg::Rt0LevelDev> rt;
    double *rt_coarse_inv = nullptr;
    double *rt_corr = nullptr;                  // vertex-patch corrections [n_vert][RT_PV][max_rhs]
    double *lf_pw = nullptr;
    int32_t *lf_rrow = nullptr, *lf_rcol = nullptr;

    // trace work vectors [n_facet][m][max_rhs]
    double *vz0 = nullptr, *vx = nullptr, *vx2 = nullptr, *vres = nullptr;
    double *vrc = nullptr;                      // the V-cycle's input in FP32 (mixed solves)
    // Krylov work
    double *kr = nullptr, *kz = nullptr, *kp = nullptr, *kw = nullptr, *klam = nullptr;
    double *kV = nullptr, *kZ = nullptr;      // FGMRES bases [(restart+1)][vec], [restart][vec]
    double *red = nullptr;                    // reduction partials
    double *scal = nullptr;                   // device scalars [slot][max_rhs]
    double *hscal = nullptr;                  // pinned host mirror
    double *hcol = nullptr;                   // FGMRES Hessenberg column [restart+1][max_rhs]
    int *gs_explicit = nullptr;               // (device) 1 when an iteration's Gram-Schmidt update ran explicitly
    double *gm = nullptr;                     // FGMRES per-RHS state (H, Givens, g)
    double *hy = nullptr;                     // FGMRES coefficients [restart][max_rhs]
    double *dbn = nullptr;                    // ||rhat|| per RHS (device)
    double *loc = nullptr;                    // condensation scratch [nt][n_cell][max_rhs]
    double *noalloc_scratch = nullptr;        // this device's static scratch (hdg_condense_noalloc)
    std::vector<double> hbn2;                 // ||rhat||^2 per RHS (host)
    double *hlag = nullptr;                   // host-mapped landing slots for reduction results [4][64]
    double *dlag = nullptr;                   // device view of hlag
    hipEvent_t lag_ev[2] = {nullptr, nullptr};
    int red_blocks = 0;

    // persistent single-launch solve of small systems (hdg_small.hip)
    bool small_ok = false;                // the context qualifies (upwind flux, LDS footprint)
    bool small_stage_ops = false;         // ... and its operators fit in LDS as well
    double *small_p1B = nullptr;          // the P1 V-cycle as a dense matrix, transposed (small hierarchies), or null
    char *small_image = nullptr;          // the operators packed in the layout of their LDS copies
    size_t small_lds = 0;                 // dynamic LDS per workgroup
    double *small_V = nullptr, *small_Z = nullptr;   // FGMRES bases per right-hand side
    double *small_info = nullptr;         // [max_rhs][4] record of each solve: device view of small_hinfo
    double *small_hinfo = nullptr;        // host-mapped memory the kernel writes
    double *stage_rhat = nullptr;         // condensed right-hand side of the multi-launch stage solve

    // learned smoother: weights [W1 (64 x K1P) | W2 (16 x 64)], FP32 master + Adam moments, BF16 copy
    int mlp_n1 = 0, mlp_n2 = 0, mlp_step = 0;
    int mlp_spl = 1;                      // samples per lane in the learned smoothing kernel
    int rhs_block = 4;                    // facet-row kernels: RHS per thread when nrhs allows (1 or 4)
    int cell_cells = 0;                   // batched cell kernels: cells per block (0 = the most that fit)
    float *mlp_w = nullptr, *mlp_m1 = nullptr, *mlp_m2 = nullptr, *mlp_g = nullptr;
    short *mlp_wb = nullptr;
    float *mlp_pdW1 = nullptr, *mlp_pdW2 = nullptr, *mlp_ploss = nullptr;
    double *mlp_loss = nullptr;           // device, one value per training step of an epoch
    double *mlp_E = nullptr, *mlp_R = nullptr;   // training: current error and S e (allocated on first use)
    double *mlp_U = nullptr, *mlp_T = nullptr;   // training: features source u and targets t
    double *p1_keep = nullptr, *p1_acc = nullptr;  // finest-P1 vectors for the training targets
    bool use_mlp_now = false;             // smoother of the current V-cycles (fallback clears it)
    // FP32 trace vectors (the same buffers, half used): vcyc32 for the V-cycle's work vectors
    // and its output z (the FGMRES Z basis), vin32 for the V-cycle's input r, kv32 for the
    // FGMRES V basis.  Mixed solves set vcyc32; the inner solve of HDG_MIXED_IR sets all three.
    bool vcyc32 = false, vin32 = false, kv32 = false;
    hdg::GsLag gs_lag;   // Gram-Schmidt step pending on the next V-cycle's input (FGMRES)

    // timing
    struct PendingEvent {
        hipEvent_t a, b;
        int kind, prec;
        double bytes;   // the launch's own algorithmic bytes (0: use the class formula)
    };
    bool timing = false;
    int timing_repeat = 1;
    std::vector<PendingEvent> pending;
    std::vector<hipEvent_t> event_pool;

    // captured Krylov iterations
    std::map<uint64_t, hipGraphExec_t> graphs;
    hipStream_t cap_stream = nullptr;
    int64_t t_launches[2][HDG_KERNEL_COUNT] = {};
    int t_nb[2][HDG_KERNEL_COUNT] = {};   // nrhs of the last timed launch per class
    int t_sx[2][HDG_KERNEL_COUNT] = {};   // bytes per input-vector entry of that launch (8 or 4)
    int t_sy[2][HDG_KERNEL_COUNT] = {};   // bytes per output-vector entry
    double t_ms[2][HDG_KERNEL_COUNT] = {};
    double t_bytes[2][HDG_KERNEL_COUNT] = {};     // sum of the launches' own algorithmic bytes
    int64_t t_blaunch[2][HDG_KERNEL_COUNT] = {};  // launches that stated their bytes
};
