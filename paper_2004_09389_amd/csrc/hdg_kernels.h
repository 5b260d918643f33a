// Launch wrappers of the device kernels (see hdg_kernels.hip).
#pragma once

#include <type_traits>

#include "hdg_internal.h"

namespace hdg {

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own L2.
// The trace and cell kernels remap the block index so that every XCD streams
// one contiguous range of facets (cells): the neighbour gathers of a facet row
// then hit the L2 that already holds them.  Launchers pad the grid to a
// multiple of 8 blocks; threads past the end return.
constexpr int N_XCD = 8;
__device__ __forceinline__ int xcd_block() {
    const int per = gridDim.x / N_XCD;
    return (blockIdx.x % N_XCD) * per + blockIdx.x / N_XCD;
}

// Trace vectors are [facet][node][rhs], stored as double (FP64 paths) or
// float (the FP32 inner solve of HDG_MIXED_IR); values are converted to and
// from double in registers.  With one right-hand side the M values of a facet
// are contiguous: load and store them as 16-byte (or 8-byte) groups when M
// allows.  base = facet * M * nb + rhs.
typedef double trace_dbl2_t __attribute__((ext_vector_type(2)));
typedef float trace_flt2_t __attribute__((ext_vector_type(2)));
typedef float trace_flt4_t __attribute__((ext_vector_type(4)));
template <int M, bool NB1, typename T, typename D>
__device__ __forceinline__ void load_trace(const T *__restrict__ v, size_t base, int nb, D (&d)[M]) {
    if constexpr (NB1 && std::is_same<T, double>::value && M % 2 == 0) {
#pragma unroll
        for (int j = 0; j < M; j += 2) {
            const trace_dbl2_t a = *reinterpret_cast<const trace_dbl2_t *>(v + base + j);
            d[j] = a.x;
            d[j + 1] = a.y;
        }
    } else if constexpr (NB1 && std::is_same<T, float>::value && M % 4 == 0) {
#pragma unroll
        for (int j = 0; j < M; j += 4) {
            const trace_flt4_t a = *reinterpret_cast<const trace_flt4_t *>(v + base + j);
            d[j] = a.x;
            d[j + 1] = a.y;
            d[j + 2] = a.z;
            d[j + 3] = a.w;
        }
    } else if constexpr (NB1 && std::is_same<T, float>::value && M % 2 == 0) {
#pragma unroll
        for (int j = 0; j < M; j += 2) {
            const trace_flt2_t a = *reinterpret_cast<const trace_flt2_t *>(v + base + j);
            d[j] = a.x;
            d[j + 1] = a.y;
        }
    } else {
#pragma unroll
        for (int j = 0; j < M; ++j) d[j] = (D)v[base + (size_t)(NB1 ? j : j * nb)];
    }
}
template <int M, bool NB1, typename T, typename D>
__device__ __forceinline__ void store_trace(T *__restrict__ v, size_t base, int nb, const D (&d)[M]) {
    if constexpr (NB1 && std::is_same<T, double>::value && M % 2 == 0) {
#pragma unroll
        for (int j = 0; j < M; j += 2)
            *reinterpret_cast<trace_dbl2_t *>(v + base + j) = trace_dbl2_t{d[j], d[j + 1]};
    } else if constexpr (NB1 && std::is_same<T, float>::value && M % 4 == 0) {
#pragma unroll
        for (int j = 0; j < M; j += 4)
            *reinterpret_cast<trace_flt4_t *>(v + base + j) =
                trace_flt4_t{(float)d[j], (float)d[j + 1], (float)d[j + 2], (float)d[j + 3]};
    } else if constexpr (NB1 && std::is_same<T, float>::value && M % 2 == 0) {
#pragma unroll
        for (int j = 0; j < M; j += 2)
            *reinterpret_cast<trace_flt2_t *>(v + base + j) = trace_flt2_t{(float)d[j], (float)d[j + 1]};
    } else {
#pragma unroll
        for (int j = 0; j < M; ++j) v[base + (size_t)(NB1 ? j : j * nb)] = (T)d[j];
    }
}

// Value at trace node k of the linear interpolant of q0 (start vertex) and
// q1 (end vertex): the injection pi of a P1 function.  The rounding is fixed
// here (one product, one fused multiply-add) so that every kernel applying
// pi produces identical bits.
template <int P>
__device__ __forceinline__ double p1_node(int k, double q0, double q1) {
    const double t = (double)k / P;
    return __builtin_fma(t, q1, (1.0 - t) * q0);
}
template <int P>
__device__ __forceinline__ float p1_node(int k, float q0, float q1) {
    const float t = (float)k / P;
    return __builtin_fmaf(t, q1, (1.0f - t) * q0);
}

// Coefficients of the generalised smoothing sweep
//   y = a0 x' + a1 z0 - a3 T x' + a2 xprev'
// with x' = x + pi qc (prolongation term optional), xprev' = xprev + pi qcprev
// (own facet only, optional), z0 = omega D^-1 r, T x the stored off-diagonal
// rows omega D^-1 S_j x_j.  Damped block-Jacobi: (1 - omega, 1, 1, 0);
// the correction alone: (-omega, 1, 1, 0); Chebyshev steps: see vcycle_cheb.
struct SweepCoef {
    double a0, a1, a3, a2;
    const void *xprev;        // trace vector of the sweep's vector type
    const void *qcprev;       // P1 vector, also of the sweep's vector type
};
// the sweep's output combination with its rounding fixed (every launch shape
// produces the same bits)
__device__ __forceinline__ double sweep_combine(const SweepCoef &cf, double x, double z, double acc) {
    return __builtin_fma(-cf.a3, acc, __builtin_fma(cf.a0, x, cf.a1 * z));
}
// Sweeps on FP32 vectors (the mixed V-cycle) evaluate the same formulas in FP32:
// the combination, the prolongation term and the previous-iterate term.
__device__ __forceinline__ float sweep_combine(const SweepCoef &cf, float x, float z, float acc) {
    return __builtin_fmaf(-(float)cf.a3, acc, __builtin_fmaf((float)cf.a0, x, (float)cf.a1 * z));
}
__device__ __forceinline__ double sweep_prev(double a2, double pv, double out) { return __builtin_fma(a2, pv, out); }
__device__ __forceinline__ float sweep_prev(double a2, float pv, float out) {
    return __builtin_fmaf((float)a2, pv, out);
}
// the arithmetic type of a sweep on vectors of type VT
template <typename VT>
using SweepT = typename std::conditional<std::is_same<VT, float>::value, float, double>::type;

// The condensation rows Zr (C A^-1 Mtilde, length nc per trace row) are stored
// in 16-byte pairs [entry / 2][n_cell][2], rows padded to an even length.
// (The recovery matrices stay one entry per lane: measured faster there.)
constexpr int cell_zw(int p) { return ((3 * (p + 1) * (p + 2) / 2) + 1) / 2 * 2; }

// padded component count of a facet-row matrix stored with v entries per 16 bytes
constexpr int wide_padded(int c, int v) { return (c + v - 1) / v * v; }

struct CellParams {
    double kappa, tau, dt, f0, omega, hscale;
    int geom;
};

// nu: trace components per node (1 upwind, 2 Lax-Friedrichs)
// With Aout non-null the kernel only assembles and stores A_K ([nc][nc][nk]) and -B_K
// ([nc][nt][nk], into Bnout), skipping the condensation.
void launch_cell_condense(int p, int nu, int nk, const double *corners, const double *ref, CellParams cp,
                          double *Sloc, double *Zr, double *Ar, double *Wr, int *err, hipStream_t s,
                          double *Aout = nullptr, double *Bnout = nullptr);
void launch_facet_rows(int p, int nu, int ne, int nk, const double *Sloc, const int *facet_cell,
                       const int *facet_loc, const int *cell_facet, const int8_t *cell_rev, double omega,
                       double *S64, double *T64, double *Dw64, float *S32, __hip_bfloat16 *T16, float *Dw32,
                       int *nbr, int8_t *prev, int *err, hipStream_t s);

// facet-row kernels: M = trace unknowns per facet (2, 3, 4, 6 or 8)
// VT: element type of the trace vectors (double, or float in the FP32 inner solve)
// y = S x or y = b - S x; x may be held in another type than b and y
template <typename MT, typename XT, typename YT>
void launch_trace_apply(int M, int ne, int nb, const MT *S, const int *nbr, const XT *x, const YT *b, YT *y,
                        hipStream_t s, int rhs_block = 1);
// z0 = omega D^-1 r (r / scale, written back to rs, when scale is given); rc (may be null)
// receives the scaled input in z0's type
template <typename MT, typename RT, typename ZT>
void launch_jacobi0(int M, int ne, int nb, const MT *Dw, const RT *r, const double *scale, RT *rs, ZT *rc, ZT *z0,
                    hipStream_t s, GsLag gs = GsLag{});
// qc (a P1 vector, may be null) holds values of the sweep's vector type VT in its buffer
template <typename MT, typename VT>
void launch_sweep(int M, int ne, int nb, const MT *T, const int *nbr, const VT *x, const VT *z0, const double *qc,
                  const int *fvert, SweepCoef cf, VT *y, hipStream_t s, int rhs_block = 1);
// FP64 residual y = b - S x with the FP64 operator, stored as FP32
void launch_trace_residual_f32(int M, int ne, int nb, const double *S, const int *nbr, const double *x,
                               const double *b, float *y, hipStream_t s, int rhs_block = 1);
// pi^T res onto the P1 vertices; rc receives values of the residual's type VT
template <typename VT>
void launch_restrict_trace(int p, int nv, int nb, const int *vf_row, const int *vf_col, const VT *res, double *rc,
                           hipStream_t s);

// P1 level kernels; f32: the level vectors (b, x, y, xc, r, bc) hold float values
// in their double buffers (the V-cycle of a mixed-precision solve)
// P1 level launchers: rb == 4 with nb % 4 == 0 takes four right-hand sides per
// thread (the same bits as rb == 1).
void launch_p1_first(int n, int nb, const double *dinv, double omega, const double *b, double *x, hipStream_t s,
                     bool f32 = false, int rb = 1);
void launch_p1_pre2(int n, int W, int nb, const int *col, const double *val, const double *diag,
                    const double *dinv, double omega, const double *b, double *x, hipStream_t s, bool f32 = false,
                    int rb = 1);
// y = x + w D^-1 (b - A x); with xc != nullptr, x is first updated in place to x + P xc (with one
// right-hand side the prolonged values are formed inside the sweep instead and x is left as it is)
void launch_p1_sweep(int n, int W, int nb, const int *col, const double *val, const double *diag,
                     const double *dinv, double omega, const double *b, double *x, const double *xc,
                     const int *parents, double *y, hipStream_t s, bool f32 = false, int rb = 1);
void launch_p1_resid(int n, int W, int nb, const int *col, const double *val, const double *diag,
                     const double *b, const double *x, double *y, hipStream_t s, bool f32 = false,
                     int rb = 1);
void launch_p1_restrict(int nc, int nb, const int *crow, const int *ccol, const double *cw, const double *r,
                        double *bc, hipStream_t s, bool f32 = false, int rb = 1);
// one right-hand side: bc = R (b - A x) from the fine level to the coarse one in one launch
void launch_p1_resid_restrict(int n, int W, const int *col, const double *val, const double *diag, const double *b,
                              const double *x, int nc, const int *crow, const int *ccol, const double *cw, double *bc,
                              hipStream_t s, bool f32 = false);
void launch_dense_mv(int n, int nb, const double *Ainv, const double *b, double *x, hipStream_t s, bool f32 = false);
void launch_p1_tail(const P1Tail &T, int nb, hipStream_t s, bool f32 = false);

// cells: cells per block of the batched (nb >= 2) cell kernels; 0 = the most
// that fit (256 threads, 64 KiB of staged rows), larger requests are clamped
void launch_condense(int p, int nu, int nk, int ne, int nb, const double *Zr, const double *rc, double *loc,
                     const int *facet_cell, const int *facet_loc, double *rhat, hipStream_t s, int cells = 0);
void launch_recover(int p, int nu, int nk, int nb, const double *Ar, const double *Wr, const int *cell_facet,
                    const int8_t *cell_rev, const double *rc, const double *lam, double *q, hipStream_t s,
                    int cells = 0);

int red_grid(int64_t len, int nb);
template <typename VT>
void launch_dots(int64_t len, int nb, int nd, const VT *X, int64_t xstride, const VT *y, double *partial,
                 double *out, double *host, hipStream_t s);
// ||w - sum_d h_d V_d|| of an orthonormal basis from the dot products alone
// (hcol[j + 1] holds ||w||^2: the norm is sqrt(||w||^2 - sum_{d <= j} h_d^2)), then
// the Givens step of FGMRES column j
// Used only when the remaining norm keeps at least `floor` of ||w||^2 for every
// right-hand side: then *expl = 0 and the update is left to the next V-cycle's first
// kernel (GsLag); otherwise *expl = 1 and launch_gs_norm_givens with run = expl does it.
void launch_pyth_givens(int nb, int j, int restart, double floor, const double *hcol, double *hn, double *gm,
                        const double *bnorm, double *resid_host, int *expl, hipStream_t s);
template <typename VT>
void launch_gs_norm_givens(int64_t len, int nb, int nd, const double *h, const VT *V, int64_t vstride, VT *w,
                           double *partial, double *hn, int j, int restart, double *gm, const double *bnorm,
                           double *resid_host, hipStream_t s, const int *run = nullptr);
void launch_pcg_update_norm(int64_t len, int nb, const double *num, const double *den, const double *p,
                            const double *w, double *x, double *res, double *partial, double *rr_host,
                            hipStream_t s);
void launch_pcg_dir(int64_t n, int nb, const double *num, const double *den, const double *z, double *p,
                    hipStream_t s);
template <typename VT>
void launch_lincomb(int64_t n, int nb, int nd, const double *y, const VT *Z, int64_t zstride, double *x,
                    hipStream_t s);
void launch_copy(int64_t n, const double *src, double *dst, hipStream_t s);
void launch_gmres_start(int nb, int restart, const double *beta2, double *gm, double *beta, hipStream_t s);
void launch_gmres_solve(int nb, int k, int restart, const double *gm, double *y, hipStream_t s);
void launch_sqrt(int nb, const double *in, double *out, hipStream_t s);

// persistent single-workgroup solve of small trace systems (hdg_small.hip)
constexpr int SMALL_THREADS = 256;    // threads per workgroup (one workgroup per right-hand side)
constexpr int SMALL_MAXR = 32;        // largest FGMRES restart length of the persistent solve
constexpr int SMALL_P1_DENSE = 64;    // finest P1 levels up to this size apply the V-cycle as its matrix
// The operators the persistent solve copies into LDS, packed once at setup into
// one device image in the order and 16-byte alignment of their LDS copies, so
// that the copy at the start of a launch is one loop with many loads in flight.
// small_image_walk calls f(part, level, byte offset, bytes) for each operator in
// image order (the levels only without the dense V-cycle matrix B, B only with
// it) and returns the image size; the host packs with it and the kernel
// publishes the LDS addresses with it (no per-level tables in private memory).
enum SmallPart { SP_S, SP_T, SP_DW, SP_NBR, SP_FVERT, SP_VF_ROW, SP_VF_COL, SP_B, SP_COL, SP_VAL, SP_DIAG, SP_DINV,
                 SP_PARENTS, SP_CROW, SP_CCOL, SP_CW, SP_AINV };
template <typename F>
__host__ __device__ inline size_t small_image_walk(int ne, int m, const P1Lev *lev, int nlev, int nB, F &&f) {
    size_t o = 0;
    auto put = [&](SmallPart part, int l, size_t bytes) {
        f(part, l, o, bytes);
        o += (bytes + 15) / 16 * 16;
    };
    const auto pad2 = [](int c) { return (size_t)((c + 1) / 2 * 2); };
    const size_t NE = (size_t)ne;
    put(SP_S, 0, 8 * pad2(5 * m * m) * NE);
    put(SP_T, 0, 8 * pad2(4 * m * m) * NE);
    put(SP_DW, 0, 8 * pad2(m * m) * NE);
    put(SP_NBR, 0, 16 * NE);
    put(SP_FVERT, 0, 8 * NE);
    put(SP_VF_ROW, 0, 4 * ((size_t)lev[nlev - 1].n + 1));
    put(SP_VF_COL, 0, 8 * NE);
    if (nB) {
        put(SP_B, 0, 8 * (size_t)nB * nB);
    } else {
        for (int l = 0; l < nlev; ++l) {
            const size_t n = lev[l].n, w = lev[l].w;
            put(SP_COL, l, 4 * w * n);
            put(SP_VAL, l, 8 * w * n);
            put(SP_DIAG, l, 8 * n);
            put(SP_DINV, l, 8 * n);
            if (l > 0) {
                put(SP_PARENTS, l, 8 * n);
                put(SP_CROW, l, 4 * ((size_t)lev[l - 1].n + 1));
                put(SP_CCOL, l, 8 * n);
                put(SP_CW, l, 16 * n);
            }
        }
        put(SP_AINV, 0, 8 * (size_t)lev[0].n * lev[0].n);
    }
    return o;
}
__host__ __device__ inline size_t small_image_bytes(int ne, int m, const P1Lev *lev, int nlev, int nB) {
    return small_image_walk(ne, m, lev, nlev, nB, [](SmallPart, int, size_t, size_t) {});
}

struct SmallArgs {
    int ne, m, nk, nb, nlev;
    int stage_ops;                      // copy the operators below into LDS at the start
    const char *image;                  // with stage_ops: the packed operators (small_image_walk order)
    int krylov, restart, maxit, nu_pre, nu_post, p1_nu;
    double omega, p1_omega, rtol;
    const double *S, *T, *Dw;           // FP64 facet rows (16-byte groups)
    const int *nbr, *fvert, *vf_row, *vf_col;
    P1Lev lev[P1_TAIL_LEVELS];          // P1 levels, 0 coarsest (work vectors unused: LDS)
    const double *Ainv;                 // dense inverse of level 0
    const double *p1B;                  // the whole P1 V-cycle as a matrix, transposed [j][i] (finest level), or null
    // Steps 1 and 3 inside the launch (stage solve)
    const double *Zr, *Ar, *Wr;
    const int *fcell, *floc, *cell_facet;
    const int8_t *cell_rev;
    const double *r_cell;               // [n_cell][3][n_loc][nb]
    double *q_cell;
    // the trace system
    const double *rhat;                 // [n_facet][m][nb] (solve only)
    double *lam;                        // [n_facet][m][nb]: initial guess (solve) and solution
    double *V, *Z;                      // FGMRES bases [nb][SMALL_MAXR + 1][n_facet m], [nb][SMALL_MAXR][...]
    double *info;                       // [nb][4]: iterations, restarts, status, final relative residual
};
// dynamic LDS of one workgroup for a mesh with ne facets, m unknowns per facet and the P1 levels
// (sizes and ELL widths), with or without the staged copies of the operators
size_t small_lds_bytes(int ne, int m, const P1Lev *lev, int nlev, bool stage_ops, int nB);
void launch_solve_small(int p, bool stage, const SmallArgs &A, size_t lds, hipStream_t s);
// opt the kernels of degree p into lds bytes of dynamic LDS
hipError_t small_prepare(int p, size_t lds);

// learned smoother (hdg_mlp.hip)
int mlp_k1p(int p);
int mlp_grad_waves(int ne, int nb);
template <typename VT>
void launch_mlp_smooth(int p, int ne, int nb, int spl, const VT *u, const VT *xi, const double *qc,
                       const int *fvert, const int *nbr, const int8_t *prev, const short *W1b, const short *W2b,
                       VT *xo, hipStream_t s);
void launch_mlp_grad(int p, int ne, int nb, const double *u, const double *t, const int *nbr, const int8_t *prev,
                     const short *W1b, const short *W2b, float *pdW1, float *pdW2, float *ploss, float *g,
                     double *loss, hipStream_t s);
void launch_adam(int p, const float *g, float gscale, float *w, float *m1, float *m2, float lr, int step,
                 short *wb, hipStream_t s);
void launch_to_bf16(int n, const float *w, short *wb, hipStream_t s);
void launch_prolong_trace(int p, int ne, int nb, const int *fvert, const double *qc, double *x, hipStream_t s);
template <typename VT>
void launch_lin3(int64_t n, double a, const VT *x, double b, const VT *y, double c, const VT *z, VT *out,
                 hipStream_t s);

}  // namespace hdg
