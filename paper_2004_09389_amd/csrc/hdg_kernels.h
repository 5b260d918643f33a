// Launch wrappers of the device kernels (see hdg_kernels.hip).
#pragma once

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

// Trace vectors are [facet][node][rhs].  With one right-hand side the M
// values of a facet are contiguous and (M even) 16-byte aligned: load and
// store them as pairs.  base = facet * M * nb + rhs.
typedef double trace_dbl2_t __attribute__((ext_vector_type(2)));
template <int M, bool NB1>
__device__ __forceinline__ void load_trace(const double *__restrict__ v, size_t base, int nb, double (&d)[M]) {
    if constexpr (NB1 && M % 2 == 0) {
#pragma unroll
        for (int j = 0; j < M; j += 2) {
            const trace_dbl2_t a = *reinterpret_cast<const trace_dbl2_t *>(v + base + j);
            d[j] = a.x;
            d[j + 1] = a.y;
        }
    } else {
#pragma unroll
        for (int j = 0; j < M; ++j) d[j] = v[base + (size_t)(NB1 ? j : j * nb)];
    }
}
template <int M, bool NB1>
__device__ __forceinline__ void store_trace(double *__restrict__ v, size_t base, int nb, const double (&d)[M]) {
    if constexpr (NB1 && M % 2 == 0) {
#pragma unroll
        for (int j = 0; j < M; j += 2)
            *reinterpret_cast<trace_dbl2_t *>(v + base + j) = trace_dbl2_t{d[j], d[j + 1]};
    } else {
#pragma unroll
        for (int j = 0; j < M; ++j) v[base + (size_t)(NB1 ? j : j * nb)] = d[j];
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

// Coefficients of the generalised smoothing sweep
//   y = a0 x' + a1 z0 - a3 T x' + a2 xprev'
// with x' = x + pi qc (prolongation term optional), xprev' = xprev + pi qcprev
// (own facet only, optional), z0 = omega D^-1 r, T x the stored off-diagonal
// rows omega D^-1 S_j x_j.  Damped block-Jacobi: (1 - omega, 1, 1, 0);
// the correction alone: (-omega, 1, 1, 0); Chebyshev steps: see vcycle_cheb.
struct SweepCoef {
    double a0, a1, a3, a2;
    const double *xprev, *qcprev;
};
// the sweep's output combination with its rounding fixed (every launch shape
// produces the same bits)
__device__ __forceinline__ double sweep_combine(const SweepCoef &cf, double x, double z, double acc) {
    return __builtin_fma(-cf.a3, acc, __builtin_fma(cf.a0, x, cf.a1 * z));
}

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
void launch_cell_condense(int p, int nu, int nk, const double *corners, const double *ref, CellParams cp,
                          double *Sloc, double *Zr, double *Ar, double *Wr, int *err, hipStream_t s);
void launch_facet_rows(int p, int nu, int ne, int nk, const double *Sloc, const int *facet_cell,
                       const int *facet_loc, const int *cell_facet, const int8_t *cell_rev, double omega,
                       double *S64, double *T64, double *Dw64, float *S32, __hip_bfloat16 *T16, float *Dw32,
                       int *nbr, int8_t *prev, int *err, hipStream_t s);

// facet-row kernels: M = trace unknowns per facet (2, 3, 4, 6 or 8)
template <typename MT>
void launch_trace_apply(int M, int ne, int nb, const MT *S, const int *nbr, const double *x, const double *b,
                        double *y, hipStream_t s, int rhs_block = 1);
template <typename MT>
void launch_jacobi0(int M, int ne, int nb, const MT *Dw, const double *r, const double *scale, double *rs,
                    double *z0, hipStream_t s);
template <typename MT>
void launch_sweep(int M, int ne, int nb, const MT *T, const int *nbr, const double *x, const double *z0,
                  const double *qc, const int *fvert, SweepCoef cf, double *y, hipStream_t s, int rhs_block = 1);
void launch_restrict_trace(int p, int nv, int nb, const int *vf_row, const int *vf_col, const double *res,
                           double *rc, hipStream_t s);

void launch_p1_first(int n, int nb, const double *dinv, double omega, const double *b, double *x, hipStream_t s);
void launch_p1_pre2(int n, int W, int nb, const int *col, const double *val, const double *diag,
                    const double *dinv, double omega, const double *b, double *x, hipStream_t s);
void launch_p1_sweep(int n, int W, int nb, const int *col, const double *val, const double *diag,
                     const double *dinv, double omega, const double *b, const double *x, const double *xc,
                     const int *parents, double *y, hipStream_t s);
void launch_p1_resid(int n, int W, int nb, const int *col, const double *val, const double *diag,
                     const double *b, const double *x, double *y, hipStream_t s);
void launch_p1_restrict(int nc, int nb, const int *crow, const int *ccol, const double *cw, const double *r,
                        double *bc, hipStream_t s);
void launch_dense_mv(int n, int nb, const double *Ainv, const double *b, double *x, hipStream_t s);
void launch_p1_tail(const P1Tail &T, int nb, hipStream_t s);

void launch_condense(int p, int nu, int nk, int ne, int nb, const double *Zr, const double *rc, double *loc,
                     const int *facet_cell, const int *facet_loc, double *rhat, hipStream_t s);
void launch_recover(int p, int nu, int nk, int nb, const double *Ar, const double *Wr, const int *cell_facet,
                    const int8_t *cell_rev, const double *rc, const double *lam, double *q, hipStream_t s);

int red_grid(int64_t len, int nb);
void launch_dots(int64_t len, int nb, int nd, const double *X, int64_t xstride, const double *y, double *partial,
                 double *out, double *host, hipStream_t s);
void launch_gs_norm_givens(int64_t len, int nb, int nd, const double *h, const double *V, int64_t vstride,
                           double *w, double *partial, double *hn, int j, int restart, double *gm,
                           const double *bnorm, double *resid_host, hipStream_t s);
void launch_pcg_update_norm(int64_t len, int nb, const double *num, const double *den, const double *p,
                            const double *w, double *x, double *res, double *partial, double *rr_host,
                            hipStream_t s);
void launch_pcg_dir(int64_t n, int nb, const double *num, const double *den, const double *z, double *p,
                    hipStream_t s);
void launch_lincomb(int64_t n, int nb, int nd, const double *y, const double *Z, int64_t zstride, double *x,
                    hipStream_t s);
void launch_copy(int64_t n, const double *src, double *dst, hipStream_t s);
void launch_gmres_start(int nb, int restart, const double *beta2, double *gm, double *beta, hipStream_t s);
void launch_gmres_solve(int nb, int k, int restart, const double *gm, double *y, hipStream_t s);
void launch_sqrt(int nb, const double *in, double *out, hipStream_t s);

// learned smoother (hdg_mlp.hip)
int mlp_k1p(int p);
int mlp_grad_waves(int ne, int nb);
void launch_mlp_smooth(int p, int ne, int nb, int spl, const double *u, const double *xi, const double *qc,
                       const int *fvert, const int *nbr, const int8_t *prev, const short *W1b, const short *W2b,
                       double *xo, hipStream_t s);
void launch_mlp_grad(int p, int ne, int nb, const double *u, const double *t, const int *nbr, const int8_t *prev,
                     const short *W1b, const short *W2b, float *pdW1, float *pdW2, float *ploss, float *g,
                     double *loss, hipStream_t s);
void launch_adam(int p, const float *g, float gscale, float *w, float *m1, float *m2, float lr, int step,
                 short *wb, hipStream_t s);
void launch_to_bf16(int n, const float *w, short *wb, hipStream_t s);
void launch_prolong_trace(int p, int ne, int nb, const int *fvert, const double *qc, double *x, hipStream_t s);
void launch_lin3(int64_t n, double a, const double *x, double b, const double *y, double c, const double *z,
                 double *out, hipStream_t s);

}  // namespace hdg
