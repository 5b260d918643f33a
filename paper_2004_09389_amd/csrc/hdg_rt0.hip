// Lax-Friedrichs coarse correction on the GPU: restriction pi^T of a vector-
// trace residual onto RT0 fluxes, prolongation pi of an RT0 field back onto
// the trace nodes, and the RT0 geometric-multigrid V-cycle (additive vertex-
// patch smoothing, exact flux transfer between nested levels, dense inverse
// on the coarsest level).  Vectors are [unknown][nrhs].
#include "hdg_kernels.h"
#include "hdg_rt0.h"

namespace hdg {

namespace {

#define GRID8(n, b) dim3((unsigned)((((n) + (b) - 1) / (b) + N_XCD - 1) / N_XCD * N_XCD)), dim3(b)

// rc[e'] = sum over the (e, slot) pairs whose row patch holds e' of
// sum_a pw[slot][a][e] res[e][a]   (pi^T; code = 8 e + slot)
template <int M, typename VT>
__global__ __launch_bounds__(256) void k_lf_restrict(int ne, int nb, const double *__restrict__ pw,
                                                     const int *__restrict__ rrow, const int *__restrict__ rcol,
                                                     const VT *__restrict__ res, double *__restrict__ rc) {
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= ne * nb) return;
    const int ep = t / nb, r = t - ep * nb;
    const size_t NE = (size_t)ne;
    double acc = 0.0;
    for (int q = rrow[ep]; q < rrow[ep + 1]; ++q) {
        const int code = rcol[q], e = code >> 3, slot = code & 7;
#pragma unroll
        for (int a = 0; a < M; ++a)
            acc += pw[((size_t)slot * M + a) * NE + e] * (double)res[((size_t)e * M + a) * nb + r];
    }
    rc[t] = acc;
}

// out = x + pi xc  (x may be null): the average of the two cells' RT0 fields at
// the facet's nodes, from the five fluxes of the facet's row patch
// value of an RT0 iterate at facet e: x[e] plus, when the level's last smoothing
// update is still pending (corr != null), omega times the facet's two patch corrections
__device__ __forceinline__ double rt_value(int e, int r, int nb, int ne, const double *__restrict__ x,
                                           const int *__restrict__ fs, double omega,
                                           const double *__restrict__ corr) {
    double v = x[(size_t)e * nb + r];
    if (corr) {
        const int s0 = fs[e], s1 = fs[ne + e];
        double c = corr[(size_t)s0 * nb + r];
        if (s1 != s0) c += corr[(size_t)s1 * nb + r];
        v += omega * c;
    }
    return v;
}

template <int M, typename VT>
__global__ __launch_bounds__(256) void k_lf_prolong(int ne, int nb, const double *__restrict__ pw,
                                                    const int *__restrict__ nbr, const double *__restrict__ xc,
                                                    const int *__restrict__ cfs, double omega,
                                                    const double *__restrict__ ccorr, const VT *__restrict__ x,
                                                    VT *__restrict__ out) {
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= ne * nb) return;
    const int e = t / nb, r = t - e * nb;
    const size_t NE = (size_t)ne;
    double c[5];
    c[0] = rt_value(e, r, nb, ne, xc, cfs, omega, ccorr);
#pragma unroll
    for (int j = 0; j < 4; ++j) c[j + 1] = rt_value(nbr[j * NE + e], r, nb, ne, xc, cfs, omega, ccorr);
#pragma unroll
    for (int a = 0; a < M; ++a) {
        const size_t o = ((size_t)e * M + a) * nb + r;
        double v = x ? (double)x[o] : 0.0;
#pragma unroll
        for (int j = 0; j < 5; ++j) v += pw[((size_t)j * M + a) * NE + e] * c[j];
        out[o] = (VT)v;
    }
}

// (b - A x) at facet e of an RT0 level (x == null: b)
__device__ __forceinline__ double rt_resid_at(int e, int r, int nb, size_t NE, const double *__restrict__ val,
                                              const int *__restrict__ nbr, const double *__restrict__ b,
                                              const double *__restrict__ x) {
    double v = b[(size_t)e * nb + r];
    if (x) {
        double ax = val[e] * x[(size_t)e * nb + r];
#pragma unroll
        for (int j = 0; j < 4; ++j) ax += val[(j + 1) * NE + e] * x[(size_t)nbr[j * NE + e] * nb + r];
        v -= ax;
    }
    return v;
}

// vertex-patch corrections c_v = A_v^-1 (b - A x)|patch(v), written as
// corr[v][slot][rhs]; the padded slots of a patch carry zero rows and columns
__global__ __launch_bounds__(256) void k_rt_patch(int nv, int ne, int nb, const int *__restrict__ pf,
                                                  const double *__restrict__ pinv, const double *__restrict__ val,
                                                  const int *__restrict__ nbr, const double *__restrict__ b,
                                                  const double *__restrict__ x, double *__restrict__ corr) {
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= nv * nb) return;
    const int v = t / nb, r = t - v * nb;
    const size_t NV = (size_t)nv, NE = (size_t)ne;
    double rv[RT_PV];
#pragma unroll
    for (int j = 0; j < RT_PV; ++j) {
        const int e = pf[j * NV + v];
        rv[j] = e >= 0 ? rt_resid_at(e, r, nb, NE, val, nbr, b, x) : 0.0;
    }
#pragma unroll
    for (int i = 0; i < RT_PV; ++i) {
        double y = 0.0;
#pragma unroll
        for (int j = 0; j < RT_PV; ++j) y += pinv[(size_t)(i * RT_PV + j) * NV + v] * rv[j];
        corr[((size_t)v * RT_PV + i) * nb + r] = y;
    }
}

// x_out = x_in + omega (c at the facet's slot in both end vertices' patches)
__global__ __launch_bounds__(256) void k_rt_update(int ne, int nb, const int *__restrict__ fs, double omega,
                                                   const double *__restrict__ corr, const double *__restrict__ xin,
                                                   double *__restrict__ xout) {
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= ne * nb) return;
    const int e = t / nb, r = t - e * nb;
    const int s0 = fs[e], s1 = fs[ne + e];
    double c = corr[(size_t)s0 * nb + r];
    if (s1 != s0) c += corr[(size_t)s1 * nb + r];
    xout[t] = (xin ? xin[t] : 0.0) + omega * c;
}

// last pre-smoothing step fused with the residual: x_out = x_in + omega c at the
// facet (x_in may be null: zero), written, and res = b - A x_out with the
// neighbours' x_out formed on the fly
__global__ __launch_bounds__(256) void k_rt_update_resid(int ne, int nb, const int *__restrict__ fs, double omega,
                                                         const double *__restrict__ corr,
                                                         const double *__restrict__ xin,
                                                         const double *__restrict__ val,
                                                         const int *__restrict__ nbr, const double *__restrict__ b,
                                                         double *__restrict__ xout, double *__restrict__ res) {
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= ne * nb) return;
    const int e = t / nb, r = t - e * nb;
    const size_t NE = (size_t)ne;
    auto xnew = [&](int f) {
        const int s0 = fs[f], s1 = fs[ne + f];
        double c = corr[(size_t)s0 * nb + r];
        if (s1 != s0) c += corr[(size_t)s1 * nb + r];
        return (xin ? xin[(size_t)f * nb + r] : 0.0) + omega * c;
    };
    const double xe = xnew(e);
    double ax = val[e] * xe;
#pragma unroll
    for (int j = 0; j < 4; ++j) ax += val[(j + 1) * NE + e] * xnew(nbr[j * NE + e]);
    res[t] = b[t] - ax;
    xout[t] = xe;
}

__global__ __launch_bounds__(256) void k_rt_resid(int ne, int nb, const double *__restrict__ val,
                                                  const int *__restrict__ nbr, const double *__restrict__ b,
                                                  const double *__restrict__ x, double *__restrict__ res) {
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= ne * nb) return;
    const int e = t / nb, r = t - e * nb;
    res[t] = rt_resid_at(e, r, nb, (size_t)ne, val, nbr, b, x);
}

// bc[c] = sum over the fine facets fed by coarse facet c of w * r_fine  (P^T)
__global__ __launch_bounds__(256) void k_rt_restrict(int nc, int nb, const int *__restrict__ crow,
                                                     const int *__restrict__ ccol, const double *__restrict__ cw,
                                                     const double *__restrict__ r, double *__restrict__ bc) {
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= nc * nb) return;
    const int c = t / nb, rr = t - c * nb;
    double acc = 0.0;
    for (int q = crow[c]; q < crow[c + 1]; ++q) acc += cw[q] * r[(size_t)ccol[q] * nb + rr];
    bc[t] = acc;
}

// x += P xc: the coarse field's flux through each fine facet (xc with the coarse
// level's pending update when ccorr is given)
__global__ __launch_bounds__(256) void k_rt_prolong(int ne, int nb, const int *__restrict__ pc,
                                                    const double *__restrict__ pw, int nec,
                                                    const double *__restrict__ xc, const int *__restrict__ cfs,
                                                    double omega, const double *__restrict__ ccorr,
                                                    double *__restrict__ x) {
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= ne * nb) return;
    const int e = t / nb, r = t - e * nb;
    double v = x[t];
#pragma unroll
    for (int j = 0; j < 3; ++j)
        v += pw[(size_t)j * ne + e] * rt_value(pc[(size_t)j * ne + e], r, nb, nec, xc, cfs, omega, ccorr);
    x[t] = v;
}

}  // namespace

template <typename VT>
void launch_lf_restrict(int M, int ne, int nb, const double *pw, const int *rrow, const int *rcol, const VT *res,
                        double *rc, hipStream_t s) {
#define LR(MM) hipLaunchKernelGGL((k_lf_restrict<MM, VT>), GRID8(ne * nb, 256), 0, s, ne, nb, pw, rrow, rcol, res, rc)
    switch (M) { case 4: LR(4); break; case 6: LR(6); break; case 8: LR(8); break; }
#undef LR
}

template <typename VT>
void launch_lf_prolong(int M, int ne, int nb, const double *pw, const int *nbr, const double *xc, const int *cfs,
                       double omega, const double *ccorr, const VT *x, VT *out, hipStream_t s) {
#define LP(MM) hipLaunchKernelGGL((k_lf_prolong<MM, VT>), GRID8(ne * nb, 256), 0, s, ne, nb, pw, nbr, xc, cfs, omega, ccorr, x, out)
    switch (M) { case 4: LP(4); break; case 6: LP(6); break; case 8: LP(8); break; }
#undef LP
}
template void launch_lf_restrict<double>(int, int, int, const double *, const int *, const int *, const double *,
                                         double *, hipStream_t);
template void launch_lf_restrict<float>(int, int, int, const double *, const int *, const int *, const float *,
                                        double *, hipStream_t);
template void launch_lf_prolong<double>(int, int, int, const double *, const int *, const double *, const int *,
                                        double, const double *, const double *, double *, hipStream_t);
template void launch_lf_prolong<float>(int, int, int, const double *, const int *, const double *, const int *,
                                       double, const double *, const float *, float *, hipStream_t);

void launch_rt_patch(const Rt0LevelDev &L, int nb, const double *b, const double *x, double *corr, hipStream_t s) {
    hipLaunchKernelGGL(k_rt_patch, GRID8(L.nv * nb, 256), 0, s, L.nv, L.ne, nb, L.pf, L.pinv, L.val, L.nbr, b, x,
                       corr);
}
void launch_rt_update(const Rt0LevelDev &L, int nb, double omega, const double *corr, const double *xin,
                      double *xout, hipStream_t s) {
    hipLaunchKernelGGL(k_rt_update, GRID8(L.ne * nb, 256), 0, s, L.ne, nb, L.fs, omega, corr, xin, xout);
}
void launch_rt_update_resid(const Rt0LevelDev &L, int nb, double omega, const double *corr, const double *xin,
                            double *xout, double *res, hipStream_t s) {
    hipLaunchKernelGGL(k_rt_update_resid, GRID8(L.ne * nb, 256), 0, s, L.ne, nb, L.fs, omega, corr, xin, L.val, L.nbr,
                       L.b, xout, res);
}
void launch_rt_resid(const Rt0LevelDev &L, int nb, const double *b, const double *x, double *res, hipStream_t s) {
    hipLaunchKernelGGL(k_rt_resid, GRID8(L.ne * nb, 256), 0, s, L.ne, nb, L.val, L.nbr, b, x, res);
}
void launch_rt_restrict(const Rt0LevelDev &F, int nc, int nb, const double *r, double *bc, hipStream_t s) {
    hipLaunchKernelGGL(k_rt_restrict, GRID8(nc * nb, 256), 0, s, nc, nb, F.crow, F.ccol, F.cw, r, bc);
}
void launch_rt_prolong(const Rt0LevelDev &F, const Rt0LevelDev &C, int nb, const double *xc, double omega,
                       const double *ccorr, double *x, hipStream_t s) {
    hipLaunchKernelGGL(k_rt_prolong, GRID8(F.ne * nb, 256), 0, s, F.ne, nb, F.pc, F.pw, C.ne, xc, C.fs, omega, ccorr,
                       x);
}

}  // namespace hdg
