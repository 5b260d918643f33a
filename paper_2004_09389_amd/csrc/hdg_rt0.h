// Launch wrappers of the Lax-Friedrichs coarse-correction kernels (hdg_rt0.hip).
#pragma once

#include "hdg_internal.h"

namespace hdg {

// pi^T: trace residual (M = 2(p+1) unknowns per facet) -> RT0 fluxes of the finest level
template <typename VT>
void launch_lf_restrict(int M, int ne, int nb, const double *pw, const int *rrow, const int *rcol, const VT *res,
                        double *rc, hipStream_t s);
// out = x + pi xc (x may be null); ccorr (may be null): the finest RT0 level's pending last
// smoothing update, xc + omega (corrections at the facet's two vertex patches, slots cfs)
template <typename VT>
void launch_lf_prolong(int M, int ne, int nb, const double *pw, const int *nbr, const double *xc, const int *cfs,
                       double omega, const double *ccorr, const VT *x, VT *out, hipStream_t s);
// RT0 level operations
void launch_rt_patch(const Rt0LevelDev &L, int nb, const double *b, const double *x, double *corr, hipStream_t s);
void launch_rt_update(const Rt0LevelDev &L, int nb, double omega, const double *corr, const double *xin,
                      double *xout, hipStream_t s);
void launch_rt_resid(const Rt0LevelDev &L, int nb, const double *b, const double *x, double *res, hipStream_t s);
// xout = xin + omega c (xin may be null) and res = L.b - A xout, in one pass
void launch_rt_update_resid(const Rt0LevelDev &L, int nb, double omega, const double *corr, const double *xin,
                            double *xout, double *res, hipStream_t s);
void launch_rt_restrict(const Rt0LevelDev &F, int nc, int nb, const double *r, double *bc, hipStream_t s);
// x += P xc, xc taken with level C's pending update when ccorr is given
void launch_rt_prolong(const Rt0LevelDev &F, const Rt0LevelDev &C, int nb, const double *xc, double omega,
                       const double *ccorr, double *x, hipStream_t s);

}  // namespace hdg
