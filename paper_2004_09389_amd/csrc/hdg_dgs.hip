// Non-hybridised DG baseline: restarted flexible GMRES on the standard DG
// stage system with the approximate Schur-complement preconditioner of the
// native DG section (Eqs. native_dg_system, native_matrix_representation,
// S_approx_diag).
//
// Operator.  The standard upwind DG system is the HDG cell system with the
// trace replaced by the DG trace lam(q) = {{phi}} + [[u]] / (2 tau) (the two
// forms coincide, Eq. linear_hybridized), so one application is the trace
// shares of q at the facet nodes, their sum per facet, and per cell
// A_K q_K + B_K lam_K with the stored cell matrices (the recovery kernel with
// (A, -B) in place of (A^-1 M, A^-1 B)).  Vectors use the symmetric variables
// (phi = h sqrt(g/H), u) in the cell layout [n_cell][3][n_loc][nrhs].
//
// Preconditioner (three steps): V = A_uu~^-1 R_u;  Phi = S~^-1 (R_phi - A_pu V);
// U = A_uu~^-1 (R_u - A_up Phi), with
//   A_uu~^-1  the exact inverse of each cell's diagonal block of A_uu;
//   S = A_pp - A_pu diag(A_uu)^-1 A_up, applied as two operator applications;
//   S~^-1     one two-level cycle: Chebyshev(nu_pre) smoothing preconditioned by
//             the inverse of each cell's own block of S on [0.1, 1.1] lambda_max,
//             the coarse correction on P1 with the Galerkin operator
//             P^T S P = M_1 + kappa^2 sum_K sum_d beta_Kd d_d phi d_d psi,
//             beta_Kd = sum_i (int_K phi_i)^2 / diag(A_uu)_(K,d,i) (exact for
//             continuous P1 fields: the facet terms cancel and A_up P phi is
//             kappa M grad phi), one P1 V-cycle with Galerkin coarsening, and
//             Chebyshev(nu_post) again.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <map>
#include <string>
#include <vector>

#include "hdg_kernels.h"

namespace hdg {
namespace {

constexpr int DGS_MAX_RHS = 64;



inline dim3 grid_for(int64_t n, int block) { return dim3((unsigned)((n + block - 1) / block)); }

// lattice coordinates (i, j) of DG node `node` (j-major, then i)
template <int P>
__device__ __forceinline__ void lattice(int node, int &i, int &j) {
    j = 0;
    while (node > P - j) {
        node -= P + 1 - j;
        ++j;
    }
    i = node;
}

// barycentric weight of corner c at lattice node (i, j) / P
template <int P>
__device__ __forceinline__ double corner_weight(int c, int i, int j) {
    return c == 0 ? 1.0 - (double)(i + j) / P : (c == 1 ? (double)i / P : (double)j / P);
}

// ------------------------------------------------------------------ kernels

__global__ void k_dgs_trace_sum(int64_t cnt, int Mnb, const double *__restrict__ half, double *__restrict__ lam) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const int64_t e = t / Mnb, w = t - e * Mnb;
    lam[t] = half[(2 * e) * Mnb + w] + half[(2 * e + 1) * Mnb + w];
}

// Gauss-Jordan with partial pivoting on an LDS matrix a[rows][ld] (columns
// 0..cols-1, the first `rows` of them the matrix), one wavefront, rows <= 64.
__device__ bool wave_gauss_jordan(double *a, int rows, int ld, int cols, double *fac, int lane) {
    for (int k = 0; k < rows; ++k) {
        double best = (lane >= k && lane < rows) ? fabs(a[lane * ld + k]) : -1.0;
        int bi = lane;
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        if (!(best > 0.0)) return false;
        if (bi != k)
            for (int c = lane; c < cols; c += 64) {
                const double t = a[k * ld + c];
                a[k * ld + c] = a[bi * ld + c];
                a[bi * ld + c] = t;
            }
        __syncthreads();
        const double ip = 1.0 / a[k * ld + k];
        __syncthreads();
        for (int c = lane; c < cols; c += 64) a[k * ld + c] *= ip;
        for (int r = lane; r < rows; r += 64) fac[r] = a[r * ld + k];
        __syncthreads();
        for (int idx = lane; idx < rows * (cols - k); idx += 64) {
            const int r = idx / (cols - k), c = k + idx % (cols - k);
            if (r != k) a[r * ld + c] -= fac[r] * a[k * ld + c];
        }
        __syncthreads();
    }
    return true;
}

// Per cell (one wavefront): the cell-diagonal block of the DG matrix
// G = A + B Lambda (Lambda: this cell's share of lam at its facet nodes,
// 1/2 for phi and n_d / (2 tau) for u_d), then diag(A_uu), the inverse of
// G_uu, the inverse of the own block G_pp - G_pu diag(A_uu)^-1 G_up, and
// beta_Kd = sum_i (int phi_i)^2 / diag(A_uu)_(d,i).
template <int P>
__global__ __launch_bounds__(64) void k_dgs_local(int nk, int geom, double tau, const double *__restrict__ corners,
                                                  const double *__restrict__ A, const double *__restrict__ Bn,
                                                  double *__restrict__ Auu_inv, double *__restrict__ Sown_inv,
                                                  double *__restrict__ Dinv, double *__restrict__ beta,
                                                  int *__restrict__ err) {
    constexpr int n = (P + 1) * (P + 2) / 2, m = P + 1, nc = 3 * n, nt = 3 * m, n2 = 2 * n;
    __shared__ double G[nc * nc];
    __shared__ double au[n2 * 2 * n2];
    __shared__ double as[n * 2 * n];
    __shared__ double D[n2];
    __shared__ double fac[n2];
    __shared__ double nrm[3][2];
    __shared__ int tnode[nt];
    const int K = blockIdx.x, lane = threadIdx.x;
    if (K >= nk) return;
    const size_t NK = (size_t)nk;
    if (lane < 3) {
        const int f = lane;
        const double *X = corners + 9 * (size_t)K;
        double ab[3], ac[3];
        for (int d = 0; d < 3; ++d) {
            ab[d] = X[3 + d] - X[d];
            ac[d] = X[6 + d] - X[d];
        }
        double e1[3] = {1.0, 0.0, 0.0}, e2[3] = {0.0, 1.0, 0.0};
        if (geom == HDG_SPHERE) {
            double kn[3] = {ab[1] * ac[2] - ab[2] * ac[1], ab[2] * ac[0] - ab[0] * ac[2], ab[0] * ac[1] - ab[1] * ac[0]};
            const double il = 1.0 / sqrt(kn[0] * kn[0] + kn[1] * kn[1] + kn[2] * kn[2]);
            for (int d = 0; d < 3; ++d) kn[d] *= il;
            const double la = 1.0 / sqrt(ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]);
            for (int d = 0; d < 3; ++d) e1[d] = ab[d] * la;
            e2[0] = kn[1] * e1[2] - kn[2] * e1[1];
            e2[1] = kn[2] * e1[0] - kn[0] * e1[2];
            e2[2] = kn[0] * e1[1] - kn[1] * e1[0];
        }
        const double Px[3] = {0.0, ab[0] * e1[0] + ab[1] * e1[1] + ab[2] * e1[2],
                              ac[0] * e1[0] + ac[1] * e1[1] + ac[2] * e1[2]};
        const double Py[3] = {0.0, ab[0] * e2[0] + ab[1] * e2[1] + ab[2] * e2[2],
                              ac[0] * e2[0] + ac[1] * e2[1] + ac[2] * e2[2]};
        const double tx = Px[(f + 2) % 3] - Px[(f + 1) % 3], ty = Py[(f + 2) % 3] - Py[(f + 1) % 3];
        const double L = sqrt(tx * tx + ty * ty);
        nrm[f][0] = ty / L;
        nrm[f][1] = -tx / L;
    }
    if (lane < nt) {
        const int f = lane / m, k = lane % m;
        const int i = f == 0 ? P - k : (f == 1 ? 0 : k);
        const int j = f == 0 ? k : (f == 1 ? P - k : 0);
        tnode[lane] = j * (P + 1) - j * (j - 1) / 2 + i;
    }
    __syncthreads();
    const double it2 = 0.5 / tau;
    for (int idx = lane; idx < nc * nc; idx += 64) {
        const int a = idx / nc, b = idx - a * nc, fb = b / n, ib = b - fb * n;
        double s = A[(size_t)idx * NK + K];
        for (int t = 0; t < nt; ++t) {
            if (tnode[t] != ib) continue;
            const double coef = fb == 0 ? 0.5 : nrm[t / m][fb - 1] * it2;
            s -= Bn[(size_t)(a * nt + t) * NK + K] * coef;
        }
        G[idx] = s;
    }
    __syncthreads();
    if (lane < n2) {
        D[lane] = G[(n + lane) * nc + n + lane];
        Dinv[(size_t)K * n2 + lane] = 1.0 / D[lane];
    }
    for (int idx = lane; idx < n2 * 2 * n2; idx += 64) {
        const int r = idx / (2 * n2), c = idx - r * 2 * n2;
        au[idx] = c < n2 ? G[(n + r) * nc + n + c] : (c - n2 == r ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int idx = lane; idx < n * 2 * n; idx += 64) {
        const int r = idx / (2 * n), c = idx - r * 2 * n;
        double v = 0.0;
        if (c < n) {
            v = G[r * nc + c];
            for (int j = 0; j < n2; ++j) v -= G[r * nc + n + j] * G[(n + j) * nc + c] / D[j];
        } else {
            v = (c - n == r) ? 1.0 : 0.0;
        }
        as[idx] = v;
    }
    if (lane < 2) {
        double bsum = 0.0;
        for (int i = 0; i < n; ++i) {
            double rs = 0.0;
            for (int j = 0; j < n; ++j) rs += A[(size_t)((n + i) * nc + n + j) * NK + K];   // cell mass row sum
            bsum += rs * rs / D[lane * n + i];
        }
        beta[2 * (size_t)K + lane] = bsum;
    }
    __syncthreads();
    if (!wave_gauss_jordan(au, n2, 2 * n2, 2 * n2, fac, lane)) {
        if (lane == 0) atomicOr(err, 1);
        return;
    }
    if (!wave_gauss_jordan(as, n, 2 * n, 2 * n, fac, lane)) {
        if (lane == 0) atomicOr(err, 2);
        return;
    }
    for (int idx = lane; idx < n2 * n2; idx += 64) {
        const int r = idx / n2, c = idx - r * n2;
        Auu_inv[(size_t)idx * NK + K] = au[r * 2 * n2 + n2 + c];
    }
    for (int idx = lane; idx < n * n; idx += 64) {
        const int r = idx / n, c = idx - r * n;
        Sown_inv[(size_t)idx * NK + K] = as[r * 2 * n + n + c];
    }
}

// out[K][off + a][r] = sum_b Minv_K[a][b] in[K][off + b][r], a, b < R (other fields untouched)
template <int R>
__global__ __launch_bounds__(256) void k_dgs_block_mv(int nk, int nb, int nc, int off, const double *__restrict__ Minv,
                                                      const double *__restrict__ in, double *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nk * nb) return;
    const int K = (int)(t / nb), r = (int)(t - (int64_t)K * nb);
    const size_t NK = (size_t)nk;
    double x[R];
#pragma unroll
    for (int b = 0; b < R; ++b) x[b] = in[((size_t)K * nc + off + b) * nb + r];
    for (int a = 0; a < R; ++a) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < R; ++b) s += Minv[(size_t)(a * R + b) * NK + K] * x[b];
        out[((size_t)K * nc + off + a) * nb + r] = s;
    }
}

// out = (a x + b y) on the fields f0 <= f < f1 (x, y may be null = 0); with dinv
// the velocity fields are also multiplied by 1 / diag(A_uu)
__global__ __launch_bounds__(256) void k_dgs_lin(int64_t cnt, int n, int nb, int f0, int f1, double a,
                                                 const double *__restrict__ x, double b, const double *__restrict__ y,
                                                 const double *__restrict__ dinv, double *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    const int64_t per = (int64_t)(f1 - f0) * n * nb;
    const int64_t K = t / per, w = t - K * per;
    const size_t o = (size_t)(K * 3 * n * nb + (int64_t)f0 * n * nb + w);
    double v = 0.0;
    if (x) v = a * x[o];
    if (y) v = __builtin_fma(b, y[o], v);
    if (dinv) {
        const int fld = f0 + (int)(w / ((int64_t)n * nb));
        if (fld >= 1) {
            const int node = (int)((w % ((int64_t)n * nb)) / nb);
            v *= dinv[(size_t)K * 2 * n + (fld - 1) * n + node];
        }
    }
    out[o] = v;
}

// R = Mtilde r: per cell the mass matrix (the u1-u1 block of A_K) times each
// field, the phi field also times hscale
__global__ __launch_bounds__(256) void k_dgs_load(int nk, int n, int nb, double hscale, const double *__restrict__ A,
                                                  const double *__restrict__ r, double *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nk * 3 * n * nb) return;
    const int rr = (int)(t % nb);
    const int64_t q = t / nb;
    const int i = (int)(q % n), fld = (int)((q / n) % 3);
    const int64_t K = q / (3 * n);
    const int nc = 3 * n;
    const size_t NK = (size_t)nk;
    double s = 0.0;
    for (int j = 0; j < n; ++j)
        s += A[(size_t)((n + i) * nc + n + j) * NK + K] * r[((size_t)K * nc + fld * n + j) * nb + rr];
    out[t] = fld == 0 ? hscale * s : s;
}

// rc[v] = sum over the cells at v and their DG nodes of the corner weight times r_phi
template <int P>
__global__ __launch_bounds__(256) void k_dgs_restrict(int nv, int nb, const int *__restrict__ vrow,
                                                      const int *__restrict__ vcol, const double *__restrict__ r,
                                                      double *__restrict__ rc) {
    constexpr int n = (P + 1) * (P + 2) / 2, nc = 3 * n;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nv * nb) return;
    const int v = (int)(t / nb), rr = (int)(t - (int64_t)v * nb);
    double s = 0.0;
    for (int q = vrow[v]; q < vrow[v + 1]; ++q) {
        const int K = vcol[q] / 3, c = vcol[q] - 3 * K;
        for (int node = 0; node < n; ++node) {
            int i, j;
            lattice<P>(node, i, j);
            s += corner_weight<P>(c, i, j) * r[((size_t)K * nc + node) * nb + rr];
        }
    }
    rc[t] = s;
}

// x_phi[K][node] += sum_c w_c(node) xc[vertex of corner c]
template <int P>
__global__ __launch_bounds__(256) void k_dgs_prolong(int nk, int nb, const int *__restrict__ cvert,
                                                     const double *__restrict__ xc, double *__restrict__ x) {
    constexpr int n = (P + 1) * (P + 2) / 2, nc = 3 * n;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nk * nb) return;
    const int K = (int)(t / nb), rr = (int)(t - (int64_t)K * nb);
    const double c0 = xc[(size_t)cvert[3 * K] * nb + rr], c1 = xc[(size_t)cvert[3 * K + 1] * nb + rr],
                 c2 = xc[(size_t)cvert[3 * K + 2] * nb + rr];
    for (int node = 0; node < n; ++node) {
        int i, j;
        lattice<P>(node, i, j);
        const double v = corner_weight<P>(0, i, j) * c0 + corner_weight<P>(1, i, j) * c1 + corner_weight<P>(2, i, j) * c2;
        x[((size_t)K * nc + node) * nb + rr] += v;
    }
}

// out[i][r] = x[i][r] * c[r]  (c: per right-hand side, by value)
struct Cols {
    double v[DGS_MAX_RHS];
};
__global__ __launch_bounds__(256) void k_dgs_scale(int64_t cnt, int nb, Cols c, const double *__restrict__ x,
                                                   double *__restrict__ out) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    out[t] = x[t] * c.v[t % nb];
}

// ------------------------------------------------------------------ host helpers

struct Dgs {
    hdg_ctx *c;
    int nb;
    hipStream_t s;
    int64_t len;    // rows of a cell vector (n_cell * nc)
    double *tmp(int i) const { return c->dgs_tmp[i]; }
};

void lin(const Dgs &g, int f0, int f1, double a, const double *x, double b, const double *y, bool dinv, double *out) {
    const int64_t cnt = (int64_t)g.c->n_cell * (f1 - f0) * g.c->n * g.nb;
    hipLaunchKernelGGL(k_dgs_lin, grid_for(cnt, 256), dim3(256), 0, g.s, cnt, g.c->n, g.nb, f0, f1, a, x, b, y,
                       dinv ? g.c->dgs_Dinv : nullptr, out);
    check_kernel_launch();
}

// y = A x, the DG stage operator (symmetric variables)
void dgs_apply(const Dgs &g, const double *x, double *y) {
    hdg_ctx *c = g.c;
    launch_dg_half(c, g.nb, 1.0, x, c->dgs_half, g.s);
    const int64_t cnt = (int64_t)c->n_facet * c->m * g.nb;
    hipLaunchKernelGGL(k_dgs_trace_sum, grid_for(cnt, 256), dim3(256), 0, g.s, cnt, c->m * g.nb, c->dgs_half,
                       c->dgs_lam);
    check_kernel_launch();
    launch_recover(c->p, 1, c->n_cell, g.nb, c->dgs_A, c->dgs_Bn, c->cell_facet, c->cell_rev, x, c->dgs_lam, y, g.s);
    check_kernel_launch();
}

void block_mv(const Dgs &g, bool velocity, const double *in, double *out) {
    hdg_ctx *c = g.c;
    const int64_t cnt = (int64_t)c->n_cell * g.nb;
    const int n = c->n;
#define BMV(R, M, OFF) \
    hipLaunchKernelGGL(k_dgs_block_mv<R>, grid_for(cnt, 256), dim3(256), 0, g.s, c->n_cell, g.nb, c->nc, OFF, M, in, out)
    if (velocity) {
        switch (c->p) {
            case 1: BMV(6, c->dgs_Auu_inv, n); break;
            case 2: BMV(12, c->dgs_Auu_inv, n); break;
            default: BMV(20, c->dgs_Auu_inv, n); break;
        }
    } else {
        switch (c->p) {
            case 1: BMV(3, c->dgs_Sown_inv, 0); break;
            case 2: BMV(6, c->dgs_Sown_inv, 0); break;
            default: BMV(10, c->dgs_Sown_inv, 0); break;
        }
    }
#undef BMV
    check_kernel_launch();
}

// y_phi = S x_phi (x in the phi field of x; its velocity fields must be zero).
// Uses tmp 6, 7, 11.
void s_apply(const Dgs &g, const double *x, double *y) {
    double *t1 = g.tmp(6), *w = g.tmp(7), *t3 = g.tmp(11);
    dgs_apply(g, x, t1);                                  // t1 = (A_pp x, A_up x)
    lin(g, 0, 1, 0.0, nullptr, 0.0, nullptr, false, w);
    lin(g, 1, 3, 1.0, t1, 0.0, nullptr, true, w);         // w = (0, D^-1 A_up x)
    dgs_apply(g, w, t3);                                  // t3_phi = A_pu D^-1 A_up x
    lin(g, 0, 1, 1.0, t1, -1.0, t3, false, y);            // y_phi = A_pp x - A_pu D^-1 A_up x
}

double *p1_cycle(std::vector<P1LevelDev> &lev, const double *coarse_inv, int l, int nb, int nu, double w,
                 hipStream_t s) {
    P1LevelDev &L = lev[l];
    if (l == 0) {
        launch_dense_mv(L.n, nb, coarse_inv, L.b, L.x, s);
        return L.x;
    }
    double *x = L.x, *y = L.y;
    if (nu == 1) {
        launch_p1_first(L.n, nb, L.dinv, w, L.b, x, s);
    } else {
        launch_p1_pre2(L.n, L.w, nb, L.col, L.val, L.diag, L.dinv, w, L.b, x, s);
        for (int k = 2; k < nu; ++k) {
            launch_p1_sweep(L.n, L.w, nb, L.col, L.val, L.diag, L.dinv, w, L.b, x, nullptr, nullptr, y, s);
            std::swap(x, y);
        }
    }
    launch_p1_resid(L.n, L.w, nb, L.col, L.val, L.diag, L.b, x, y, s);
    P1LevelDev &C = lev[l - 1];
    launch_p1_restrict(C.n, nb, L.crow, L.ccol, L.cw, y, C.b, s);
    const double *xc = p1_cycle(lev, coarse_inv, l - 1, nb, nu, w, s);
    for (int k = 0; k < nu; ++k) {
        launch_p1_sweep(L.n, L.w, nb, L.col, L.val, L.diag, L.dinv, w, L.b, x, k == 0 ? xc : nullptr, L.parents, y,
                        s);
        std::swap(x, y);
    }
    return x;
}

// k Chebyshev steps for S x = b (phi fields; x updated in place), preconditioned by
// the own-block inverses on [0.1, 1.1] lambda_max.  Uses tmp 3, 4, 5 (and 6, 7).
void chebyshev(const Dgs &g, const double *b, double *x, int k, bool x_zero) {
    const double lo = 0.1 * g.c->dgs_lmax, hi = 1.1 * g.c->dgs_lmax;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    double rho = 1.0 / sigma;
    double *res = g.tmp(3), *d = g.tmp(4), *z = g.tmp(5);
    if (x_zero) {
        lin(g, 0, 1, 1.0, b, 0.0, nullptr, false, res);
    } else {
        s_apply(g, x, res);
        lin(g, 0, 1, 1.0, b, -1.0, res, false, res);
    }
    block_mv(g, false, res, z);
    lin(g, 0, 1, 1.0 / theta, z, 0.0, nullptr, false, d);
    for (int step = 0; step < k; ++step) {
        lin(g, 0, 1, 1.0, x, 1.0, d, false, x);
        if (step == k - 1) break;
        const double rho_new = 1.0 / (2.0 * sigma - rho);
        s_apply(g, x, res);
        lin(g, 0, 1, 1.0, b, -1.0, res, false, res);
        block_mv(g, false, res, z);
        lin(g, 0, 1, rho_new * rho, d, 2.0 * rho_new / delta, z, false, d);
        rho = rho_new;
    }
}

// x_phi = S~^-1 b_phi (one two-level cycle from zero); x's velocity fields are zeroed
void s_cycle(const Dgs &g, const double *b, double *x) {
    hdg_ctx *c = g.c;
    lin(g, 0, 3, 0.0, nullptr, 0.0, nullptr, false, x);
    chebyshev(g, b, x, c->opt.nu_pre, true);
    double *res = g.tmp(3);
    s_apply(g, x, res);
    lin(g, 0, 1, 1.0, b, -1.0, res, false, res);
    const int L = (int)c->dgs_lev.size() - 1;
    P1LevelDev &F = c->dgs_lev[L];
#define RESTRICT(P)                                                                                                \
    hipLaunchKernelGGL(k_dgs_restrict<P>, grid_for((int64_t)F.n * g.nb, 256), dim3(256), 0, g.s, F.n, g.nb,         \
                       c->dgs_vrow, c->dgs_vcol, res, F.b)
#define PROLONG(P)                                                                                                 \
    hipLaunchKernelGGL(k_dgs_prolong<P>, grid_for((int64_t)c->n_cell * g.nb, 256), dim3(256), 0, g.s, c->n_cell, \
                       g.nb, c->dgs_cvert, xc, x)
    switch (c->p) {
        case 1: RESTRICT(1); break;
        case 2: RESTRICT(2); break;
        default: RESTRICT(3); break;
    }
    check_kernel_launch();
    const double *xc = p1_cycle(c->dgs_lev, c->dgs_coarse_inv, L, g.nb, c->opt.p1_nu, c->opt.p1_omega, g.s);
    switch (c->p) {
        case 1: PROLONG(1); break;
        case 2: PROLONG(2); break;
        default: PROLONG(3); break;
    }
#undef RESTRICT
#undef PROLONG
    check_kernel_launch();
    chebyshev(g, b, x, c->opt.nu_post, false);
}

// z = P^-1 r, the three steps (tmp 0, 1, 2 and those of s_cycle)
void precondition(const Dgs &g, const double *r, double *z) {
    double *v = g.tmp(0), *t = g.tmp(1), *w = g.tmp(2);
    lin(g, 0, 1, 0.0, nullptr, 0.0, nullptr, false, v);
    block_mv(g, true, r, v);                               // v = (0, A_uu~^-1 r_u)
    dgs_apply(g, v, t);                                    // t_phi = A_pu V
    lin(g, 0, 1, 1.0, r, -1.0, t, false, w);               // w_phi = r_phi - A_pu V
    s_cycle(g, w, z);                                      // z = (Phi, 0)
    dgs_apply(g, z, t);                                    // t_u = A_up Phi
    lin(g, 1, 3, 1.0, r, -1.0, t, false, w);               // w_u = r_u - A_up Phi
    block_mv(g, true, w, z);                               // z_u = A_uu~^-1 w_u
}

std::vector<double> dots(const Dgs &g, int nd, const double *X, int64_t xstride, const double *y) {
    launch_dots<double>(g.len, g.nb, nd, X, xstride, y, g.c->dgs_red, g.c->dgs_out, nullptr, g.s);
    check_kernel_launch();
    std::vector<double> h((size_t)nd * g.nb);
    HDG_HIP_CHECK(hipMemcpyAsync(h.data(), g.c->dgs_out, h.size() * sizeof(double), hipMemcpyDeviceToHost, g.s));
    HDG_HIP_CHECK(hipStreamSynchronize(g.s));
    return h;
}

void scale_cols(const Dgs &g, const std::vector<double> &c, const double *x, double *out) {
    Cols cc{};
    for (int r = 0; r < g.nb; ++r) cc.v[r] = c[r];
    const int64_t cnt = g.len * g.nb;
    hipLaunchKernelGGL(k_dgs_scale, grid_for(cnt, 256), dim3(256), 0, g.s, cnt, g.nb, cc, x, out);
    check_kernel_launch();
}

// x += sum_d coef[d][r] Z_d
void lincomb(const Dgs &g, int nd, const std::vector<double> &coef, const double *Z, int64_t zstride, double *x) {
    HDG_HIP_CHECK(hipMemcpyAsync(g.c->dgs_coef, coef.data(), (size_t)nd * g.nb * sizeof(double),
                                 hipMemcpyHostToDevice, g.s));
    launch_lincomb<double>(g.len, g.nb, nd, g.c->dgs_coef, Z, zstride, x, g.s);
    check_kernel_launch();
}

int restart_len(const hdg_ctx *c) { return std::max(1, std::min(c->opt.restart, 64)); }

// Galerkin P1 operator of S on the finest mesh: M_1 + kappa^2 sum_K sum_d beta_Kd
// d_d lambda_i d_d lambda_j, with P1 gradients in each cell's frame
P1Host assemble_sc(const hdg_mesh &mesh, double kappa, const std::vector<double> &beta) {
    P1Host P;
    const int nv = mesh.n_vert;
    P.n = nv;
    std::vector<double> x = cell_corners(mesh);
    std::vector<std::map<int, double>> rows(nv);
    std::vector<double> diag(nv, 0.0);
    for (int K = 0; K < mesh.n_cell; ++K) {
        const double *c = &x[9 * K];
        double ab[3], ac[3];
        for (int d = 0; d < 3; ++d) {
            ab[d] = c[3 + d] - c[d];
            ac[d] = c[6 + d] - c[d];
        }
        double e1[3] = {1.0, 0.0, 0.0}, e2[3] = {0.0, 1.0, 0.0};
        if (mesh.geom == HDG_SPHERE) {
            double kn[3] = {ab[1] * ac[2] - ab[2] * ac[1], ab[2] * ac[0] - ab[0] * ac[2], ab[0] * ac[1] - ab[1] * ac[0]};
            const double il = 1.0 / std::sqrt(kn[0] * kn[0] + kn[1] * kn[1] + kn[2] * kn[2]);
            for (double &v : kn) v *= il;
            const double la = 1.0 / std::sqrt(ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]);
            for (int d = 0; d < 3; ++d) e1[d] = ab[d] * la;
            e2[0] = kn[1] * e1[2] - kn[2] * e1[1];
            e2[1] = kn[2] * e1[0] - kn[0] * e1[2];
            e2[2] = kn[0] * e1[1] - kn[1] * e1[0];
        }
        const double px[3] = {0.0, ab[0] * e1[0] + ab[1] * e1[1] + ab[2] * e1[2], ac[0] * e1[0] + ac[1] * e1[1] + ac[2] * e1[2]};
        const double py[3] = {0.0, ab[0] * e2[0] + ab[1] * e2[1] + ab[2] * e2[2], ac[0] * e2[0] + ac[1] * e2[1] + ac[2] * e2[2]};
        const double area = 0.5 * (px[1] * py[2] - py[1] * px[2]);
        double gr[3][2];
        for (int i = 0; i < 3; ++i) {
            const int a = (i + 1) % 3, b = (i + 2) % 3;
            gr[i][0] = (py[a] - py[b]) / (2.0 * area);
            gr[i][1] = (px[b] - px[a]) / (2.0 * area);
        }
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                const double kij = beta[2 * K] * gr[i][0] * gr[j][0] + beta[2 * K + 1] * gr[i][1] * gr[j][1];
                const double v = area / 12.0 * (i == j ? 2.0 : 1.0) + kappa * kappa * kij;
                const int vi = mesh.cell_vert[3 * K + i], vj = mesh.cell_vert[3 * K + j];
                if (vi == vj)
                    diag[vi] += v;
                else
                    rows[vi][vj] += v;
            }
    }
    P.rowptr.assign(nv + 1, 0);
    for (int v = 0; v < nv; ++v) P.rowptr[v + 1] = P.rowptr[v] + (int)rows[v].size();
    for (int v = 0; v < nv; ++v)
        for (auto &kv : rows[v]) {
            P.col.push_back(kv.first);
            P.val.push_back(kv.second);
        }
    P.diag = diag;
    return P;
}

void check_vec(const hdg_ctx *c, int nb) {
    HDG_REQUIRE(c->dgs_ready, "call hdg_dgs_setup first");
    HDG_REQUIRE(nb >= 1 && nb <= c->opt.max_rhs && nb <= DGS_MAX_RHS, "nrhs must be in 1..max_rhs (at most 64)");
}

}  // namespace
}  // namespace hdg

using hdg::Error;

extern "C" int hdg_dgs_setup(hdg_ctx *c, const hdg_mesh *levels, int32_t n_levels, const int32_t *const *parents) {
    if (!c) return HDG_EINVAL;
    return hdg::guarded([&] {
        if (c->dgs_ready) return;
        HDG_REQUIRE(c->flux == HDG_FLUX_UPWIND, "the DG baseline is built for the upwind flux");
        HDG_REQUIRE(levels && n_levels >= 1, "levels must be given");
        const hdg_mesh &fine = levels[n_levels - 1];
        HDG_REQUIRE(fine.n_cell == c->n_cell && fine.n_vert == c->n_vert, "the finest level must be the context's mesh");
        HDG_HIP_CHECK(hipSetDevice(c->device));
        const int nk = c->n_cell, n = c->n, nc = c->nc, nt = c->nt, mr = c->opt.max_rhs;
        HDG_REQUIRE(mr <= hdg::DGS_MAX_RHS, "max_rhs must be at most 64");
        const size_t NK = (size_t)nk;
        auto dalloc = [&](size_t count) { return static_cast<double *>(hdg::ctx_alloc(c, count * sizeof(double))); };
        c->dgs_A = dalloc((size_t)nc * nc * NK);
        c->dgs_Bn = dalloc((size_t)nc * nt * NK);
        c->dgs_Auu_inv = dalloc((size_t)4 * n * n * NK);
        c->dgs_Sown_inv = dalloc((size_t)n * n * NK);
        c->dgs_Dinv = dalloc((size_t)2 * n * NK);
        double *d_beta = dalloc(2 * NK);
        int *d_err = static_cast<int *>(hdg::ctx_alloc(c, sizeof(int)));
        HDG_HIP_CHECK(hipMemset(d_err, 0, sizeof(int)));
        hipStream_t s = nullptr;
        hdg::CellParams cp{c->kappa, c->tau, c->dt, c->prm.f0, c->prm.omega, c->hscale, c->geom};
        hdg::launch_cell_condense(c->p, 1, nk, c->corners, c->ref, cp, nullptr, nullptr, nullptr, nullptr, d_err, s,
                                  c->dgs_A, c->dgs_Bn);
        hdg::check_kernel_launch();
#define LOCAL(P)                                                                                                   \
    hipLaunchKernelGGL(hdg::k_dgs_local<P>, dim3(nk), dim3(64), 0, s, nk, c->geom, c->tau, c->corners, c->dgs_A, \
                       c->dgs_Bn, c->dgs_Auu_inv, c->dgs_Sown_inv, c->dgs_Dinv, d_beta, d_err)
        switch (c->p) {
            case 1: LOCAL(1); break;
            case 2: LOCAL(2); break;
            default: LOCAL(3); break;
        }
#undef LOCAL
        hdg::check_kernel_launch();
        HDG_HIP_CHECK(hipDeviceSynchronize());
        int herr = 0;
        HDG_HIP_CHECK(hipMemcpy(&herr, d_err, sizeof(int), hipMemcpyDeviceToHost));
        if (herr) throw Error{HDG_EINVAL, "singular cell block in the DG baseline's preconditioner"};
        std::vector<double> beta(2 * NK);
        HDG_HIP_CHECK(hipMemcpy(beta.data(), d_beta, beta.size() * sizeof(double), hipMemcpyDeviceToHost));

        // Galerkin P1 hierarchy of S
        std::vector<hdg::P1Host> ops(n_levels);
        ops[n_levels - 1] = hdg::assemble_sc(fine, c->kappa, beta);
        for (int l = n_levels - 1; l > 0; --l) {
            HDG_REQUIRE(parents && parents[l], "parents[l] must be given for every level above the coarsest");
            ops[l - 1] = hdg::galerkin_coarsen(ops[l], parents[l], levels[l - 1].n_vert);
        }
        hdg::build_p1_levels(c, levels, parents, ops, c->dgs_lev, &c->dgs_coarse_inv);

        // vertex <-> cell incidence
        std::vector<int32_t> cv(fine.cell_vert, fine.cell_vert + 3 * NK);
        std::vector<int32_t> vrow(fine.n_vert + 1, 0), vcol(3 * NK);
        for (size_t q = 0; q < 3 * NK; ++q) vrow[cv[q] + 1]++;
        for (int v = 0; v < fine.n_vert; ++v) vrow[v + 1] += vrow[v];
        std::vector<int32_t> fill(vrow.begin(), vrow.end() - 1);
        for (size_t q = 0; q < 3 * NK; ++q) vcol[fill[cv[q]]++] = (int32_t)q;
        auto iupload = [&](const std::vector<int32_t> &v) {
            int32_t *p = static_cast<int32_t *>(hdg::ctx_alloc(c, v.size() * sizeof(int32_t)));
            HDG_HIP_CHECK(hipMemcpy(p, v.data(), v.size() * sizeof(int32_t), hipMemcpyHostToDevice));
            return p;
        };
        c->dgs_cvert = iupload(cv);
        c->dgs_vrow = iupload(vrow);
        c->dgs_vcol = iupload(vcol);

        // work buffers
        const size_t cellv = (size_t)nk * nc * mr;
        c->dgs_half = dalloc((size_t)c->n_facet * 2 * c->m * mr);
        c->dgs_lam = dalloc((size_t)c->n_facet * c->m * mr);
        c->dgs_tmp.clear();
        for (int i = 0; i < 12; ++i) c->dgs_tmp.push_back(dalloc(cellv));
        const int rs = hdg::restart_len(c);
        c->dgs_V = dalloc(cellv * (rs + 1));
        c->dgs_Z = dalloc(cellv * rs);
        c->dgs_red = dalloc((size_t)hdg::red_grid((int64_t)nk * nc, mr) * (rs + 1) * mr);
        c->dgs_out = dalloc((size_t)(rs + 1) * mr);
        c->dgs_coef = dalloc((size_t)(rs + 1) * mr);
        c->dgs_ready = true;

        // lambda_max of S_own^-1 S: 20 normalised power steps from the fixed start
        // vector v_i = frac(i * 2654435761 / 2^32) - 1/2 over the phi unknowns (i = K n + node)
        hdg::Dgs g{c, 1, s, (int64_t)nk * nc};
        std::vector<double> v0((size_t)nk * nc, 0.0);
        double nrm = 0.0;
        for (int K = 0; K < nk; ++K)
            for (int i = 0; i < n; ++i) {
                const uint64_t idx = (uint64_t)K * n + i;
                const double val = (double)((idx * 2654435761ull) % 4294967296ull) / 4294967296.0 - 0.5;
                v0[(size_t)K * nc + i] = val;
                nrm += val * val;
            }
        nrm = std::sqrt(nrm);
        for (double &x : v0) x /= nrm;
        double *pv = g.tmp(8), *pw = g.tmp(9), *pz = g.tmp(10);
        HDG_HIP_CHECK(hipMemcpy(pv, v0.data(), v0.size() * sizeof(double), hipMemcpyHostToDevice));
        hdg::lin(g, 1, 3, 0.0, nullptr, 0.0, nullptr, false, pz);
        double lam = 0.0;
        for (int it = 0; it < 20; ++it) {
            hdg::s_apply(g, pv, pw);
            hdg::block_mv(g, false, pw, pz);
            lam = std::sqrt(hdg::dots(g, 1, pz, 0, pz)[0]);
            hdg::lin(g, 0, 1, 1.0 / lam, pz, 0.0, nullptr, false, pv);
        }
        c->dgs_lmax = lam;
        HDG_HIP_CHECK(hipDeviceSynchronize());
    });
}

extern "C" int hdg_dgs_apply(hdg_ctx *c, int32_t nb, const double *x, double *y, void *stream) {
    if (!c) return HDG_EINVAL;
    return hdg::guarded([&] {
        hdg::check_vec(c, nb);
        HDG_REQUIRE(x && y && x != y, "x and y must be distinct non-NULL arrays");
        hdg::Dgs g{c, nb, reinterpret_cast<hipStream_t>(stream), (int64_t)c->n_cell * c->nc};
        hdg::dgs_apply(g, x, y);
    });
}

extern "C" int hdg_dgs_precondition(hdg_ctx *c, int32_t nb, const double *r, double *z, void *stream) {
    if (!c) return HDG_EINVAL;
    return hdg::guarded([&] {
        hdg::check_vec(c, nb);
        HDG_REQUIRE(r && z && r != z, "r and z must be distinct non-NULL arrays");
        hdg::Dgs g{c, nb, reinterpret_cast<hipStream_t>(stream), (int64_t)c->n_cell * c->nc};
        hdg::precondition(g, r, z);
    });
}

extern "C" int hdg_dgs_solve(hdg_ctx *c, int32_t nb, const double *r_cell, double *q_cell, hdg_solve_info *info,
                             void *stream) {
    if (!c) return HDG_EINVAL;
    int status = HDG_OK;
    const int rc = hdg::guarded([&] {
        hdg::check_vec(c, nb);
        HDG_REQUIRE(r_cell && q_cell && r_cell != q_cell, "r_cell and q_cell must be distinct non-NULL arrays");
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        const int64_t len = (int64_t)c->n_cell * c->nc;
        hdg::Dgs g{c, nb, s, len};
        const int rs = hdg::restart_len(c);
        const size_t vs = (size_t)len * nb;
        double *R = g.tmp(8), *X = g.tmp(9), *W = g.tmp(10);
        {
            const int64_t cnt = len * nb;
            hipLaunchKernelGGL(hdg::k_dgs_load, hdg::grid_for(cnt, 256), dim3(256), 0, s, c->n_cell, c->n, nb,
                               c->hscale, c->dgs_A, r_cell, R);
            hdg::check_kernel_launch();
        }
        hdg::lin(g, 0, 3, 0.0, nullptr, 0.0, nullptr, false, X);
        std::vector<double> bn = hdg::dots(g, 1, R, 0, R);
        for (double &v : bn) v = std::sqrt(v);
        std::vector<int> iters(nb, 0);
        std::vector<double> rel(nb, 1.0);
        int its = 0;
        bool done = false;
        while (!done) {
            // true residual
            hdg::dgs_apply(g, X, W);
            hdg::lin(g, 0, 3, 1.0, R, -1.0, W, false, c->dgs_V);
            std::vector<double> beta = hdg::dots(g, 1, c->dgs_V, 0, c->dgs_V);
            bool all = true;
            for (int r = 0; r < nb; ++r) {
                beta[r] = std::sqrt(beta[r]);
                rel[r] = bn[r] > 0 ? beta[r] / bn[r] : 0.0;
                all = all && rel[r] <= c->opt.rtol;
            }
            if (all || its >= c->opt.maxit) break;
            std::vector<double> inv(nb);
            for (int r = 0; r < nb; ++r) inv[r] = beta[r] > 0 ? 1.0 / beta[r] : 0.0;
            hdg::scale_cols(g, inv, c->dgs_V, c->dgs_V);
            // Arnoldi with per-RHS Givens rotations (host)
            std::vector<double> H((size_t)(rs + 1) * rs * nb, 0.0), cs((size_t)rs * nb), sn((size_t)rs * nb),
                gvec((size_t)(rs + 1) * nb, 0.0);
            for (int r = 0; r < nb; ++r) gvec[r] = beta[r];
            auto Hat = [&](int i, int k, int r) -> double & { return H[((size_t)i * rs + k) * nb + r]; };
            int k = 0;
            for (; k < rs && its < c->opt.maxit; ++k) {
                double *Vk = c->dgs_V + (size_t)k * vs, *Zk = c->dgs_Z + (size_t)k * vs, *Vn = c->dgs_V + (size_t)(k + 1) * vs;
                hdg::precondition(g, Vk, Zk);
                hdg::dgs_apply(g, Zk, Vn);
                // classical Gram-Schmidt, twice
                for (int pass = 0; pass < 2; ++pass) {
                    std::vector<double> h = hdg::dots(g, k + 1, c->dgs_V, (int64_t)vs, Vn);
                    std::vector<double> mh(h.size());
                    for (size_t q = 0; q < h.size(); ++q) mh[q] = -h[q];
                    hdg::lincomb(g, k + 1, mh, c->dgs_V, (int64_t)vs, Vn);
                    for (int j = 0; j <= k; ++j)
                        for (int r = 0; r < nb; ++r) Hat(j, k, r) += h[(size_t)j * nb + r];
                }
                std::vector<double> hn = hdg::dots(g, 1, Vn, 0, Vn);
                std::vector<double> ih(nb);
                for (int r = 0; r < nb; ++r) {
                    hn[r] = std::sqrt(hn[r]);
                    Hat(k + 1, k, r) = hn[r];
                    ih[r] = hn[r] > 0 ? 1.0 / hn[r] : 0.0;
                }
                hdg::scale_cols(g, ih, Vn, Vn);
                ++its;
                bool conv = true;
                for (int r = 0; r < nb; ++r) {
                    for (int j = 0; j < k; ++j) {
                        const double a = Hat(j, k, r), b = Hat(j + 1, k, r);
                        Hat(j, k, r) = cs[(size_t)j * nb + r] * a + sn[(size_t)j * nb + r] * b;
                        Hat(j + 1, k, r) = -sn[(size_t)j * nb + r] * a + cs[(size_t)j * nb + r] * b;
                    }
                    const double a = Hat(k, k, r), b = Hat(k + 1, k, r);
                    const double d = std::hypot(a, b);
                    const double cc = d > 0 ? a / d : 1.0, ss = d > 0 ? b / d : 0.0;
                    cs[(size_t)k * nb + r] = cc;
                    sn[(size_t)k * nb + r] = ss;
                    Hat(k, k, r) = d;
                    Hat(k + 1, k, r) = 0.0;
                    gvec[(size_t)(k + 1) * nb + r] = -ss * gvec[(size_t)k * nb + r];
                    gvec[(size_t)k * nb + r] = cc * gvec[(size_t)k * nb + r];
                    if (std::fabs(gvec[(size_t)(k + 1) * nb + r]) > c->opt.rtol * bn[r]) conv = false;
                    if (std::fabs(gvec[(size_t)(k + 1) * nb + r]) <= c->opt.rtol * bn[r] && iters[r] == 0) iters[r] = its;
                }
                if (conv) {
                    ++k;
                    break;
                }
            }
            // x += Z y, y from the triangular system per RHS
            std::vector<double> y((size_t)k * nb, 0.0);
            for (int r = 0; r < nb; ++r)
                for (int i = k - 1; i >= 0; --i) {
                    double v = gvec[(size_t)i * nb + r];
                    for (int j = i + 1; j < k; ++j) v -= Hat(i, j, r) * y[(size_t)j * nb + r];
                    y[(size_t)i * nb + r] = Hat(i, i, r) != 0.0 ? v / Hat(i, i, r) : 0.0;
                }
            hdg::lincomb(g, k, y, c->dgs_Z, (int64_t)vs, X);
            if (its >= c->opt.maxit) {
                hdg::dgs_apply(g, X, W);
                hdg::lin(g, 0, 3, 1.0, R, -1.0, W, false, c->dgs_V);
                std::vector<double> b2 = hdg::dots(g, 1, c->dgs_V, 0, c->dgs_V);
                for (int r = 0; r < nb; ++r) rel[r] = bn[r] > 0 ? std::sqrt(b2[r]) / bn[r] : 0.0;
                done = true;
            }
        }
        // q = (phi / hscale, u)
        hdg::lin(g, 0, 1, 1.0 / c->hscale, X, 0.0, nullptr, false, q_cell);
        hdg::lin(g, 1, 3, 1.0, X, 0.0, nullptr, false, q_cell);
        HDG_HIP_CHECK(hipStreamSynchronize(s));
        for (int r = 0; r < nb; ++r) {
            const bool ok = rel[r] <= c->opt.rtol;
            if (!ok) status = HDG_ENOTCONV;
            if (info) {
                info[r].iters = iters[r] ? iters[r] : its;
                info[r].refinements = 0;
                info[r].fallbacks = 0;
                info[r].status = ok ? HDG_OK : HDG_ENOTCONV;
                info[r].rel_res = rel[r];
            }
        }
    });
    if (rc != HDG_OK) return rc;
    return status;
}
