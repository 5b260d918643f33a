// Device kernels of the HDG trace-multigrid library, written for gfx950
// (64-wide wavefronts).  Layout conventions:
//   per-cell matrices  component-major [row][col][n_cell]  (lanes = cells, coalesced)
//   facet block rows   component-major [slot][a][b][n_facet]
//   vectors            [item][dof][nrhs]  (RHS innermost)
#include <algorithm>
#include <type_traits>

#include "hdg_device.h"
#include "hdg_kernels.h"

namespace hdg {

// ------------------------------------------------------------------ setup: per-cell condensation
//
// Two cells per wavefront: each 32-lane half takes a cell, a lane per row of
// the local system, the row held in registers.  The local HDG blocks (Eq.
// ABCMform) are assembled from reference-element tables and the cell's affine map:
//   A = [[M + k t sum_f E_f,  k G_1,  k G_2],
//        [-k G_1^T,           M,     -dt Mf],
//        [-k G_2^T,           dt Mf,  M   ]]
//   B = [-k t T_f ; k n_f1 T_f ; k n_f2 T_f],   C = [t T_f^T, n_f1 T_f^T, n_f2 T_f^T],
//   Mt = t F_f (block diagonal),
// with k = kappa, t = tau, G_d[i][j] = (d_d phi_j, phi_i), E_f / T_f / F_f the
// facet mass / facet-trace / trace mass on local facet f.  (This is the HDG
// form of Eq. bilinear_HDG_upwind after integrating the volume flux term by
// parts.)  [A | B | Mtilde] is reduced by Gauss-Jordan with partial pivoting
// across the lanes of the half, giving W = A^-1 B and A^-1 Mtilde, then
// S_K = Mt + C W (Step 2 operator) and C A^-1 Mtilde (Step 1 map) are formed.
//
// NU = 2: the Lax-Friedrichs form (Eq. bilinear_HDG_lax) with the vector
// trace uhat, local trace unknown (f, d, k) at f*2m + d*m + k:
//   A = [[M,                    -k G_1^T,          -k G_2^T        ],
//        [-k G_1 + k n_f1 E_f,   M + k t sum_f E_f, -dt Mf          ],
//        [-k G_2 + k n_f2 E_f,   dt Mf,             M + k t sum_f E_f]]
//   (G_d^T[i][j] = (phi_j, d_d phi_i): the psi row keeps -k (u, grad psi)),
//   B = [k n_fd T_f ; -k t T_f on component d],  C = [n_fd T_f^T, t T_f^T on
//   component d],  Mt = t F_f per facet and component.

constexpr int CONDENSE_XB = 14;   // solution columns staged per round of the products

// DPP lane moves (all lanes have a source): xor 1 and xor 2 within a quad,
// lane i <-> 7 - i within 8, lane i <-> 15 - i within 16
constexpr int DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_HALF_MIRROR = 0x141, DPP_MIRROR = 0x140;
template <int CTRL>
__device__ __forceinline__ int dpp_i32(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)dpp_i32<CTRL>((int)b), hi = (unsigned)dpp_i32<CTRL>((int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// one of three per-facet values without indexing a register array at run time
__device__ __forceinline__ double facet_sel(const double (&v)[3], int f) { return f == 0 ? v[0] : (f == 1 ? v[1] : v[2]); }

template <int P, int NU>
__global__ __launch_bounds__(64) void k_cell_condense(int nk, const double *__restrict__ corners,
                                                      const double *__restrict__ ref, CellParams cp,
                                                      double *__restrict__ Sloc, double *__restrict__ Zr,
                                                      double *__restrict__ Ar, double *__restrict__ Wr,
                                                      int *__restrict__ err, double *__restrict__ Aout,
                                                      double *__restrict__ Bnout) {
    constexpr int n = (P + 1) * (P + 2) / 2, m = P + 1, nc = 3 * n, M = NU * m, nt = 3 * M, nq = (P + 3) * (P + 3);
    constexpr int LD = nc + nt + nc, NX = nt + nc, XB = CONDENSE_XB, NR = (NX + XB - 1) / XB, ZW = cell_zw(P);
    static_assert(nc <= 32, "a 32-lane half holds the rows of a cell");
    // pool: the reference tables and basis values while the rows are assembled,
    // then the pivot rows [2][LD] and a round of solution columns [2][nc][XB]
    constexpr int TAB = 6 * n * n + 3 * n * m, POOL_A = TAB + nq * n, POOL_B = 2 * LD + 2 * nc * XB;
    __shared__ double pool[POOL_A > POOL_B ? POOL_A : POOL_B];
    __shared__ double fq[2][nq];
    __shared__ double Mf[2][n * n];   // (f phi_j, phi_i)_K
    __shared__ double Cm[2][nt * nc];
    double *const tM = pool, *const tG = tM + n * n, *const tE = tG + 2 * n * n, *const tT = tE + 3 * n * n;
    double *const sphi = pool + TAB;   // reference basis values at the quadrature points
    const int lane = threadIdx.x, h = lane >> 5, r = lane & 31;
    double *const prow = pool + h * LD;   // this half's pivot row (set by the lane that takes it)
    auto xs = [&](int row, int u) -> double & { return pool[2 * LD + (h * nc + row) * XB + u]; };
    // each XCD takes a contiguous range of cell pairs, so the outputs (component-major,
    // cells fastest) of neighbouring cells meet in one L2 before they are written back
    const int pair = xcd_block();
    if (2 * pair >= nk) return;   // the whole wavefront
    const bool live = 2 * pair + h < nk;
    const int K = live ? 2 * pair + h : nk - 1;   // a spare half repeats the last cell and writes nothing

    const double *rM = ref;
    const double *rF = rM + 6 * n * n + 3 * n * m;
    const double *rq = rF + m * m;
    const double *rw = rq + 2 * nq;
    const double *rPhi = rw + nq;
    for (int t = lane; t < TAB + nq * n; t += 64) pool[t] = t < TAB ? rM[t] : rPhi[t - TAB];   // M, G, E, T; basis

    // ---- geometry of the flat cell
    const double *X = corners + 9 * (size_t)K;
    double ab[3], ac[3];
    for (int d = 0; d < 3; ++d) {
        ab[d] = X[3 + d] - X[d];
        ac[d] = X[6 + d] - X[d];
    }
    double e1[3], e2[3];
    if (cp.geom == HDG_TORUS) {
        e1[0] = 1; e1[1] = 0; e1[2] = 0;
        e2[0] = 0; e2[1] = 1; e2[2] = 0;
    } else {
        double kn[3] = {ab[1] * ac[2] - ab[2] * ac[1], ab[2] * ac[0] - ab[0] * ac[2], ab[0] * ac[1] - ab[1] * ac[0]};
        double il = 1.0 / sqrt(kn[0] * kn[0] + kn[1] * kn[1] + kn[2] * kn[2]);
        for (int d = 0; d < 3; ++d) kn[d] *= il;
        double la = 1.0 / sqrt(ab[0] * ab[0] + ab[1] * ab[1] + ab[2] * ab[2]);
        for (int d = 0; d < 3; ++d) e1[d] = ab[d] * la;
        e2[0] = kn[1] * e1[2] - kn[2] * e1[1];
        e2[1] = kn[2] * e1[0] - kn[0] * e1[2];
        e2[2] = kn[0] * e1[1] - kn[1] * e1[0];
    }
    const double Pbx = ab[0] * e1[0] + ab[1] * e1[1] + ab[2] * e1[2];
    const double Pby = ab[0] * e2[0] + ab[1] * e2[1] + ab[2] * e2[2];
    const double Pcx = ac[0] * e1[0] + ac[1] * e1[1] + ac[2] * e1[2];
    const double Pcy = ac[0] * e2[0] + ac[1] * e2[1] + ac[2] * e2[2];
    const double det = Pbx * Pcy - Pby * Pcx;
    const bool det_ok = det > 0.0;   // otherwise the cell is reported and nothing of it written
    // Jinv[r][d] = d xi_r / d x_d
    const double J00 = Pcy / det, J01 = -Pcx / det, J10 = -Pby / det, J11 = Pbx / det;
    double L[3], nx[3], ny[3];
    {
        const double Px[3] = {0.0, Pbx, Pcx}, Py[3] = {0.0, Pby, Pcy};
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            double tx = Px[(f + 2) % 3] - Px[(f + 1) % 3], ty = Py[(f + 2) % 3] - Py[(f + 1) % 3];
            L[f] = sqrt(tx * tx + ty * ty);
            nx[f] = ty / L[f];
            ny[f] = -tx / L[f];
        }
    }
    const double kap = cp.kappa, tau = cp.tau, dt = cp.dt;
    for (int q = r; q < nq; q += 32) {
        double f = cp.f0;
        if (cp.geom == HDG_SPHERE && cp.omega != 0.0) {
            double x0 = X[0] + rq[2 * q] * ab[0] + rq[2 * q + 1] * ac[0];
            double x1 = X[1] + rq[2 * q] * ab[1] + rq[2 * q + 1] * ac[1];
            double x2 = X[2] + rq[2 * q] * ab[2] + rq[2 * q + 1] * ac[2];
            f += 2.0 * cp.omega * x2 / sqrt(x0 * x0 + x1 * x1 + x2 * x2);
        }
        fq[h][q] = f * rw[q];
    }
    __syncthreads();
    for (int t = r; t < n * n; t += 32) {
        const int i = t / n, j = t - (t / n) * n;
        double mf = 0.0;
        for (int q = 0; q < nq; ++q) mf += fq[h][q] * sphi[q * n + i] * sphi[q * n + j];
        Mf[h][t] = mf * det;
    }
    for (int idx = r; idx < nt * nc; idx += 32) {
        const int row = idx / nc, col = idx % nc;
        const int f = row / M, d = (row % M) / m, k = row % m, fc = col / n, j = col % n;
        const double t = facet_sel(L, f) * tT[f * n * m + j * m + k];
        if constexpr (NU == 1)
            Cm[h][idx] = fc == 0 ? tau * t : (fc == 1 ? facet_sel(nx, f) : facet_sel(ny, f)) * t;
        else
            Cm[h][idx] = fc == 0 ? (d == 0 ? facet_sel(nx, f) : facet_sel(ny, f)) * t : (fc == d + 1 ? tau * t : 0.0);
    }
    __syncthreads();

    // ---- row r of [A | B | Mtilde] of this half's cell, in registers
    const bool row_ok = r < nc;
    const int fr = row_ok ? r / n : 0, i = row_ok ? r % n : 0;
    // (d_d phi_jj, phi_ii)_K / det for d = 0, 1
    auto grad_ij = [&](int d, int ii, int jj) {
        const double c0 = d == 0 ? J00 : J01, c1 = d == 0 ? J10 : J11;
        return c0 * tG[ii * n + jj] + c1 * tG[n * n + ii * n + jj];
    };
    auto entry = [&](int col) -> double {
        double v = 0.0;
        if (col < nc) {
            const int fc = col / n, j = col % n;
            if constexpr (NU == 1) {
                if (fr == 0 && fc == 0) {
                    v = det * tM[i * n + j];
                    for (int f = 0; f < 3; ++f) v += kap * tau * L[f] * tE[f * n * n + i * n + j];
                } else if (fr == 0) {
                    v = kap * det * grad_ij(fc - 1, i, j);
                } else if (fc == 0) {
                    v = -kap * det * grad_ij(fr - 1, j, i);
                } else if (fr == fc) {
                    v = det * tM[i * n + j];
                } else {
                    v = (fr == 1) ? -dt * Mf[h][i * n + j] : dt * Mf[h][i * n + j];
                }
            } else {
                if (fr == 0 && fc == 0) {
                    v = det * tM[i * n + j];
                } else if (fr == 0) {
                    v = -kap * det * grad_ij(fc - 1, j, i);
                } else if (fc == 0) {
                    v = -kap * det * grad_ij(fr - 1, j, i);
                    for (int f = 0; f < 3; ++f)
                        v += kap * (fr == 1 ? nx[f] : ny[f]) * L[f] * tE[f * n * n + i * n + j];
                } else if (fr == fc) {
                    v = det * tM[i * n + j];
                    for (int f = 0; f < 3; ++f) v += kap * tau * L[f] * tE[f * n * n + i * n + j];
                } else {
                    v = (fr == 1) ? -dt * Mf[h][i * n + j] : dt * Mf[h][i * n + j];
                }
            }
        } else if (col < nc + nt) {
            const int c = col - nc, f = c / M, d = (c % M) / m, k = c % m;
            const double t = L[f] * tT[f * n * m + i * m + k];
            if constexpr (NU == 1)
                v = fr == 0 ? -kap * tau * t : kap * (fr == 1 ? nx[f] : ny[f]) * t;
            else
                v = fr == 0 ? kap * (d == 0 ? nx[f] : ny[f]) * t : (fr == d + 1 ? -kap * tau * t : 0.0);
        } else {
            const int c = col - nc - nt, fc = c / n, j = c % n;
            if (fc == fr) v = (fr == 0 ? cp.hscale : 1.0) * det * tM[i * n + j];
        }
        return v;
    };
    double a[LD];
#pragma unroll
    for (int c = 0; c < LD; ++c) a[c] = row_ok ? entry(c) : 0.0;
    __syncthreads();   // the tables are done with: the pool now holds pivot rows

    const size_t NK = (size_t)nk;
    if (Aout) {   // store A and -B only (the standard DG operator is A q + B lam(q))
        if (live && det_ok && row_ok) {
#pragma unroll
            for (int c = 0; c < nc; ++c) Aout[(size_t)(r * nc + c) * NK + K] = a[c];
#pragma unroll
            for (int c = 0; c < nt; ++c) Bnout[(size_t)(r * nt + c) * NK + K] = -a[nc + c];
        }
        if (live && !det_ok && r == 0) atomicOr(err, 1);
        return;
    }

    // ---- Gauss-Jordan with partial pivoting.  Rows stay in their lanes: the
    // pivot of column k is the unused row of largest magnitude (lowest row on
    // ties), found by a reduction over the half (DPP moves within 16 lanes,
    // then one exchange between the 16-lane rows); its lane posts its row and
    // the pivot's reciprocal ip, and every other row is eliminated with the
    // scaled row, the factor ip folded into its multiplier.  The pivot's lane
    // keeps its row unscaled with the factor beside it (myip): later
    // eliminations of that row are the same either way.  The lane that took
    // pivot k then holds row k of A^-1 [A | B | Mtilde] divided by myip.
    // Columns <= k are not read again once pivot k is taken.
    bool used = !row_ok, bad = false;
    int myk = -1;
    double myip = 1.0;
#pragma unroll
    for (int k = 0; k < nc; ++k) {
        const double ip = 1.0 / a[k];   // every lane: the pivot's lane is not known yet
        double best = used ? -1.0 : fabs(a[k]);
        int bl = r;
        // (value, row) pairs ordered by value, then by lower row: the
        // combination is associative and commutative, so any pairing works
        auto take = [&](double ob, int ol) {
            if (ob > best || (ob == best && ol < bl)) {
                best = ob;
                bl = ol;
            }
        };
        take(dpp_f64<DPP_XOR1>(best), dpp_i32<DPP_XOR1>(bl));
        take(dpp_f64<DPP_XOR2>(best), dpp_i32<DPP_XOR2>(bl));
        take(dpp_f64<DPP_HALF_MIRROR>(best), dpp_i32<DPP_HALF_MIRROR>(bl));
        take(dpp_f64<DPP_MIRROR>(best), dpp_i32<DPP_MIRROR>(bl));
        take(__shfl_xor(best, 16, 64), __shfl_xor(bl, 16, 64));
        bad |= !(best > 0.0);
        if (r == bl) {
#pragma unroll
            for (int c = k + 1; c < LD; ++c) prow[c] = a[c];
            prow[k] = ip;
            used = true;
            myk = k;
            myip = ip;
        }
        __syncthreads();
        if (r != bl) {   // (a branch, not a zero multiplier: it keeps the register count down)
            const double g = a[k] * prow[k];
#pragma unroll
            for (int c = k + 1; c < LD; ++c) a[c] -= g * prow[c];
        }
        __syncthreads();
    }
    const bool hbad = ((__ballot(bad) >> (32 * h)) & 0xffffffffull) != 0;
    if (live && r == 0) {
        if (!det_ok) atomicOr(err, 1);
        else if (hbad) atomicOr(err, 2);
    }
    const bool ok = live && det_ok && !hbad;

    // ---- outputs: A^-1 Mtilde and W = A^-1 B (scaled back to the unscaled
    // depth unknown) from the registers, then S_K = Mt + C W and C A^-1 Mtilde
    // from the solution staged through LDS a round of columns at a time
    const double ih = 1.0 / cp.hscale;
    if (ok && myk >= 0) {
        const double sc = myk < n ? ih : 1.0;
#pragma unroll
        for (int b = 0; b < nc; ++b) Ar[(size_t)(myk * nc + b) * NK + K] = sc * (myip * a[nc + nt + b]);
#pragma unroll
        for (int b = 0; b < nt; ++b) Wr[(size_t)(myk * nt + b) * NK + K] = sc * (myip * a[nc + b]);
    }
#pragma unroll
    for (int rho = 0; rho < NR; ++rho) {
        const int lo = rho * XB, hi = lo + XB < NX ? lo + XB : NX;
        __syncthreads();
        if (myk >= 0) {
#pragma unroll
            for (int u = 0; u < XB; ++u)
                if (lo + u < hi) xs(myk, u) = myip * a[nc + lo + u];
        }
        __syncthreads();
        if (!ok) continue;
        if (lo < nt) {   // S_K columns [lo, min(hi, nt))
            const int b1 = hi < nt ? hi : nt, w = b1 - lo;
            for (int t = r; t < nt * w; t += 32) {
                const int aa = t / w, b = lo + t % w;
                double s = 0.0;
                if (aa / m == b / m) s = tau * facet_sel(L, aa / M) * rF[(aa % m) * m + (b % m)];   // same facet and component
                for (int j = 0; j < nc; ++j) s += Cm[h][aa * nc + j] * xs(j, b - lo);
                Sloc[(size_t)(aa * nt + b) * NK + K] = s;
            }
        }
        if (hi > nt) {   // C A^-1 Mtilde columns [max(lo, nt), hi) - nt, rows padded to ZW, 16-byte pairs
            const int x0 = lo > nt ? lo : nt, w = hi - x0;
            for (int t = r; t < nt * w; t += 32) {
                const int aa = t / w, b = x0 - nt + t % w;
                double s = 0.0;
                for (int j = 0; j < nc; ++j) s += Cm[h][aa * nc + j] * xs(j, nt + b - lo);
                const int idx = aa * ZW + b;
                Zr[((size_t)(idx / 2) * NK + K) * 2 + idx % 2] = s;
            }
        }
    }
    if constexpr (ZW > nc) {
        for (int t = r; ok && t < nt * (ZW - nc); t += 32) {
            const int idx = (t / (ZW - nc)) * ZW + nc + t % (ZW - nc);
            Zr[((size_t)(idx / 2) * NK + K) * 2 + idx % 2] = 0.0;
        }
    }
}

// ------------------------------------------------------------------ setup: facet block rows
//
// Row block of facet e: S restricted to (e, e') for the five facets e' of the
// two cells adjacent to e.  The diagonal block sums both cells'
// contributions; the four off-diagonal slots hold the other two facets of the
// owner cell, then of the second cell.  Also forms omega D_e^-1 and
// omega D_e^-1 S_{e,j} used by the block-Jacobi sweep.

template <int M>
__device__ bool small_inverse(double (&a)[M][M], double (&inv)[M][M]) {
    for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) inv[i][j] = i == j ? 1.0 : 0.0;
    for (int k = 0; k < M; ++k) {
        int p = k;
        for (int i = k + 1; i < M; ++i)
            if (fabs(a[i][k]) > fabs(a[p][k])) p = i;
        if (!(fabs(a[p][k]) > 0.0)) return false;
        if (p != k)
            for (int j = 0; j < M; ++j) {
                double t = a[k][j]; a[k][j] = a[p][j]; a[p][j] = t;
                t = inv[k][j]; inv[k][j] = inv[p][j]; inv[p][j] = t;
            }
        double d = 1.0 / a[k][k];
        for (int j = 0; j < M; ++j) { a[k][j] *= d; inv[k][j] *= d; }
        for (int i = 0; i < M; ++i) {
            if (i == k) continue;
            double f = a[i][k];
            for (int j = 0; j < M; ++j) { a[i][j] -= f * a[k][j]; inv[i][j] -= f * inv[k][j]; }
        }
    }
    return true;
}

template <int P, int NU>
__global__ void k_facet_rows(int ne, int nk, const double *__restrict__ Sloc, const int *__restrict__ facet_cell,
                             const int *__restrict__ facet_loc, const int *__restrict__ cell_facet,
                             const int8_t *__restrict__ cell_rev, double omega, double *__restrict__ S64,
                             double *__restrict__ T64, double *__restrict__ Dw64, float *__restrict__ S32,
                             __hip_bfloat16 *__restrict__ T16, float *__restrict__ Dw32, int *__restrict__ nbr,
                             int8_t *__restrict__ prev, int *__restrict__ err) {
    constexpr int m = P + 1, M = NU * m, nt = 3 * M;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const size_t NK = (size_t)nk, NE = (size_t)ne;
    // diagonal block: both cells' contributions
    double D[M][M] = {};
    for (int s = 0; s < 2; ++s) {
        const int K = facet_cell[2 * e + s], i = facet_loc[2 * e + s];
        for (int a = 0; a < M; ++a) {
            const int ra = loc_trace<P, NU>(i, a, s);
            for (int b = 0; b < M; ++b) D[a][b] += Sloc[(size_t)(ra * nt + loc_trace<P, NU>(i, b, s)) * NK + K];
        }
    }
    double Dc[M][M], Di[M][M];
    for (int a = 0; a < M; ++a)
        for (int b = 0; b < M; ++b) Dc[a][b] = D[a][b];
    if (!small_inverse<M>(Dc, Di)) {
        atomicOr(err, 4);
        return;
    }
    for (int a = 0; a < M; ++a)
        for (int b = 0; b < M; ++b) {
            const int c = a * M + b;
            S64[widx(c, e, NE, 2)] = D[a][b];
            S32[widx(c, e, NE, 4)] = (float)D[a][b];
            Dw64[widx(c, e, NE, 2)] = omega * Di[a][b];
            Dw32[widx(c, e, NE, 4)] = (float)(omega * Di[a][b]);
        }
    // off-diagonal slots j = 2 s + jj - 1: the other two facets of the owner, then of the second cell
    for (int s = 0; s < 2; ++s) {
        const int K = facet_cell[2 * e + s], i = facet_loc[2 * e + s];
        for (int jj = 1; jj < 3; ++jj) {
            const int j = 2 * s + jj - 1;
            const int i2 = (i + jj) % 3;
            const int e2 = cell_facet[i2 * NK + K];
            const int rev2 = cell_rev[i2 * NK + K];
            nbr[j * NE + e] = e2;
            // learned-smoother patch: list this slot's nodes counter-clockwise around cell K
            prev[j * NE + e] = (int8_t)rev2;
            double Off[M][M];
            for (int a = 0; a < M; ++a) {
                const int ra = loc_trace<P, NU>(i, a, s);
                for (int b = 0; b < M; ++b)
                    Off[a][b] = Sloc[(size_t)(ra * nt + loc_trace<P, NU>(i2, b, rev2)) * NK + K];
            }
            for (int a = 0; a < M; ++a)
                for (int b = 0; b < M; ++b) {
                    double t = 0.0;
                    for (int c = 0; c < M; ++c) t += Di[a][c] * Off[c][b];
                    const int cs = ((j + 1) * M + a) * M + b;
                    const int ct = (j * M + a) * M + b;
                    S64[widx(cs, e, NE, 2)] = Off[a][b];
                    S32[widx(cs, e, NE, 4)] = (float)Off[a][b];
                    T64[widx(ct, e, NE, 2)] = omega * t;
                    T16[widx(ct, e, NE, 8)] = __float2bfloat16((float)(omega * t));
                }
        }
    }
    // zero the padding up to a whole 16-byte group
    for (int c = 5 * M * M; c < padded(5 * M * M, 4); ++c) {
        if (c < padded(5 * M * M, 2)) S64[widx(c, e, NE, 2)] = 0.0;
        S32[widx(c, e, NE, 4)] = 0.f;
    }
    for (int c = M * M; c < padded(M * M, 4); ++c) {
        if (c < padded(M * M, 2)) Dw64[widx(c, e, NE, 2)] = 0.0;
        Dw32[widx(c, e, NE, 4)] = 0.f;
    }
    for (int c = 4 * M * M; c < padded(4 * M * M, 8); ++c) {
        if (c < padded(4 * M * M, 2)) T64[widx(c, e, NE, 2)] = 0.0;
        T16[widx(c, e, NE, 8)] = __float2bfloat16(0.f);
    }
}

// ------------------------------------------------------------------ trace-level operators
//
// Pull formulation: each (facet, RHS) thread gathers the trace values of the
// five facets of its block row and produces all m rows, so every matrix
// entry is read exactly once per apply and there are no write conflicts.

template <int M, typename MT, typename XT, typename YT, bool NB1, typename BT = YT>
__global__ __launch_bounds__(256) void k_trace_apply(int ne, int nb, const MT *__restrict__ S,
                                                     const int *__restrict__ nbr, const XT *__restrict__ x,
                                                     const BT *__restrict__ b, YT *__restrict__ y) {
    using AT = typename Acc<MT>::type;
    constexpr int V = Wide<MT>::V, C = 5 * M * M, G = padded(C, V) / V;
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= ne * nb) return;
    const int e = NB1 ? t : t / nb, r = NB1 ? 0 : t - e * nb;
    const size_t NE = (size_t)ne, MB = (size_t)M * (NB1 ? 1 : nb);
    int id[5];
    id[0] = e;
#pragma unroll
    for (int j = 0; j < 4; ++j) id[j + 1] = nbr[j * NE + e];
    double xd[5][M];
#pragma unroll
    for (int j = 0; j < 5; ++j) load_trace<M, NB1>(x, id[j] * MB + r, nb, xd[j]);
    AT acc[M];
#pragma unroll
    for (int a = 0; a < M; ++a) acc[a] = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        AT w[V];
        Wide<MT>::load(S + ((size_t)g * NE + e) * V, w);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int c = g * V + v;
            if (c < C) {
                const int j = c / (M * M), a = (c / M) % M, k = c % M;
                acc[a] += w[v] * (AT)xd[j][k];
            }
        }
    }
    double out[M];
    if (b) {   // residual b - S x
        double bv[M];
        load_trace<M, NB1>(b, e * MB + r, nb, bv);
#pragma unroll
        for (int a = 0; a < M; ++a) out[a] = bv[a] - (double)acc[a];
    } else {
#pragma unroll
        for (int a = 0; a < M; ++a) out[a] = (double)acc[a];
    }
    store_trace<M, NB1>(y, e * MB + r, nb, out);
}

// z0 = omega D^-1 r  (first sweep from a zero guess).  With scale != nullptr
// the input is r / scale[rhs], and the scaled input is also written to rs
// (normalisation of a Krylov basis vector fused into its first use).
// rc (may be null): a copy of the scaled input in z0's type
template <int M, typename MT, typename RT, typename ZT>
__global__ __launch_bounds__(256) void k_jacobi0(int ne, int nb, const MT *__restrict__ Dw,
                                                 const RT *__restrict__ r, const double *__restrict__ scale,
                                                 RT *__restrict__ rs, ZT *__restrict__ rc, ZT *__restrict__ z0,
                                                 GsLag gs) {
    using AT = typename Acc<MT>::type;
    constexpr int V = Wide<MT>::V, C = M * M, G = padded(C, V) / V;
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= ne * nb) return;
    const int e = t / nb, rr = t - e * nb;
    const size_t NE = (size_t)ne;
    double rv[M];
    const double sc = scale ? (scale[rr] != 0.0 ? 1.0 / scale[rr] : 0.0) : 1.0;
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const size_t o = ((size_t)e * M + k) * nb + rr;
        double rk = (double)r[o];
        const int gnd = (gs.done && *gs.done) ? 0 : gs.nd;
        for (int d = 0; d < gnd; ++d)
            rk -= gs.h[(size_t)d * nb + rr] * (double)static_cast<const RT *>(gs.V)[(size_t)d * gs.vstride + o];
        const RT v = (RT)(rk * sc);             // the scaled vector as stored
        if (scale) rs[o] = v;
        const ZT vz = (ZT)v;                    // ... and as the V-cycle reads it
        if (rc) rc[o] = vz;
        rv[k] = (double)vz;
    }
    AT acc[M];
#pragma unroll
    for (int a = 0; a < M; ++a) acc[a] = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        AT w[V];
        Wide<MT>::load(Dw + ((size_t)g * NE + e) * V, w);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int c = g * V + v;
            if (c < C) acc[c / M] += w[v] * (AT)rv[c % M];
        }
    }
#pragma unroll
    for (int a = 0; a < M; ++a) z0[((size_t)e * M + a) * nb + rr] = (ZT)(double)acc[a];
}

// Block-Jacobi sweep  y = x + omega D^-1 (r - S x) = (1 - omega) x + z0 - sum_j T_j x_j,
// with T_j = omega D^-1 S_j over the four off-diagonal slots and z0 = omega D^-1 r.
// With qc != nullptr the input is x + pi qc (prolongation of the P1 correction
// fused in, pi the injection of a P1 function onto the trace nodes).
template <int M, typename MT, typename VT, bool NB1>
__global__ __launch_bounds__(256) void k_sweep(int ne, int nb, const MT *__restrict__ T,
                                               const int *__restrict__ nbr, const VT *__restrict__ x,
                                               const VT *__restrict__ z0, const VT *__restrict__ qc,
                                               const int *__restrict__ fvert, SweepCoef cf,
                                               VT *__restrict__ y) {
    using AT = typename Acc<MT>::type;
    using CT = SweepT<VT>;
    constexpr int P = M - 1;
    constexpr int V = Wide<MT>::V, C = 4 * M * M, G = padded(C, V) / V;
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= ne * nb) return;
    const int e = NB1 ? t : t / nb, r = NB1 ? 0 : t - e * nb;
    const size_t NE = (size_t)ne, MB = (size_t)M * (NB1 ? 1 : nb);
    int id[5];
    id[0] = e;
#pragma unroll
    for (int j = 0; j < 4; ++j) id[j + 1] = nbr[j * NE + e];
    CT xv[5][M];
#pragma unroll
    for (int j = 0; j < 5; ++j) {
        load_trace<M, NB1>(x, id[j] * MB + r, nb, xv[j]);
        if (qc) {
            const CT q0 = (CT)qc[(size_t)fvert[2 * id[j]] * nb + r];
            const CT q1 = (CT)qc[(size_t)fvert[2 * id[j] + 1] * nb + r];
#pragma unroll
            for (int k = 0; k < M; ++k) xv[j][k] += p1_node<P>(k, q0, q1);
        }
    }
    AT acc[M];
#pragma unroll
    for (int a = 0; a < M; ++a) acc[a] = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        AT w[V];
        Wide<MT>::load(T + ((size_t)g * NE + e) * V, w);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int c = g * V + v;
            if (c < C) {
                const int j = c / (M * M), a = (c / M) % M, k = c % M;
                acc[a] += w[v] * (AT)xv[j + 1][k];
            }
        }
    }
    CT zv[M], out[M];
    load_trace<M, NB1>(z0, e * MB + r, nb, zv);
#pragma unroll
    for (int a = 0; a < M; ++a) out[a] = sweep_combine(cf, xv[0][a], zv[a], (CT)acc[a]);
    if (cf.xprev) {
        CT pv[M];
        load_trace<M, NB1>(static_cast<const VT *>(cf.xprev), e * MB + r, nb, pv);
        if (cf.qcprev) {
            const VT *qp = static_cast<const VT *>(cf.qcprev);
            const CT q0 = (CT)qp[(size_t)fvert[2 * e] * nb + r], q1 = (CT)qp[(size_t)fvert[2 * e + 1] * nb + r];
#pragma unroll
            for (int a = 0; a < M; ++a) pv[a] += p1_node<P>(a, q0, q1);
        }
#pragma unroll
        for (int a = 0; a < M; ++a) out[a] = sweep_prev(cf.a2, pv[a], out[a]);
    }
    store_trace<M, NB1>(y, e * MB + r, nb, out);
}

// Restriction pi^T of a trace residual onto the P1 vertices:
// rc[v] = sum over facet ends at v of sum_k w_end(k) res[e][k], w_0 = 1 - k/p, w_1 = k/p.
// The facet ends of a vertex (5-7 on these meshes) are taken up to eight at a
// time with every load in flight together (index clamped into the list, the
// surplus ends not added; the sum keeps its order).
template <int M, typename VT>
__global__ void k_restrict_trace(int nv, int nb, const int *__restrict__ vf_row, const int *__restrict__ vf_col,
                                 const VT *__restrict__ res, VT *__restrict__ rc) {
    constexpr int P = M - 1, U = 8;
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= nv * nb) return;
    const int v = t / nb, r = t - v * nb;
    const int c0 = vf_row[v], cnt = vf_row[v + 1] - c0;
    double acc = 0.0;
    for (int k0 = 0; k0 < cnt; k0 += U) {
        int code[U];
        double val[U][M];
#pragma unroll
        for (int u = 0; u < U; ++u) code[u] = vf_col[c0 + min(k0 + u, cnt - 1)];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < M; ++k) val[u][k] = (double)res[((size_t)(code[u] >> 1) * M + k) * nb + r];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int end = code[u] & 1;
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const double w = end ? (double)k / P : 1.0 - (double)k / P;
                acc = k0 + u < cnt ? acc + w * val[u][k] : acc;
            }
        }
    }
    rc[(size_t)v * nb + r] = (VT)acc;
}

// ------------------------------------------------------------------ P1 levels
//
// Coarse problem S_c q = r_c of the upwind case, solved by one geometric
// multigrid V-cycle: damped Jacobi smoothing, linear-interpolation transfer
// from the nested hierarchy's parent map, dense inverse on the coarsest
// level.  Large levels run as one kernel per step; all levels with at most
// P1_TAIL_MAX vertices (and the dense solve) run inside one single-workgroup
// kernel, because at that size a launch costs more than the work.
// The per-level kernels hand each XCD one contiguous range of vertices, so the
// neighbour rows that nearby vertices share are fetched into one L2.

// Level matrices are stored off-diagonal in ELL form, [W][n] column-major
// (padding entries point at the row itself with value 0), so the neighbour
// indices of a row are independent coalesced loads.  WT > 0 fixes the width at
// compile time (6 on the icosahedral and torus meshes), so a row's loads are
// all issued before the first one is used; WT = 0 takes the width W at run time.
template <int WT, typename VT>
__device__ __forceinline__ double p1_ax(int v, int n, int W, int nb, int r, const int *ell_col,
                                        const double *ell_val, const double *diag, const VT *x) {
    if (WT) W = WT;
    double s = diag[v] * (double)x[(size_t)v * nb + r];
#pragma unroll
    for (int k = 0; k < W; ++k)
        s += ell_val[(size_t)k * n + v] * (double)x[(size_t)ell_col[(size_t)k * n + v] * nb + r];
    return s;
}

template <typename VT>
__global__ void k_p1_first(int n, int nb, const double *__restrict__ dinv, double omega,
                           const VT *__restrict__ b, VT *__restrict__ x) {
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= n * nb) return;
    x[t] = (VT)(omega * dinv[t / nb] * (double)b[t]);
}

// two sweeps from a zero guess: x1 = w D^-1 b, x2 = x1 + w D^-1 (b - A x1)
template <int WT, typename VT>
__global__ void k_p1_pre2(int n, int W, int nb, const int *__restrict__ ell_col, const double *__restrict__ ell_val,
                          const double *__restrict__ diag, const double *__restrict__ dinv, double omega,
                          const VT *__restrict__ b, VT *__restrict__ x) {
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= n * nb) return;
    const int v = t / nb, r = t - v * nb;
    if (WT) W = WT;
    const double bv = (double)b[t];
    double ax = diag[v] * omega * dinv[v] * bv;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const int u = ell_col[(size_t)k * n + v];
        ax += ell_val[(size_t)k * n + v] * omega * dinv[u] * (double)b[(size_t)u * nb + r];
    }
    const double x1 = omega * dinv[v] * bv;
    x[t] = (VT)(x1 + omega * dinv[v] * (bv - ax));
}

// y = x + w D^-1 (b - A x)
template <int WT, typename VT>
__global__ void k_p1_sweep(int n, int W, int nb, const int *__restrict__ ell_col, const double *__restrict__ ell_val,
                           const double *__restrict__ diag, const double *__restrict__ dinv, double omega,
                           const VT *__restrict__ b, const VT *__restrict__ x, VT *__restrict__ y) {
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= n * nb) return;
    const int v = t / nb, r = t - v * nb;
    y[t] = (VT)((double)x[t] + omega * dinv[v] * ((double)b[t] - p1_ax<WT>(v, n, W, nb, r, ell_col, ell_val, diag, x)));
}

// x += P xc: each vertex takes half of each of its two coarse parents (an
// inherited vertex lists its parent twice)
template <typename VT>
__global__ void k_p1_prolong(int n, int nb, const int *__restrict__ parents, const VT *__restrict__ xc,
                             VT *__restrict__ x) {
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= n * nb) return;
    const int v = t / nb, r = t - v * nb;
    x[t] = (VT)((double)x[t] + 0.5 * ((double)xc[(size_t)parents[2 * v] * nb + r] +
                                     (double)xc[(size_t)parents[2 * v + 1] * nb + r]));
}

template <int WT, typename VT>
__global__ void k_p1_resid(int n, int W, int nb, const int *__restrict__ ell_col, const double *__restrict__ ell_val,
                           const double *__restrict__ diag, const VT *__restrict__ b, const VT *__restrict__ x,
                           VT *__restrict__ y) {
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= n * nb) return;
    const int v = t / nb, r = t - v * nb;
    y[t] = (VT)((double)b[t] - p1_ax<WT>(v, n, W, nb, r, ell_col, ell_val, diag, x));
}

// One right-hand side (nb == 1), where a level's kernels are a few waves and a
// launch costs more than its work: the residual fused into the restriction.
// Eight lanes per coarse vertex each evaluate one child's residual in place (the
// expression of k_p1_resid, rounded to the vector type as it stores it) and the
// weighted values are summed by shuffles within the eight lanes.
template <int WT, typename VT>
__global__ void k_p1_resid_restrict(int n, int W, const int *__restrict__ ell_col, const double *__restrict__ ell_val,
                                    const double *__restrict__ diag, const VT *__restrict__ b,
                                    const VT *__restrict__ x, int nc, const int *__restrict__ crow,
                                    const int *__restrict__ ccol, const double *__restrict__ cw,
                                    VT *__restrict__ bc) {
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    const int c = t >> 3, sub = t & 7;
    double v = 0.0;   // every lane of a group takes part in the shuffles below
    if (c < nc) {
        const int k0 = crow[c], cnt = crow[c + 1] - k0;
        for (int k = sub; k < cnt; k += 8) {
            const int u = ccol[k0 + k];
            const VT ru = (VT)((double)b[u] - p1_ax<WT>(u, n, W, 1, 0, ell_col, ell_val, diag, x));
            v += cw[k0 + k] * (double)ru;
        }
    }
    v += __shfl_xor(v, 1, 8);
    v += __shfl_xor(v, 2, 8);
    v += __shfl_xor(v, 4, 8);
    if (c < nc && sub == 0) bc[c] = (VT)v;
}

// One right-hand side: the first post-sweep with the prolongation x' = x + P xc
// evaluated at the vertex and its neighbours in place (rounded to the vector type
// as k_p1_prolong stores it: the same bits as the two kernels)
template <int WT, typename VT>
__global__ void k_p1_sweep_prolong(int n, int W, const int *__restrict__ ell_col, const double *__restrict__ ell_val,
                                   const double *__restrict__ diag, const double *__restrict__ dinv, double omega,
                                   const VT *__restrict__ b, const VT *__restrict__ x, const int *__restrict__ parents,
                                   const VT *__restrict__ xc, VT *__restrict__ y) {
    const int v = xcd_block() * blockDim.x + threadIdx.x;
    if (v >= n) return;
    if (WT) W = WT;
    auto xp = [&](int u) {
        return (double)(VT)((double)x[u] + 0.5 * ((double)xc[parents[2 * u]] + (double)xc[parents[2 * u + 1]]));
    };
    const double xv = xp(v);
    double s = diag[v] * xv;
#pragma unroll
    for (int k = 0; k < W; ++k) s += ell_val[(size_t)k * n + v] * xp(ell_col[(size_t)k * n + v]);
    y[v] = (VT)(xv + omega * dinv[v] * ((double)b[v] - s));
}

// bc[c] = sum over children of w * r[child]  (transpose of the interpolation); the
// children (7 on the icosahedral hierarchy) are read eight at a time, all loads in flight
template <typename VT>
__global__ void k_p1_restrict(int nc, int nb, const int *__restrict__ crow, const int *__restrict__ ccol,
                              const double *__restrict__ cw, const VT *__restrict__ r,
                              VT *__restrict__ bc) {
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= nc * nb) return;
    const int c = t / nb, rr = t - c * nb;
    const int k0 = crow[c];
    bc[t] = (VT)acc_row<8>(0.0, crow[c + 1] - k0,
                           [&](int k) { return cw[k0 + k] * (double)r[(size_t)ccol[k0 + k] * nb + rr]; });
}

// x = Ainv b on the coarsest level when it is too large for the tail kernel:
// one wavefront per (row, RHS), lanes stride over the row, shuffle reduction.
// x = Ainv b on the coarsest level: one wavefront per (row, chunk of up to CH
// right-hand sides), lanes striding the row; each matrix row is read once per
// chunk and a lane reads the chunk's values of b[j] contiguously.
template <int CH, typename VT>
__global__ void k_dense_mv(int n, int nb, const double *__restrict__ Ainv, const VT *__restrict__ b,
                           VT *__restrict__ x) {
    const int nch = (nb + CH - 1) / CH;
    const int w = (blockIdx.x * blockDim.x + threadIdx.x) / 64;
    const int lane = threadIdx.x & 63;
    if (w >= n * nch) return;
    const int i = w / nch, r0 = (w - i * nch) * CH;
    const int cnt = min(CH, nb - r0);
    double s[CH];
#pragma unroll
    for (int q = 0; q < CH; ++q) s[q] = 0.0;
    for (int j = lane; j < n; j += 64) {
        const double a = Ainv[(size_t)i * n + j];
        const VT *bj = b + (size_t)j * nb + r0;
#pragma unroll
        for (int q = 0; q < CH; ++q)
            if (q < cnt) s[q] += a * (double)bj[q];
    }
#pragma unroll
    for (int q = 0; q < CH; ++q)
        for (int off = 32; off > 0; off >>= 1) s[q] += __shfl_xor(s[q], off, 64);
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < CH; ++q)
            if (q < cnt) x[(size_t)i * nb + r0 + q] = (VT)s[q];
}

// All levels 0..top of the hierarchy in one workgroup: the complete V-cycle
// below and including level `top`, input lev[top].b, result in lev[top].x.
template <typename VT>
__global__ __launch_bounds__(1024) void k_p1_tail(const P1Tail Targ, int nb) {
    __shared__ VT *xs[P1_TAIL_LEVELS];
    __shared__ P1Tail T;   // level descriptors staged in LDS (runtime-indexed below)
    const int tid = threadIdx.x, nth = blockDim.x;
    if (tid == 0) T = Targ;
    __syncthreads();
    const double w = T.omega;
    for (int l = T.top; l >= 1; --l) {
        const P1Lev &L = T.lev[l];
        const int N = L.n * nb;
        const VT *b = reinterpret_cast<const VT *>(L.b);
        VT *x = reinterpret_cast<VT *>(L.x), *y = reinterpret_cast<VT *>(L.y);
        for (int t = tid; t < N; t += nth) x[t] = (VT)(w * L.dinv[t / nb] * (double)b[t]);
        __syncthreads();
        for (int k = 1; k < T.nu; ++k) {
            for (int t = tid; t < N; t += nth) {
                const int v = t / nb, r = t - v * nb;
                y[t] = (VT)((double)x[t] + w * L.dinv[v] * ((double)b[t] - p1_ax<0>(v, L.n, L.w, nb, r, L.col, L.val, L.diag, x)));
            }
            __syncthreads();
            VT *tmp = x; x = y; y = tmp;
        }
        for (int t = tid; t < N; t += nth) {
            const int v = t / nb, r = t - v * nb;
            y[t] = (VT)((double)b[t] - p1_ax<0>(v, L.n, L.w, nb, r, L.col, L.val, L.diag, x));
        }
        __syncthreads();
        const P1Lev &C = T.lev[l - 1];
        for (int t = tid; t < C.n * nb; t += nth) {
            const int c = t / nb, rr = t - c * nb;
            double acc = 0.0;
            for (int k = L.crow[c]; k < L.crow[c + 1]; ++k) acc += L.cw[k] * (double)y[(size_t)L.ccol[k] * nb + rr];
            reinterpret_cast<VT *>(C.b)[t] = (VT)acc;
        }
        if (tid == 0) xs[l] = x;
        __syncthreads();
    }
    {
        const P1Lev &L0 = T.lev[0];
        const int n0 = L0.n;
        for (int t = tid; t < n0 * nb; t += nth) {
            const int i = t / nb, r = t - i * nb;
            double s = 0.0;
            for (int j = 0; j < n0; ++j) s += T.Ainv[(size_t)i * n0 + j] * (double)reinterpret_cast<const VT *>(L0.b)[(size_t)j * nb + r];
            reinterpret_cast<VT *>(L0.x)[t] = (VT)s;
        }
        if (tid == 0) xs[0] = reinterpret_cast<VT *>(L0.x);
        __syncthreads();
    }
    for (int l = 1; l <= T.top; ++l) {
        const P1Lev &L = T.lev[l];
        const int N = L.n * nb;
        const VT *b = reinterpret_cast<const VT *>(L.b);
        VT *x = xs[l];
        VT *y = (x == reinterpret_cast<VT *>(L.x)) ? reinterpret_cast<VT *>(L.y) : reinterpret_cast<VT *>(L.x);
        const VT *xc = xs[l - 1];
        for (int k = 0; k < T.nu; ++k) {
            for (int t = tid; t < N; t += nth) {
                const int v = t / nb, r = t - v * nb;
                auto xin = [&](int u) -> double {
                    double s = (double)x[(size_t)u * nb + r];
                    if (k == 0)
                        s += 0.5 * ((double)xc[(size_t)L.parents[2 * u] * nb + r] +
                                    (double)xc[(size_t)L.parents[2 * u + 1] * nb + r]);
                    return s;
                };
                double ax = 0.0;
                for (int k = 0; k < L.w; ++k) ax += L.val[(size_t)k * L.n + v] * xin(L.col[(size_t)k * L.n + v]);
                const double xv = xin(v);
                ax += L.diag[v] * xv;
                y[t] = (VT)(xv + w * L.dinv[v] * ((double)b[t] - ax));
            }
            __syncthreads();
            VT *tmp = x; x = y; y = tmp;
        }
        if (tid == 0) xs[l] = x;
        __syncthreads();
    }
    const P1Lev &Lt = T.lev[T.top];
    if (T.top > 0 && xs[T.top] != reinterpret_cast<VT *>(Lt.x)) {
        for (int t = tid; t < Lt.n * nb; t += nth) reinterpret_cast<VT *>(Lt.x)[t] = xs[T.top][t];
    }
}

// ------------------------------------------------------------------ condensation / recovery (per solve)

// loc[rho][K][r] = sum_j Zr[rho][j][K] r_cell[K][j][r]   (Step 1, cell part)
constexpr int RECOVER_TILE = 128;   // cells per block of the one-right-hand-side cell kernels

// Condensation at one right-hand side: the block's cells read their inputs
// through LDS (coalesced global loads).  NU trace components per node (1:
// upwind, 2: Lax-Friedrichs).
template <int P, int NU>
__global__ __launch_bounds__(RECOVER_TILE) void k_condense_cell_n1(int nk, const double *__restrict__ Zr,
                                                                  const double *__restrict__ rc,
                                                                  double *__restrict__ loc) {
    constexpr int n = (P + 1) * (P + 2) / 2, m = P + 1, nc = 3 * n, nt = 3 * NU * m, ZW = cell_zw(P);
    __shared__ double buf[RECOVER_TILE * nc];
    const int K0 = xcd_block() * RECOVER_TILE, tid = threadIdx.x, K = K0 + tid;
    const int cnt = min(RECOVER_TILE, nk - K0);
    const size_t NK = (size_t)nk;
    for (int i = tid; i < cnt * nc; i += RECOVER_TILE) buf[i] = rc[(size_t)K0 * nc + i];
    __syncthreads();
    if (tid >= cnt) return;
    double f[ZW];
#pragma unroll
    for (int j = 0; j < ZW; ++j) f[j] = j < nc ? buf[tid * nc + j] : 0.0;
#pragma unroll
    for (int a = 0; a < nt; ++a) {
        double s = 0.0;
#pragma unroll
        for (int jp = 0; jp < ZW / 2; ++jp) {
            double w[2];
            Wide<double>::load(Zr + ((size_t)(a * ZW / 2 + jp) * NK + K) * 2, w);
            s += w[0] * f[2 * jp];
            if (2 * jp + 1 < nc) s += w[1] * f[2 * jp + 1];
        }
        loc[(size_t)a * NK + K] = s;
    }
}

// rhat[e][a][r] = sum of the two cells' local contributions (orientation mapped)
template <int P, int NU>
__global__ void k_condense_gather(int ne, int nk, int nb, const int *__restrict__ facet_cell,
                                  const int *__restrict__ facet_loc, const double *__restrict__ loc,
                                  double *__restrict__ rhat) {
    constexpr int M = NU * (P + 1);
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= ne * M * nb) return;
    const int r = t % nb, ea = t / nb, e = ea / M, a = ea - e * M;
    const size_t NK = (size_t)nk;
    const int K0 = facet_cell[2 * e], i0 = facet_loc[2 * e];
    const int K1 = facet_cell[2 * e + 1], i1 = facet_loc[2 * e + 1];
    const double v0 = loc[((size_t)loc_trace<P, NU>(i0, a, 0) * NK + K0) * nb + r];
    const double v1 = loc[((size_t)loc_trace<P, NU>(i1, a, 1) * NK + K1) * nb + r];
    rhat[t] = v0 + v1;
}

// Recovery q = Ar r_cell - Wr lam_K (Step 3) with one right-hand side: the
// block's cells read their inputs and write their outputs through LDS, so the
// global traffic of r_cell and q (nc consecutive values per cell) is coalesced.
template <int P, int NU>
__global__ __launch_bounds__(RECOVER_TILE) void k_recover_n1(int nk, const double *__restrict__ Ar,
                                                            const double *__restrict__ Wr,
                                                            const int *__restrict__ cell_facet,
                                                            const int8_t *__restrict__ cell_rev,
                                                            const double *__restrict__ rc,
                                                            const double *__restrict__ lam, double *__restrict__ q) {
    constexpr int n = (P + 1) * (P + 2) / 2, m = P + 1, nc = 3 * n, M = NU * m, nt = 3 * M;
    __shared__ double buf[RECOVER_TILE * nc];
    const int K0 = xcd_block() * RECOVER_TILE, tid = threadIdx.x, K = K0 + tid;
    const int cnt = min(RECOVER_TILE, nk - K0);   // may be <= 0 in the padding blocks
    const size_t NK = (size_t)nk;
    for (int i = tid; i < cnt * nc; i += RECOVER_TILE) buf[i] = rc[(size_t)K0 * nc + i];
    __syncthreads();
    double f[nc], l[nt];
    const bool live = tid < cnt;
#pragma unroll
    for (int j = 0; j < nc; ++j) f[j] = live ? buf[tid * nc + j] : 0.0;
    if (live) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int e = cell_facet[i * NK + K];
            const int rev = cell_rev[i * NK + K];
#pragma unroll
            for (int a = 0; a < M; ++a) l[loc_trace<P, NU>(i, a, rev)] = lam[(size_t)e * M + a];
        }
    }
    __syncthreads();
    if (live) {
#pragma unroll 1
        for (int a = 0; a < nc; ++a) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < nc; ++j) s += ldm(Ar + (size_t)(a * nc + j) * NK + K) * f[j];
#pragma unroll
            for (int j = 0; j < nt; ++j) s -= ldm(Wr + (size_t)(a * nt + j) * NK + K) * l[j];
            buf[tid * nc + a] = s;
        }
    }
    __syncthreads();
    for (int i = tid; i < cnt * nc; i += RECOVER_TILE) q[(size_t)K0 * nc + i] = buf[i];
}

// Batched cell kernels (nrhs >= 2): a block holds CB cells x nrhs threads
// (right-hand side fastest) and streams the cells' matrix rows through LDS in
// chunks of CELL_ROWS rows, loaded once per block with coalesced reads; every
// thread keeps its right-hand side's inputs in registers.  Same arithmetic
// order as the one-thread-per-(cell, rhs) kernels.
// Condensation: when a chunk is at most CELL_PF entries per thread (6 rl <= 8 nb:
// 32 right-hand sides at p = 3), the next chunk is loaded into registers while
// the current one is used, through two LDS buffers and one barrier per chunk
// (recovery keeps one buffer: with the prefetch registers it would drop from
// four waves per SIMD to three, and measured slower).
constexpr int CELL_ROWS = 6, CELL_PF = 8;
// cells per block for row length rl: at most 256 threads and 64 KiB of staged rows
inline int cell_block_cells(int nb, int rl) {
    return std::max(1, std::min(std::min(32, 256 / nb), 65536 / (int)(sizeof(double) * CELL_ROWS * rl)));
}
// cells per block actually launched: a request (tuning) of at most the default
inline int cell_cells(int nb, int rl, int req) {
    const int mx = cell_block_cells(nb, rl);
    return req > 0 && req < mx ? req : mx;
}
__host__ __device__ constexpr bool cell_prefetch(int nb, int rl) { return CELL_ROWS * rl <= CELL_PF * nb; }
// dynamic LDS of a batched cell kernel with cb cells per block: one or two staging buffers
inline size_t cell_stage_bytes(int nb, int rl, int cb) {
    return sizeof(double) * CELL_ROWS * rl * cb * (cell_prefetch(nb, rl) ? 2 : 1);
}

template <int P, int NU>
__global__ __launch_bounds__(256) void k_recover_b(int nk, int nb, int cb, const double *__restrict__ Ar,
                                                   const double *__restrict__ Wr, const int *__restrict__ cell_facet,
                                                   const int8_t *__restrict__ cell_rev, const double *__restrict__ rc,
                                                   const double *__restrict__ lam, double *__restrict__ q) {
    constexpr int n = (P + 1) * (P + 2) / 2, m = P + 1, nc = 3 * n, M = NU * m, nt = 3 * M, RL = nc + nt;
    extern __shared__ double sm[];   // [row][entry][cell], CELL_ROWS * RL * cb doubles
    const int K0 = xcd_block() * cb, tid = threadIdx.x;
    const int cl = tid / nb, r = tid - cl * nb, K = K0 + cl;
    const bool live = cl < cb && K < nk;
    const size_t NK = (size_t)nk;
    double f[nc], l[nt];
    if (live) {
#pragma unroll
        for (int j = 0; j < nc; ++j) f[j] = rc[((size_t)K * nc + j) * nb + r];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const int e = cell_facet[i * NK + K];
            const int rev = cell_rev[i * NK + K];
#pragma unroll
            for (int a = 0; a < M; ++a) l[loc_trace<P, NU>(i, a, rev)] = lam[((size_t)e * M + a) * nb + r];
        }
    }
    for (int a0 = 0; a0 < nc; a0 += CELL_ROWS) {
        const int rows = min(CELL_ROWS, nc - a0);
        __syncthreads();
        for (int i = tid; i < rows * RL * cb; i += blockDim.x) {
            const int c = i % cb, jr = i / cb, row = jr / RL, j = jr - row * RL, Kc = K0 + c;
            double v = 0.0;
            if (Kc < nk) {
                const int a = a0 + row;
                v = j < nc ? ldm(Ar + (size_t)(a * nc + j) * NK + Kc) : ldm(Wr + (size_t)(a * nt + j - nc) * NK + Kc);
            }
            sm[(row * RL + j) * cb + c] = v;
        }
        __syncthreads();
        if (live) {
            for (int row = 0; row < rows; ++row) {
                double s = 0.0;
#pragma unroll
                for (int j = 0; j < nc; ++j) s += sm[(row * RL + j) * cb + cl] * f[j];
#pragma unroll
                for (int j = 0; j < nt; ++j) s -= sm[(row * RL + nc + j) * cb + cl] * l[j];
                q[((size_t)K * nc + a0 + row) * nb + r] = s;
            }
        }
    }
}

template <int P, int NU>
__global__ __launch_bounds__(256) void k_condense_cell_b(int nk, int nb, int cb, const double *__restrict__ Zr,
                                                         const double *__restrict__ rc, double *__restrict__ loc) {
    constexpr int n = (P + 1) * (P + 2) / 2, m = P + 1, nc = 3 * n, nt = 3 * NU * m, ZW = cell_zw(P);
    extern __shared__ double sm[];   // [row][entry][cell], CELL_ROWS * ZW * cb doubles (twice with prefetch)
    const int K0 = xcd_block() * cb, tid = threadIdx.x;
    const int cl = tid / nb, r = tid - cl * nb, K = K0 + cl;
    const bool live = cl < cb && K < nk;
    const size_t NK = (size_t)nk;
    double f[ZW];
#pragma unroll
    for (int j = 0; j < ZW; ++j) f[j] = (live && j < nc) ? rc[((size_t)K * nc + j) * nb + r] : 0.0;
    // staged entry i of the chunk at row a0 (its LDS slot is i: [row][entry][cell])
    auto entry = [&](int a0, int i) {
        const int c = i % cb, jr = i / cb, row = jr / ZW, j = jr - row * ZW, Kc = K0 + c;
        const int idx = (a0 + row) * ZW + j;   // pair layout [idx / 2][NK][2]
        return Kc < nk ? Zr[((size_t)(idx / 2) * NK + Kc) * 2 + idx % 2] : 0.0;
    };
    auto use = [&](const double *buf, int a0, int rows) {
        for (int row = 0; row < rows; ++row) {
            double s = 0.0;
#pragma unroll
            for (int jp = 0; jp < ZW / 2; ++jp) {
                s += buf[(row * ZW + 2 * jp) * cb + cl] * f[2 * jp];
                if (2 * jp + 1 < nc) s += buf[(row * ZW + 2 * jp + 1) * cb + cl] * f[2 * jp + 1];
            }
            loc[((size_t)(a0 + row) * NK + K) * nb + r] = s;
        }
    };
    if (cell_prefetch(nb, ZW)) {
        const int per = CELL_ROWS * ZW * cb, nthr = blockDim.x;
        double v[CELL_PF];
        auto fetch = [&](int a0) {
            const int cnt = min(CELL_ROWS, nt - a0) * ZW * cb;
#pragma unroll
            for (int u = 0; u < CELL_PF; ++u) v[u] = tid + u * nthr < cnt ? entry(a0, tid + u * nthr) : 0.0;
        };
        auto put = [&](int a0, double *buf) {
            const int cnt = min(CELL_ROWS, nt - a0) * ZW * cb;
#pragma unroll
            for (int u = 0; u < CELL_PF; ++u)
                if (tid + u * nthr < cnt) buf[tid + u * nthr] = v[u];
        };
        fetch(0);
        put(0, sm);
        __syncthreads();
        for (int a0 = 0, ch = 0; a0 < nt; a0 += CELL_ROWS, ++ch) {
            const bool more = a0 + CELL_ROWS < nt;
            if (more) fetch(a0 + CELL_ROWS);
            if (live) use(sm + (ch & 1) * per, a0, min(CELL_ROWS, nt - a0));
            if (more) put(a0 + CELL_ROWS, sm + ((ch + 1) & 1) * per);
            __syncthreads();
        }
        return;
    }
    for (int a0 = 0; a0 < nt; a0 += CELL_ROWS) {
        const int rows = min(CELL_ROWS, nt - a0);
        __syncthreads();
        for (int i = tid; i < rows * ZW * cb; i += blockDim.x) sm[i] = entry(a0, i);
        __syncthreads();
        if (live) use(sm, a0, rows);
    }
}

// ------------------------------------------------------------------ Krylov vector kernels
//
// Vectors are [len][nb]; per-RHS reductions run in two deterministic passes
// (block partials, then one block per RHS), so repeated solves are bitwise
// identical.

__device__ __forceinline__ int rows_per_block(int nb) {
    int r = 1;
    while (r * 2 * nb <= 256) r *= 2;
    return r;
}

// Per-RHS reductions over trace vectors run in two deterministic passes:
// block partials (fixed row split), then one block per output summing the
// partials in block order.  Repeated solves are bitwise identical.

constexpr int RED_CHUNK = 8;   // dot products accumulated per pass over the rows
constexpr int MDOT_ROWS = 4;   // rows each thread loads per step of the dot-product kernel
constexpr int GS_ROWS = 2;     // rows each thread updates per step of the Gram-Schmidt kernel

// sh[k][tid] -> per-RHS block sums for k < kc in sh[k][r], r < nb
__device__ __forceinline__ void block_rhs_sums(double (*sh)[256], int kc, int nb, int rpb) {
    const int tid = threadIdx.x;
    const int rl = tid / nb;
    __syncthreads();
    for (int s = rpb / 2; s > 0; s >>= 1) {
        if (rl < s)
            for (int k = 0; k < kc; ++k) sh[k][tid] += sh[k][tid + s * nb];
        __syncthreads();
    }
}

// partial[blk][d][r] = this block's share of sum_i X_d[i][r] y[i][r], d < nd
template <typename VT>
__global__ __launch_bounds__(256) void k_mdot_partial(int64_t len, int nb, int nd, const VT *__restrict__ X,
                                                      int64_t xstride, const VT *__restrict__ y,
                                                      double *__restrict__ partial) {
    __shared__ double sh[RED_CHUNK][256];
    const int rpb = rows_per_block(nb);
    const int tid = threadIdx.x;
    const int rl = tid / nb, r = tid - rl * nb;
    for (int d0 = 0; d0 < nd; d0 += RED_CHUNK) {
        const int kc = min(RED_CHUNK, nd - d0);
        double acc[RED_CHUNK];
#pragma unroll
        for (int k = 0; k < RED_CHUNK; ++k) acc[k] = 0.0;
        if (rl < rpb) {
            // MDOT_ROWS rows per pass (more loads in flight per wave)
            const int64_t stride = (int64_t)gridDim.x * rpb;
            for (int64_t i = (int64_t)blockIdx.x * rpb + rl; i < len; i += MDOT_ROWS * stride) {
                size_t tt[MDOT_ROWS];
                double yy[MDOT_ROWS];
#pragma unroll
                for (int u = 0; u < MDOT_ROWS; ++u) {
                    const int64_t iu = i + u * stride;
                    const bool ok = iu < len;
                    tt[u] = (size_t)(ok ? iu : i) * nb + r;
                    yy[u] = ok ? (double)y[tt[u]] : 0.0;
                }
#pragma unroll
                for (int k = 0; k < RED_CHUNK; ++k)
                    if (k < kc) {
                        double a[MDOT_ROWS];
#pragma unroll
                        for (int u = 0; u < MDOT_ROWS; ++u) a[u] = (double)X[(size_t)(d0 + k) * xstride + tt[u]];
#pragma unroll
                        for (int u = 0; u < MDOT_ROWS; ++u) acc[k] += a[u] * yy[u];
                    }
            }
        }
#pragma unroll
        for (int k = 0; k < RED_CHUNK; ++k) sh[k][tid] = (rl < rpb) ? acc[k] : 0.0;
        block_rhs_sums(sh, kc, nb, rpb);
        if (tid < nb)
            for (int k = 0; k < kc; ++k) partial[((size_t)blockIdx.x * nd + d0 + k) * nb + tid] = sh[k][tid];
        __syncthreads();
    }
}

__device__ __forceinline__ double block_sum_partials(const double *partial, int nblk, int nout, int o) {
    __shared__ double sh[256];
    double acc = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) acc += partial[(size_t)b * nout + o];
    sh[threadIdx.x] = acc;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

// out[o] = sum over blocks, one block per output o = d * nb + r (grid nd * nb);
// host (may be null) receives a copy in host-mapped memory.
__global__ __launch_bounds__(256) void k_sum_final(int nblk, int nout, const double *__restrict__ partial,
                                                   double *__restrict__ out, double *__restrict__ host) {
    const int o = blockIdx.x;
    const double v = block_sum_partials(partial, nblk, nout, o);
    if (threadIdx.x == 0) {
        if (out) out[o] = v;
        if (host) host[o] = v;
    }
}

__device__ void givens_column(int r, int nb, int j, int restart, const double *hcol, double hn, double *gm,
                              const double *bnorm, double *resid) {
    const int stride = (restart + 1) * restart + 2 * restart + (restart + 1);
    double *H = gm + (size_t)r * stride;
    double *cs = H + (restart + 1) * restart;
    double *sn = cs + restart;
    double *g = sn + restart;
    double col[65];
    for (int i = 0; i <= j; ++i) col[i] = hcol[(size_t)i * nb + r];
    col[j + 1] = hn;
    for (int i = 0; i < j; ++i) {
        const double a = col[i], b = col[i + 1];
        col[i] = cs[i] * a + sn[i] * b;
        col[i + 1] = -sn[i] * a + cs[i] * b;
    }
    const double a = col[j], b = col[j + 1];
    const double d = sqrt(a * a + b * b);
    const double c = d > 0.0 ? a / d : 1.0, s = d > 0.0 ? b / d : 0.0;
    cs[j] = c;
    sn[j] = s;
    col[j] = d;
    for (int i = 0; i <= j; ++i) H[(size_t)i * restart + j] = col[i];
    const double gj = g[j];
    g[j] = c * gj;
    g[j + 1] = -s * gj;
    const double bn = bnorm[r];
    resid[r] = bn > 0.0 ? fabs(g[j + 1]) / bn : 0.0;
}

// w -= sum_d h[d] V_d (classical Gram-Schmidt) and block partials of ||w||^2
template <typename VT>
__global__ __launch_bounds__(256) void k_gs_update_norm(int64_t len, int nb, int nd, const double *__restrict__ h,
                                                        const VT *__restrict__ V, int64_t vstride,
                                                        VT *__restrict__ w, double *__restrict__ partial,
                                                        const int *__restrict__ run) {
    if (run && !*run) return;   // the lagged step was taken instead (k_pyth_givens)
    __shared__ double sh[1][256];
    const int rpb = rows_per_block(nb);
    const int tid = threadIdx.x;
    const int rl = tid / nb, r = tid - rl * nb;
    double acc = 0.0;
    if (rl < rpb) {
        // GS_ROWS rows per pass (more loads in flight per wave)
        const int64_t stride = (int64_t)gridDim.x * rpb;
        for (int64_t i = (int64_t)blockIdx.x * rpb + rl; i < len; i += GS_ROWS * stride) {
            size_t tt[GS_ROWS];
            bool ok[GS_ROWS];
            double s[GS_ROWS];
#pragma unroll
            for (int u = 0; u < GS_ROWS; ++u) {
                const int64_t iu = i + u * stride;
                ok[u] = iu < len;
                tt[u] = (size_t)(ok[u] ? iu : i) * nb + r;
                s[u] = (double)w[tt[u]];
            }
            for (int d = 0; d < nd; ++d) {
                const double hd = h[(size_t)d * nb + r];
#pragma unroll
                for (int u = 0; u < GS_ROWS; ++u) s[u] -= hd * (double)V[(size_t)d * vstride + tt[u]];
            }
#pragma unroll
            for (int u = 0; u < GS_ROWS; ++u)
                if (ok[u]) {
                    const VT sv = (VT)s[u];   // the norm is that of the vector as stored
                    w[tt[u]] = sv;
                    acc += (double)sv * (double)sv;
                }
        }
    }
    sh[0][tid] = (rl < rpb) ? acc : 0.0;
    block_rhs_sums(sh, 1, nb, rpb);
    if (tid < nb) partial[(size_t)blockIdx.x * nb + tid] = sh[0][tid];
}

// one block per RHS: ||w|| from the partials, then the Givens step of column j
// (FGMRES); the relative residual estimate goes to host-mapped memory.
__global__ __launch_bounds__(256) void k_norm_givens(int nblk, int nb, const double *__restrict__ partial,
                                                     double *__restrict__ hn, int j, int restart,
                                                     const double *__restrict__ hcol, double *__restrict__ gm,
                                                     const double *__restrict__ bnorm, double *__restrict__ resid,
                                                     const int *__restrict__ run) {
    if (run && !*run) return;
    const int r = blockIdx.x;
    const double v = block_sum_partials(partial, nblk, nb, r);
    if (threadIdx.x == 0) {
        const double n = sqrt(fmax(v, 0.0));
        hn[r] = n;
        givens_column(r, nb, j, restart, hcol, n, gm, bnorm, resid);
    }
}

// The norm of w - sum_{d <= j} h_d V_d from the dot products of the same pass
// (hcol[j + 1] = ||w||^2): ||w||^2 - sum h_d^2, exact for an orthonormal basis.
// Its rounding error grows with the basis' loss of orthogonality relative to the
// remaining norm, so it is used only when that norm keeps at least `floor` of
// ||w||^2 for every right-hand side; then the Givens step follows and *expl = 0
// (the update is left to the next V-cycle's first kernel).  Otherwise *expl = 1
// and the explicit update pass (k_gs_update_norm, k_norm_givens) does both.
// One block of 64 threads, nb <= 64.
__global__ __launch_bounds__(64) void k_pyth_givens(int nb, int j, int restart, double floor,
                                                    const double *__restrict__ hcol, double *__restrict__ hn,
                                                    double *__restrict__ gm, const double *__restrict__ bnorm,
                                                    double *__restrict__ resid, int *__restrict__ expl) {
    __shared__ int bad;
    const int r = threadIdx.x;
    if (r == 0) bad = 0;
    __syncthreads();
    double s = 0.0;
    if (r < nb) {
        const double w2 = hcol[(size_t)(j + 1) * nb + r];
        s = w2;
        for (int i = 0; i <= j; ++i) {
            const double h = hcol[(size_t)i * nb + r];
            s -= h * h;
        }
        if (!(s >= floor * w2)) atomicOr(&bad, 1);
    }
    __syncthreads();
    if (r == 0) *expl = bad;
    if (bad || r >= nb) return;
    const double n = sqrt(s);
    hn[r] = n;
    givens_column(r, nb, j, restart, hcol, n, gm, bnorm, resid);
}

// PCG update x += alpha p, r -= alpha w (alpha = num/den) and partials of ||r||^2
__global__ __launch_bounds__(256) void k_pcg_update_norm(int64_t len, int nb, const double *__restrict__ num,
                                                         const double *__restrict__ den,
                                                         const double *__restrict__ p, const double *__restrict__ w,
                                                         double *__restrict__ x, double *__restrict__ res,
                                                         double *__restrict__ partial) {
    __shared__ double sh[1][256];
    const int rpb = rows_per_block(nb);
    const int tid = threadIdx.x;
    const int rl = tid / nb, r = tid - rl * nb;
    double acc = 0.0;
    if (rl < rpb) {
        const double d = den[r];
        const double al = d != 0.0 ? num[r] / d : 0.0;
        for (int64_t i = (int64_t)blockIdx.x * rpb + rl; i < len; i += (int64_t)gridDim.x * rpb) {
            const size_t t = (size_t)i * nb + r;
            x[t] += al * p[t];
            const double v = res[t] - al * w[t];
            res[t] = v;
            acc += v * v;
        }
    }
    sh[0][tid] = (rl < rpb) ? acc : 0.0;
    block_rhs_sums(sh, 1, nb, rpb);
    if (tid < nb) partial[(size_t)blockIdx.x * nb + tid] = sh[0][tid];
}


// p = z + beta p, beta[r] = num[r] / den[r]
__global__ void k_pcg_dir(int64_t n, int nb, const double *__restrict__ num, const double *__restrict__ den,
                          const double *__restrict__ z, double *__restrict__ p) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nb) return;
    const int r = (int)(t % nb);
    const double d = den[r];
    const double be = d != 0.0 ? num[r] / d : 0.0;
    p[t] = z[t] + be * p[t];
}

// x += sum_{d < nd} y[d][r] Z_d
template <typename VT>
__global__ void k_lincomb(int64_t n, int nb, int nd, const double *__restrict__ y, const VT *__restrict__ Z,
                          int64_t zstride, double *__restrict__ x) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nb) return;
    const int r = (int)(t % nb);
    double s = x[t];
    for (int d = 0; d < nd; ++d) s += y[(size_t)d * nb + r] * (double)Z[(size_t)d * zstride + t];
    x[t] = s;
}


__global__ void k_copy(int64_t n, const double *__restrict__ src, double *__restrict__ dst) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < n) dst[t] = src[t];
}

// start of a cycle: g = (beta, 0, ...), beta = ||r0||
__global__ void k_gmres_start(int nb, int restart, const double *__restrict__ beta2, double *__restrict__ gm,
                              double *__restrict__ beta) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nb) return;
    const int stride = (restart + 1) * restart + 2 * restart + (restart + 1);
    double *g = gm + (size_t)r * stride + (restart + 1) * restart + 2 * restart;
    const double b = sqrt(fmax(beta2[r], 0.0));
    for (int i = 0; i <= restart; ++i) g[i] = 0.0;
    g[0] = b;
    beta[r] = b;
}

// y = H(0:k,0:k)^-1 g(0:k) by back substitution, written as y[i][r]
__global__ void k_gmres_solve(int nb, int k, int restart, const double *__restrict__ gm, double *__restrict__ y) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nb) return;
    const int stride = (restart + 1) * restart + 2 * restart + (restart + 1);
    const double *H = gm + (size_t)r * stride;
    const double *g = H + (restart + 1) * restart + 2 * restart;
    double yy[64];
    for (int i = k - 1; i >= 0; --i) {
        double s = g[i];
        for (int l = i + 1; l < k; ++l) s -= H[(size_t)i * restart + l] * yy[l];
        const double d = H[(size_t)i * restart + i];
        yy[i] = d != 0.0 ? s / d : 0.0;
    }
    for (int i = 0; i < k; ++i) y[(size_t)i * nb + r] = yy[i];
}

__global__ void k_sqrt(int nb, const double *__restrict__ in, double *__restrict__ out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < nb) out[r] = sqrt(fmax(in[r], 0.0));
}

// ------------------------------------------------------------------ explicit instantiations via launchers

#define GRID(n, b) dim3((unsigned)(((n) + (b) - 1) / (b))), dim3(b)
// grid padded to a multiple of N_XCD blocks, for kernels indexed through xcd_block()

// ------------------------------------------------------------------ RHS-blocked facet-row kernels
//
// With many right-hand sides the per-(facet, rhs) kernels above re-read the
// facet's matrix row once per right-hand side.  These variants give each
// thread RB = 4 consecutive right-hand sides of one facet (two 16-byte loads
// per facet node) and stage the rows of the block's 64 facets in LDS with
// coalesced 16-byte loads, so every row leaves L2 once per block.
// Block = 64 facets x (nb / RB) threads; nb / RB must be a power of two <= 16.
constexpr int RB_FACETS = 64;

template <typename MT>
__device__ __forceinline__ float lds_entry_f(const MT *p) { return (float)*p; }
template <>
__device__ __forceinline__ float lds_entry_f<__hip_bfloat16>(const __hip_bfloat16 *p) {
    return __uint_as_float(((unsigned)*reinterpret_cast<const unsigned short *>(p)) << 16);
}
template <typename MT>
__device__ __forceinline__ typename Acc<MT>::type lds_entry(const MT *p) {
    if constexpr (std::is_same<MT, double>::value) return *p;
    else return lds_entry_f<MT>(p);
}

// stage the G 16-byte groups of the rows of facets f0 .. f0 + 63 as [g][64][V]
template <typename MT, int G>
__device__ __forceinline__ void stage_rows(MT *sm, const MT *__restrict__ S, int f0, int ne) {
    // four 16-byte loads per lane go out before their LDS stores
    constexpr int V = Wide<MT>::V, W = G * RB_FACETS, U = 4;
    const size_t NE = (size_t)ne;
    const int step = blockDim.x;
    for (int i0 = threadIdx.x; i0 < W; i0 += U * step) {
        u32x4_t v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * step, g = i / RB_FACETS, e = f0 + (i - g * RB_FACETS);
            v[u] = u32x4_t{0u, 0u, 0u, 0u};
            if (i < W && e < ne) v[u] = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t *>(S + ((size_t)g * NE + e) * V));
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = i0 + u * step;
            if (i < W) *reinterpret_cast<u32x4_t *>(sm + (size_t)i * V) = v[u];
        }
    }
}

template <int RB, typename T>
__device__ __forceinline__ void load_rb(const T *__restrict__ p, double (&d)[RB]) {
    if constexpr (std::is_same<T, double>::value) {
#pragma unroll
        for (int q = 0; q < RB; q += 2) {
            const dbl2_t a = *reinterpret_cast<const dbl2_t *>(p + q);
            d[q] = a.x;
            d[q + 1] = a.y;
        }
    } else {
#pragma unroll
        for (int q = 0; q < RB; q += 4) {
            const trace_flt4_t a = *reinterpret_cast<const trace_flt4_t *>(p + q);
            d[q] = a.x;
            d[q + 1] = a.y;
            d[q + 2] = a.z;
            d[q + 3] = a.w;
        }
    }
}
template <int RB, typename T>
__device__ __forceinline__ void store_rb(T *__restrict__ p, const double (&d)[RB]) {
    // streaming stores: the outputs are not read again by this launch
    if constexpr (std::is_same<T, double>::value) {
#pragma unroll
        for (int q = 0; q < RB; q += 2)
            __builtin_nontemporal_store(dbl2_t{d[q], d[q + 1]}, reinterpret_cast<dbl2_t *>(p + q));
    } else {
#pragma unroll
        for (int q = 0; q < RB; q += 4)
            __builtin_nontemporal_store(trace_flt4_t{(float)d[q], (float)d[q + 1], (float)d[q + 2], (float)d[q + 3]},
                                        reinterpret_cast<trace_flt4_t *>(p + q));
    }
}

// RB consecutive values in their stored type, 16 bytes per load
template <int RB, typename T>
__device__ __forceinline__ void load_raw(const T *__restrict__ p, T (&d)[RB]) {
    if constexpr (std::is_same<T, double>::value) {
#pragma unroll
        for (int q = 0; q < RB; q += 2) {
            const dbl2_t a = *reinterpret_cast<const dbl2_t *>(p + q);
            d[q] = a.x;
            d[q + 1] = a.y;
        }
    } else {
#pragma unroll
        for (int q = 0; q < RB; q += 4) {
            const trace_flt4_t a = *reinterpret_cast<const trace_flt4_t *>(p + q);
            d[q] = a.x;
            d[q + 1] = a.y;
            d[q + 2] = a.z;
            d[q + 3] = a.w;
        }
    }
}

// RB consecutive values in their stored type, 16 bytes per store
template <int RB, typename T>
__device__ __forceinline__ void store_raw(T *__restrict__ p, const T (&d)[RB]) {
    if constexpr (std::is_same<T, double>::value) {
#pragma unroll
        for (int q = 0; q < RB; q += 2) *reinterpret_cast<dbl2_t *>(p + q) = dbl2_t{d[q], d[q + 1]};
    } else {
#pragma unroll
        for (int q = 0; q < RB; q += 4)
            *reinterpret_cast<trace_flt4_t *>(p + q) = trace_flt4_t{d[q], d[q + 1], d[q + 2], d[q + 3]};
    }
}

// RB consecutive values of a sweep's vectors in its arithmetic type (SweepT):
// FP32 vectors stay FP32, FP64 vectors (or FP32 ones in an FP64 sweep) are read as double
template <int RB, typename T, typename C>
__device__ __forceinline__ void load_ct(const T *__restrict__ p, C (&d)[RB]) {
    if constexpr (std::is_same<C, double>::value) load_rb<RB>(p, d);
    else load_raw<RB>(p, d);
}
template <int RB, typename T, typename C>
__device__ __forceinline__ void store_ct(T *__restrict__ p, const C (&d)[RB]) {
    if constexpr (std::is_same<C, double>::value) {
        store_rb<RB>(p, d);
    } else {
#pragma unroll
        for (int q = 0; q < RB; q += 4)
            __builtin_nontemporal_store(trace_flt4_t{d[q], d[q + 1], d[q + 2], d[q + 3]},
                                        reinterpret_cast<trace_flt4_t *>(p + q));
    }
}

// ---------------------------------------------------------------- P1 levels, four right-hand sides per thread
// With nb % 4 == 0 a thread of the P1 level kernels takes four consecutive
// right-hand sides of one vertex: each index and matrix entry is loaded once
// for four values, vector values move in 16-byte loads (32 bytes for FP64
// vectors), and a launch has a quarter of the wavefronts of the per-(vertex,
// rhs) form, each with four times the loads in flight.  The arithmetic per
// entry is the per-(vertex, rhs) kernels', so the two shapes give the same bits.

template <typename VT>
__device__ __forceinline__ void p1_st4(VT *__restrict__ p, const double (&d)[4]) {
    if constexpr (std::is_same<VT, double>::value) {
        *reinterpret_cast<dbl2_t *>(p) = dbl2_t{d[0], d[1]};
        *reinterpret_cast<dbl2_t *>(p + 2) = dbl2_t{d[2], d[3]};
    } else {
        *reinterpret_cast<trace_flt4_t *>(p) = trace_flt4_t{(float)d[0], (float)d[1], (float)d[2], (float)d[3]};
    }
}

// s = (A x)[v] at right-hand sides r0..r0+3: diagonal term first, then the ELL entries in order
template <int WT, typename VT>
__device__ __forceinline__ void p1_ax4(int v, int n, int W, int nb, int r0, const int *ell_col,
                                       const double *ell_val, const double *diag, const VT *x, double (&s)[4]) {
    if (WT) W = WT;
    double xv[4];
    load_rb<4>(x + (size_t)v * nb + r0, xv);
    const double d = diag[v];
#pragma unroll
    for (int q = 0; q < 4; ++q) s[q] = d * xv[q];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const double a = ell_val[(size_t)k * n + v];
        double xu[4];
        load_rb<4>(x + (size_t)ell_col[(size_t)k * n + v] * nb + r0, xu);
#pragma unroll
        for (int q = 0; q < 4; ++q) s[q] += a * xu[q];
    }
}

// thread -> (vertex v, first right-hand side r0); false past the end
__device__ __forceinline__ bool p1_thread4(int n, int nb, int &v, int &r0) {
    const int tpv = nb >> 2;
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= n * tpv) return false;
    v = t / tpv;
    r0 = (t - v * tpv) * 4;
    return true;
}

template <typename VT>
__global__ void k_p1_first4(int n, int nb, const double *__restrict__ dinv, double omega,
                            const VT *__restrict__ b, VT *__restrict__ x) {
    int v, r0;
    if (!p1_thread4(n, nb, v, r0)) return;
    const size_t o = (size_t)v * nb + r0;
    double bv[4], out[4];
    load_rb<4>(b + o, bv);
    const double dv = dinv[v];
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = omega * dv * bv[q];
    p1_st4(x + o, out);
}

template <int WT, typename VT>
__global__ void k_p1_pre2_4(int n, int W, int nb, const int *__restrict__ ell_col, const double *__restrict__ ell_val,
                            const double *__restrict__ diag, const double *__restrict__ dinv, double omega,
                            const VT *__restrict__ b, VT *__restrict__ x) {
    int v, r0;
    if (!p1_thread4(n, nb, v, r0)) return;
    if (WT) W = WT;
    const size_t o = (size_t)v * nb + r0;
    double bv[4], ax[4], out[4];
    load_rb<4>(b + o, bv);
    const double dv = dinv[v], dd = diag[v];
#pragma unroll
    for (int q = 0; q < 4; ++q) ax[q] = dd * omega * dv * bv[q];
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const int u = ell_col[(size_t)k * n + v];
        const double a = ell_val[(size_t)k * n + v], du = dinv[u];
        double bu[4];
        load_rb<4>(b + (size_t)u * nb + r0, bu);
#pragma unroll
        for (int q = 0; q < 4; ++q) ax[q] += a * omega * du * bu[q];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const double x1 = omega * dv * bv[q];
        out[q] = x1 + omega * dv * (bv[q] - ax[q]);
    }
    p1_st4(x + o, out);
}

template <int WT, typename VT>
__global__ void k_p1_sweep4(int n, int W, int nb, const int *__restrict__ ell_col, const double *__restrict__ ell_val,
                            const double *__restrict__ diag, const double *__restrict__ dinv, double omega,
                            const VT *__restrict__ b, const VT *__restrict__ x, VT *__restrict__ y) {
    int v, r0;
    if (!p1_thread4(n, nb, v, r0)) return;
    const size_t o = (size_t)v * nb + r0;
    double ax[4], xv[4], bv[4], out[4];
    p1_ax4<WT>(v, n, W, nb, r0, ell_col, ell_val, diag, x, ax);
    load_rb<4>(x + o, xv);
    load_rb<4>(b + o, bv);
    const double dv = dinv[v];
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = xv[q] + omega * dv * (bv[q] - ax[q]);
    p1_st4(y + o, out);
}

template <typename VT>
__global__ void k_p1_prolong4(int n, int nb, const int *__restrict__ parents, const VT *__restrict__ xc,
                              VT *__restrict__ x) {
    int v, r0;
    if (!p1_thread4(n, nb, v, r0)) return;
    const size_t o = (size_t)v * nb + r0;
    double xv[4], c0[4], c1[4], out[4];
    load_rb<4>(x + o, xv);
    load_rb<4>(xc + (size_t)parents[2 * v] * nb + r0, c0);
    load_rb<4>(xc + (size_t)parents[2 * v + 1] * nb + r0, c1);
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = xv[q] + 0.5 * (c0[q] + c1[q]);
    p1_st4(x + o, out);
}

template <int WT, typename VT>
__global__ void k_p1_resid4(int n, int W, int nb, const int *__restrict__ ell_col, const double *__restrict__ ell_val,
                            const double *__restrict__ diag, const VT *__restrict__ b, const VT *__restrict__ x,
                            VT *__restrict__ y) {
    int v, r0;
    if (!p1_thread4(n, nb, v, r0)) return;
    const size_t o = (size_t)v * nb + r0;
    double ax[4], bv[4], out[4];
    p1_ax4<WT>(v, n, W, nb, r0, ell_col, ell_val, diag, x, ax);
    load_rb<4>(b + o, bv);
#pragma unroll
    for (int q = 0; q < 4; ++q) out[q] = bv[q] - ax[q];
    p1_st4(y + o, out);
}

// the children of a coarse vertex eight at a time (index clamped, surplus terms
// dropped), summed in list order as in the per-(vertex, rhs) restriction
template <typename VT>
__global__ void k_p1_restrict4(int nc, int nb, const int *__restrict__ crow, const int *__restrict__ ccol,
                               const double *__restrict__ cw, const VT *__restrict__ r, VT *__restrict__ bc) {
    int c, r0;
    if (!p1_thread4(nc, nb, c, r0)) return;
    const int k0 = crow[c], cnt = crow[c + 1] - k0;
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int g = 0; g < cnt; g += 8) {
        double t[8][4];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + min(g + u, cnt - 1);
            const double w = cw[k];
            double rv[4];
            load_rb<4>(r + (size_t)ccol[k] * nb + r0, rv);
#pragma unroll
            for (int q = 0; q < 4; ++q) t[u][q] = w * rv[q];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u)
#pragma unroll
            for (int q = 0; q < 4; ++q) s[q] = g + u < cnt ? s[q] + t[u][q] : s[q];
    }
    p1_st4(bc + (size_t)c * nb + r0, s);
}

// x = Ainv b on the coarsest level, one 256-thread block per row i.  A thread
// takes G consecutive right-hand sides (G = 4 when nb = 4 NQ with NQ a power of
// two, G = 1 when nb = 1) and one of the block's 256 / NQ phases j = phase +
// k (256 / NQ), four columns' loads in flight at a time.  The partial sums are
// combined by a butterfly within each wavefront and then over the four
// wavefronts in order: a fixed summation order for a given nb.
template <int G, typename VT>
__global__ __launch_bounds__(256) void k_dense_row(int n, int nb, const double *__restrict__ Ainv,
                                                   const VT *__restrict__ b, VT *__restrict__ x) {
    __shared__ double part[4][64];
    const int i = blockIdx.x, tid = threadIdx.x;
    const int NQ = nb / G, JP = 256 / NQ;
    const int rq = tid & (NQ - 1), jp = tid / NQ, r0 = rq * G;
    const double *Ai = Ainv + (size_t)i * n;
    double s[G];
#pragma unroll
    for (int g = 0; g < G; ++g) s[g] = 0.0;
    for (int j0 = jp; j0 < n; j0 += 4 * JP) {
        double a[4], bv[4][G];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = min(j0 + u * JP, n - 1);
            a[u] = Ai[j];
            if constexpr (G == 4) load_rb<4>(b + (size_t)j * nb + r0, bv[u]);
            else bv[u][0] = (double)b[j];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (j0 + u * JP < n)
#pragma unroll
                for (int g = 0; g < G; ++g) s[g] += a[u] * bv[u][g];
    }
    for (int off = NQ; off < 64; off <<= 1)
#pragma unroll
        for (int g = 0; g < G; ++g) s[g] += __shfl_xor(s[g], off, 64);
    const int wv = tid >> 6, lane = tid & 63;
    if (lane < NQ)
#pragma unroll
        for (int g = 0; g < G; ++g) part[wv][lane * G + g] = s[g];
    __syncthreads();
    if (tid < nb) x[(size_t)i * nb + tid] = (VT)(((part[0][tid] + part[1][tid]) + part[2][tid]) + part[3][tid]);
}

// y = S x or y = b - S x
//
// Latency: a lane requests its four neighbour ids and its own facet's values
// before the block stages its rows, so those waits overlap the staging; each
// neighbour then costs one wait (its values), not two (id, then values).
template <int M, typename MT, typename XT, typename YT, int RB, typename BT = YT>
__global__ __launch_bounds__(1024) void k_trace_apply_rb(int ne, int nb, const MT *__restrict__ S,
                                                         const int *__restrict__ nbr, const XT *__restrict__ x,
                                                         const BT *__restrict__ b, YT *__restrict__ y) {
    using AT = typename Acc<MT>::type;
    constexpr int V = Wide<MT>::V, C = 5 * M * M, G = padded(C, V) / V;
    __shared__ __attribute__((aligned(16))) MT sm[G * RB_FACETS * V];
    const int f0 = xcd_block() * RB_FACETS;
    const int tpf = nb / RB;
    const int el = threadIdx.x / tpf, r0 = (threadIdx.x - el * tpf) * RB, e = f0 + el;
    const bool live = e < ne;
    const size_t NE = (size_t)ne;
    int id[4] = {0, 0, 0, 0};
    XT xa[M][RB];
    auto fetch = [&](int f, XT (&xv)[M][RB]) {
#pragma unroll
        for (int k = 0; k < M; ++k) load_raw<RB>(x + ((size_t)f * M + k) * nb + r0, xv[k]);
    };
    if (live) {
#pragma unroll
        for (int j = 0; j < 4; ++j) id[j] = nbr[(size_t)j * NE + e];
        fetch(e, xa);
    }
    stage_rows<MT, G>(sm, S, f0, ne);
    __syncthreads();
    if (!live) return;
    AT acc[M][RB];
#pragma unroll
    for (int a = 0; a < M; ++a)
#pragma unroll
        for (int q = 0; q < RB; ++q) acc[a][q] = 0;
    auto mac = [&](int j, const XT (&xv)[M][RB]) {
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const int c = (j * M + a) * M + k;
                const AT w = lds_entry<MT>(sm + ((size_t)(c / V) * RB_FACETS + el) * V + c % V);
#pragma unroll
                for (int q = 0; q < RB; ++q) acc[a][q] += w * (AT)xv[k][q];
            }
    };
    mac(0, xa);
#pragma unroll 1
    for (int j = 1; j < 5; ++j) {   // one neighbour's values in flight at a time keeps the registers in bounds
        const int f = j == 1 ? id[0] : j == 2 ? id[1] : j == 3 ? id[2] : id[3];
        fetch(f, xa);
        mac(j, xa);
    }
#pragma unroll
    for (int a = 0; a < M; ++a) {
        const size_t o = ((size_t)e * M + a) * nb + r0;
        double out[RB];
        if (b) {
            double bv[RB];
            load_rb<RB>(b + o, bv);
#pragma unroll
            for (int q = 0; q < RB; ++q) out[q] = bv[q] - (double)acc[a][q];
        } else {
#pragma unroll
            for (int q = 0; q < RB; ++q) out[q] = (double)acc[a][q];
        }
        store_rb<RB>(y + o, out);
    }
}

// the generalised sweep y = a0 x' + a1 z0 - a3 sum_j T_j x'_j + a2 xprev' (SweepCoef)
// The FP32 sweep with bf16 rows is held to 80 registers (six waves per SIMD).
template <typename MT, typename VT>
constexpr int sweep_rb_waves() { return std::is_same<MT, __hip_bfloat16>::value && std::is_same<VT, float>::value ? 6 : 1; }
template <int M, typename MT, typename VT, int RB>
__global__ __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(sweep_rb_waves<MT, VT>(), 8))) void k_sweep_rb(int ne, int nb, const MT *__restrict__ T,
                                                   const int *__restrict__ nbr, const VT *__restrict__ x,
                                                   const VT *__restrict__ z0, const VT *__restrict__ qc,
                                                   const int *__restrict__ fvert, SweepCoef cf,
                                                   VT *__restrict__ y) {
    using AT = typename Acc<MT>::type;
    using CT = SweepT<VT>;
    constexpr int P = M - 1;
    constexpr int V = Wide<MT>::V, C = 4 * M * M, G = padded(C, V) / V;
    __shared__ __attribute__((aligned(16))) MT sm[G * RB_FACETS * V];
    const int f0 = xcd_block() * RB_FACETS;
    const int tpf = nb / RB;
    const int el = threadIdx.x / tpf, r0 = (threadIdx.x - el * tpf) * RB, e = f0 + el;
    const bool live = e < ne;
    const size_t NE = (size_t)ne;
    // Neighbour ids (and, with a fused prolongation, their vertex ids) are
    // requested before the rows are staged.  Neighbour values are held in the
    // accumulation type (the same rounding as converting at the product), and
    // the own facet's values are read node by node in the epilogue: both keep
    // the register count, and so the number of waves in flight, up.
    int id[4] = {0, 0, 0, 0}, iv[4][2] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
    if (live) {
#pragma unroll
        for (int j = 0; j < 4; ++j) id[j] = nbr[(size_t)j * NE + e];
        if (qc)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                iv[j][0] = fvert[2 * id[j]];
                iv[j][1] = fvert[2 * id[j] + 1];
            }
    }
    stage_rows<MT, G>(sm, T, f0, ne);
    __syncthreads();
    if (!live) return;
    AT acc[M][RB];
#pragma unroll
    for (int a = 0; a < M; ++a)
#pragma unroll
        for (int q = 0; q < RB; ++q) acc[a][q] = 0;
#pragma unroll 1
    for (int j = 0; j < 4; ++j) {   // one neighbour's values in flight at a time keeps the registers in bounds
        const int f = j == 0 ? id[0] : j == 1 ? id[1] : j == 2 ? id[2] : id[3];
        VT raw[M][RB];
        AT xv[M][RB];
#pragma unroll
        for (int k = 0; k < M; ++k) load_raw<RB>(x + ((size_t)f * M + k) * nb + r0, raw[k]);
        if (qc) {
            const int v0 = j == 0 ? iv[0][0] : j == 1 ? iv[1][0] : j == 2 ? iv[2][0] : iv[3][0];
            const int v1 = j == 0 ? iv[0][1] : j == 1 ? iv[1][1] : j == 2 ? iv[2][1] : iv[3][1];
            CT q0[RB], q1[RB];
            load_ct<RB>(qc + (size_t)v0 * nb + r0, q0);
            load_ct<RB>(qc + (size_t)v1 * nb + r0, q1);
#pragma unroll
            for (int k = 0; k < M; ++k)
#pragma unroll
                for (int q = 0; q < RB; ++q) xv[k][q] = (AT)((CT)raw[k][q] + p1_node<P>(k, q0[q], q1[q]));
        } else {
#pragma unroll
            for (int k = 0; k < M; ++k)
#pragma unroll
                for (int q = 0; q < RB; ++q) xv[k][q] = (AT)raw[k][q];
        }
#pragma unroll
        for (int a = 0; a < M; ++a)
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const int c = (j * M + a) * M + k;
                const AT w = lds_entry<MT>(sm + ((size_t)(c / V) * RB_FACETS + el) * V + c % V);
#pragma unroll
                for (int q = 0; q < RB; ++q) acc[a][q] += w * xv[k][q];
            }
    }
    CT q0[RB], q1[RB], p0[RB], p1[RB];
    if (qc) {
        load_ct<RB>(qc + (size_t)fvert[2 * e] * nb + r0, q0);
        load_ct<RB>(qc + (size_t)fvert[2 * e + 1] * nb + r0, q1);
    }
    if (cf.xprev && cf.qcprev) {
        const VT *qp = static_cast<const VT *>(cf.qcprev);
        load_ct<RB>(qp + (size_t)fvert[2 * e] * nb + r0, p0);
        load_ct<RB>(qp + (size_t)fvert[2 * e + 1] * nb + r0, p1);
    }
#pragma unroll
    for (int a = 0; a < M; ++a) {
        const size_t o = ((size_t)e * M + a) * nb + r0;
        CT xe[RB], zv[RB], out[RB];
        load_ct<RB>(x + o, xe);
        load_ct<RB>(z0 + o, zv);
        if (qc)
#pragma unroll
            for (int q = 0; q < RB; ++q) xe[q] += p1_node<P>(a, q0[q], q1[q]);
#pragma unroll
        for (int q = 0; q < RB; ++q) out[q] = sweep_combine(cf, xe[q], zv[q], (CT)acc[a][q]);
        if (cf.xprev) {
            CT pv[RB];
            load_ct<RB>(static_cast<const VT *>(cf.xprev) + o, pv);
            if (cf.qcprev)
#pragma unroll
                for (int q = 0; q < RB; ++q) pv[q] += p1_node<P>(a, p0[q], p1[q]);
#pragma unroll
            for (int q = 0; q < RB; ++q) out[q] = sweep_prev(cf.a2, pv[q], out[q]);
        }
        store_ct<RB>(y + o, out);
    }
}

// z0 = omega D^-1 r with RB consecutive right-hand sides per thread (16-byte
// loads and stores of r, rs, rc and z0); the same arithmetic per entry as k_jacobi0,
// so the two shapes give the same bits.
template <int M, typename MT, typename RT, typename ZT, int RB>
__global__ __launch_bounds__(256) void k_jacobi0_rb(int ne, int nb, const MT *__restrict__ Dw,
                                                    const RT *__restrict__ r, const double *__restrict__ scale,
                                                    RT *__restrict__ rs, ZT *__restrict__ rc, ZT *__restrict__ z0,
                                                    GsLag gs) {
    using AT = typename Acc<MT>::type;
    constexpr int V = Wide<MT>::V, C = M * M, G = padded(C, V) / V;
    const int tpf = nb / RB;
    const int t = xcd_block() * blockDim.x + threadIdx.x;
    if (t >= ne * tpf) return;
    const int e = t / tpf, r0 = (t - e * tpf) * RB;
    const size_t NE = (size_t)ne;
    double sc[RB];
#pragma unroll
    for (int q = 0; q < RB; ++q) sc[q] = scale ? (scale[r0 + q] != 0.0 ? 1.0 / scale[r0 + q] : 0.0) : 1.0;
    ZT rz[M][RB];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        const size_t o = ((size_t)e * M + k) * nb + r0;
        RT v[RB];
        load_raw<RB>(r + o, v);
        double rk[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) rk[q] = (double)v[q];
        const int gnd = (gs.done && *gs.done) ? 0 : gs.nd;
        for (int d = 0; d < gnd; ++d) {
            RT vd[RB];
            load_raw<RB>(static_cast<const RT *>(gs.V) + (size_t)d * gs.vstride + o, vd);
#pragma unroll
            for (int q = 0; q < RB; ++q) rk[q] -= gs.h[(size_t)d * nb + r0 + q] * (double)vd[q];
        }
#pragma unroll
        for (int q = 0; q < RB; ++q) {
            v[q] = (RT)(rk[q] * sc[q]);          // the scaled vector as stored
            rz[k][q] = (ZT)v[q];                 // ... and as the V-cycle reads it
        }
        if (scale) store_raw<RB>(rs + o, v);
        if (rc) store_raw<RB>(rc + o, rz[k]);
    }
    AT acc[M][RB];
#pragma unroll
    for (int a = 0; a < M; ++a)
#pragma unroll
        for (int q = 0; q < RB; ++q) acc[a][q] = 0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        AT w[V];
        Wide<MT>::load(Dw + ((size_t)g * NE + e) * V, w);
#pragma unroll
        for (int v = 0; v < V; ++v) {
            const int c = g * V + v;
            if (c < C)
#pragma unroll
                for (int q = 0; q < RB; ++q) acc[c / M][q] += w[v] * (AT)(double)rz[c % M][q];
        }
    }
#pragma unroll
    for (int a = 0; a < M; ++a) {
        ZT out[RB];
#pragma unroll
        for (int q = 0; q < RB; ++q) out[q] = (ZT)(double)acc[a][q];
        store_raw<RB>(z0 + ((size_t)e * M + a) * nb + r0, out);
    }
}

// RHS-blocked launch applies when nb / 4 is a power of two <= 16
bool rhs_blocked(int nb, int rhs_block) {
    if (rhs_block != 4 || nb < 4 || nb % 4 != 0) return false;
    const int t = nb / 4;
    return t <= 16 && (t & (t - 1)) == 0;
}

#define GRID_RB(ne, nb) dim3((unsigned)((((ne) + RB_FACETS - 1) / RB_FACETS + N_XCD - 1) / N_XCD * N_XCD)), dim3(RB_FACETS * ((nb) / 4))

#define GRID8(n, b) dim3((unsigned)((((n) + (b) - 1) / (b) + N_XCD - 1) / N_XCD * N_XCD)), dim3(b)

void launch_cell_condense(int p, int nu, int nk, const double *corners, const double *ref, CellParams cp,
                          double *Sloc, double *Zr, double *Ar, double *Wr, int *err, hipStream_t s, double *Aout,
                          double *Bnout) {
    const int pairs = (nk + 1) / 2;   // two cells per wavefront
#define CK(P, NU) hipLaunchKernelGGL((k_cell_condense<P, NU>), dim3((unsigned)((pairs + N_XCD - 1) / N_XCD * N_XCD)), dim3(64), 0, s, nk, corners, ref, cp, Sloc, Zr, Ar, Wr, err, Aout, Bnout)
    if (nu == 1) { switch (p) { case 1: CK(1, 1); break; case 2: CK(2, 1); break; case 3: CK(3, 1); break; } }
    else { switch (p) { case 1: CK(1, 2); break; case 2: CK(2, 2); break; case 3: CK(3, 2); break; } }
#undef CK
}

void launch_facet_rows(int p, int nu, int ne, int nk, const double *Sloc, const int *facet_cell,
                       const int *facet_loc, const int *cell_facet, const int8_t *cell_rev, double omega,
                       double *S64, double *T64, double *Dw64, float *S32, __hip_bfloat16 *T16, float *Dw32,
                       int *nbr, int8_t *prev, int *err, hipStream_t s) {
#define FR(P, NU) hipLaunchKernelGGL((k_facet_rows<P, NU>), GRID(ne, 128), 0, s, ne, nk, Sloc, facet_cell, facet_loc, cell_facet, cell_rev, omega, S64, T64, Dw64, S32, T16, Dw32, nbr, prev, err)
    if (nu == 1) { switch (p) { case 1: FR(1, 1); break; case 2: FR(2, 1); break; case 3: FR(3, 1); break; } }
    else { switch (p) { case 1: FR(1, 2); break; case 2: FR(2, 2); break; case 3: FR(3, 2); break; } }
#undef FR
}

// Facet-row launchers take M, the trace unknowns per facet: p + 1 (upwind) or
// 2 (p + 1) (Lax-Friedrichs).  The RHS-blocked forms stage 64 facets' rows in
// LDS and are built for M <= 4.
bool rhs_blocked_m(int M, int nb, int rhs_block) { return M <= 4 && rhs_blocked(nb, rhs_block); }

#define M_SWITCH(X) \
    switch (M) { case 2: X(2); break; case 3: X(3); break; case 4: X(4); break; case 6: X(6); break; case 8: X(8); break; }
#define M_SWITCH_RB(X) switch (M) { case 2: X(2); break; case 3: X(3); break; case 4: X(4); break; }

template <typename MT, typename XT, typename YT>
void launch_trace_apply(int M, int ne, int nb, const MT *S, const int *nbr, const XT *x, const YT *b, YT *y,
                        hipStream_t s, int rhs_block) {
    if (rhs_blocked_m(M, nb, rhs_block)) {
#define TAB(MM) hipLaunchKernelGGL((k_trace_apply_rb<MM, MT, XT, YT, 4>), GRID_RB(ne, nb), 0, s, ne, nb, S, nbr, x, b, y)
        M_SWITCH_RB(TAB)
#undef TAB
        return;
    }
#define TA(MM)                                                                                          \
    if (nb == 1) hipLaunchKernelGGL((k_trace_apply<MM, MT, XT, YT, true>), GRID8(ne * nb, 256), 0, s, ne, nb, S, nbr, x, b, y); \
    else hipLaunchKernelGGL((k_trace_apply<MM, MT, XT, YT, false>), GRID8(ne * nb, 256), 0, s, ne, nb, S, nbr, x, b, y)
    M_SWITCH(TA)
#undef TA
}
// FP64 residual b - S x rounded once to FP32 on output (the first vector of the
// FP32 inner solve of a refinement step)
void launch_trace_residual_f32(int M, int ne, int nb, const double *S, const int *nbr, const double *x,
                               const double *b, float *y, hipStream_t s, int rhs_block) {
    if (rhs_blocked_m(M, nb, rhs_block)) {
#define TAB(MM) hipLaunchKernelGGL((k_trace_apply_rb<MM, double, double, float, 4, double>), GRID_RB(ne, nb), 0, s, ne, nb, S, nbr, x, b, y)
        M_SWITCH_RB(TAB)
#undef TAB
        return;
    }
#define TA(MM)                                                                                          \
    if (nb == 1) hipLaunchKernelGGL((k_trace_apply<MM, double, double, float, true, double>), GRID8(ne * nb, 256), 0, s, ne, nb, S, nbr, x, b, y); \
    else hipLaunchKernelGGL((k_trace_apply<MM, double, double, float, false, double>), GRID8(ne * nb, 256), 0, s, ne, nb, S, nbr, x, b, y)
    M_SWITCH(TA)
#undef TA
}
#define INST_TA(MT, XT, YT) \
    template void launch_trace_apply<MT, XT, YT>(int, int, int, const MT *, const int *, const XT *, const YT *, YT *, hipStream_t, int);
INST_TA(double, double, double)
INST_TA(float, double, double)
INST_TA(double, float, float)
INST_TA(float, float, float)
INST_TA(double, float, double)
INST_TA(float, float, double)
INST_TA(double, double, float)
INST_TA(float, double, float)
#undef INST_TA

template <typename MT, typename RT, typename ZT>
void launch_jacobi0(int M, int ne, int nb, const MT *Dw, const RT *r, const double *scale, RT *rs, ZT *rc, ZT *z0,
                    hipStream_t s, GsLag gs) {
    if (M <= 4 && nb % 4 == 0) {   // four right-hand sides per thread
#define J0B(MM) hipLaunchKernelGGL((k_jacobi0_rb<MM, MT, RT, ZT, 4>), GRID8(ne * (nb / 4), 256), 0, s, ne, nb, Dw, r, scale, rs, rc, z0, gs)
        M_SWITCH_RB(J0B)
#undef J0B
        return;
    }
#define J0(MM) hipLaunchKernelGGL((k_jacobi0<MM, MT, RT, ZT>), GRID8(ne * nb, 256), 0, s, ne, nb, Dw, r, scale, rs, rc, z0, gs)
    M_SWITCH(J0)
#undef J0
}
#define INST_J0(MT, RT, ZT) \
    template void launch_jacobi0<MT, RT, ZT>(int, int, int, const MT *, const RT *, const double *, RT *, ZT *, ZT *, hipStream_t, GsLag);
INST_J0(double, double, double)
INST_J0(float, double, double)
INST_J0(double, float, float)
INST_J0(float, float, float)
INST_J0(double, double, float)
INST_J0(float, double, float)
INST_J0(double, float, double)
INST_J0(float, float, double)
#undef INST_J0

// qc (the fused P1 prolongation) applies to the upwind trace only: M = p + 1.
template <typename MT, typename VT>
void launch_sweep(int M, int ne, int nb, const MT *T, const int *nbr, const VT *x, const VT *z0, const double *qc,
                  const int *fvert, SweepCoef cf, VT *y, hipStream_t s, int rhs_block) {
    const VT *qv = reinterpret_cast<const VT *>(qc);   // P1 values in the sweep's vector type
    if (rhs_blocked_m(M, nb, rhs_block)) {
#define SWB(MM) hipLaunchKernelGGL((k_sweep_rb<MM, MT, VT, 4>), GRID_RB(ne, nb), 0, s, ne, nb, T, nbr, x, z0, qv, fvert, cf, y)
        M_SWITCH_RB(SWB)
#undef SWB
        return;
    }
#define SW(MM)                                                                                                \
    if (nb == 1) hipLaunchKernelGGL((k_sweep<MM, MT, VT, true>), GRID8(ne * nb, 256), 0, s, ne, nb, T, nbr, x, z0, qv, fvert, cf, y); \
    else hipLaunchKernelGGL((k_sweep<MM, MT, VT, false>), GRID8(ne * nb, 256), 0, s, ne, nb, T, nbr, x, z0, qv, fvert, cf, y)
    M_SWITCH(SW)
#undef SW
}
template void launch_sweep<double, double>(int, int, int, const double *, const int *, const double *, const double *, const double *, const int *, SweepCoef, double *, hipStream_t, int);
template void launch_sweep<__hip_bfloat16, double>(int, int, int, const __hip_bfloat16 *, const int *, const double *, const double *, const double *, const int *, SweepCoef, double *, hipStream_t, int);
template void launch_sweep<__hip_bfloat16, float>(int, int, int, const __hip_bfloat16 *, const int *, const float *, const float *, const double *, const int *, SweepCoef, float *, hipStream_t, int);
template void launch_sweep<double, float>(int, int, int, const double *, const int *, const float *, const float *, const double *, const int *, SweepCoef, float *, hipStream_t, int);

template <typename VT>
void launch_restrict_trace(int p, int nv, int nb, const int *vf_row, const int *vf_col, const VT *res, double *rc,
                           hipStream_t s) {
    VT *rcv = reinterpret_cast<VT *>(rc);   // the P1 vector in the residual's type
#define RT(P) hipLaunchKernelGGL((k_restrict_trace<P + 1, VT>), GRID8(nv * nb, 256), 0, s, nv, nb, vf_row, vf_col, res, rcv)
    switch (p) { case 1: RT(1); break; case 2: RT(2); break; case 3: RT(3); break; }
#undef RT
}
template void launch_restrict_trace<double>(int, int, int, const int *, const int *, const double *, double *, hipStream_t);
template void launch_restrict_trace<float>(int, int, int, const int *, const int *, const float *, double *, hipStream_t);


// P1 launchers: the level vectors hold double values, or float values in the
// same buffers when f32 is set (the V-cycle of a mixed-precision solve).
template <typename VT>
static VT *pv(double *p) { return reinterpret_cast<VT *>(p); }
template <typename VT>
static const VT *pv(const double *p) { return reinterpret_cast<const VT *>(p); }
#define P1_TYPED(CALL) \
    if (f32) { using VT = float; CALL; } else { using VT = double; CALL; }

// rb == 4 with nb % 4 == 0: four right-hand sides per thread (same bits)
static bool p1_r4(int rb, int nb) { return rb == 4 && nb % 4 == 0; }
#define P1_GRID(n, nb, r4) GRID8((int64_t)(n) * ((r4) ? (nb) / 4 : (nb)), 256)

void launch_p1_first(int n, int nb, const double *dinv, double omega, const double *b, double *x, hipStream_t s,
                     bool f32, int rb) {
    const bool r4 = p1_r4(rb, nb);
    P1_TYPED(if (r4) hipLaunchKernelGGL(k_p1_first4<VT>, P1_GRID(n, nb, r4), 0, s, n, nb, dinv, omega, pv<VT>(b),
                                        pv<VT>(x));
             else hipLaunchKernelGGL(k_p1_first<VT>, P1_GRID(n, nb, r4), 0, s, n, nb, dinv, omega, pv<VT>(b),
                                     pv<VT>(x)))
}
void launch_p1_pre2(int n, int W, int nb, const int *col, const double *val, const double *diag,
                    const double *dinv, double omega, const double *b, double *x, hipStream_t s, bool f32, int rb) {
    const bool r4 = p1_r4(rb, nb);
#define PRE2(K, WW) hipLaunchKernelGGL((K<WW, VT>), P1_GRID(n, nb, r4), 0, s, n, W, nb, col, val, diag, dinv, omega, \
                                       pv<VT>(b), pv<VT>(x))
    P1_TYPED(if (r4) { if (W == 6) PRE2(k_p1_pre2_4, 6); else PRE2(k_p1_pre2_4, 0); }
             else { if (W == 6) PRE2(k_p1_pre2, 6); else PRE2(k_p1_pre2, 0); })
#undef PRE2
}
#define SWPP(WW) hipLaunchKernelGGL((k_p1_sweep_prolong<WW, VT>), P1_GRID(n, 1, false), 0, s, n, W, col, val, diag, \
                                    dinv, omega, pv<VT>(b), pv<VT>(x), parents, pv<VT>(xc), pv<VT>(y))
void launch_p1_sweep(int n, int W, int nb, const int *col, const double *val, const double *diag,
                     const double *dinv, double omega, const double *b, double *x, const double *xc,
                     const int *parents, double *y, hipStream_t s, bool f32, int rb) {
    const bool r4 = p1_r4(rb, nb);
#define SWP(K, WW) hipLaunchKernelGGL((K<WW, VT>), P1_GRID(n, nb, r4), 0, s, n, W, nb, col, val, diag, dinv, omega, \
                                      pv<VT>(b), pv<VT>(x), pv<VT>(y))
    P1_TYPED(
        if (xc && nb == 1) {
            if (W == 6) SWPP(6); else SWPP(0);
            return;
        }
        if (xc) {
            if (r4) hipLaunchKernelGGL(k_p1_prolong4<VT>, P1_GRID(n, nb, r4), 0, s, n, nb, parents, pv<VT>(xc), pv<VT>(x));
            else hipLaunchKernelGGL(k_p1_prolong<VT>, P1_GRID(n, nb, r4), 0, s, n, nb, parents, pv<VT>(xc), pv<VT>(x));
        }
        if (r4) { if (W == 6) SWP(k_p1_sweep4, 6); else SWP(k_p1_sweep4, 0); }
        else { if (W == 6) SWP(k_p1_sweep, 6); else SWP(k_p1_sweep, 0); })
#undef SWP
}
#undef SWPP
void launch_p1_resid(int n, int W, int nb, const int *col, const double *val, const double *diag,
                     const double *b, const double *x, double *y, hipStream_t s, bool f32, int rb) {
    const bool r4 = p1_r4(rb, nb);
#define RES(K, WW) hipLaunchKernelGGL((K<WW, VT>), P1_GRID(n, nb, r4), 0, s, n, W, nb, col, val, diag, pv<VT>(b), \
                                      pv<VT>(x), pv<VT>(y))
    P1_TYPED(if (r4) { if (W == 6) RES(k_p1_resid4, 6); else RES(k_p1_resid4, 0); }
             else { if (W == 6) RES(k_p1_resid, 6); else RES(k_p1_resid, 0); })
#undef RES
}
void launch_p1_restrict(int nc, int nb, const int *crow, const int *ccol, const double *cw, const double *r,
                        double *bc, hipStream_t s, bool f32, int rb) {
    const bool r4 = p1_r4(rb, nb);
    P1_TYPED(if (r4) hipLaunchKernelGGL(k_p1_restrict4<VT>, P1_GRID(nc, nb, r4), 0, s, nc, nb, crow, ccol, cw,
                                        pv<VT>(r), pv<VT>(bc));
             else hipLaunchKernelGGL(k_p1_restrict<VT>, P1_GRID(nc, nb, r4), 0, s, nc, nb, crow, ccol, cw, pv<VT>(r),
                                     pv<VT>(bc)))
}
void launch_p1_resid_restrict(int n, int W, const int *col, const double *val, const double *diag, const double *b,
                              const double *x, int nc, const int *crow, const int *ccol, const double *cw, double *bc,
                              hipStream_t s, bool f32) {
#define RR(WW) hipLaunchKernelGGL((k_p1_resid_restrict<WW, VT>), P1_GRID((int64_t)nc * 8, 1, false), 0, s, n, W, col, \
                                  val, diag, \
                                  pv<VT>(b), pv<VT>(x), nc, crow, ccol, cw, pv<VT>(bc))
    P1_TYPED(if (W == 6) RR(6); else RR(0))
#undef RR
}
#undef P1_GRID
// the row-block product for nb = 1 and nb = 4 NQ (NQ = 1, 2, 4, 8, 16), else a
// wavefront per (row, chunk of 8 right-hand sides)
void launch_dense_mv(int n, int nb, const double *Ainv, const double *b, double *x, hipStream_t s, bool f32) {
    const int nq = nb / 4;
    const bool g4 = nb % 4 == 0 && nq <= 16 && (nq & (nq - 1)) == 0;
    P1_TYPED(if (nb == 1) hipLaunchKernelGGL((k_dense_row<1, VT>), dim3(n), dim3(256), 0, s, n, nb, Ainv, pv<VT>(b),
                                              pv<VT>(x));
             else if (g4) hipLaunchKernelGGL((k_dense_row<4, VT>), dim3(n), dim3(256), 0, s, n, nb, Ainv, pv<VT>(b),
                                             pv<VT>(x));
             else hipLaunchKernelGGL((k_dense_mv<8, VT>), GRID((int64_t)n * ((nb + 7) / 8) * 64, 256), 0, s, n, nb,
                                     Ainv, pv<VT>(b), pv<VT>(x)))
}
void launch_p1_tail(const P1Tail &T, int nb, hipStream_t s, bool f32) {
    P1_TYPED(hipLaunchKernelGGL(k_p1_tail<VT>, dim3(1), dim3(1024), 0, s, T, nb))
}
#undef P1_TYPED

void launch_condense(int p, int nu, int nk, int ne, int nb, const double *Zr, const double *rc, double *loc,
                     const int *facet_cell, const int *facet_loc, double *rhat, hipStream_t s, int cells) {
#define CC(P, NU)                                                                                                 \
    if (nb == 1)                                                                                                  \
        hipLaunchKernelGGL((k_condense_cell_n1<P, NU>), GRID8(nk, RECOVER_TILE), 0, s, nk, Zr, rc, loc);          \
    else                                                                                                          \
        hipLaunchKernelGGL((k_condense_cell_b<P, NU>), GRID8((int64_t)nk * nb, cell_cells(nb, cell_zw(P), cells) * nb), \
                           cell_stage_bytes(nb, cell_zw(P), cell_cells(nb, cell_zw(P), cells)), s, nk, nb,          \
                           cell_cells(nb, cell_zw(P), cells), Zr, rc, loc);                                       \
    hipLaunchKernelGGL((k_condense_gather<P, NU>), GRID8(ne * NU * (P + 1) * nb, 256), 0, s, ne, nk, nb,          \
                       facet_cell, facet_loc, loc, rhat)
    if (nu == 1) { switch (p) { case 1: CC(1, 1); break; case 2: CC(2, 1); break; case 3: CC(3, 1); break; } }
    else { switch (p) { case 1: CC(1, 2); break; case 2: CC(2, 2); break; case 3: CC(3, 2); break; } }
#undef CC
}

#define RL_REC(P, NU) (3 * (P + 1) * (P + 2) / 2 + 3 * (NU) * (P + 1))   // recovery row: A^-1 Mt and W entries
void launch_recover(int p, int nu, int nk, int nb, const double *Ar, const double *Wr, const int *cell_facet,
                    const int8_t *cell_rev, const double *rc, const double *lam, double *q, hipStream_t s,
                    int cells) {
#define RC(P, NU)                                                                                              \
    if (nb == 1)                                                                                               \
        hipLaunchKernelGGL((k_recover_n1<P, NU>), GRID8(nk, RECOVER_TILE), 0, s, nk, Ar, Wr, cell_facet, cell_rev, \
                           rc, lam, q);                                                                        \
    else                                                                                                       \
        hipLaunchKernelGGL((k_recover_b<P, NU>), GRID8((int64_t)nk * nb, cell_cells(nb, RL_REC(P, NU), cells) * nb), \
                           sizeof(double) * CELL_ROWS * RL_REC(P, NU) * cell_cells(nb, RL_REC(P, NU), cells), s, nk, \
                           nb, cell_cells(nb, RL_REC(P, NU), cells), Ar, Wr, cell_facet, cell_rev, rc, lam, q)
    if (nu == 1) { switch (p) { case 1: RC(1, 1); break; case 2: RC(2, 1); break; case 3: RC(3, 1); break; } }
    else { switch (p) { case 1: RC(1, 2); break; case 2: RC(2, 2); break; case 3: RC(3, 2); break; } }
#undef RC
}

int red_grid(int64_t len, int nb) {
    // about four rows per thread; the final pass sums one partial per block
    const int rpb = [&] { int r = 1; while (r * 2 * nb <= 256) r *= 2; return r; }();
    int64_t blocks = (len + (int64_t)rpb * 4 - 1) / ((int64_t)rpb * 4);
    if (blocks < 1) blocks = 1;
    if (blocks > 2048) blocks = 2048;
    return (int)blocks;
}

template <typename VT>
void launch_dots(int64_t len, int nb, int nd, const VT *X, int64_t xstride, const VT *y, double *partial,
                 double *out, double *host, hipStream_t s) {
    const int g = red_grid(len, nb);
    hipLaunchKernelGGL(k_mdot_partial<VT>, dim3(g), dim3(256), 0, s, len, nb, nd, X, xstride, y, partial);
    hipLaunchKernelGGL(k_sum_final, dim3(nd * nb), dim3(256), 0, s, g, nd * nb, partial, out, host);
}
template <typename VT>
void launch_gs_norm_givens(int64_t len, int nb, int nd, const double *h, const VT *V, int64_t vstride, VT *w,
                           double *partial, double *hn, int j, int restart, double *gm, const double *bnorm,
                           double *resid_host, hipStream_t s, const int *run) {
    const int g = red_grid(len, nb);
    hipLaunchKernelGGL(k_gs_update_norm<VT>, dim3(g), dim3(256), 0, s, len, nb, nd, h, V, vstride, w, partial, run);
    hipLaunchKernelGGL(k_norm_givens, dim3(nb), dim3(256), 0, s, g, nb, partial, hn, j, restart, h, gm, bnorm,
                       resid_host, run);
}
void launch_pyth_givens(int nb, int j, int restart, double floor, const double *hcol, double *hn, double *gm,
                        const double *bnorm, double *resid_host, int *expl, hipStream_t s) {
    hipLaunchKernelGGL(k_pyth_givens, dim3(1), dim3(64), 0, s, nb, j, restart, floor, hcol, hn, gm, bnorm, resid_host,
                       expl);
}
void launch_pcg_update_norm(int64_t len, int nb, const double *num, const double *den, const double *p,
                            const double *w, double *x, double *res, double *partial, double *rr_host,
                            hipStream_t s) {
    const int g = red_grid(len, nb);
    hipLaunchKernelGGL(k_pcg_update_norm, dim3(g), dim3(256), 0, s, len, nb, num, den, p, w, x, res, partial);
    hipLaunchKernelGGL(k_sum_final, dim3(nb), dim3(256), 0, s, g, nb, partial, (double *)nullptr, rr_host);
}

void launch_pcg_dir(int64_t n, int nb, const double *num, const double *den, const double *z, double *p,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_pcg_dir, GRID(n * nb, 256), 0, s, n, nb, num, den, z, p);
}
template <typename VT>
void launch_lincomb(int64_t n, int nb, int nd, const double *y, const VT *Z, int64_t zstride, double *x,
                    hipStream_t s) {
    hipLaunchKernelGGL(k_lincomb<VT>, GRID(n * nb, 256), 0, s, n, nb, nd, y, Z, zstride, x);
}
template void launch_dots<double>(int64_t, int, int, const double *, int64_t, const double *, double *, double *,
                                  double *, hipStream_t);
template void launch_dots<float>(int64_t, int, int, const float *, int64_t, const float *, double *, double *,
                                 double *, hipStream_t);
template void launch_gs_norm_givens<double>(int64_t, int, int, const double *, const double *, int64_t, double *,
                                            double *, double *, int, int, double *, const double *, double *,
                                            hipStream_t, const int *);
template void launch_gs_norm_givens<float>(int64_t, int, int, const double *, const float *, int64_t, float *,
                                           double *, double *, int, int, double *, const double *, double *,
                                           hipStream_t, const int *);
template void launch_lincomb<double>(int64_t, int, int, const double *, const double *, int64_t, double *,
                                     hipStream_t);
template void launch_lincomb<float>(int64_t, int, int, const double *, const float *, int64_t, double *,
                                    hipStream_t);
void launch_copy(int64_t n, const double *src, double *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_copy, GRID(n, 256), 0, s, n, src, dst);
}
void launch_gmres_start(int nb, int restart, const double *beta2, double *gm, double *beta, hipStream_t s) {
    hipLaunchKernelGGL(k_gmres_start, GRID(nb, 64), 0, s, nb, restart, beta2, gm, beta);
}
void launch_gmres_solve(int nb, int k, int restart, const double *gm, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_gmres_solve, GRID(nb, 64), 0, s, nb, k, restart, gm, y);
}
void launch_sqrt(int nb, const double *in, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_sqrt, GRID(nb, 64), 0, s, nb, in, out);
}

}  // namespace hdg
