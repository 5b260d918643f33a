// Persistent solve of small trace systems: one workgroup per right-hand side
// runs the whole Krylov solve -- and optionally the condensation before it and
// the recovery after it (Steps 1-3) -- in a single launch.
//
// Below a few thousand trace unknowns every kernel of the multi-launch solve
// is a few waves and a solve is a chain of ~10 dependent launches per Krylov
// iteration, so its time is launch latency.  Here the trace vectors of the
// Krylov method and the V-cycle and the vectors of every P1 level live in LDS;
// the operator rows (facet blocks of S, omega D^-1 S_j, omega D^-1), the P1
// level matrices and the dense coarsest inverse are read from global memory,
// where they stay cached after the first iteration.  A workgroup of 512
// threads owns the facets (vertices, cells) thread-cyclically, and every phase
// whose output is read at other items ends with a workgroup barrier.
//
// The arithmetic is the multi-launch path's: PCG (symmetric case) or flexible
// GMRES with one classical Gram-Schmidt pass, both stopping on the FP64 true
// relative residual; the non-nested V-cycle of Alg. twolevel_vcycle with
// damped facet block-Jacobi sweeps, restriction pi^T, one P1 multigrid V-cycle
// (damped Jacobi, linear-interpolation transfers, dense coarsest inverse) and
// prolongation pi fused into the first post-sweep.  Only the order of the
// reduction sums differs (one workgroup instead of block partials).
#include "hdg_device.h"
#include "hdg_kernels.h"

namespace hdg {

namespace {

constexpr int SW = SMALL_THREADS / 64;   // wavefronts per workgroup

// The trace unknowns a thread owns: the m unknowns of facets tid, tid + SMALL_THREADS, ...
// -- the items the facet kernels below write -- so that element-wise updates
// read only values the same thread wrote (no barrier needed between them).
template <int M, typename F>
__device__ __forceinline__ void for_own(int ne, F &&f) {
    for (int e = threadIdx.x; e < ne; e += SMALL_THREADS)
#pragma unroll
        for (int a = 0; a < M; ++a) f(e * M + a);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Block-wide sum of one partial value per thread, slot i of the reduction
// area; every thread receives the total (fixed summation order).
__device__ __forceinline__ double block_sum(double v, double *red) {
    const double s = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < SW; ++q) t += red[q];
    return t;
}

__device__ __forceinline__ void ld2(const double *p, double (&o)[2]) {
    const dbl2_t v = *reinterpret_cast<const dbl2_t *>(p);
    o[0] = v.x;
    o[1] = v.y;
}

// y = S x  (b == nullptr) or y = b - S x over this thread's facets; x in LDS
template <int M>
__device__ void s_apply(const SmallArgs &A, const double *x, const double *b, double *y) {
    constexpr int C = 5 * M * M, G = padded(C, 2) / 2;
    const size_t NE = (size_t)A.ne;
    for (int e = threadIdx.x; e < A.ne; e += SMALL_THREADS) {
        int id[5];
        id[0] = e;
#pragma unroll
        for (int j = 0; j < 4; ++j) id[j + 1] = A.nbr[j * NE + e];
        double acc[M];
#pragma unroll
        for (int a = 0; a < M; ++a) acc[a] = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            double w[2];
            ld2(A.S + ((size_t)g * NE + e) * 2, w);
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int c = 2 * g + v;
                if (c < C) {
                    const int j = c / (M * M), a = (c / M) % M, k = c % M;
                    acc[a] += w[v] * x[id[j] * M + k];
                }
            }
        }
#pragma unroll
        for (int a = 0; a < M; ++a) y[e * M + a] = b ? b[e * M + a] - acc[a] : acc[a];
    }
}

// z0 = omega D^-1 r
template <int M>
__device__ void s_jacobi0(const SmallArgs &A, const double *r, double *z0) {
    constexpr int C = M * M, G = padded(C, 2) / 2;
    const size_t NE = (size_t)A.ne;
    for (int e = threadIdx.x; e < A.ne; e += SMALL_THREADS) {
        double rv[M], acc[M];
#pragma unroll
        for (int k = 0; k < M; ++k) {
            rv[k] = r[e * M + k];
            acc[k] = 0.0;
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            double w[2];
            ld2(A.Dw + ((size_t)g * NE + e) * 2, w);
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int c = 2 * g + v;
                if (c < C) acc[c / M] += w[v] * rv[c % M];
            }
        }
#pragma unroll
        for (int a = 0; a < M; ++a) z0[e * M + a] = acc[a];
    }
}

// damped block-Jacobi sweep y = (1 - omega) x' + z0 - sum_j T_j x'_j, x' = x + pi qc
template <int M>
__device__ void s_sweep(const SmallArgs &A, const double *x, const double *z0, const double *qc, double *y) {
    constexpr int P = M - 1, C = 4 * M * M, G = padded(C, 2) / 2;
    const size_t NE = (size_t)A.ne;
    const double a0 = 1.0 - A.omega;
    for (int e = threadIdx.x; e < A.ne; e += SMALL_THREADS) {
        int id[5];
        id[0] = e;
#pragma unroll
        for (int j = 0; j < 4; ++j) id[j + 1] = A.nbr[j * NE + e];
        double xv[5][M];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
#pragma unroll
            for (int k = 0; k < M; ++k) xv[j][k] = x[id[j] * M + k];
            if (qc) {
                const double q0 = qc[A.fvert[2 * id[j]]], q1 = qc[A.fvert[2 * id[j] + 1]];
#pragma unroll
                for (int k = 0; k < M; ++k) xv[j][k] += p1_node<P>(k, q0, q1);
            }
        }
        double acc[M];
#pragma unroll
        for (int a = 0; a < M; ++a) acc[a] = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            double w[2];
            ld2(A.T + ((size_t)g * NE + e) * 2, w);
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int c = 2 * g + v;
                if (c < C) {
                    const int j = c / (M * M), a = (c / M) % M, k = c % M;
                    acc[a] += w[v] * xv[j + 1][k];
                }
            }
        }
        const SweepCoef cf{a0, 1.0, 1.0, 0.0, nullptr, nullptr};
#pragma unroll
        for (int a = 0; a < M; ++a) y[e * M + a] = sweep_combine(cf, xv[0][a], z0[e * M + a], acc[a]);
    }
}

// pi^T: rc[v] = sum over facet ends at v of sum_k w_end(k) res[e][k]
template <int M>
__device__ void s_restrict_trace(const SmallArgs &A, const P1Lev *lev, const double *res, double *rc) {
    constexpr int P = M - 1;
    for (int v = threadIdx.x; v < lev[A.nlev - 1].n; v += SMALL_THREADS) {
        double acc = 0.0;
        for (int c = A.vf_row[v]; c < A.vf_row[v + 1]; ++c) {
            const int code = A.vf_col[c], e = code >> 1, end = code & 1;
#pragma unroll
            for (int k = 0; k < M; ++k) {
                const double w = end ? (double)k / P : 1.0 - (double)k / P;
                acc += w * res[e * M + k];
            }
        }
        rc[v] = acc;
    }
}

__device__ __forceinline__ double s_p1_ax(const P1Lev &L, int v, const double *x) {
    double s = L.diag[v] * x[v];
    for (int k = 0; k < L.w; ++k) s += L.val[(size_t)k * L.n + v] * x[L.col[(size_t)k * L.n + v]];
    return s;
}

// Level vectors of the P1 hierarchy in LDS: b, x, y of level l and the vector
// holding the level's result (tables in LDS, runtime-indexed).
struct P1Vecs {
    double *b[P1_TAIL_LEVELS], *x[P1_TAIL_LEVELS], *y[P1_TAIL_LEVELS], *res[P1_TAIL_LEVELS];
};

// One P1 multigrid V-cycle from the finest level's right-hand side; returns the
// LDS vector holding the result.
__device__ double *s_p1_vcycle(const SmallArgs &A, const P1Lev *lev, P1Vecs *pv) {
    const int top = A.nlev - 1, tid = threadIdx.x;
    const double w = A.p1_omega;
    for (int l = top; l >= 1; --l) {
        const P1Lev &L = lev[l];
        double *x = pv->x[l], *y = pv->y[l];
        const double *b = pv->b[l];
        for (int v = tid; v < L.n; v += SMALL_THREADS) x[v] = w * L.dinv[v] * b[v];
        __syncthreads();
        for (int k = 1; k < A.p1_nu; ++k) {
            for (int v = tid; v < L.n; v += SMALL_THREADS) y[v] = x[v] + w * L.dinv[v] * (b[v] - s_p1_ax(L, v, x));
            __syncthreads();
            double *t = x;
            x = y;
            y = t;
        }
        for (int v = tid; v < L.n; v += SMALL_THREADS) y[v] = b[v] - s_p1_ax(L, v, x);
        __syncthreads();
        const P1Lev &Cl = lev[l - 1];
        double *bc = pv->b[l - 1];
        for (int c = tid; c < Cl.n; c += SMALL_THREADS) {
            double acc = 0.0;
            for (int k = L.crow[c]; k < L.crow[c + 1]; ++k) acc += L.cw[k] * y[L.ccol[k]];
            bc[c] = acc;
        }
        if (tid == 0) pv->res[l] = x;
        __syncthreads();
    }
    {
        const int n0 = lev[0].n;
        const double *b0 = pv->b[0];
        double *x0 = pv->x[0];
        for (int i = tid; i < n0; i += SMALL_THREADS) {
            double s = 0.0;
            for (int j = 0; j < n0; ++j) s += A.Ainv[(size_t)i * n0 + j] * b0[j];
            x0[i] = s;
        }
        if (tid == 0) pv->res[0] = x0;
        __syncthreads();
    }
    for (int l = 1; l <= top; ++l) {
        const P1Lev &L = lev[l];
        double *x = pv->res[l];
        double *y = (x == pv->x[l]) ? pv->y[l] : pv->x[l];
        const double *xc = pv->res[l - 1], *b = pv->b[l];
        for (int k = 0; k < A.p1_nu; ++k) {
            for (int v = tid; v < L.n; v += SMALL_THREADS) {
                auto xin = [&](int u) -> double {
                    double s = x[u];
                    if (k == 0) s += 0.5 * (xc[L.parents[2 * u]] + xc[L.parents[2 * u + 1]]);
                    return s;
                };
                double ax = 0.0;
                for (int q = 0; q < L.w; ++q) ax += L.val[(size_t)q * L.n + v] * xin(L.col[(size_t)q * L.n + v]);
                const double xv = xin(v);
                ax += L.diag[v] * xv;
                y[v] = xv + w * L.dinv[v] * (b[v] - ax);
            }
            __syncthreads();
            double *t = x;
            x = y;
            y = t;
        }
        if (tid == 0) pv->res[l] = x;
        __syncthreads();
    }
    return pv->res[top];
}

// Shared-memory layout of one workgroup (all doubles).
struct SmallLds {
    const P1Lev *lev;   // level descriptors (copied from the kernel arguments)
    P1Vecs *pv;         // level vectors
    double *lam, *r, *z, *p, *w, *z0, *x, *x2, *res, *b;
    double *red;     // [2][SMALL_MAXR + 1][SW] reduction partials
    double *hv;      // [SMALL_MAXR + 1] Gram-Schmidt coefficients
    double *H;       // [SMALL_MAXR + 1][SMALL_MAXR] Hessenberg (column-major by column j)
    double *cs, *sn, *g, *y;
    double *scal;    // broadcast scalars
};

__device__ SmallLds carve(const SmallArgs &A, const P1Lev *lev, P1Vecs *pv, double *base) {
    SmallLds L;
    L.lev = lev;
    L.pv = pv;
    const int nt = A.ne * A.m;
    double *q = base;
    double **vec[10] = {&L.lam, &L.r, &L.z, &L.p, &L.w, &L.z0, &L.x, &L.x2, &L.res, &L.b};
    for (int i = 0; i < 10; ++i) {
        *vec[i] = q;
        q += nt;
    }
    for (int l = 0; l < A.nlev; ++l) {
        const int n = lev[l].n;
        if (threadIdx.x == 0) {
            pv->b[l] = q;
            pv->x[l] = q + n;
            pv->y[l] = q + 2 * n;
        }
        q += 3 * n;
    }
    L.red = q;
    q += 2 * (SMALL_MAXR + 1) * SW;
    L.hv = q;
    q += SMALL_MAXR + 1;
    L.H = q;
    q += (SMALL_MAXR + 1) * SMALL_MAXR;
    L.cs = q;
    q += SMALL_MAXR;
    L.sn = q;
    q += SMALL_MAXR;
    L.g = q;
    q += SMALL_MAXR + 1;
    L.y = q;
    q += SMALL_MAXR;
    L.scal = q;
    return L;
}

// z = V(r) (r read at this thread's facets only; z in LDS)
template <int M>
__device__ void s_vcycle(const SmallArgs &A, SmallLds &L, const double *r, double *z) {
    s_jacobi0<M>(A, r, L.z0);
    __syncthreads();
    double *bufs[2] = {L.x, L.x2};
    int bi = 0;
    double *cur = L.z0;
    for (int k = 1; k < A.nu_pre; ++k) {
        double *out = bufs[bi];
        bi ^= 1;
        s_sweep<M>(A, cur, L.z0, nullptr, out);
        __syncthreads();
        cur = out;
    }
    s_apply<M>(A, cur, r, L.res);
    __syncthreads();
    const int top = A.nlev - 1;
    s_restrict_trace<M>(A, L.lev, L.res, L.pv->b[top]);
    __syncthreads();
    const double *xl = s_p1_vcycle(A, L.lev, L.pv);
    for (int k = 0; k < A.nu_post; ++k) {
        double *out;
        if (k == A.nu_post - 1) {
            out = z;
        } else {
            out = bufs[bi];
            if (out == cur) {
                bi ^= 1;
                out = bufs[bi];
            }
            bi ^= 1;
        }
        s_sweep<M>(A, cur, L.z0, k == 0 ? xl : nullptr, out);
        __syncthreads();
        cur = out;
    }
}

template <int P, bool STAGE>
__global__ __launch_bounds__(SMALL_THREADS) void k_solve_small(const SmallArgs A) {
    constexpr int M = P + 1, n = (P + 1) * (P + 2) / 2, nc = 3 * n, nt = 3 * M, ZW = cell_zw(P);
    extern __shared__ double lds[];
    __shared__ P1Lev slev[P1_TAIL_LEVELS];
    __shared__ P1Vecs spv;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int l = 0; l < P1_TAIL_LEVELS; ++l) slev[l] = A.lev[l];
    }
    __syncthreads();
    SmallLds L = carve(A, slev, &spv, lds);
    __syncthreads();
    const int tid = threadIdx.x, rh = blockIdx.x, nb = A.nb, ne = A.ne;
    const size_t NK = (size_t)A.nk;
    double *red0 = L.red, *red1 = L.red + (SMALL_MAXR + 1) * SW;
    int rsel = 0;
    auto red = [&]() {   // alternate the reduction areas (a barrier always separates reuse)
        rsel ^= 1;
        return rsel ? red1 : red0;
    };

    // ---- right-hand side of the trace system and the initial guess
    if (STAGE) {
        // Step 1: rhat = sum over the facet's two cells of C A^-1 (r, v)_K, row of the facet's node
        for (int e = tid; e < ne; e += SMALL_THREADS) {
#pragma unroll
            for (int a = 0; a < M; ++a) {
                double s = 0.0;
                for (int side = 0; side < 2; ++side) {
                    const int K = A.fcell[2 * e + side], i = A.floc[2 * e + side];
                    const int row = loc_trace<P, 1>(i, a, side);
                    double t = 0.0;
                    for (int j = 0; j < nc; ++j) {
                        const int idx = row * ZW + j;
                        t += A.Zr[((size_t)(idx / 2) * NK + K) * 2 + idx % 2] * A.r_cell[((size_t)K * nc + j) * nb + rh];
                    }
                    s += t;
                }
                L.b[e * M + a] = s;
                L.lam[e * M + a] = 0.0;
            }
        }
    } else {
        for_own<M>(ne, [&](int i) {
            L.b[i] = A.rhat[(size_t)i * nb + rh];
            L.lam[i] = A.lam[(size_t)i * nb + rh];
        });
    }
    __syncthreads();
    double part = 0.0;
    for_own<M>(ne, [&](int i) { part += L.b[i] * L.b[i]; });
    const double bn2 = block_sum(part, red());
    const double rtol = A.rtol;
    int its = 0, restarts = 0, status = HDG_OK;
    double rel = 0.0;
    double *Vb = A.V + (size_t)rh * (SMALL_MAXR + 1) * ne * M;   // this right-hand side's bases (FGMRES)
    double *Zb = A.Z + (size_t)rh * SMALL_MAXR * ne * M;

    while (true) {
        // true residual r = b - S lam (FP64)
        s_apply<M>(A, L.lam, L.b, L.r);
        part = 0.0;
        for_own<M>(ne, [&](int i) { part += L.r[i] * L.r[i]; });
        const double rr = block_sum(part, red());
        rel = bn2 > 0 ? sqrt(rr / bn2) : sqrt(rr);
        if (!isfinite(rel)) {
            status = HDG_EBREAKDOWN;
            break;
        }
        if (rel <= rtol) break;
        if (its >= A.maxit) {
            status = HDG_ENOTCONV;
            break;
        }
        ++restarts;
        if (A.krylov == HDG_KRYLOV_PCG) {
            s_vcycle<M>(A, L, L.r, L.z);
            part = 0.0;
            for_own<M>(ne, [&](int i) {
                part += L.r[i] * L.z[i];
                L.p[i] = L.z[i];
            });
            double rz = block_sum(part, red());
            while (its < A.maxit) {
                s_apply<M>(A, L.p, nullptr, L.w);
                part = 0.0;
                for_own<M>(ne, [&](int i) { part += L.p[i] * L.w[i]; });
                const double pw = block_sum(part, red());
                const double alpha = rz / pw;
                part = 0.0;
                for_own<M>(ne, [&](int i) {
                    L.lam[i] += alpha * L.p[i];
                    L.r[i] -= alpha * L.w[i];
                    part += L.r[i] * L.r[i];
                });
                const double rrk = block_sum(part, red());
                ++its;
                if (!isfinite(rrk) || rrk <= rtol * rtol * bn2) break;
                s_vcycle<M>(A, L, L.r, L.z);
                part = 0.0;
                for_own<M>(ne, [&](int i) { part += L.r[i] * L.z[i]; });
                const double rzn = block_sum(part, red());
                const double beta = rzn / rz;
                rz = rzn;
                for_own<M>(ne, [&](int i) { L.p[i] = L.z[i] + beta * L.p[i]; });
                __syncthreads();
            }
        } else {
            // flexible GMRES(R), classical Gram-Schmidt, the basis vectors in global memory
            const int R = A.restart;
            const double beta = sqrt(rr);
            for_own<M>(ne, [&](int i) { Vb[i] = L.r[i] / beta; });
            if (tid == 0) L.g[0] = beta;
            int k = 0;
            for (int j = 0; j < R && its < A.maxit; ++j) {
                const double *Vj = Vb + (size_t)j * ne * M;
                s_vcycle<M>(A, L, Vj, L.z);
                double *Zj = Zb + (size_t)j * ne * M;
                for_own<M>(ne, [&](int i) { Zj[i] = L.z[i]; });
                s_apply<M>(A, L.z, nullptr, L.w);
                // h_i = V_i . w (this thread's items were written by this thread)
                double *rd = red();
                for (int q = 0; q <= j; ++q) {
                    const double *Vq = Vb + (size_t)q * ne * M;
                    double s = 0.0;
                    for_own<M>(ne, [&](int i) { s += Vq[i] * L.w[i]; });
                    s = wave_sum(s);
                    if ((tid & 63) == 0) rd[q * SW + (tid >> 6)] = s;
                }
                __syncthreads();
                if (tid <= j) {
                    double s = 0.0;
#pragma unroll
                    for (int q = 0; q < SW; ++q) s += rd[tid * SW + q];
                    L.hv[tid] = s;
                }
                __syncthreads();
                part = 0.0;
                for_own<M>(ne, [&](int i) {
                    double wv = L.w[i];
                    for (int q = 0; q <= j; ++q) wv -= L.hv[q] * Vb[(size_t)q * ne * M + i];
                    L.w[i] = wv;
                    part += wv * wv;
                });
                const double hn = sqrt(block_sum(part, red()));
                double *Vn = Vb + (size_t)(j + 1) * ne * M;
                const double inv = hn > 0 ? 1.0 / hn : 0.0;
                for_own<M>(ne, [&](int i) { Vn[i] = L.w[i] * inv; });
                if (tid == 0) {
                    // Givens rotations on column j of the Hessenberg matrix
                    double *Hj = L.H + (size_t)j * (SMALL_MAXR + 1);
                    for (int q = 0; q <= j; ++q) Hj[q] = L.hv[q];
                    Hj[j + 1] = hn;
                    for (int q = 0; q < j; ++q) {
                        const double t0 = L.cs[q] * Hj[q] + L.sn[q] * Hj[q + 1];
                        Hj[q + 1] = -L.sn[q] * Hj[q] + L.cs[q] * Hj[q + 1];
                        Hj[q] = t0;
                    }
                    const double d = sqrt(Hj[j] * Hj[j] + Hj[j + 1] * Hj[j + 1]);
                    const double cj = d > 0 ? Hj[j] / d : 1.0, sj = d > 0 ? Hj[j + 1] / d : 0.0;
                    L.cs[j] = cj;
                    L.sn[j] = sj;
                    Hj[j] = d;
                    Hj[j + 1] = 0.0;
                    L.g[j + 1] = -sj * L.g[j];
                    L.g[j] = cj * L.g[j];
                    const double bn = sqrt(bn2);
                    L.scal[0] = bn > 0 ? fabs(L.g[j + 1]) / bn : fabs(L.g[j + 1]);
                }
                __syncthreads();
                ++its;
                k = j + 1;
                const double est = L.scal[0];
                if (!isfinite(est) || est <= rtol) break;
            }
            // y = H^-1 g (upper triangular k x k), then lam += Z y
            if (tid == 0) {
                for (int q = k - 1; q >= 0; --q) {
                    double s = L.g[q];
                    for (int t = q + 1; t < k; ++t) s -= L.H[(size_t)t * (SMALL_MAXR + 1) + q] * L.y[t];
                    L.y[q] = s / L.H[(size_t)q * (SMALL_MAXR + 1) + q];
                }
            }
            __syncthreads();
            for_own<M>(ne, [&](int i) {
                double s = L.lam[i];
                for (int q = 0; q < k; ++q) s += L.y[q] * Zb[(size_t)q * ne * M + i];
                L.lam[i] = s;
            });
            __syncthreads();
        }
    }

    // ---- outputs: lam, the info record, and (stage) the recovered cell fields
    for_own<M>(ne, [&](int i) { A.lam[(size_t)i * nb + rh] = L.lam[i]; });
    if (tid == 0) {
        A.info[4 * rh + 0] = its;
        A.info[4 * rh + 1] = restarts;
        A.info[4 * rh + 2] = status;
        A.info[4 * rh + 3] = rel;
    }
    if (STAGE) {
        __syncthreads();
        // Step 3: q = Ar r_cell - Wr lam_K per cell
        for (int K = tid; K < A.nk; K += SMALL_THREADS) {
            double l[nt];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int e = A.cell_facet[i * NK + K];
                const int rev = A.cell_rev[i * NK + K];
#pragma unroll
                for (int a = 0; a < M; ++a) l[loc_trace<P, 1>(i, a, rev)] = L.lam[e * M + a];
            }
            for (int a = 0; a < nc; ++a) {
                double s = 0.0;
                for (int j = 0; j < nc; ++j) s += A.Ar[(size_t)(a * nc + j) * NK + K] * A.r_cell[((size_t)K * nc + j) * nb + rh];
#pragma unroll
                for (int j = 0; j < nt; ++j) s -= A.Wr[(size_t)(a * nt + j) * NK + K] * l[j];
                A.q_cell[((size_t)K * nc + a) * nb + rh] = s;
            }
        }
    }
}

}  // namespace

size_t small_lds_bytes(int ne, int m, const int *level_n, int nlev) {
    size_t d = (size_t)10 * ne * m;
    for (int l = 0; l < nlev; ++l) d += 3 * (size_t)level_n[l];
    d += 2 * (SMALL_MAXR + 1) * SW + (SMALL_MAXR + 1) + (SMALL_MAXR + 1) * SMALL_MAXR + 3 * SMALL_MAXR +
         (SMALL_MAXR + 1) + 8;
    return d * sizeof(double);
}

hipError_t small_prepare(int p, size_t lds) {
    // dynamic LDS above the default 64 KiB needs the kernels' opt-in
    auto set = [&](const void *f) {
        return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    };
    hipError_t e1 = hipSuccess, e2 = hipSuccess;
    switch (p) {
    case 1: e1 = set((const void *)k_solve_small<1, false>); e2 = set((const void *)k_solve_small<1, true>); break;
    case 2: e1 = set((const void *)k_solve_small<2, false>); e2 = set((const void *)k_solve_small<2, true>); break;
    case 3: e1 = set((const void *)k_solve_small<3, false>); e2 = set((const void *)k_solve_small<3, true>); break;
    default: return hipErrorInvalidValue;
    }
    return e1 != hipSuccess ? e1 : e2;
}

void launch_solve_small(int p, bool stage, const SmallArgs &A, size_t lds, hipStream_t s) {
    const dim3 grid(A.nb), block(SMALL_THREADS);
    switch (p * 2 + (stage ? 1 : 0)) {
    case 2: k_solve_small<1, false><<<grid, block, lds, s>>>(A); break;
    case 3: k_solve_small<1, true><<<grid, block, lds, s>>>(A); break;
    case 4: k_solve_small<2, false><<<grid, block, lds, s>>>(A); break;
    case 5: k_solve_small<2, true><<<grid, block, lds, s>>>(A); break;
    case 6: k_solve_small<3, false><<<grid, block, lds, s>>>(A); break;
    case 7: k_solve_small<3, true><<<grid, block, lds, s>>>(A); break;
    default: break;
    }
}

}  // namespace hdg
