// Persistent solve of small trace systems: one workgroup per right-hand side
// runs the whole Krylov solve -- and optionally the condensation before it and
// the recovery after it (Steps 1-3) -- in a single launch.
//
// Below a few thousand trace unknowns every kernel of the multi-launch solve
// is a few waves and a solve is a chain of ~10 dependent launches per Krylov
// iteration, so its time is launch latency.  Here the trace vectors of the
// Krylov method and the V-cycle and the vectors of every P1 level live in LDS,
// and so do, when they fit, the operators themselves: the facet rows of S,
// omega D^-1 S_j and omega D^-1, the neighbour and vertex tables, the P1 level
// matrices and the dense coarsest inverse (otherwise they are read from global
// memory, where they stay cached after the first iteration).  A workgroup of
// 256 threads owns the facets (vertices, cells) thread-cyclically, and every
// phase whose output is read at other items ends with a workgroup barrier.
//
// The arithmetic is the multi-launch path's: PCG (symmetric case) or flexible
// GMRES with one classical Gram-Schmidt pass, both stopping on the FP64 true
// relative residual; the non-nested V-cycle of Alg. twolevel_vcycle with
// damped facet block-Jacobi sweeps (the first one from zero fused with
// omega D^-1 r), restriction pi^T, one P1 multigrid V-cycle (damped Jacobi,
// its first two sweeps fused, linear-interpolation transfers, dense coarsest
// inverse) and prolongation pi fused into the first post-sweep.  Only the
// rounding differs: the order of the reduction sums (one workgroup instead of
// block partials) and, for hierarchies of at most SMALL_P1_DENSE finest
// vertices, the P1 V-cycle applied as its matrix (formed on the host by
// applying the same cycle to unit vectors, stored transposed).
#include "hdg_device.h"
#include "hdg_kernels.h"

namespace hdg {

namespace {

constexpr int SW = SMALL_THREADS / 64;   // wavefronts per workgroup
static_assert(SW == 4 && SMALL_P1_DENSE <= 64, "the dense P1 phase: four wavefronts, a row per lane");

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

// Block-wide sum of one partial value per thread; every thread receives the
// total (fixed summation order, so every thread holds the same bits).
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

// Operator loads.  When the operators are staged in LDS (OL) their addresses
// are still generic pointers (published through a shared table), which would
// compile to flat instructions; the loads below cast them to the local address
// space, so that they compile to LDS instructions.
typedef __attribute__((address_space(3))) const double lds_double;
typedef __attribute__((address_space(3))) const int lds_int;
typedef __attribute__((address_space(3))) const dbl2_t lds_double2;
typedef __attribute__((address_space(3))) double lds_dbl;   // P1 level vectors (always in LDS)

template <bool OL>
__device__ __forceinline__ void opr2(const double *p, double (&o)[2]) {
    if constexpr (OL) {
        const dbl2_t v = *(const lds_double2 *)p;
        o[0] = v.x;
        o[1] = v.y;
    } else {
        ld2(p, o);
    }
}
template <bool OL>
__device__ __forceinline__ int opri(const int *p) {
    if constexpr (OL) return *(const lds_int *)p;
    else return *p;
}
template <bool OL>
__device__ __forceinline__ double oprd(const double *p) {
    if constexpr (OL) return *(const lds_double *)p;
    else return *p;
}

// The operators as the phases read them: global memory, or the LDS copies.
struct Ops {
    const double *S, *T, *Dw, *Ainv, *B;
    const int *nbr, *fvert, *vf_row, *vf_col;
    P1Lev lev[P1_TAIL_LEVELS];
};

// y = S x  (b == nullptr) or y = b - S x over this thread's facets; x in LDS
template <int M, bool OL>
__device__ void s_apply(int ne, const Ops &O, const double *x, const double *b, double *y) {
    constexpr int C = 5 * M * M, G = padded(C, 2) / 2;
    const size_t NE = (size_t)ne;
    const double *S = O.S;
    const int *nbr = O.nbr;
    for (int e = threadIdx.x; e < ne; e += SMALL_THREADS) {
        int id[5];
        id[0] = e;
#pragma unroll
        for (int j = 0; j < 4; ++j) id[j + 1] = opri<OL>(nbr + j * NE + e);
        double acc[M];
#pragma unroll
        for (int a = 0; a < M; ++a) acc[a] = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            double w[2];
            opr2<OL>(S + ((size_t)g * NE + e) * 2, w);
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

// PCG direction and operator in one phase: pn = z + beta po at this thread's
// facets and w = S pn, pn at the patch facets evaluated in place (the same
// expression, so the same bits); returns this thread's part of pn . w
template <int M, bool OL>
__device__ double s_apply_dir(int ne, const Ops &O, const double *z, double beta, const double *po, double *pn,
                              double *w) {
    constexpr int C = 5 * M * M, G = padded(C, 2) / 2;
    const size_t NE = (size_t)ne;
    const double *S = O.S;
    const int *nbr = O.nbr;
    double part = 0.0;
    for (int e = threadIdx.x; e < ne; e += SMALL_THREADS) {
        int id[5];
        id[0] = e;
#pragma unroll
        for (int j = 0; j < 4; ++j) id[j + 1] = opri<OL>(nbr + j * NE + e);
        double xv[5][M];
#pragma unroll
        for (int j = 0; j < 5; ++j)
#pragma unroll
            for (int k = 0; k < M; ++k) xv[j][k] = z[id[j] * M + k] + beta * po[id[j] * M + k];
        double acc[M];
#pragma unroll
        for (int a = 0; a < M; ++a) acc[a] = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            double wv[2];
            opr2<OL>(S + ((size_t)g * NE + e) * 2, wv);
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int c = 2 * g + v;
                if (c < C) {
                    const int j = c / (M * M), a = (c / M) % M, k = c % M;
                    acc[a] += wv[v] * xv[j][k];
                }
            }
        }
#pragma unroll
        for (int a = 0; a < M; ++a) {
            pn[e * M + a] = xv[0][a];
            w[e * M + a] = acc[a];
            part += xv[0][a] * acc[a];
        }
    }
    return part;
}

// omega D_f^-1 r_f at facet f (the multi-launch first sweep's arithmetic)
template <int M, bool OL>
__device__ __forceinline__ void jacobi_at(const Ops &O, size_t NE, int f, const double *r, double (&z)[M]) {
    constexpr int C = M * M, G = padded(C, 2) / 2;
    const double *Dw = O.Dw;
    double rv[M];
#pragma unroll
    for (int k = 0; k < M; ++k) {
        rv[k] = r[f * M + k];
        z[k] = 0.0;
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
        double w[2];
        opr2<OL>(Dw + ((size_t)g * NE + f) * 2, w);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int c = 2 * g + v;
            if (c < C) z[c / M] += w[v] * rv[c % M];
        }
    }
}

// omega D_f^-1 rv for the values rv of facet f
template <int M, bool OL>
__device__ __forceinline__ void jacobi_of(const Ops &O, size_t NE, int f, const double (&rv)[M], double (&z)[M]) {
    constexpr int C = M * M, G = padded(C, 2) / 2;
    const double *Dw = O.Dw;
#pragma unroll
    for (int k = 0; k < M; ++k) z[k] = 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        double w[2];
        opr2<OL>(Dw + ((size_t)g * NE + f) * 2, w);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            const int c = 2 * g + v;
            if (c < C) z[c / M] += w[v] * rv[c % M];
        }
    }
}

// The PCG update fused with the first V-cycle phase of the next preconditioner
// application: at this thread's facets lam += alpha p and rn = r - alpha w (into
// a second buffer: the old r is still read at the patch facets), then z0 =
// omega D^-1 rn and, with y != nullptr, the first sweep from zero, rn at the
// patch facets evaluated in place (the same expression, so the same bits).
// Returns this thread's part of rn . rn.
template <int M, bool OL>
__device__ double s_update_first_sweep(int ne, const Ops &O, double omega, double alpha, const double *p,
                                       const double *w, const double *r, double *rn, double *lam, double *z0,
                                       double *y) {
    constexpr int C = 4 * M * M, G = padded(C, 2) / 2;
    const size_t NE = (size_t)ne;
    const double *T = O.T;
    const int *nbr = O.nbr;
    const SweepCoef cf{1.0 - omega, 1.0, 1.0, 0.0, nullptr, nullptr};
    double part = 0.0;
    for (int e = threadIdx.x; e < ne; e += SMALL_THREADS) {
        double rv[M], zv[5][M];
#pragma unroll
        for (int a = 0; a < M; ++a) {
            const int i = e * M + a;
            rv[a] = r[i] - alpha * w[i];
            rn[i] = rv[a];
            lam[i] += alpha * p[i];
            part += rv[a] * rv[a];
        }
        jacobi_of<M, OL>(O, NE, e, rv, zv[0]);
#pragma unroll
        for (int a = 0; a < M; ++a) z0[e * M + a] = zv[0][a];
        if (!y) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int f = opri<OL>(nbr + j * NE + e);
            double rj[M];
#pragma unroll
            for (int k = 0; k < M; ++k) rj[k] = r[f * M + k] - alpha * w[f * M + k];
            jacobi_of<M, OL>(O, NE, f, rj, zv[j + 1]);
        }
        double acc[M];
#pragma unroll
        for (int a = 0; a < M; ++a) acc[a] = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            double wt[2];
            opr2<OL>(T + ((size_t)g * NE + e) * 2, wt);
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int c = 2 * g + v;
                if (c < C) {
                    const int j = c / (M * M), a = (c / M) % M, k = c % M;
                    acc[a] += wt[v] * zv[j + 1][k];
                }
            }
        }
#pragma unroll
        for (int a = 0; a < M; ++a) y[e * M + a] = sweep_combine(cf, zv[0][a], zv[0][a], acc[a]);
    }
    return part;
}

// z0 = omega D^-1 r at this thread's facets and, with y != nullptr, the first
// damped block-Jacobi sweep from zero y = (1 - omega) z0 + z0 - sum_j T_j z0_j
// (z0 at the patch facets computed in place)
template <int M, bool OL>
__device__ void s_first_sweep(int ne, const Ops &O, double omega, const double *r, double *z0, double *y) {
    constexpr int C = 4 * M * M, G = padded(C, 2) / 2;
    const size_t NE = (size_t)ne;
    const double *T = O.T;
    const int *nbr = O.nbr;
    const SweepCoef cf{1.0 - omega, 1.0, 1.0, 0.0, nullptr, nullptr};
    for (int e = threadIdx.x; e < ne; e += SMALL_THREADS) {
        double zv[5][M];
        jacobi_at<M, OL>(O, NE, e, r, zv[0]);
#pragma unroll
        for (int a = 0; a < M; ++a) z0[e * M + a] = zv[0][a];
        if (!y) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) jacobi_at<M, OL>(O, NE, opri<OL>(nbr + j * NE + e), r, zv[j + 1]);
        double acc[M];
#pragma unroll
        for (int a = 0; a < M; ++a) acc[a] = 0.0;
#pragma unroll
        for (int g = 0; g < G; ++g) {
            double w[2];
            opr2<OL>(T + ((size_t)g * NE + e) * 2, w);
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int c = 2 * g + v;
                if (c < C) {
                    const int j = c / (M * M), a = (c / M) % M, k = c % M;
                    acc[a] += w[v] * zv[j + 1][k];
                }
            }
        }
#pragma unroll
        for (int a = 0; a < M; ++a) y[e * M + a] = sweep_combine(cf, zv[0][a], zv[0][a], acc[a]);
    }
}

// damped block-Jacobi sweep y = (1 - omega) x' + z0 - sum_j T_j x'_j, x' = x + pi qc;
// returns this thread's part of d . y when d is given
template <int M, bool OL>
__device__ double s_sweep(int ne, const Ops &O, double omega, const double *x, const double *z0, const lds_dbl *qc,
                          double *y, const double *d = nullptr) {
    double part = 0.0;
    const double *T = O.T;
    const int *nbr = O.nbr, *fvert = O.fvert;
    constexpr int P = M - 1, C = 4 * M * M, G = padded(C, 2) / 2;
    const size_t NE = (size_t)ne;
    const SweepCoef cf{1.0 - omega, 1.0, 1.0, 0.0, nullptr, nullptr};
    for (int e = threadIdx.x; e < ne; e += SMALL_THREADS) {
        int id[5];
        id[0] = e;
#pragma unroll
        for (int j = 0; j < 4; ++j) id[j + 1] = opri<OL>(nbr + j * NE + e);
        double xv[5][M];
#pragma unroll
        for (int j = 0; j < 5; ++j) {
#pragma unroll
            for (int k = 0; k < M; ++k) xv[j][k] = x[id[j] * M + k];
            if (qc) {
                const double q0 = qc[opri<OL>(fvert + 2 * id[j])], q1 = qc[opri<OL>(fvert + 2 * id[j] + 1)];
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
            opr2<OL>(T + ((size_t)g * NE + e) * 2, w);
#pragma unroll
            for (int v = 0; v < 2; ++v) {
                const int c = 2 * g + v;
                if (c < C) {
                    const int j = c / (M * M), a = (c / M) % M, k = c % M;
                    acc[a] += w[v] * xv[j + 1][k];
                }
            }
        }
#pragma unroll
        for (int a = 0; a < M; ++a) {
            const double v = sweep_combine(cf, xv[0][a], z0[e * M + a], acc[a]);
            y[e * M + a] = v;
            if (d) part += d[e * M + a] * v;
        }
    }
    return part;
}

// pi^T: rc[v] = sum over facet ends at v of sum_k w_end(k) res[e][k].  Four lanes
// per vertex take every fourth facet end and add their sums by shuffles, so that
// the whole workgroup shares the short per-vertex lists.
template <int M, bool OL>
__device__ void s_restrict_trace(int nv, const Ops &O, const double *res, lds_dbl *rc) {
    constexpr int P = M - 1;
    const int *vf_row = O.vf_row, *vf_col = O.vf_col;
    const int nvr = (nv + SMALL_THREADS / 4 - 1) / (SMALL_THREADS / 4) * (SMALL_THREADS / 4);   // uniform trip count
    for (int v0 = 0; v0 < nvr; v0 += SMALL_THREADS / 4) {
        const int v = v0 + (threadIdx.x >> 2), sub = threadIdx.x & 3;
        double acc = 0.0;
        if (v < nv) {
            const int c1 = opri<OL>(vf_row + v + 1);
            for (int k = opri<OL>(vf_row + v) + sub; k < c1; k += 4) {
                const int code = opri<OL>(vf_col + k), e = code >> 1, end = code & 1;
#pragma unroll
                for (int q = 0; q < M; ++q) {
                    const double w = end ? (double)q / P : 1.0 - (double)q / P;
                    acc += w * res[e * M + q];
                }
            }
        }
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        if (v < nv && sub == 0) rc[v] = acc;
    }
}

// Short index ranges (ELL rows, vertex and child lists: 5-7 entries on these
// meshes) are walked UNROLL entries at a time with the index clamped into the
// range and the surplus terms multiplied by zero, so that all loads of a row
// are in flight together instead of one dependent pair after the other.
constexpr int UNROLL = 8;

// sum over k in [0, cnt) of f(k); cnt >= 0
template <typename F>
__device__ __forceinline__ double range_sum(int cnt, F &&f) {
    double s = 0.0;
    for (int k0 = 0; k0 < cnt; k0 += UNROLL) {
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int k = min(k0 + u, cnt - 1);
            const double t = f(k);
            s += k0 + u < cnt ? t : 0.0;
        }
    }
    return s;
}

template <bool OL>
__device__ __forceinline__ double s_p1_ax(const P1Lev &L, int v, const lds_dbl *x) {
    const double s = oprd<OL>(L.diag + v) * x[v];
    return s + range_sum(L.w, [&](int k) {
        return oprd<OL>(L.val + (size_t)k * L.n + v) * x[opri<OL>(L.col + (size_t)k * L.n + v)];
    });
}

// Level vectors of the P1 hierarchy in LDS: b, x, y of level l (tables in LDS,
// runtime-indexed).  Which of x, y holds a level's iterate follows from the
// sweep count alone, so no pointer has to be published between the phases.
struct P1Vecs {
    lds_dbl *b[P1_TAIL_LEVELS], *x[P1_TAIL_LEVELS], *y[P1_TAIL_LEVELS];
};

// One P1 multigrid V-cycle from the finest level's right-hand side; returns the
// LDS vector holding the result.
template <bool OL>
__device__ lds_dbl *s_p1_vcycle(int nlev, int nu, double w, const Ops &O, const P1Vecs *pv) {
    const int top = nlev - 1, tid = threadIdx.x;
    // after pre-smoothing the iterate is in x when the sweeps after the first
    // fused pair are even in number; after post-smoothing in that buffer when nu is even
    const bool pre_x = nu == 1 || (nu - 2) % 2 == 0, fin_pre = nu % 2 == 0;
    auto pre = [&](int l) { return pre_x ? pv->x[l] : pv->y[l]; };
    auto other = [&](int l) { return pre_x ? pv->y[l] : pv->x[l]; };
    auto fin = [&](int l) { return l == 0 ? pv->x[0] : (fin_pre ? pre(l) : other(l)); };
    for (int l = top; l >= 1; --l) {
        const P1Lev &L = O.lev[l];
        lds_dbl *x = pv->x[l], *y = pv->y[l];
        const lds_dbl *b = pv->b[l];
        auto dinv = [&](int v) { return oprd<OL>(L.dinv + v); };
        if (nu == 1) {
            for (int v = tid; v < L.n; v += SMALL_THREADS) x[v] = w * dinv(v) * b[v];
        } else {
            // two sweeps from zero: x1 = w D^-1 b (evaluated where needed), x2 = x1 + w D^-1 (b - A x1)
            for (int v = tid; v < L.n; v += SMALL_THREADS) {
                const double x1 = w * dinv(v) * b[v];
                const double ax = oprd<OL>(L.diag + v) * x1 + range_sum(L.w, [&](int k) {
                    const int u = opri<OL>(L.col + (size_t)k * L.n + v);
                    return oprd<OL>(L.val + (size_t)k * L.n + v) * (w * dinv(u) * b[u]);
                });
                x[v] = x1 + w * dinv(v) * (b[v] - ax);
            }
        }
        __syncthreads();
        for (int k = 2; k < nu; ++k) {
            for (int v = tid; v < L.n; v += SMALL_THREADS) y[v] = x[v] + w * dinv(v) * (b[v] - s_p1_ax<OL>(L, v, x));
            __syncthreads();
            lds_dbl *t = x;
            x = y;
            y = t;
        }
        for (int v = tid; v < L.n; v += SMALL_THREADS) y[v] = b[v] - s_p1_ax<OL>(L, v, x);
        __syncthreads();
        const P1Lev &Cl = O.lev[l - 1];
        lds_dbl *bc = pv->b[l - 1];
        for (int c = tid; c < Cl.n; c += SMALL_THREADS) {
            const int k0 = opri<OL>(L.crow + c);
            bc[c] = range_sum(opri<OL>(L.crow + c + 1) - k0,
                              [&](int k) { return oprd<OL>(L.cw + k0 + k) * y[opri<OL>(L.ccol + k0 + k)]; });
        }
        __syncthreads();
    }
    {
        const int n0 = O.lev[0].n;
        const lds_dbl *b0 = pv->b[0];
        lds_dbl *x0 = pv->x[0];
        for (int i = tid; i < n0; i += SMALL_THREADS)
            x0[i] = range_sum(n0, [&](int j) { return oprd<OL>(O.Ainv + (size_t)i * n0 + j) * b0[j]; });
        __syncthreads();
    }
    for (int l = 1; l <= top; ++l) {
        const P1Lev &L = O.lev[l];
        lds_dbl *x = pre(l), *y = other(l);
        const lds_dbl *xc = fin(l - 1), *b = pv->b[l];
        for (int k = 0; k < nu; ++k) {
            for (int v = tid; v < L.n; v += SMALL_THREADS) {
                auto xin = [&](int u) -> double {
                    double s = x[u];
                    if (k == 0)
                        s += 0.5 * (xc[opri<OL>(L.parents + 2 * u)] + xc[opri<OL>(L.parents + 2 * u + 1)]);
                    return s;
                };
                double ax = range_sum(L.w, [&](int q) {
                    return oprd<OL>(L.val + (size_t)q * L.n + v) * xin(opri<OL>(L.col + (size_t)q * L.n + v));
                });
                const double xv = xin(v);
                ax += oprd<OL>(L.diag + v) * xv;
                y[v] = xv + w * oprd<OL>(L.dinv + v) * (b[v] - ax);
            }
            __syncthreads();
            lds_dbl *t = x;
            x = y;
            y = t;
        }
    }
    return fin(top);
}

// Shared-memory layout of one workgroup (all doubles, then the staged operators).
struct SmallLds {
    const Ops *ops;
    P1Vecs *pv;
    double *lam, *r, *r2, *z, *p, *p2, *w, *z0, *x, *x2, *res, *b;
    double *red;     // [2][SMALL_MAXR + 1][SW] reduction partials
    double *dpart;   // [4][64] partial sums of the dense P1 product
    double *hv;      // [SMALL_MAXR + 1] Gram-Schmidt coefficients
    double *H;       // Hessenberg, column j at H + j (SMALL_MAXR + 1)
    double *cs, *sn, *g, *y;
    double *scal;    // broadcast scalars
    char *img;       // LDS copy of the operator image (stage_ops), else null
};

constexpr size_t small_fixed_doubles() {
    return 2 * (SMALL_MAXR + 1) * SW + 4 * 64 + (SMALL_MAXR + 1) + (SMALL_MAXR + 1) * SMALL_MAXR + 3 * SMALL_MAXR +
           (SMALL_MAXR + 1) + 8;
}

__device__ SmallLds carve(const SmallArgs &A, Ops *ops, P1Vecs *pv, double *base) {
    SmallLds L;
    L.ops = ops;
    L.pv = pv;
    const int nt = A.ne * A.m;
    double *q = base;
    double **vec[12] = {&L.lam, &L.r, &L.r2, &L.z, &L.p, &L.p2, &L.w, &L.z0, &L.x, &L.x2, &L.res, &L.b};
    for (int i = 0; i < 12; ++i) {
        *vec[i] = q;
        q += nt;
    }
    for (int l = 0; l < A.nlev; ++l) {
        const int n = ops->lev[l].n;
        if (threadIdx.x == 0) {
            pv->b[l] = (lds_dbl *)q;
            pv->x[l] = (lds_dbl *)(q + n);
            pv->y[l] = (lds_dbl *)(q + 2 * n);
        }
        q += 3 * n;
    }
    L.red = q;
    q += 2 * (SMALL_MAXR + 1) * SW;
    L.dpart = q;
    q += 4 * 64;
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
    q += 8;
    L.img = nullptr;
    if (A.stage_ops) {
        // the operator image goes after the vectors, 16-byte aligned (copied by the kernel)
        char *c = reinterpret_cast<char *>(q);
        c += (16 - (reinterpret_cast<uintptr_t>(c) & 15)) & 15;
        L.img = c;
    }
    return L;
}

// z = V(r): r and z in LDS.  With d given, returns this thread's part of d . z and
// leaves the barrier after the last sweep to the caller's reduction.
// The V-cycle after its first phase (z0 and the first sweep from zero in L.z0, L.x).
template <int M, bool OL>
__device__ double s_vcycle_rest(const SmallArgs &A, SmallLds &L, const double *r, double *z, const double *d) {
    const Ops &O = *L.ops;
    const int ne = A.ne, tid = threadIdx.x;
    double *bufs[2] = {L.x, L.x2};
    int bi = 0;
    double *cur = L.z0;
    if (A.nu_pre >= 2) {
        cur = L.x;
        bi = 1;
    }
    for (int k = 2; k < A.nu_pre; ++k) {
        double *out = bufs[bi];
        bi ^= 1;
        s_sweep<M, OL>(ne, O, A.omega, cur, L.z0, nullptr, out);
        __syncthreads();
        cur = out;
    }
    s_apply<M, OL>(ne, O, cur, r, L.res);
    __syncthreads();
    const int top = A.nlev - 1;
    s_restrict_trace<M, OL>(O.lev[top].n, O, L.res, L.pv->b[top]);
    __syncthreads();
    const lds_dbl *xl;
    if (O.B) {
        // the P1 V-cycle as its matrix, stored transposed: lane i of each wavefront takes
        // row i (consecutive doubles across the lanes: no LDS bank conflicts), wavefront w
        // a quarter of the columns; the four partial sums are added in a second step
        const int nv = O.lev[top].n;
        const lds_dbl *bv = L.pv->b[top];
        const double *BT = O.B;
        lds_dbl *xv = L.pv->x[top];
        const int wv = tid >> 6, lane = tid & 63, jc = (nv + 3) / 4, j0 = wv * jc, j1 = min(nv, j0 + jc);
        double s = 0.0;
        if (lane < nv) {
#pragma unroll 8
            for (int j = j0; j < j1; ++j) s += oprd<OL>(BT + (size_t)j * nv + lane) * bv[j];
        }
        L.dpart[wv * 64 + lane] = s;
        __syncthreads();
        if (tid < nv) xv[tid] = (L.dpart[tid] + L.dpart[64 + tid]) + (L.dpart[128 + tid] + L.dpart[192 + tid]);
        __syncthreads();
        xl = xv;
    } else {
        xl = s_p1_vcycle<OL>(A.nlev, A.p1_nu, A.p1_omega, O, L.pv);
    }
    double part = 0.0;
    for (int k = 0; k < A.nu_post; ++k) {
        const bool last = k == A.nu_post - 1;
        double *out;
        if (last) {
            out = z;
        } else {
            out = bufs[bi];
            if (out == cur) {
                bi ^= 1;
                out = bufs[bi];
            }
            bi ^= 1;
        }
        part = s_sweep<M, OL>(ne, O, A.omega, cur, L.z0, k == 0 ? xl : nullptr, out, last ? d : nullptr);
        if (!(last && d)) __syncthreads();
        cur = out;
    }
    return part;
}

template <int M, bool OL>
__device__ double s_vcycle(const SmallArgs &A, SmallLds &L, const double *r, double *z, const double *d = nullptr) {
    s_first_sweep<M, OL>(A.ne, *L.ops, A.omega, r, L.z0, A.nu_pre >= 2 ? L.x : nullptr);
    __syncthreads();
    return s_vcycle_rest<M, OL>(A, L, r, z, d);
}

// thread 0 points the operator table at the LDS copy of the image
__device__ void publish_image(const SmallArgs &A, Ops *ops, const char *c) {
    const int nB = A.p1B ? ops->lev[A.nlev - 1].n : 0;
    small_image_walk(A.ne, A.m, ops->lev, A.nlev, nB, [&](SmallPart part, int l, size_t off, size_t) {
        const char *a = c + off;
        const double *d = reinterpret_cast<const double *>(a);
        const int *k = reinterpret_cast<const int *>(a);
        P1Lev &D = ops->lev[l];
        switch (part) {
        case SP_S: ops->S = d; break;
        case SP_T: ops->T = d; break;
        case SP_DW: ops->Dw = d; break;
        case SP_NBR: ops->nbr = k; break;
        case SP_FVERT: ops->fvert = k; break;
        case SP_VF_ROW: ops->vf_row = k; break;
        case SP_VF_COL: ops->vf_col = k; break;
        case SP_B: ops->B = d; break;
        case SP_COL: D.col = k; break;
        case SP_VAL: D.val = d; break;
        case SP_DIAG: D.diag = d; break;
        case SP_DINV: D.dinv = d; break;
        case SP_PARENTS: D.parents = k; break;
        case SP_CROW: D.crow = k; break;
        case SP_CCOL: D.ccol = k; break;
        case SP_CW: D.cw = d; break;
        case SP_AINV: ops->Ainv = d; break;
        }
    });
}

template <int P, bool STAGE, bool OL>
__global__ __launch_bounds__(SMALL_THREADS) void k_solve_small(const SmallArgs A) {
    constexpr int M = P + 1, n = (P + 1) * (P + 2) / 2, nc = 3 * n, nt = 3 * M, ZW = cell_zw(P);
    extern __shared__ double lds[];
    __shared__ Ops sops;
    __shared__ P1Vecs spv;
    // the operator table into LDS: the level descriptors one per lane (their argument
    // loads in flight together), the rest by the next lane
    if (threadIdx.x < A.nlev) sops.lev[threadIdx.x] = A.lev[threadIdx.x];
    if (threadIdx.x == 63) {
        sops.S = A.S;
        sops.T = A.T;
        sops.Dw = A.Dw;
        sops.Ainv = A.Ainv;
        sops.B = A.p1B;
        sops.nbr = A.nbr;
        sops.fvert = A.fvert;
        sops.vf_row = A.vf_row;
        sops.vf_col = A.vf_col;
    }
    __syncthreads();
    SmallLds L = carve(A, &sops, &spv, lds);
    __syncthreads();
    const Ops &O = sops;
    const int tid = threadIdx.x, rh = blockIdx.x, nb = A.nb, ne = A.ne;
    // The packed operator image into LDS: the first up-to-32 16-byte loads per thread
    // go out before the right-hand side below is read, so that both are in flight
    // together; their stores, any further rounds and the table follow it.
    typedef unsigned u4 __attribute__((ext_vector_type(4)));
    constexpr int IU = 32;
    const int n16 = L.img ? (int)(small_image_bytes(ne, A.m, sops.lev, A.nlev, A.p1B ? sops.lev[A.nlev - 1].n : 0) / 16)
                          : 0;
    const u4 *isrc = reinterpret_cast<const u4 *>(A.image);   // device allocations are 256-byte aligned
    u4 *idst = reinterpret_cast<u4 *>(L.img);
    u4 iv[IU];
#pragma unroll
    for (int u = 0; u < IU; ++u) {
        const int i = tid + u * SMALL_THREADS;
        if (i < n16) iv[u] = isrc[i];
    }
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
#pragma unroll
    for (int u = 0; u < IU; ++u) {
        const int i = tid + u * SMALL_THREADS;
        if (i < n16) idst[i] = iv[u];
    }
    for (int i0 = tid + IU * SMALL_THREADS; i0 < n16; i0 += IU * SMALL_THREADS) {
#pragma unroll
        for (int u = 0; u < IU; ++u) {
            const int i = i0 + u * SMALL_THREADS;
            if (i < n16) iv[u] = isrc[i];
        }
#pragma unroll
        for (int u = 0; u < IU; ++u) {
            const int i = i0 + u * SMALL_THREADS;
            if (i < n16) idst[i] = iv[u];
        }
    }
    __syncthreads();   // every thread has read the level sizes above
    if (L.img && tid == 0) publish_image(A, &sops, L.img);
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
        s_apply<M, OL>(ne, O, L.lam, L.b, L.r);
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
            // p_0 = z_0; then per iteration: p = z + beta p (fused into w = S p), alpha = rz / p.w,
            // lam += alpha p, r -= alpha w, z = V(r), beta = r.z / rz
            // (the update of lam and r rides in the first phase of the next V-cycle;
            // r alternates between two buffers)
            double rz = block_sum(s_vcycle<M, OL>(A, L, L.r, L.z, L.r), red());
            double beta = 0.0;
            double *pbuf[2] = {L.p, L.p2};
            double *rc = L.r, *rnx = L.r2;
            int pc = 0;
            const double *po = L.z;   // first direction: z itself (beta = 0)
            while (its < A.maxit) {
                double *pn = pbuf[pc];
                const double pw = block_sum(s_apply_dir<M, OL>(ne, O, L.z, beta, po, pn, L.w), red());
                const double alpha = rz / pw;
                const double rrk = block_sum(s_update_first_sweep<M, OL>(ne, O, A.omega, alpha, pn, L.w, rc, rnx, L.lam,
                                                                         L.z0, A.nu_pre >= 2 ? L.x : nullptr),
                                             red());
                ++its;
                if (!isfinite(rrk) || rrk <= rtol * rtol * bn2) break;
                const double rzn = block_sum(s_vcycle_rest<M, OL>(A, L, rnx, L.z, rnx), red());
                beta = rzn / rz;
                rz = rzn;
                po = pn;
                pc ^= 1;
                double *t = rc;
                rc = rnx;
                rnx = t;
            }
        } else {
            // flexible GMRES(R), classical Gram-Schmidt; the basis in global memory
            // (each thread reads back only the items it wrote), the current basis
            // vector also in LDS (L.p) as the V-cycle's input
            const int R = A.restart;
            const double beta = sqrt(rr);
            for_own<M>(ne, [&](int i) {
                const double v = L.r[i] / beta;
                Vb[i] = v;
                L.p[i] = v;
            });
            if (tid == 0) L.g[0] = beta;
            __syncthreads();
            int k = 0;
            for (int j = 0; j < R && its < A.maxit; ++j) {
                s_vcycle<M, OL>(A, L, L.p, L.z);
                double *Zj = Zb + (size_t)j * ne * M;
                for_own<M>(ne, [&](int i) { Zj[i] = L.z[i]; });
                s_apply<M, OL>(ne, O, L.z, nullptr, L.w);
                // h_q = V_q . w for q <= j
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
                for_own<M>(ne, [&](int i) {
                    const double v = L.w[i] * inv;
                    Vn[i] = v;
                    L.p[i] = v;
                });
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

    // ---- outputs: lam, (stage) the recovered cell fields, then the info record
    for_own<M>(ne, [&](int i) { A.lam[(size_t)i * nb + rh] = L.lam[i]; });
    if (STAGE) {
        __syncthreads();
        // Step 3: q = Ar r_cell - Wr lam_K per cell.  The cell's right-hand side is
        // read once; outputs go three at a time, each group's row loads issued
        // together before its stores (which could alias them).
        constexpr int QG = 3;
        static_assert(nc % QG == 0, "three fields per node");
        for (int K = tid; K < A.nk; K += SMALL_THREADS) {
            double l[nt], rc[nc];
#pragma unroll
            for (int j = 0; j < nc; ++j) rc[j] = A.r_cell[((size_t)K * nc + j) * nb + rh];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const int e = A.cell_facet[i * NK + K];
                const int rev = A.cell_rev[i * NK + K];
#pragma unroll
                for (int t = 0; t < M; ++t) l[i * M + t] = L.lam[e * M + (rev ? P - t : t)];   // l[loc_trace(i, a, rev)] = lam[e][a]
            }
            for (int a0 = 0; a0 < nc; a0 += QG) {
                double s[QG];
#pragma unroll
                for (int g = 0; g < QG; ++g) {
                    const int a = a0 + g;
                    s[g] = 0.0;
#pragma unroll
                    for (int j = 0; j < nc; ++j) s[g] += A.Ar[(size_t)(a * nc + j) * NK + K] * rc[j];
#pragma unroll
                    for (int j = 0; j < nt; ++j) s[g] -= A.Wr[(size_t)(a * nt + j) * NK + K] * l[j];
                }
#pragma unroll
                for (int g = 0; g < QG; ++g) A.q_cell[((size_t)K * nc + a0 + g) * nb + rh] = s[g];
            }
        }
    }
    // the record goes to host-mapped memory last, its status after a system-scope
    // fence: the host returns once every right-hand side's status has arrived
    __syncthreads();
    if (tid == 0) {
        A.info[4 * rh + 0] = its;
        A.info[4 * rh + 1] = restarts;
        A.info[4 * rh + 3] = rel;
        __threadfence_system();
        A.info[4 * rh + 2] = status;
    }
}

size_t round16(size_t b) { return (b + 15) / 16 * 16; }

}  // namespace

size_t small_lds_bytes(int ne, int m, const P1Lev *lev, int nlev, bool stage_ops, int nB) {
    size_t d = (size_t)12 * ne * m;
    for (int l = 0; l < nlev; ++l) d += 3 * (size_t)lev[l].n;
    size_t bytes = (d + small_fixed_doubles()) * sizeof(double);
    if (stage_ops) bytes += 16 + small_image_bytes(ne, m, lev, nlev, nB);   // alignment + the operator image
    return bytes;
}

template <int P, bool STAGE, bool OL>
hipError_t prepare_one(size_t bytes) {
    return hipFuncSetAttribute((const void *)k_solve_small<P, STAGE, OL>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)bytes);
}

template <int P>
hipError_t prepare_p(size_t bytes) {
    const hipError_t e[4] = {prepare_one<P, false, false>(bytes), prepare_one<P, false, true>(bytes),
                             prepare_one<P, true, false>(bytes), prepare_one<P, true, true>(bytes)};
    for (hipError_t x : e)
        if (x != hipSuccess) return x;
    return hipSuccess;
}

hipError_t small_prepare(int p, size_t bytes) {
    // dynamic LDS above the default 64 KiB needs the kernels' opt-in
    switch (p) {
    case 1: return prepare_p<1>(bytes);
    case 2: return prepare_p<2>(bytes);
    case 3: return prepare_p<3>(bytes);
    default: return hipErrorInvalidValue;
    }
}

template <int P>
void launch_p(bool stage, const SmallArgs &A, size_t bytes, hipStream_t s) {
    const dim3 grid(A.nb), block(SMALL_THREADS);
    if (stage) {
        if (A.stage_ops) k_solve_small<P, true, true><<<grid, block, bytes, s>>>(A);
        else k_solve_small<P, true, false><<<grid, block, bytes, s>>>(A);
    } else {
        if (A.stage_ops) k_solve_small<P, false, true><<<grid, block, bytes, s>>>(A);
        else k_solve_small<P, false, false><<<grid, block, bytes, s>>>(A);
    }
}

void launch_solve_small(int p, bool stage, const SmallArgs &A, size_t bytes, hipStream_t s) {
    switch (p) {
    case 1: launch_p<1>(stage, A, bytes, s); break;
    case 2: launch_p<2>(stage, A, bytes, s); break;
    case 3: launch_p<3>(stage, A, bytes, s); break;
    default: break;
    }
}

}  // namespace hdg
