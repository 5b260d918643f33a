// IMEX time stepping around the HDG stage solve (Eqs. IMEX_HDG_I, IMEX_HDG_II,
// theta_method) and the explicit flux evaluation it needs for an explicit
// first stage.
//
// A step is a short host loop over the stages: one elementwise kernel builds
// the stage's right-hand side in DG coefficients, then condense / solve /
// recover give the stage.  The flux term of an implicit stage is never
// evaluated: dt M^-1 L(Q_j) = (Q_j - R_j) / at_jj follows from the stage
// equation itself, and the explicit source M^-1 N_0 = -f k x u is a rotation
// of the velocity coefficients.  Both enter later stages through the same
// combination kernel, which reads every input once per DG node (HBM-bound,
// coalesced over the [cell][field][node][rhs] layout).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <functional>
#include <string>
#include <vector>

#include "hdg_internal.h"

namespace hdg {
namespace {

constexpr int TEND_MAX_RHS = 64;
constexpr int COMBINE_MAX = 2 * HDG_IMEX_MAX_STAGES;




// ------------------------------------------------------------------ kernels

// Each side's share of the DG trace at the nodes of one of its facets, in the
// facet's direction: upwind  phi / 2 + u.n / (2 tau),  Lax-Friedrichs
// u_d / 2 + phi n_d / (2 tau).  The trace of q is the sum of the two shares.
// Nodal Lagrange bases make the cell's values at the facet nodes its
// coefficients at the lattice nodes on that side.  One thread per
// (cell, local facet, rhs); half is [facet][side][facet_dofs][nrhs], side 0
// for the owner (which runs along the facet), 1 for the other cell.
template <int P, int NU>
__global__ __launch_bounds__(256) void k_dg_half(int nk, int nb, int geom, double tau, double hscale,
                                                 const double *__restrict__ corners,
                                                 const int *__restrict__ cell_facet,
                                                 const int8_t *__restrict__ cell_rev, const double *__restrict__ q,
                                                 double *__restrict__ half) {
    constexpr int n = (P + 1) * (P + 2) / 2, m = P + 1, M = NU * m;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nk * 3 * nb) return;
    const int r = (int)(t % nb);
    const int kf = (int)(t / nb), K = kf / 3, f = kf % 3;
    const size_t NK = (size_t)nk;

    // outward unit normal of local facet f in the cell's frame
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
    const double Px[3] = {0.0, ab[0] * e1[0] + ab[1] * e1[1] + ab[2] * e1[2], ac[0] * e1[0] + ac[1] * e1[1] + ac[2] * e1[2]};
    const double Py[3] = {0.0, ab[0] * e2[0] + ab[1] * e2[1] + ab[2] * e2[2], ac[0] * e2[0] + ac[1] * e2[1] + ac[2] * e2[2]};
    const double tx = Px[(f + 2) % 3] - Px[(f + 1) % 3], ty = Py[(f + 2) % 3] - Py[(f + 1) % 3];
    const double L = sqrt(tx * tx + ty * ty);
    const double nx = ty / L, ny = -tx / L;

    const int e = cell_facet[f * NK + K];
    const int rev = cell_rev[f * NK + K];
    const double *qK = q + (size_t)K * 3 * n * nb + r;
    double *hK = half + ((size_t)e * 2 + rev) * M * nb + r;
    const double it2 = 0.5 / tau;
#pragma unroll
    for (int k = 0; k <= P; ++k) {
        // lattice node (i, j) at counter-clockwise parameter k / P along facet f
        const int i = f == 0 ? P - k : (f == 1 ? 0 : k);
        const int j = f == 0 ? k : (f == 1 ? P - k : 0);
        const int node = j * (P + 1) - j * (j - 1) / 2 + i;
        const double phi = hscale * qK[(size_t)node * nb];
        const double u1 = qK[(size_t)(n + node) * nb], u2 = qK[(size_t)(2 * n + node) * nb];
        const int kk = rev ? P - k : k;
        if constexpr (NU == 1) {
            hK[(size_t)kk * nb] = 0.5 * phi + (u1 * nx + u2 * ny) * it2;
        } else {
            hK[(size_t)kk * nb] = 0.5 * u1 + phi * nx * it2;
            hK[(size_t)(m + kk) * nb] = 0.5 * u2 + phi * ny * it2;
        }
    }
}

// Local trace index of unknown a of local facet i for a cell running along
// (rev = 0) or against (rev = 1) the facet's direction.
template <int P, int NU>
__device__ __forceinline__ int tend_loc(int i, int a, int rev) {
    constexpr int m = P + 1;
    const int k = a % m;
    return i * NU * m + (a - k) + (rev ? P - k : k);
}

// out = scale (q - r) with r the right-hand side for which the recovery
// q = Ar r - Wr lam returns q:  Ar r = q + Wr lam,  solved per cell by
// Gauss-Jordan with partial pivoting in LDS (one wavefront per cell, all
// right-hand sides as extra columns).
template <int P, int NU>
__global__ __launch_bounds__(64) void k_dg_tendency(int nk, int nb, double scale, const double *__restrict__ Ar,
                                                    const double *__restrict__ Wr,
                                                    const int *__restrict__ cell_facet,
                                                    const int8_t *__restrict__ cell_rev,
                                                    const double *__restrict__ q, const double *__restrict__ half,
                                                    double *__restrict__ out, int *__restrict__ err) {
    constexpr int n = (P + 1) * (P + 2) / 2, m = P + 1, nc = 3 * n, M = NU * m, nt = 3 * M;
    // LDS sized for the call's nb (tend_lds_bytes): [nc][nc + nb] | [nt][nb] | [nc]
    extern __shared__ double tsm[];
    const int LD = nc + nb, W = nc + nb;
    double *aug = tsm, *lam = tsm + nc * LD, *fac = lam + nt * nb;
    const int K = blockIdx.x, lane = threadIdx.x;
    if (K >= nk) return;
    const size_t NK = (size_t)nk;

    for (int idx = lane; idx < nt * nb; idx += 64) {
        const int g = idx / nb, r = idx - g * nb, i = g / M, a = g - i * M;
        const int e = cell_facet[i * NK + K], rev = cell_rev[i * NK + K];
        const double v = half[(((size_t)e * 2 + 0) * M + a) * nb + r] + half[(((size_t)e * 2 + 1) * M + a) * nb + r];
        lam[tend_loc<P, NU>(i, a, rev) * nb + r] = v;
    }
    for (int idx = lane; idx < nc * nc; idx += 64) aug[(idx / nc) * LD + idx % nc] = Ar[(size_t)idx * NK + K];
    __syncthreads();
    for (int idx = lane; idx < nc * nb; idx += 64) {
        const int a = idx / nb, r = idx - a * nb;
        double s = q[((size_t)K * nc + a) * nb + r];
        for (int j = 0; j < nt; ++j) s += Wr[(size_t)(a * nt + j) * NK + K] * lam[j * nb + r];
        aug[a * LD + nc + r] = s;
    }
    __syncthreads();

    for (int k = 0; k < nc; ++k) {
        double best = (lane >= k && lane < nc) ? fabs(aug[lane * LD + k]) : -1.0;
        int bi = lane;
        for (int off = 32; off > 0; off >>= 1) {
            const double ob = __shfl_xor(best, off, 64);
            const int oi = __shfl_xor(bi, off, 64);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        if (!(best > 0.0)) {
            if (lane == 0) atomicOr(err, 1);
            return;
        }
        if (bi != k) {
            for (int c = lane; c < W; c += 64) {
                const double t = aug[k * LD + c];
                aug[k * LD + c] = aug[bi * LD + c];
                aug[bi * LD + c] = t;
            }
        }
        __syncthreads();
        const double ip = 1.0 / aug[k * LD + k];
        __syncthreads();
        for (int c = lane; c < W; c += 64) aug[k * LD + c] *= ip;
        for (int rr = lane; rr < nc; rr += 64) fac[rr] = aug[rr * LD + k];
        __syncthreads();
        for (int idx = lane; idx < nc * (W - k); idx += 64) {
            const int rr = idx / (W - k), c = k + idx % (W - k);
            if (rr != k) aug[rr * LD + c] -= fac[rr] * aug[k * LD + c];
        }
        __syncthreads();
    }
    for (int idx = lane; idx < nc * nb; idx += 64) {
        const int a = idx / nb, r = idx - a * nb;
        const size_t o = ((size_t)K * nc + a) * nb + r;
        out[o] = scale * (q[o] - aug[a * LD + nc + r]);
    }
}

// out = cb base + sum_j crot_j R(rot_j) + sum_j cdif_j (dq_j - dr_j)  at every
// DG node, with R(u) = (0, u_2, -u_1) (the explicit source with f folded into
// crot) and dr_j optional (null reads as zero).  Terms are added in this
// fixed order.  out may alias any input: each thread reads its own node only.
struct Combine {
    const double *base;
    double cb;
    int nrot, ndif;
    const double *rot[COMBINE_MAX];
    double crot[COMBINE_MAX];
    const double *dq[COMBINE_MAX];
    const double *dr[COMBINE_MAX];
    double cdif[COMBINE_MAX];
};

__global__ __launch_bounds__(256) void k_imex_combine(int64_t npt, int64_t stride, Combine t,
                                                      double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npt) return;
    const int64_t K = i / stride, rest = i - K * stride;
    const size_t o0 = (size_t)(K * 3 * stride + rest), o1 = o0 + stride, o2 = o1 + stride;
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    if (t.base) {
        v0 = t.cb * t.base[o0];
        v1 = t.cb * t.base[o1];
        v2 = t.cb * t.base[o2];
    }
    for (int j = 0; j < t.nrot; ++j) {
        const double *u = t.rot[j];
        const double a1 = u[o1], a2 = u[o2];
        v1 = __builtin_fma(t.crot[j], a2, v1);
        v2 = __builtin_fma(-t.crot[j], a1, v2);
    }
    for (int j = 0; j < t.ndif; ++j) {
        const double *x = t.dq[j], *y = t.dr[j];
        const double c = t.cdif[j];
        if (y) {
            v0 = __builtin_fma(c, x[o0] - y[o0], v0);
            v1 = __builtin_fma(c, x[o1] - y[o1], v1);
            v2 = __builtin_fma(c, x[o2] - y[o2], v2);
        } else {
            v0 = __builtin_fma(c, x[o0], v0);
            v1 = __builtin_fma(c, x[o1], v1);
            v2 = __builtin_fma(c, x[o2], v2);
        }
    }
    out[o0] = v0;
    out[o1] = v1;
    out[o2] = v2;
}

// ------------------------------------------------------------------ host helpers

void launch_combine(const hdg_ctx *c, int nb, const Combine &t, double *out, hipStream_t s) {
    const int64_t stride = (int64_t)c->n * nb;
    const int64_t npt = (int64_t)c->n_cell * stride;
    const int block = 256;
    const int64_t grid = (npt + block - 1) / block;
    hipLaunchKernelGGL(k_imex_combine, dim3((unsigned)grid), dim3(block), 0, s, npt, stride, t, out);
    check_kernel_launch();
}

void check_nb(const hdg_ctx *c, int nb) {
    HDG_REQUIRE(nb >= 1 && nb <= c->opt.max_rhs,
                "nrhs must be in 1..max_rhs (" + std::to_string(c->opt.max_rhs) + ")");
}

double *half_buffer(hdg_ctx *c) {
    // [n_facet][2][m][max_rhs], allocated on first use and owned by the context
    if (c->dg_half) return c->dg_half;
    const size_t count = (size_t)c->n_facet * 2 * c->m * c->opt.max_rhs;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, count * sizeof(double));
    if (e != hipSuccess) throw Error{HDG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
    c->allocations.push_back(p);
    c->device_bytes += (int64_t)(count * sizeof(double));
    c->dg_half = static_cast<double *>(p);
    return c->dg_half;
}

void dg_tendency(hdg_ctx *c, int nb, double dt, const double *q, double *out, hipStream_t s) {
    double *half = half_buffer(c);
    int *err = c->dg_err;
    if (!err) {
        void *p = nullptr;
        HDG_HIP_CHECK(hipMalloc(&p, sizeof(int)));
        c->allocations.push_back(p);
        c->device_bytes += (int64_t)sizeof(int);
        c->dg_err = err = static_cast<int *>(p);
    }
    HDG_HIP_CHECK(hipMemsetAsync(err, 0, sizeof(int), s));
    const int64_t nth = (int64_t)c->n_cell * 3 * nb;
    const int block = 256;
    const unsigned grid = (unsigned)((nth + block - 1) / block);
    const double scale = dt / c->dt;
#define HALF(P, NU)                                                                                              \
    hipLaunchKernelGGL((k_dg_half<P, NU>), dim3(grid), dim3(block), 0, s, c->n_cell, nb, c->geom, c->tau, c->hscale, \
                       c->corners, c->cell_facet, c->cell_rev, q, half)
    const size_t lds = (size_t)(c->nc * (c->nc + nb) + c->nt * nb + c->nc) * sizeof(double);
#define TEND(P, NU)                                                                                               \
    hipLaunchKernelGGL((k_dg_tendency<P, NU>), dim3(c->n_cell), dim3(64), lds, s, c->n_cell, nb, scale, c->Ar, c->Wr, \
                       c->cell_facet, c->cell_rev, q, half, out, err)
    if (c->nu == 1) {
        switch (c->p) {
            case 1: HALF(1, 1); check_kernel_launch(); TEND(1, 1); break;
            case 2: HALF(2, 1); check_kernel_launch(); TEND(2, 1); break;
            default: HALF(3, 1); check_kernel_launch(); TEND(3, 1); break;
        }
    } else {
        switch (c->p) {
            case 1: HALF(1, 2); check_kernel_launch(); TEND(1, 2); break;
            case 2: HALF(2, 2); check_kernel_launch(); TEND(2, 2); break;
            default: HALF(3, 2); check_kernel_launch(); TEND(3, 2); break;
        }
    }
#undef HALF
#undef TEND
    check_kernel_launch();
}

struct Plan {
    int s = 0;
    double gamma = 0.0;
    bool need_tend = false;   // explicit first stage whose flux term is used
    bool fsal = false;        // carry the flux term of the last stage to the next step
};

Plan make_plan(const hdg_imex_tableau *tab) {
    HDG_REQUIRE(tab, "tableau must not be NULL");
    Plan pl;
    pl.s = tab->stages;
    HDG_REQUIRE(pl.s >= 1 && pl.s <= HDG_IMEX_MAX_STAGES, "stages must be in 1..5");
    const int s = pl.s;
    for (int i = 0; i < s; ++i)
        for (int j = 0; j < s; ++j) {
            HDG_REQUIRE(std::isfinite(tab->a[i][j]) && std::isfinite(tab->at[i][j]), "non-finite tableau entry");
            if (j >= i) HDG_REQUIRE(tab->a[i][j] == 0.0, "a must be strictly lower triangular");
            if (j > i) HDG_REQUIRE(tab->at[i][j] == 0.0, "at must be lower triangular");
        }
    for (int i = 0; i < s; ++i) {
        const double d = tab->at[i][i];
        if (d == 0.0) continue;
        if (pl.gamma == 0.0) pl.gamma = d;
        HDG_REQUIRE(std::fabs(d - pl.gamma) <= 1e-14 * std::fabs(pl.gamma),
                    "the nonzero diagonal entries of at must be equal (one stage operator)");
    }
    HDG_REQUIRE(pl.gamma > 0.0, "the tableau needs an implicit stage with a positive diagonal entry");
    for (int j = 1; j < s; ++j) {
        if (tab->at[j][j] != 0.0) continue;
        bool used = tab->bt[j] != 0.0;
        for (int i = j + 1; i < s; ++i) used = used || tab->at[i][j] != 0.0;
        HDG_REQUIRE(!used, "an explicit stage after the first may not feed the implicit part");
    }
    if (tab->at[0][0] == 0.0) {
        bool used = tab->bt[0] != 0.0;
        for (int i = 1; i < s; ++i) used = used || tab->at[i][0] != 0.0;
        pl.need_tend = used;
    }
    if (pl.need_tend && tab->at[s - 1][s - 1] != 0.0) {
        bool sa = true;
        for (int j = 0; j < s; ++j) sa = sa && tab->b[j] == tab->a[s - 1][j] && tab->bt[j] == tab->at[s - 1][j];
        pl.fsal = sa;
    }
    return pl;
}

size_t even(size_t x) { return (x + 1) & ~(size_t)1; }

}  // namespace

void launch_dg_half(const hdg_ctx *c, int nb, double hscale, const double *q, double *half, hipStream_t s) {
    const int64_t nth = (int64_t)c->n_cell * 3 * nb;
    const int block = 256;
    const unsigned grid = (unsigned)((nth + block - 1) / block);
#define HALF(P, NU)                                                                                           \
    hipLaunchKernelGGL((k_dg_half<P, NU>), dim3(grid), dim3(block), 0, s, c->n_cell, nb, c->geom, c->tau, hscale, \
                       c->corners, c->cell_facet, c->cell_rev, q, half)
    if (c->nu == 1) {
        switch (c->p) {
            case 1: HALF(1, 1); break;
            case 2: HALF(2, 1); break;
            default: HALF(3, 1); break;
        }
    } else {
        switch (c->p) {
            case 1: HALF(1, 2); break;
            case 2: HALF(2, 2); break;
            default: HALF(3, 2); break;
        }
    }
#undef HALF
    check_kernel_launch();
}

}  // namespace hdg

using hdg::Error;

extern "C" int hdg_imex_tableau_get(int32_t method, double theta, hdg_imex_tableau *out) {
    return hdg::guarded([&] {
        HDG_REQUIRE(out, "out must not be NULL");
        hdg_imex_tableau t{};
        switch (method) {
            case HDG_IMEX_THETA:
                HDG_REQUIRE(theta > 0.0 && theta <= 1.0, "theta must be in (0, 1]");
                t.stages = 2;
                t.a[1][0] = 1.0;
                t.at[1][0] = 1.0 - theta;
                t.at[1][1] = theta;
                t.b[0] = 1.0;
                t.bt[0] = 1.0 - theta;
                t.bt[1] = theta;
                break;
            case HDG_IMEX_ARS232: {
                const double g = 1.0 - 1.0 / std::sqrt(2.0), d = -2.0 * std::sqrt(2.0) / 3.0;
                t.stages = 3;
                t.a[1][0] = g;
                t.a[2][0] = d;
                t.a[2][1] = 1.0 - d;
                t.at[1][1] = g;
                t.at[2][1] = 1.0 - g;
                t.at[2][2] = g;
                t.b[1] = t.bt[1] = 1.0 - g;
                t.b[2] = t.bt[2] = g;
                break;
            }
            case HDG_IMEX_SSP322:
                t.stages = 3;
                t.a[2][1] = 1.0;
                t.at[0][0] = 0.5;
                t.at[1][0] = -0.5;
                t.at[1][1] = 0.5;
                t.at[2][1] = 0.5;
                t.at[2][2] = 0.5;
                t.b[1] = t.bt[1] = 0.5;
                t.b[2] = t.bt[2] = 0.5;
                break;
            case HDG_IMEX_ARS443: {
                t.stages = 5;
                const double a[5][5] = {{0, 0, 0, 0, 0},
                                        {1.0 / 2, 0, 0, 0, 0},
                                        {11.0 / 18, 1.0 / 18, 0, 0, 0},
                                        {5.0 / 6, -5.0 / 6, 1.0 / 2, 0, 0},
                                        {1.0 / 4, 7.0 / 4, 3.0 / 4, -7.0 / 4, 0}};
                const double at[5][5] = {{0, 0, 0, 0, 0},
                                         {0, 1.0 / 2, 0, 0, 0},
                                         {0, 1.0 / 6, 1.0 / 2, 0, 0},
                                         {0, -1.0 / 2, 1.0 / 2, 1.0 / 2, 0},
                                         {0, 3.0 / 2, -3.0 / 2, 1.0 / 2, 1.0 / 2}};
                for (int i = 0; i < 5; ++i)
                    for (int j = 0; j < 5; ++j) {
                        t.a[i][j] = a[i][j];
                        t.at[i][j] = at[i][j];
                    }
                for (int j = 0; j < 5; ++j) {
                    t.b[j] = a[4][j];
                    t.bt[j] = at[4][j];
                }
                break;
            }
            default:
                throw Error{HDG_EINVAL, "unknown IMEX method"};
        }
        *out = t;
    });
}

extern "C" int hdg_imex_work_size(const hdg_ctx *c, const hdg_imex_tableau *tab, int32_t nb, int64_t *doubles) {
    if (!c) return HDG_EINVAL;
    return hdg::guarded([&] {
        HDG_REQUIRE(doubles, "doubles must not be NULL");
        hdg::check_nb(c, nb);
        const hdg::Plan pl = hdg::make_plan(tab);
        const size_t cell = hdg::even((size_t)c->n_cell * c->nc * nb);
        const size_t trace = hdg::even((size_t)c->n_facet * c->m * nb);
        *doubles = (int64_t)((2 * pl.s + 1) * cell + 2 * trace);
    });
}

extern "C" int hdg_dg_tendency(hdg_ctx *c, int32_t nb, double dt, const double *q, double *out, void *stream) {
    if (!c) return HDG_EINVAL;
    return hdg::guarded([&] {
        hdg::check_nb(c, nb);
        HDG_REQUIRE(nb <= hdg::TEND_MAX_RHS, "nrhs must be at most 64");
        HDG_REQUIRE(q && out && q != out, "q and out must be distinct non-NULL arrays");
        HDG_REQUIRE(std::isfinite(dt), "dt must be finite");
        hipStream_t s = reinterpret_cast<hipStream_t>(stream);
        hdg::dg_tendency(c, nb, dt, q, out, s);
        int herr = 0;
        HDG_HIP_CHECK(hipMemcpyAsync(&herr, c->dg_err, sizeof(int), hipMemcpyDeviceToHost, s));
        HDG_HIP_CHECK(hipStreamSynchronize(s));
        if (herr) throw Error{HDG_EBREAKDOWN, "singular recovery matrix in the flux evaluation"};
    });
}

extern "C" int hdg_imex_run(hdg_ctx *c, const hdg_imex_tableau *tab, double dt, double f, int32_t nb,
                            int32_t steps, double *q, double *work, hdg_imex_info *info, void *stream) {
    if (!c) return HDG_EINVAL;
    int status = HDG_OK;
    const int rc = hdg::guarded([&] {
        hdg::check_nb(c, nb);
        const hdg::Plan pl = hdg::make_plan(tab);
        HDG_REQUIRE(q && work, "q and work must not be NULL");
        HDG_REQUIRE(((uintptr_t)work & 15) == 0, "work must be 16-byte aligned");
        HDG_REQUIRE(steps >= 0, "steps must be >= 0");
        HDG_REQUIRE(dt > 0.0 && std::isfinite(dt) && std::isfinite(f), "dt must be positive and f finite");
        HDG_REQUIRE(c->prm.f0 == 0.0 && c->prm.omega == 0.0,
                    "IMEX stepping treats Coriolis explicitly: set the context up with f0 = omega = 0");
        HDG_REQUIRE(std::fabs(c->prm.dt - pl.gamma * dt) <= 1e-12 * pl.gamma * dt,
                    "the context's dt must be gamma * dt (gamma: the implicit diagonal of the tableau)");
        HDG_REQUIRE(!pl.need_tend || nb <= hdg::TEND_MAX_RHS, "nrhs must be at most 64");
        const int s = pl.s;
        const size_t cell = hdg::even((size_t)c->n_cell * c->nc * nb);
        const size_t trace = hdg::even((size_t)c->n_facet * c->m * nb);
        double *R[HDG_IMEX_MAX_STAGES], *Q[HDG_IMEX_MAX_STAGES];
        for (int i = 0; i < s; ++i) {
            R[i] = work + (size_t)(2 * i) * cell;
            Q[i] = work + (size_t)(2 * i + 1) * cell;
        }
        double *tend = work + (size_t)(2 * s) * cell;
        double *rhat = tend + cell;
        double *lam = rhat + trace;
        hipStream_t st = reinterpret_cast<hipStream_t>(stream);
        std::vector<hdg_solve_info> si(nb);
        hdg_imex_info acc{};
        acc.status = HDG_OK;
        const double(*a)[5] = tab->a;
        const double(*at)[5] = tab->at;
        const double *stage_q[HDG_IMEX_MAX_STAGES];

        for (int step = 0; step < steps; ++step) {
            if (pl.need_tend && (step == 0 || !pl.fsal)) {
                hdg::dg_tendency(c, nb, dt, q, tend, st);
                int herr = 0;
                HDG_HIP_CHECK(hipMemcpyAsync(&herr, c->dg_err, sizeof(int), hipMemcpyDeviceToHost, st));
                HDG_HIP_CHECK(hipStreamSynchronize(st));
                if (herr) throw Error{HDG_EBREAKDOWN, "singular recovery matrix in the flux evaluation"};
            }
            for (int i = 0; i < s; ++i) {
                if (i == 0 && at[0][0] == 0.0) {
                    stage_q[0] = q;   // explicit first stage: Q_1 = q_n
                    continue;
                }
                hdg::Combine t{};
                t.base = q;
                t.cb = 1.0;
                for (int j = 0; j < i; ++j) {
                    if (a[i][j] != 0.0 && f != 0.0) {
                        t.rot[t.nrot] = stage_q[j];
                        t.crot[t.nrot++] = dt * a[i][j] * f;
                    }
                    if (at[i][j] != 0.0) {
                        if (at[j][j] != 0.0) {
                            t.dq[t.ndif] = Q[j];
                            t.dr[t.ndif] = R[j];
                            t.cdif[t.ndif++] = at[i][j] / at[j][j];
                        } else {   // j == 0, the carried flux term dt M^-1 L(q_n)
                            t.dq[t.ndif] = tend;
                            t.dr[t.ndif] = nullptr;
                            t.cdif[t.ndif++] = at[i][j];
                        }
                    }
                }
                hdg::launch_combine(c, nb, t, R[i], st);
                if (at[i][i] == 0.0) {
                    stage_q[i] = R[i];
                    continue;
                }
                hdg::check_abi(hdg_condense(c, nb, R[i], rhat, stream));
                HDG_HIP_CHECK(hipMemsetAsync(lam, 0, (size_t)c->n_facet * c->m * nb * sizeof(double), st));
                const int src = hdg_solve(c, nb, rhat, lam, si.data(), stream);
                hdg::check_abi(src);
                if (src == HDG_ENOTCONV) acc.status = HDG_ENOTCONV;
                int it = 0;
                for (int r = 0; r < nb; ++r) {
                    it = std::max(it, (int)si[r].iters);
                    acc.rel_res_max = std::max(acc.rel_res_max, si[r].rel_res);
                }
                acc.solves++;
                acc.iters_total += it;
                acc.iters_max = std::max(acc.iters_max, it);
                hdg::check_abi(hdg_recover(c, nb, R[i], lam, Q[i], stream));
                stage_q[i] = Q[i];
            }
            // q_{n+1} = q_n + dt sum_i b_i N_0(Q_i) + dt sum_i bt_i L(Q_i), in place
            hdg::Combine t{};
            t.base = q;
            t.cb = 1.0;
            for (int i = 0; i < s; ++i) {
                if (tab->b[i] != 0.0 && f != 0.0) {
                    t.rot[t.nrot] = stage_q[i];
                    t.crot[t.nrot++] = dt * tab->b[i] * f;
                }
                if (tab->bt[i] != 0.0) {
                    if (at[i][i] != 0.0) {
                        t.dq[t.ndif] = Q[i];
                        t.dr[t.ndif] = R[i];
                        t.cdif[t.ndif++] = tab->bt[i] / at[i][i];
                    } else {
                        t.dq[t.ndif] = tend;
                        t.dr[t.ndif] = nullptr;
                        t.cdif[t.ndif++] = tab->bt[i];
                    }
                }
            }
            hdg::launch_combine(c, nb, t, q, st);
            if (pl.fsal) {   // dt M^-1 L(q_{n+1}) from the last stage
                hdg::Combine u{};
                u.dq[0] = Q[s - 1];
                u.dr[0] = R[s - 1];
                u.cdif[0] = 1.0 / at[s - 1][s - 1];
                u.ndif = 1;
                hdg::launch_combine(c, nb, u, tend, st);
            }
            acc.steps++;
        }
        HDG_HIP_CHECK(hipStreamSynchronize(st));
        status = acc.status;
        if (info) *info = acc;
    });
    if (rc != HDG_OK) return rc;
    return status;
}
