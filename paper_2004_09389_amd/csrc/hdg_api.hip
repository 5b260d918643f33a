// C ABI of the HDG trace-multigrid library: setup, the three-step Schur
// solve (condense, Krylov on the trace system, recover), the non-nested
// V-cycle and measurement helpers.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <utility>

#include "hdg_kernels.h"
#include "hdg_rt0.h"

using hdg::Error;

namespace {

// ------------------------------------------------------------------ static scratch of hdg_condense_noalloc
//
// The condensation stages each cell's contribution to its facets before the
// facet gather (3 facet_dofs values per cell and right-hand side).
// hdg_condense keeps that buffer in the context; hdg_condense_noalloc uses
// this fixed array instead, so that the call itself allocates nothing.  Every
// GPU the library runs on holds its own copy until the process ends.  The
// array's name is a host-side stand-in: host code uses only the device address
// hipGetSymbolAddress returns for it, resolved once per device by hdg_setup
// with that device current.
constexpr size_t NOALLOC_SCRATCH_DOUBLES = (size_t)4 << 20;   // 32 MiB
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_DOUBLES];
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[MAX_DEVICES] = {};

// device address of scratch on device dev (the current device); resolved on first use
double *scratch_on(int dev) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    HDG_REQUIRE(dev >= 0 && dev < MAX_DEVICES, "device id out of range for the static scratch");
    if (!g_scratch_dev[dev]) {
        void *ptr = nullptr;
        HDG_HIP_CHECK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        HDG_REQUIRE(ptr != nullptr, "hipGetSymbolAddress returned no address for the static scratch");
        g_scratch_dev[dev] = static_cast<double *>(ptr);
    }
    return g_scratch_dev[dev];
}

// ------------------------------------------------------------------ allocation helpers

template <typename T>
T *dev_alloc(hdg_ctx *c, size_t count) {
    if (count == 0) count = 1;
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, count * sizeof(T));
    if (e != hipSuccess) throw Error{HDG_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)};
    c->allocations.push_back(p);
    c->device_bytes += (int64_t)(count * sizeof(T));
    return static_cast<T *>(p);
}

template <typename T>
T *dev_upload(hdg_ctx *c, const std::vector<T> &v) {
    T *p = dev_alloc<T>(c, v.size());
    if (!v.empty()) HDG_HIP_CHECK(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
}

void dev_release(hdg_ctx *c, void *p, size_t bytes) {
    auto it = std::find(c->allocations.begin(), c->allocations.end(), p);
    if (it != c->allocations.end()) {
        c->allocations.erase(it);
        c->device_bytes -= (int64_t)bytes;
        (void)hipFree(p);
    }
}

int guard(const std::function<void()> &fn) {
    try {
        fn();
        return HDG_OK;
    } catch (const Error &e) {
        hdg::set_error(e.msg);
        return e.code;
    } catch (const std::bad_alloc &) {
        hdg::set_error("host allocation failed");
        return HDG_ENOMEM;
    } catch (const std::exception &e) {
        hdg::set_error(e.what());
        return HDG_EINVAL;
    }
}

inline hipStream_t as_stream(void *s) { return reinterpret_cast<hipStream_t>(s); }

void check_launch() {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) throw Error{HDG_EHIP, std::string("kernel launch: ") + hipGetErrorString(e)};
}

// ------------------------------------------------------------------ HIP graphs
//
// A Krylov iteration is a fixed sequence of ~25 small launches.  It is
// captured once per (kind, nrhs, precision, index) on a private stream and
// replayed into the caller's stream; the pointers it bakes in are all
// context-owned buffers, so replays stay valid for the context's lifetime.
// Nothing captured clears memory with a memset node.
void run_step(hdg_ctx *c, uint64_t key, hipStream_t s, const std::function<void(hipStream_t)> &body) {
    if (!c->opt.use_graph || c->timing) {
        body(s);
        return;
    }
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        if (!c->cap_stream) HDG_HIP_CHECK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
        // order the capture stream after work already queued on s
        HDG_HIP_CHECK(hipStreamSynchronize(s));
        hipGraph_t g = nullptr;
        HDG_HIP_CHECK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
        body(c->cap_stream);
        HDG_HIP_CHECK(hipStreamEndCapture(c->cap_stream, &g));
        hipGraphExec_t ex = nullptr;
        HDG_HIP_CHECK(hipGraphInstantiate(&ex, g, nullptr, nullptr, 0));
        HDG_HIP_CHECK(hipGraphDestroy(g));
        it = c->graphs.emplace(key, ex).first;
    }
    HDG_HIP_CHECK(hipGraphLaunch(it->second, s));
}

void drop_graphs(hdg_ctx *c) {
    for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.second);
    c->graphs.clear();
}

uint64_t graph_key(int kind, int nb, int prec, int idx) {
    return ((uint64_t)kind << 48) | ((uint64_t)nb << 32) | ((uint64_t)prec << 24) | (uint64_t)idx;
}

// ------------------------------------------------------------------ kernel timing

hipEvent_t pool_event(hdg_ctx *c) {
    if (!c->event_pool.empty()) {
        hipEvent_t e = c->event_pool.back();
        c->event_pool.pop_back();
        return e;
    }
    hipEvent_t e;
    HDG_HIP_CHECK(hipEventCreate(&e));
    return e;
}

// Brackets one launch with events on its own stream when timing is enabled.
// The instrumented launches are idempotent (their outputs never alias their
// inputs), so with a repeat count R the launch is issued R times back to back
// between the two events and the duration is divided by R: the per-launch
// cost of recording the events is spread over R launches.
struct Timed {
    hdg_ctx *c;
    int kind, prec;
    hipStream_t s;
    hipEvent_t a = nullptr;
    double bytes;
    // sx, sy: bytes per entry of the launch's input and output trace vectors; bytes
    // (> 0): this launch's own algorithmic bytes, when they differ from the class formula
    Timed(hdg_ctx *c_, int kind_, int prec_, hipStream_t s_, int nb, int sx = 8, int sy = 8, double bytes_ = 0.0)
        : c(c_), kind(kind_), prec(prec_), s(s_), bytes(bytes_) {
        if (!c->timing) return;
        c->t_nb[prec][kind] = nb;
        c->t_sx[prec][kind] = sx;
        c->t_sy[prec][kind] = sy;
        a = pool_event(c);
        HDG_HIP_CHECK(hipEventRecord(a, s));
    }
    int repeats() const { return a ? c->timing_repeat : 1; }
    ~Timed() {
        if (!a) return;
        hipEvent_t b = pool_event(c);
        (void)hipEventRecord(b, s);
        c->pending.push_back({a, b, kind, prec, bytes});
    }
};

void collect_timing(hdg_ctx *c) {
    if (c->pending.empty()) return;
    HDG_HIP_CHECK(hipEventSynchronize(c->pending.back().b));
    for (auto &p : c->pending) {
        float ms = 0.f;
        HDG_HIP_CHECK(hipEventElapsedTime(&ms, p.a, p.b));
        c->t_ms[p.prec][p.kind] += ms / c->timing_repeat;
        c->t_launches[p.prec][p.kind] += 1;
        if (p.bytes > 0) {
            c->t_bytes[p.prec][p.kind] += p.bytes;
            c->t_blaunch[p.prec][p.kind] += 1;
        }
        c->event_pool.push_back(p.a);
        c->event_pool.push_back(p.b);
    }
    c->pending.clear();
}

// ------------------------------------------------------------------ trace-level operators
//
// Trace vectors are FP64 or, under the flags vcyc32 / vin32 / kv32 (see
// hdg_ctx), FP32 in the same buffers.  vt_call runs f with a null pointer of
// the element type selected by flag; vt2_call with two.
template <typename F>
void vt_call(bool f32, F &&f) {
    if (f32)
        f(static_cast<float *>(nullptr));
    else
        f(static_cast<double *>(nullptr));
}
template <typename F>
void vt2_call(bool a32, bool b32, F &&f) {
    vt_call(a32, [&](auto ta) { vt_call(b32, [&](auto tb) { f(ta, tb); }); });
}
template <typename VT>
const VT *vt(const double *p) { return reinterpret_cast<const VT *>(p); }
template <typename VT>
VT *vt(double *p) { return reinterpret_cast<VT *>(p); }

// y = S x (b == nullptr) or y = b - S x; x32 / y32: x, and b and y, held in FP32
void op_apply(hdg_ctx *c, int nb, int prec, const double *x, const double *b, double *y, hipStream_t s, int kind,
              bool x32 = false, bool y32 = false) {
    Timed t(c, kind, prec, s, nb, x32 ? 4 : 8, y32 ? 4 : 8);
    for (int rep = 0; rep < t.repeats(); ++rep)
        vt2_call(x32, y32, [&](auto tx, auto ty) {
            using XT = std::remove_pointer_t<decltype(tx)>;
            using YT = std::remove_pointer_t<decltype(ty)>;
            if (prec == HDG_MIXED)
                hdg::launch_trace_apply<float, XT, YT>(c->m, c->n_facet, nb, c->S32, c->nbr, vt<XT>(x), vt<YT>(b),
                                                       vt<YT>(y), s, c->rhs_block);
            else
                hdg::launch_trace_apply<double, XT, YT>(c->m, c->n_facet, nb, c->S64, c->nbr, vt<XT>(x), vt<YT>(b),
                                                        vt<YT>(y), s, c->rhs_block);
        });
    check_launch();
}
// the V-cycle's residual r - S x (work vectors)
void op_resid_v(hdg_ctx *c, int nb, int prec, const double *x, const double *r, double *y, hipStream_t s) {
    op_apply(c, nb, prec, x, r, y, s, HDG_KERNEL_RESIDUAL, c->vcyc32, c->vcyc32);
}

// damped block-Jacobi sweep y = x' + omega D^-1 (r - S x')
hdg::SweepCoef bj_coef(const hdg_ctx *c) { return {1.0 - c->opt.omega, 1.0, 1.0, 0.0, nullptr, nullptr}; }

void op_sweep(hdg_ctx *c, int nb, int prec, const double *x, const double *z0, const double *qc, double *y,
              hipStream_t s, const hdg::SweepCoef &cf) {
    // algorithmic bytes of this launch: the rows and ids once; x (own and neighbour values),
    // z0 (once, or not at all when it is x itself) and y; the P1 correction, the previous
    // iterate and its P1 correction with the facets' vertex ids when present
    const double m = c->m, ne = c->n_facet, nv = c->n_vert, sv = c->vcyc32 ? 4.0 : 8.0;
    const double st = prec == HDG_MIXED ? 2.0 : 8.0;
    double bytes = ne * (4 * m * m * st + 4 * 4) + nb * ne * m * sv * (x == z0 ? 2 : 3);
    if (qc) bytes += nb * nv * sv;
    if (cf.xprev) bytes += nb * ne * m * sv;
    if (cf.qcprev) bytes += nb * nv * sv;
    if (qc || cf.qcprev) bytes += ne * 2 * 4;
    Timed t(c, HDG_KERNEL_SWEEP, prec, s, nb, c->vcyc32 ? 4 : 8, c->vcyc32 ? 4 : 8, bytes);
    for (int rep = 0; rep < t.repeats(); ++rep)
        vt_call(c->vcyc32, [&](auto tag) {
            using VT = std::remove_pointer_t<decltype(tag)>;
            if (prec == HDG_MIXED)
                hdg::launch_sweep<__hip_bfloat16, VT>(c->m, c->n_facet, nb, c->T16, c->nbr, vt<VT>(x), vt<VT>(z0), qc,
                                                      c->facet_vert, cf, vt<VT>(y), s, c->rhs_block);
            else
                hdg::launch_sweep<double, VT>(c->m, c->n_facet, nb, c->T64, c->nbr, vt<VT>(x), vt<VT>(z0), qc,
                                              c->facet_vert, cf, vt<VT>(y), s, c->rhs_block);
        });
    check_launch();
}

// One P1 geometric-multigrid V-cycle on level l (input lev[l].b); returns the
// buffer holding the result.  Damped-Jacobi pre-smoothing (first two sweeps
// fused), residual, restriction, recursion, prolongation, post-smoothing.
// Levels small enough for the tail kernel are handled by it in one launch,
// dense coarsest solve included.  f32: the level vectors hold float values
// (inside a V-cycle whose trace vectors are FP32, the P1 vectors are too).
double *p1_vcycle(hdg_ctx *c, int l, int nb, hipStream_t s, bool f32) {
    hdg::P1LevelDev &L = c->lev[l];
    if (l == c->tail_top && (int64_t)nb * L.n <= hdg::P1_TAIL_MAX) {   // one workgroup: few values only
        hdg::launch_p1_tail(c->tail, nb, s, f32);
        return L.x;
    }
    if (l == 0) {
        hdg::launch_dense_mv(L.n, nb, c->coarse_inv, L.b, L.x, s, f32);
        return L.x;
    }
    const double w = c->opt.p1_omega;
    const int rb = c->rhs_block;
    double *x = L.x, *y = L.y;
    if (c->opt.p1_nu == 1) {
        hdg::launch_p1_first(L.n, nb, L.dinv, w, L.b, x, s, f32, rb);
    } else {
        hdg::launch_p1_pre2(L.n, L.w, nb, L.col, L.val, L.diag, L.dinv, w, L.b, x, s, f32, rb);
        for (int k = 2; k < c->opt.p1_nu; ++k) {
            hdg::launch_p1_sweep(L.n, L.w, nb, L.col, L.val, L.diag, L.dinv, w, L.b, x, nullptr, nullptr, y, s, f32,
                                 rb);
            std::swap(x, y);
        }
    }
    hdg::P1LevelDev &C = c->lev[l - 1];
    if (nb == 1) {
        hdg::launch_p1_resid_restrict(L.n, L.w, L.col, L.val, L.diag, L.b, x, C.n, L.crow, L.ccol, L.cw, C.b, s, f32);
    } else {
        hdg::launch_p1_resid(L.n, L.w, nb, L.col, L.val, L.diag, L.b, x, y, s, f32, rb);
        hdg::launch_p1_restrict(C.n, nb, L.crow, L.ccol, L.cw, y, C.b, s, f32, rb);
    }
    const double *xc = p1_vcycle(c, l - 1, nb, s, f32);
    for (int k = 0; k < c->opt.p1_nu; ++k) {
        hdg::launch_p1_sweep(L.n, L.w, nb, L.col, L.val, L.diag, L.dinv, w, L.b, x, k == 0 ? xc : nullptr,
                             L.parents, y, s, f32, rb);
        std::swap(x, y);
    }
    return x;
}

// z0 = omega D^-1 r (the first sweep from zero); with scale the input is r / scale, also written to rs
// rc (may be null): copy of the scaled input in the V-cycle's vector type.  While c->gs_lag is set
// (inside FGMRES) the input is first completed by the previous iteration's Gram-Schmidt step.
void jacobi0(hdg_ctx *c, int nb, int prec, const double *r, const double *scale, double *rs, double *rc,
             double *z0, hipStream_t s) {
    vt2_call(c->vin32, c->vcyc32, [&](auto tr, auto tz) {
        using RT = std::remove_pointer_t<decltype(tr)>;
        using ZT = std::remove_pointer_t<decltype(tz)>;
        if (prec == HDG_MIXED)
            hdg::launch_jacobi0<float, RT, ZT>(c->m, c->n_facet, nb, c->Dw32, vt<RT>(r), scale, vt<RT>(rs),
                                               vt<ZT>(rc), vt<ZT>(z0), s, c->gs_lag);
        else
            hdg::launch_jacobi0<double, RT, ZT>(c->m, c->n_facet, nb, c->Dw64, vt<RT>(r), scale, vt<RT>(rs),
                                                vt<ZT>(rc), vt<ZT>(z0), s, c->gs_lag);
    });
}
// first kernel of a V-cycle: z0 = omega D^-1 r; returns the right-hand side the cycle's
// residuals use (r itself, or its copy in the V-cycle's type when the two differ)
const double *vcycle_start(hdg_ctx *c, int nb, int prec, const double *r, const double *scale, hipStream_t s) {
    double *rs = scale ? const_cast<double *>(r) : nullptr;
    const bool copy = c->vcyc32 != c->vin32;
    jacobi0(c, nb, prec, r, scale, rs, copy ? c->vrc : nullptr, c->vz0, s);
    return copy ? c->vrc : r;
}

// pi^T of a trace residual onto the finest P1 level (upwind)
void restrict_p1(hdg_ctx *c, int nb, const double *res, double *rc, hipStream_t s) {
    vt_call(c->vcyc32, [&](auto tag) {
        using VT = std::remove_pointer_t<decltype(tag)>;
        hdg::launch_restrict_trace<VT>(c->p, c->n_vert, nb, c->vf_row, c->vf_col, vt<VT>(res), rc, s);
    });
}

// One RT0 geometric-multigrid V-cycle on level l (input rt[l].b, Lax-Friedrichs
// coarse problem); returns the buffer holding the result.  rt_nu additive
// vertex-patch steps from zero (a single one fused with the residual),
// restriction P^T, recursion, prolongation x += P x_c, rt_nu patch steps.  The
// last post-smoothing update is left pending (*pending = true): its corrections
// stay in rt_corr and the consumer of the result (the next finer level's
// prolongation, or pi) adds them as it reads.  Dense inverse on level 0.
double *rt_vcycle(hdg_ctx *c, int l, int nb, hipStream_t s, bool *pending) {
    hdg::Rt0LevelDev &L = c->rt[l];
    if (l == 0) {
        hdg::launch_dense_mv(L.ne, nb, c->rt_coarse_inv, L.b, L.x, s);
        *pending = false;
        return L.x;
    }
    const double w = c->opt.rt_omega;
    double *x = L.x;
    for (int k = 0; k < c->opt.rt_nu; ++k) {
        hdg::launch_rt_patch(L, nb, L.b, k == 0 ? nullptr : x, c->rt_corr, s);
        if (k == 0 && c->opt.rt_nu == 1) {
            // from zero the fused kernel reads no previous iterate, so it may write x in place
            hdg::launch_rt_update_resid(L, nb, w, c->rt_corr, nullptr, x, L.y, s);
        } else {
            hdg::launch_rt_update(L, nb, w, c->rt_corr, k == 0 ? nullptr : x, x, s);
            if (k + 1 == c->opt.rt_nu) hdg::launch_rt_resid(L, nb, L.b, x, L.y, s);
        }
    }
    hdg::Rt0LevelDev &C = c->rt[l - 1];
    hdg::launch_rt_restrict(L, C.ne, nb, L.y, C.b, s);
    bool cpend = false;
    const double *xc = rt_vcycle(c, l - 1, nb, s, &cpend);
    hdg::launch_rt_prolong(L, C, nb, xc, w, cpend ? c->rt_corr : nullptr, x, s);
    for (int k = 0; k < c->opt.rt_nu; ++k) {
        hdg::launch_rt_patch(L, nb, L.b, x, c->rt_corr, s);
        if (k + 1 < c->opt.rt_nu) hdg::launch_rt_update(L, nb, w, c->rt_corr, x, x, s);
    }
    *pending = true;
    return x;
}

// Lax-Friedrichs coarse correction: out = cur + pi V_RT(pi^T res)
void lf_coarse(hdg_ctx *c, int nb, const double *res, const double *cur, double *out, hipStream_t s) {
    const int L = (int)c->rt.size() - 1;
    vt_call(c->vcyc32, [&](auto tag) {
        using VT = std::remove_pointer_t<decltype(tag)>;
        hdg::launch_lf_restrict<VT>(c->m, c->n_facet, nb, c->lf_pw, c->lf_rrow, c->lf_rcol, vt<VT>(res), c->rt[L].b, s);
    });
    bool pend = false;
    const double *xr = rt_vcycle(c, L, nb, s, &pend);
    vt_call(c->vcyc32, [&](auto tag) {
        using VT = std::remove_pointer_t<decltype(tag)>;
        hdg::launch_lf_prolong<VT>(c->m, c->n_facet, nb, c->lf_pw, c->nbr, xr, c->rt[L].fs, c->opt.rt_omega,
                                   pend ? c->rt_corr : nullptr, vt<VT>(cur), vt<VT>(out), s);
    });
}

// z = V(r): Alg. twolevel_vcycle from a zero initial guess.  With scale != null
// the input is r / scale[rhs] and r is normalised in place on the way (the
// FGMRES basis vector is scaled by its first reader).
void vcycle_bj(hdg_ctx *c, int nb, int prec, const double *r, double *z, hipStream_t s,
               const double *scale = nullptr) {
    const double *rb = vcycle_start(c, nb, prec, r, scale, s);
    double *bufs[2] = {c->vx, c->vx2};
    int bi = 0;
    double *cur = c->vz0;  // first sweep from zero gives omega D^-1 r exactly
    for (int k = 1; k < c->opt.nu_pre; ++k) {
        double *out = bufs[bi];
        bi ^= 1;
        op_sweep(c, nb, prec, cur, c->vz0, nullptr, out, s, bj_coef(c));
        cur = out;
    }
    op_resid_v(c, nb, prec, cur, rb, c->vres, s);
    const double *xl = nullptr;   // P1 correction, prolonged inside the first post-sweep (upwind)
    if (c->flux == HDG_FLUX_LF) {
        double *out = cur == c->vx ? c->vx2 : c->vx;
        lf_coarse(c, nb, c->vres, cur, out, s);
        cur = out;
    } else {
        const int L = (int)c->lev.size() - 1;
        restrict_p1(c, nb, c->vres, c->lev[L].b, s);
        xl = p1_vcycle(c, L, nb, s, c->vcyc32);
    }
    for (int k = 0; k < c->opt.nu_post; ++k) {
        double *out;
        if (k == c->opt.nu_post - 1) {
            out = z;
        } else {
            out = bufs[bi];
            if (out == cur) {
                bi ^= 1;
                out = bufs[bi];
            }
            bi ^= 1;
        }
        op_sweep(c, nb, prec, cur, c->vz0, k == 0 ? xl : nullptr, out, s, bj_coef(c));
        cur = out;
    }
    check_launch();
}


// The same V-cycle with the learned smoother: every smoothing step is the
// block-Jacobi correction u = omega D^-1 (r - S x) (the sweep kernel returns
// u alone) followed by the network, x <- x + u + s MLP(patch of u).  The
// first step from zero uses u = z0 = omega D^-1 r; the prolongation
// x += pi x_P1 rides in the first post-smoothing step.
void vcycle_mlp(hdg_ctx *c, int nb, int prec, const double *r, double *z, hipStream_t s,
                const double *scale = nullptr) {
    const short *W1b = c->mlp_wb, *W2b = c->mlp_wb + c->mlp_n1;
    const double *rb = vcycle_start(c, nb, prec, r, scale, s);
    // x alternates between vx and vx2; the correction goes to vres
    double *x = c->vx, *other = c->vx2;
    auto learned = [&](const double *u, const double *xi, const double *qc, double *out) {
        Timed t(c, HDG_KERNEL_MLP, prec, s, nb, c->vcyc32 ? 4 : 8, c->vcyc32 ? 4 : 8);
        for (int rep = 0; rep < t.repeats(); ++rep)
            vt_call(c->vcyc32, [&](auto tag) {
                using VT = std::remove_pointer_t<decltype(tag)>;
                hdg::launch_mlp_smooth<VT>(c->p, c->n_facet, nb, c->mlp_spl, vt<VT>(u), vt<VT>(xi), qc, c->facet_vert,
                                           c->nbr, c->prev, W1b, W2b, vt<VT>(out), s);
            });
    };
    learned(c->vz0, nullptr, nullptr, x);
    auto step = [&](const double *qc, double *out) {
        const hdg::SweepCoef only_u{-c->opt.omega, 1.0, 1.0, 0.0, nullptr, nullptr};   // the correction alone
        op_sweep(c, nb, prec, x, c->vz0, qc, c->vres, s, only_u);
        learned(c->vres, x, qc, out);
        if (out != z) {
            other = x;
            x = out;
        }
    };
    for (int k = 1; k < c->opt.nu_pre; ++k) step(nullptr, other);
    op_resid_v(c, nb, prec, x, rb, c->vres, s);
    const int L = (int)c->lev.size() - 1;
    restrict_p1(c, nb, c->vres, c->lev[L].b, s);
    const double *xl = p1_vcycle(c, L, nb, s, c->vcyc32);
    for (int k = 0; k < c->opt.nu_post; ++k) step(k == 0 ? xl : nullptr, k == c->opt.nu_post - 1 ? z : other);
    check_launch();
}

// The V-cycle with Chebyshev smoothing of degree nu (pre and post), block-
// Jacobi preconditioned, on the interval [0.1, 1.1] lambda_max(D^-1 S):
// x_1 = x_0 + D^-1 (r - S x_0) / theta, then
// x_{k+1} = x_k + c1 (x_k - x_{k-1}) + c2 D^-1 (r - S x_k),
// c1 = rho_k rho_{k-1}, c2 = 2 rho_k / delta, rho_k = 1 / (2 sigma - rho_{k-1}),
// rho_0 = 1 / sigma, sigma = theta / delta.  Every step is one generalised
// sweep.  From a zero iterate x_1 = z0 / (theta omega) is never stored: the
// next sweep reads z0 with the factor folded into its coefficients.
void vcycle_cheb(hdg_ctx *c, int nb, int prec, const double *r, double *z, hipStream_t s,
                 const double *scale = nullptr) {
    const double *rb = vcycle_start(c, nb, prec, r, scale, s);
    const double w = c->opt.omega, lo = 0.1 * c->cheb_lmax, hi = 1.1 * c->cheb_lmax;
    const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
    struct Ref {
        const double *p;
        double sc;
        const double *qc;
    };
    auto spare = [&](const Ref &x, const Ref &xp) -> double * {
        // overwrite the previous iterate in place when it is a work buffer (each thread reads
        // it at its own facet only), else take the work buffer x does not occupy
        if (xp.p == c->vx || xp.p == c->vx2) return const_cast<double *>(xp.p);
        return x.p == c->vx ? c->vx2 : c->vx;
    };
    // pre-smoothing from zero
    Ref x{c->vz0, 1.0 / (theta * w), nullptr}, xp{nullptr, 0.0, nullptr};
    double rho = 1.0 / sigma;
    for (int k = 1; k < c->opt.nu_pre; ++k) {
        const double rn = 1.0 / (2.0 * sigma - rho), c1 = rn * rho, c2 = 2.0 * rn / delta;
        const hdg::SweepCoef cf{(1.0 + c1 - c2) * x.sc, c2 / w, c2 / w * x.sc, xp.p ? -c1 * xp.sc : 0.0, xp.p,
                                nullptr};
        double *out = spare(x, xp);
        op_sweep(c, nb, prec, x.p, c->vz0, nullptr, out, s, cf);
        xp = x;
        x = Ref{out, 1.0, nullptr};
        rho = rn;
    }
    const int64_t n = (int64_t)c->n_facet * c->m * nb;
    if (x.sc != 1.0) {
        vt_call(c->vcyc32, [&](auto tag) {
            using VT = std::remove_pointer_t<decltype(tag)>;
            hdg::launch_lin3<VT>(n, x.sc, vt<VT>(x.p), 0.0, nullptr, 0.0, nullptr, vt<VT>(c->vx), s);
        });
        x = Ref{c->vx, 1.0, nullptr};
    }
    op_resid_v(c, nb, prec, x.p, rb, c->vres, s);
    if (c->flux == HDG_FLUX_LF) {
        // post-smoothing from x + pi x_RT, formed in a work buffer
        double *out = x.p == c->vx ? c->vx2 : c->vx;
        lf_coarse(c, nb, c->vres, x.p, out, s);
        x = Ref{out, 1.0, nullptr};
    } else {
        // post-smoothing from x + pi x_P1 (the prolongation rides in the sweeps)
        const int L = (int)c->lev.size() - 1;
        restrict_p1(c, nb, c->vres, c->lev[L].b, s);
        x.qc = p1_vcycle(c, L, nb, s, c->vcyc32);
    }
    xp = Ref{nullptr, 0.0, nullptr};
    rho = 1.0 / sigma;
    for (int k = 0; k < c->opt.nu_post; ++k) {
        hdg::SweepCoef cf;
        if (k == 0) {
            cf = {1.0 - 1.0 / theta, 1.0 / (theta * w), 1.0 / (theta * w), 0.0, nullptr, nullptr};
        } else {
            const double rn = 1.0 / (2.0 * sigma - rho), c1 = rn * rho, c2 = 2.0 * rn / delta;
            cf = {1.0 + c1 - c2, c2 / w, c2 / w, -c1, xp.p, xp.qc};
            rho = rn;
        }
        double *out = (k == c->opt.nu_post - 1) ? z : spare(x, xp);
        op_sweep(c, nb, prec, x.p, c->vz0, x.qc, out, s, cf);
        xp = x;
        x = Ref{out, 1.0, nullptr};
    }
    check_launch();
}

void vcycle(hdg_ctx *c, int nb, int prec, const double *r, double *z, hipStream_t s,
            const double *scale = nullptr) {
    if (c->use_mlp_now)
        vcycle_mlp(c, nb, prec, r, z, s, scale);
    else if (c->opt.smoother == HDG_SMOOTH_CHEBYSHEV)
        vcycle_cheb(c, nb, prec, r, z, s, scale);
    else
        vcycle_bj(c, nb, prec, r, z, s, scale);
}

// ------------------------------------------------------------------ reductions and Krylov

enum { SC_RR = 0, SC_RZ0, SC_RZ1, SC_PW, SC_BETA, SC_RES, SC_HN2, SC_HN, SC_BN2, SC_COUNT };

double *scal(hdg_ctx *c, int slot) { return c->scal + (size_t)slot * c->opt.max_rhs; }
int64_t vec_len(const hdg_ctx *c) { return (int64_t)c->n_facet * c->m; }

// out (device, may be null) and host (host-mapped, may be null) receive the dots
void dots(hdg_ctx *c, int nb, int nd, const double *X, int64_t xstride, const double *y, double *out,
          hipStream_t s, double *host = nullptr) {
    vt_call(c->kv32, [&](auto tag) {
        using VT = std::remove_pointer_t<decltype(tag)>;
        hdg::launch_dots<VT>(vec_len(c), nb, nd, vt<VT>(X), xstride, vt<VT>(y), c->red, out, host, s);
    });
    check_launch();
}

// Reduction results the host needs are written by the kernels straight into
// host-mapped memory (slots of 64 doubles in c->hlag, device view c->dlag):
// no copy kernel is queued.  mark_lag() records when slot's values are final;
// wait_lag() blocks until then.  The Krylov loops look at iteration j's
// residual while iteration j+1 is already queued, so the GPU does not idle.
double *lag_dev(hdg_ctx *c, int slot) { return c->dlag + 64 * slot; }
void mark_lag(hdg_ctx *c, int slot, hipStream_t s) { HDG_HIP_CHECK(hipEventRecord(c->lag_ev[slot], s)); }
const double *wait_lag(hdg_ctx *c, int slot) {
    HDG_HIP_CHECK(hipEventSynchronize(c->lag_ev[slot]));
    return c->hlag + 64 * slot;
}

// Blocking: dots of a single pair written to host slot 2.
const double *dots_now(hdg_ctx *c, int nb, const double *x, const double *y, double *out, hipStream_t s) {
    dots(c, nb, 1, x, 0, y, out, s, lag_dev(c, 2));
    HDG_HIP_CHECK(hipStreamSynchronize(s));
    return c->hlag + 64 * 2;
}

void fill_info(hdg_solve_info *info, int nb, int its, int refinements, const std::vector<double> &rel,
               int status) {
    if (!info) return;
    for (int r = 0; r < nb; ++r) {
        info[r].iters = its;
        info[r].refinements = refinements;
        info[r].fallbacks = 0;
        info[r].status = status;
        info[r].rel_res = rel[r];
    }
}

bool all_below(const std::vector<double> &v, double tol) {
    for (double x : v)
        if (!(x <= tol)) return false;
    return true;
}

bool any_nonfinite(const std::vector<double> &v) {
    for (double x : v)
        if (!std::isfinite(x)) return true;
    return false;
}

// rel[r] = ||rhat - S lam|| / ||rhat|| with the FP64 operator; the residual stays in out.
// the true residual rhat - S lam with the FP64 operator, and its norm relative to ||rhat||;
// out32: stored as FP32 (rounded once, straight into the FP32 inner solve's first basis slot)
// and its norm taken from that FP32 vector
void true_residual(hdg_ctx *c, int nb, const double *rhat, const double *lam, double *out,
                   std::vector<double> &rel, hipStream_t s, bool out32 = false) {
    const double *h;
    if (out32) {
        const double m = c->m, ne = c->n_facet;
        Timed t(c, HDG_KERNEL_RESIDUAL, HDG_FP64, s, nb, 8, 4, ne * (5 * m * m * 8 + 16) + nb * ne * m * (8 + 8 + 4));
        for (int rep = 0; rep < t.repeats(); ++rep)
            hdg::launch_trace_residual_f32(c->m, c->n_facet, nb, c->S64, c->nbr, lam, rhat,
                                           reinterpret_cast<float *>(out), s, c->rhs_block);
        check_launch();
        hdg::launch_dots<float>(vec_len(c), nb, 1, reinterpret_cast<const float *>(out), 0,
                                reinterpret_cast<const float *>(out), c->red, scal(c, SC_RR), lag_dev(c, 2), s);
        check_launch();
        HDG_HIP_CHECK(hipStreamSynchronize(s));
        h = c->hlag + 64 * 2;
    } else {
        op_apply(c, nb, HDG_FP64, lam, rhat, out, s, HDG_KERNEL_RESIDUAL);
        h = dots_now(c, nb, out, out, scal(c, SC_RR), s);
    }
    for (int r = 0; r < nb; ++r) {
        const double bn2 = c->hbn2[r];
        rel[r] = bn2 > 0 ? std::sqrt(h[r] / bn2) : std::sqrt(h[r]);
    }
}

// Preconditioned CG (f = 0 and FP64: S symmetric positive definite, the
// V-cycle a fixed symmetric linear operator).  Convergence is judged on the
// recurrence residual, one iteration late, and confirmed on the true
// residual; PCG restarts from the true residual when the two disagree.
int solve_pcg(hdg_ctx *c, int nb, const double *rhat, double *lam_user, hdg_solve_info *info, hipStream_t s) {
    const int64_t n = vec_len(c);
    const double rtol = c->opt.rtol;
    std::vector<double> rel(nb, 0.0);
    int its = 0, restarts = 0;
    // iterate on a context-owned copy of lam so captured iterations never refer to caller memory
    double *lam = c->klam;
    hdg::launch_copy(n * nb, lam_user, lam, s);
    double *rzb[2] = {scal(c, SC_RZ0), scal(c, SC_RZ1)};
    auto finish = [&](int status) {
        hdg::launch_copy(n * nb, lam, lam_user, s);
        fill_info(info, nb, its, restarts, rel, status);
        return status;
    };
    while (true) {
        true_residual(c, nb, rhat, lam, c->kr, rel, s);
        if (any_nonfinite(rel)) return finish(HDG_EBREAKDOWN);
        if (all_below(rel, rtol)) return finish(HDG_OK);
        if (its >= c->opt.maxit) return finish(HDG_ENOTCONV);
        ++restarts;
        vcycle(c, nb, HDG_FP64, c->kr, c->kz, s);
        dots(c, nb, 1, c->kr, 0, c->kz, rzb[its & 1], s);
        hdg::launch_copy(n * nb, c->kz, c->kp, s);
        int pending = -1;
        while (its < c->opt.maxit) {
            const int slot = its & 1;
            // one iteration: w = S p, alpha = rz / (p.w), lam += alpha p, r -= alpha w, ||r||^2 -> slot,
            // z = V(r), rzn = r.z, p = z + (rzn / rz) p;  rz and rzn swap roles every iteration
            double *a = rzb[slot], *b = rzb[slot ^ 1];
            run_step(c, graph_key(1, nb, HDG_FP64, slot), s, [&](hipStream_t st) {
                op_apply(c, nb, HDG_FP64, c->kp, nullptr, c->kw, st, HDG_KERNEL_APPLY);
                dots(c, nb, 1, c->kp, 0, c->kw, scal(c, SC_PW), st);
                hdg::launch_pcg_update_norm(n, nb, a, scal(c, SC_PW), c->kp, c->kw, lam, c->kr, c->red,
                                            lag_dev(c, slot), st);
                vcycle(c, nb, HDG_FP64, c->kr, c->kz, st);
                dots(c, nb, 1, c->kr, 0, c->kz, b, st);
                hdg::launch_pcg_dir(n, nb, b, a, c->kz, c->kp, st);
                check_launch();
            });
            mark_lag(c, slot, s);
            ++its;
            if (pending >= 0) {
                const double *h = wait_lag(c, pending);
                bool done = true, bad = false;
                for (int r = 0; r < nb; ++r) {
                    if (!std::isfinite(h[r])) bad = true;
                    if (!(h[r] <= rtol * rtol * c->hbn2[r])) done = false;
                }
                if (bad || done) break;
            }
            pending = slot;
        }
    }
}

// Flexible GMRES, right preconditioned, classical Gram-Schmidt.  Every
// restart recomputes the residual with the FP64 operator.  With inner ==
// HDG_MIXED the Arnoldi process applies the FP32 operator and the
// mixed-precision V-cycle, and a cycle ends once it has reduced its own
// starting residual by inner_eta: the restarts are then FP64 iterative
// refinement around a reduced-precision inner solve.  The residual estimate
// of column j is examined while column j+1 is already queued.
int solve_fgmres(hdg_ctx *c, int nb, int vc_prec, int op_prec, double inner_eta, const double *rhat,
                 double *lam, hdg_solve_info *info, hipStream_t s) {
    const int64_t n = vec_len(c);
    const int64_t vs = n * c->opt.max_rhs;   // basis slot, in doubles
    const int R = c->opt.restart;
    const double rtol = c->opt.rtol;
    // the inner solve of HDG_MIXED_IR (FP32 operator and V-cycle) keeps its basis and the
    // V-cycle's vectors in FP32: half the vector traffic; lam and the true residual stay FP64
    const bool f32 = vc_prec == HDG_MIXED && op_prec == HDG_MIXED;
    // any solve with the mixed V-cycle keeps the V-cycle's vectors and the Z basis in FP32
    const bool z32 = vc_prec == HDG_MIXED;
    struct Vec32Off {   // FP64 vectors again (and no pending Gram-Schmidt step) when the solve returns or throws
        hdg_ctx *c;
        ~Vec32Off() {
            c->vcyc32 = c->vin32 = c->kv32 = false;
            c->gs_lag = hdg::GsLag{};
        }
    } vec32_off{c};
    auto set32 = [&](bool on) {
        c->vcyc32 = on && z32;
        c->vin32 = c->kv32 = on && f32;
    };
    const int64_t vstride = f32 ? 2 * vs : vs;   // V basis stride in elements of its type
    std::vector<double> rel(nb, 0.0), cyc0(nb, 0.0);
    int its = 0, cycles = 0, fallbacks = 0;
    auto done_info = [&](int status) {
        set32(false);
        fill_info(info, nb, its, cycles, rel, status);
        if (info)
            for (int r = 0; r < nb; ++r) info[r].fallbacks = fallbacks;
        return status;
    };
    while (true) {
        set32(false);
        true_residual(c, nb, rhat, lam, c->kV, rel, s, f32);
        if (any_nonfinite(rel)) return done_info(HDG_EBREAKDOWN);
        if (all_below(rel, rtol)) return done_info(HDG_OK);
        if (its >= c->opt.maxit) return done_info(HDG_ENOTCONV);
        ++cycles;
        cyc0 = rel;
        set32(true);
        hdg::launch_gmres_start(nb, R, scal(c, SC_RR), c->gm, scal(c, SC_BETA), s);
        int k = 0, pending = -1;
        auto converged = [&](const double *h) {
            for (int r = 0; r < nb; ++r) {
                if (!std::isfinite(h[r])) return true;   // stop the cycle; the true residual reports it
                if (!(h[r] <= std::max(rtol, inner_eta * cyc0[r]))) return false;
            }
            return true;
        };
        for (int j = 0; j < R && its < c->opt.maxit; ++j) {
            double *Vj = c->kV + (size_t)j * vs, *Vn = c->kV + (size_t)(j + 1) * vs;
            double *Zj = c->kZ + (size_t)j * vs;
            const int slot = j & 1;
            // V_j still carries its norm (beta for j = 0, the previous step's norm after);
            // the V-cycle's first kernel divides it out in place.
            // The FP32 inner solve of HDG_MIXED_IR makes one pass over the basis per
            // iteration (classical Gram-Schmidt with the update and the normalisation
            // lagged): with w = S z_j it takes the dot products with V_0..V_j and with w
            // itself in the same pass, the norm of w - sum h_d V_d from them
            // (||w||^2 - sum h_d^2, exact for an orthonormal basis), and leaves the update to
            // the next V-cycle's first kernel, which reads V_{j+1} anyway and so completes
            // and normalises it in place.  Where that norm would lose too much to rounding
            // (the remaining part of w below 1 % of w), the explicit update pass runs
            // instead, on the device's own decision (c->gs_explicit), and the next V-cycle
            // skips the lagged step.  The FP64 bases, which must reach the full tolerance in
            // one cycle, keep the explicit update and norm: there the basis' loss of
            // orthogonality over a long cycle makes the lagged norm unreliable (measured:
            // 30-44 iterations instead of 11-12 on some workloads).
            const double *vscale = (j == 0) ? scal(c, SC_BETA) : scal(c, SC_HN);
            const bool one_pass = f32;
            c->gs_lag = (j == 0 || !one_pass) ? hdg::GsLag{} : hdg::GsLag{c->kV, vstride, j, c->hcol, c->gs_explicit};
            run_step(c, graph_key(2 + (c->use_mlp_now ? 1 : 0), nb, vc_prec * 4 + op_prec, j), s, [&](hipStream_t st) {
                vcycle(c, nb, vc_prec, Vj, Zj, st, vscale);
                op_apply(c, nb, op_prec, Zj, nullptr, Vn, st, HDG_KERNEL_APPLY, c->vcyc32, c->kv32);
                dots(c, nb, one_pass ? j + 2 : j + 1, c->kV, vstride, Vn, c->hcol, st);
                if (one_pass)
                    hdg::launch_pyth_givens(nb, j, R, 1e-2, c->hcol, scal(c, SC_HN), c->gm, c->dbn, lag_dev(c, slot),
                                            c->gs_explicit, st);
                vt_call(c->kv32, [&](auto tag) {
                    using VT = std::remove_pointer_t<decltype(tag)>;
                    hdg::launch_gs_norm_givens<VT>(n, nb, j + 1, c->hcol, vt<VT>(c->kV), vstride, vt<VT>(Vn), c->red,
                                                   scal(c, SC_HN), j, R, c->gm, c->dbn, lag_dev(c, slot), st,
                                                   one_pass ? c->gs_explicit : nullptr);
                });
                check_launch();
            });
            c->gs_lag = hdg::GsLag{};
            mark_lag(c, slot, s);
            ++its;
            k = j + 1;
            if (pending >= 0) {
                const double *h = wait_lag(c, pending);
                if (converged(h)) {
                    k = j;   // column j was queued speculatively; the solution uses columns 0..j-1
                    pending = -1;
                    break;
                }
                // learned smoother judged by the mean residual reduction per iteration over
                // this restart cycle (h holds the estimate after j iterations); block-Jacobi
                // takes over for the rest of the solve when it is too weak
                if (c->use_mlp_now && j >= 2) {
                    for (int r = 0; r < nb; ++r)
                        if (cyc0[r] > 0 && std::pow(h[r] / cyc0[r], 1.0 / j) > c->opt.fallback_ratio) {
                            c->use_mlp_now = false;
                            ++fallbacks;
                            break;
                        }
                }
            }
            pending = slot;
        }
        hdg::launch_gmres_solve(nb, k, R, c->gm, c->hy, s);
        vt_call(c->vcyc32, [&](auto tag) {
            using VT = std::remove_pointer_t<decltype(tag)>;
            hdg::launch_lincomb<VT>(n, nb, k, c->hy, vt<VT>(c->kZ), c->vcyc32 ? 2 * vs : vs, lam, s);
        });
        check_launch();
    }
}

// ------------------------------------------------------------------ persistent single-launch solve

// Krylov method of a solve: PCG when the operator and the preconditioner are symmetric
int krylov_kind(const hdg_ctx *c) {
    int kry = c->opt.krylov;
    if (kry == HDG_KRYLOV_AUTO)
        kry = (c->symmetric && c->opt.precision == HDG_FP64 && c->opt.smoother != HDG_SMOOTH_MLP &&
               c->opt.nu_pre == c->opt.nu_post) ? HDG_KRYLOV_PCG : HDG_KRYLOV_FGMRES;
    return kry;
}

bool use_small(const hdg_ctx *c, int kry) {
    return c->small_ok && c->opt.precision == HDG_FP64 && c->opt.smoother == HDG_SMOOTH_BJACOBI &&
           (kry == HDG_KRYLOV_PCG || c->opt.restart <= hdg::SMALL_MAXR);
}

// One launch, one workgroup per right-hand side: the Krylov solve (stage: with
// the condensation before and the recovery after it).  Fills info and returns
// the worst status over the right-hand sides.  Synchronises the stream.
int solve_small(hdg_ctx *c, int nb, int kry, bool stage, const double *rhat, const double *r_cell, double *lam,
                double *q_cell, hdg_solve_info *info, hipStream_t s) {
    hdg::SmallArgs A{};
    A.ne = c->n_facet;
    A.m = c->m;
    A.nk = c->n_cell;
    A.nb = nb;
    A.nlev = (int)c->lev.size();
    A.stage_ops = c->small_stage_ops ? 1 : 0;
    A.image = c->small_image;
    A.p1B = c->small_p1B;
    A.krylov = kry;
    A.restart = c->opt.restart;
    A.maxit = c->opt.maxit;
    A.nu_pre = c->opt.nu_pre;
    A.nu_post = c->opt.nu_post;
    A.p1_nu = c->opt.p1_nu;
    A.omega = c->opt.omega;
    A.p1_omega = c->opt.p1_omega;
    A.rtol = c->opt.rtol;
    A.S = c->S64;
    A.T = c->T64;
    A.Dw = c->Dw64;
    A.nbr = c->nbr;
    A.fvert = c->facet_vert;
    A.vf_row = c->vf_row;
    A.vf_col = c->vf_col;
    for (int l = 0; l < A.nlev; ++l) {
        const hdg::P1LevelDev &L = c->lev[l];
        A.lev[l] = hdg::P1Lev{L.n, L.w, L.col, L.val, L.diag, L.dinv, L.parents, L.crow, L.ccol, L.cw,
                              nullptr, nullptr, nullptr};
    }
    A.Ainv = c->coarse_inv;
    A.Zr = c->Zr;
    A.Ar = c->Ar;
    A.Wr = c->Wr;
    A.fcell = c->d_fcell;
    A.floc = c->d_floc;
    A.cell_facet = c->cell_facet;
    A.cell_rev = c->cell_rev;
    A.r_cell = r_cell;
    A.q_cell = q_cell;
    A.rhat = rhat;
    A.lam = lam;
    A.V = c->small_V;
    A.Z = c->small_Z;
    A.info = c->small_info;
    // each workgroup writes its record's status last (after a system-scope fence):
    // wait for those instead of for the stream, which reports the end of the
    // launch a few microseconds later; bounded, then the stream decides
    volatile double *rec = c->small_hinfo;
    constexpr double pending = 1e300;
    for (int r = 0; r < nb; ++r) rec[4 * r + 2] = pending;
    hdg::launch_solve_small(c->p, stage, A, c->small_lds, s);
    check_launch();
    {
        const auto t0 = std::chrono::steady_clock::now();
        int r = 0;
        while (r < nb) {
            if (rec[4 * r + 2] != pending) {
                ++r;
            } else if (std::chrono::steady_clock::now() - t0 > std::chrono::seconds(2)) {
                break;
            }
        }
        if (r < nb) HDG_HIP_CHECK(hipStreamSynchronize(s));
    }
    int status = HDG_OK;
    for (int r = 0; r < nb; ++r) {
        const volatile double *h = c->small_hinfo + 4 * r;
        const int st = (int)h[2];
        if (st == HDG_EBREAKDOWN) status = HDG_EBREAKDOWN;
        else if (st == HDG_ENOTCONV && status == HDG_OK) status = HDG_ENOTCONV;
        if (info) {
            info[r].iters = (int)h[0];
            info[r].refinements = (int)h[1];
            info[r].fallbacks = 0;
            info[r].status = st;
            info[r].rel_res = h[3];
        }
    }
    return status;
}

// trace vectors are read and written as 16-byte pairs at nrhs = 1
void check_aligned(const void *p, const char *what) {
    if (reinterpret_cast<uintptr_t>(p) % 16 != 0)
        throw Error{HDG_EINVAL, std::string(what) + " must be 16-byte aligned"};
}

void check_nb(const hdg_ctx *c, int nb) {
    HDG_REQUIRE(nb >= 1 && nb <= c->opt.max_rhs, "nrhs must be in 1..max_rhs");
}

void check_prec(int prec) { HDG_REQUIRE(prec == HDG_FP64 || prec == HDG_MIXED, "precision must be HDG_FP64 or HDG_MIXED"); }

// ------------------------------------------------------------------ setup

void validate_mesh(const hdg_mesh &m) {
    HDG_REQUIRE(m.geom == HDG_TORUS || m.geom == HDG_SPHERE, "geom must be HDG_TORUS or HDG_SPHERE");
    HDG_REQUIRE(m.n_vert >= 1 && m.n_cell >= 2, "mesh needs at least one vertex and two cells");
    HDG_REQUIRE(m.vert_xyz && m.cell_vert, "mesh arrays must not be NULL");
    HDG_REQUIRE(m.geom == HDG_SPHERE || m.period > 0, "torus period must be positive");
}

// Largest eigenvalue of D^-1 S for the Chebyshev interval: 20 power steps
// v <- D^-1 S v / ||D^-1 S v|| (FP64) from the fixed start vector
// v_i = frac(i * 2654435761 / 2^32) - 1/2, estimate ||D^-1 S v||.
void estimate_lambda_max(hdg_ctx *c) {
    const int64_t n = vec_len(c);
    std::vector<double> v(n);
    double nrm = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const uint64_t h = ((uint64_t)i * 2654435761ull) % 4294967296ull;
        v[i] = (double)h / 4294967296.0 - 0.5;
        nrm += v[i] * v[i];
    }
    nrm = std::sqrt(nrm);
    for (auto &x : v) x /= nrm;
    hipStream_t s = nullptr;
    HDG_HIP_CHECK(hipMemcpy(c->vx, v.data(), n * sizeof(double), hipMemcpyHostToDevice));
    double lam = 0.0;
    for (int it = 0; it < 20; ++it) {
        op_apply(c, 1, HDG_FP64, c->vx, nullptr, c->vres, s, HDG_KERNEL_APPLY);
        jacobi0(c, 1, HDG_FP64, c->vres, nullptr, nullptr, nullptr, c->vx2, s);   // omega D^-1 S v
        const double *h = dots_now(c, 1, c->vx2, c->vx2, scal(c, SC_RR), s);
        lam = std::sqrt(h[0]) / c->opt.omega;
        HDG_REQUIRE(std::isfinite(lam) && lam > 0, "eigenvalue estimate of D^-1 S failed");
        hdg::launch_lin3<double>(n, 1.0 / (lam * c->opt.omega), c->vx2, 0.0, nullptr, 0.0, nullptr, c->vx, s);
        check_launch();
    }
    HDG_HIP_CHECK(hipStreamSynchronize(s));
    c->cheb_lmax = lam;
}

void setup_impl(const hdg_mesh *levels, int nlev, const int32_t *const *parents, const hdg_params *prm,
                const hdg_options *opt_in, hdg_ctx *c) {
    HDG_REQUIRE(levels && prm && nlev >= 1, "levels, prm must be given and n_levels >= 1");
    HDG_REQUIRE(prm->degree >= 1 && prm->degree <= 3, "degree must be 1, 2 or 3");
    HDG_REQUIRE(prm->dt > 0 && prm->g > 0 && prm->H > 0 && prm->tau > 0, "dt, g, H, tau must be positive");
    hdg_options opt;
    hdg_default_options(&opt);
    if (opt_in) opt = *opt_in;
    HDG_REQUIRE(opt.max_rhs >= 1 && opt.max_rhs <= 64, "max_rhs must be in 1..64");
    HDG_REQUIRE(opt.restart >= 1 && opt.restart <= 64, "restart must be in 1..64");
    HDG_REQUIRE(opt.nu_pre >= 1 && opt.nu_post >= 1 && opt.p1_nu >= 1, "sweep counts must be >= 1");
    HDG_REQUIRE(opt.omega > 0 && opt.p1_omega > 0, "damping factors must be positive");
    HDG_REQUIRE(opt.rtol >= 0 && opt.maxit >= 1, "rtol >= 0 and maxit >= 1 required");
    HDG_REQUIRE(opt.ir_inner_rtol > 0 && opt.ir_inner_rtol < 1, "ir_inner_rtol must be in (0, 1)");
    HDG_REQUIRE(opt.p1_tail_max >= 0 && opt.p1_tail_max <= hdg::P1_TAIL_MAX, "p1_tail_max must be in 0..4096");
    HDG_REQUIRE(opt.smoother >= HDG_SMOOTH_BJACOBI && opt.smoother <= HDG_SMOOTH_CHEBYSHEV, "unknown smoother");
    HDG_REQUIRE(opt.p1_galerkin == 0 || opt.p1_galerkin == 1, "p1_galerkin must be 0 or 1");
    HDG_REQUIRE(opt.krylov >= HDG_KRYLOV_AUTO && opt.krylov <= HDG_KRYLOV_FGMRES, "unknown krylov method");
    HDG_REQUIRE(opt.persistent == 0 || opt.persistent == 1, "persistent must be 0 or 1");
    for (int l = 0; l < nlev; ++l) validate_mesh(levels[l]);
    const hdg_mesh &fine = levels[nlev - 1];
    HDG_REQUIRE(prm->flux == HDG_FLUX_UPWIND || prm->flux == HDG_FLUX_LF, "flux must be HDG_FLUX_UPWIND or HDG_FLUX_LF");
    const bool lf = prm->flux == HDG_FLUX_LF;
    if (lf) {
        HDG_REQUIRE(fine.geom == HDG_TORUS, "the Lax-Friedrichs flux is built on the torus only");
        HDG_REQUIRE(opt.smoother != HDG_SMOOTH_MLP, "the learned smoother is built for the upwind flux only");
        HDG_REQUIRE(opt.p1_galerkin == 0, "p1_galerkin applies to the upwind flux only");
        HDG_REQUIRE(opt.rt_nu >= 1 && opt.rt_omega > 0, "rt_nu >= 1 and rt_omega > 0 required");
    }

    HDG_HIP_CHECK(hipGetDevice(&c->device));
    c->noalloc_scratch = scratch_on(c->device);
    c->prm = *prm;
    c->opt = opt;
    c->p = prm->degree;
    c->flux = prm->flux;
    c->nu = lf ? 2 : 1;
    c->m = c->nu * (c->p + 1);
    c->n = (c->p + 1) * (c->p + 2) / 2;
    c->nc = 3 * c->n;
    c->nt = 3 * c->m;
    c->geom = fine.geom;
    c->tau = prm->tau;
    c->dt = prm->dt;
    c->kappa = std::sqrt(prm->g * prm->H) * prm->dt;
    c->hscale = std::sqrt(prm->g / prm->H);
    c->symmetric = (fine.geom == HDG_TORUS ? prm->f0 == 0.0 : (prm->f0 == 0.0 && prm->omega == 0.0));

    // ---- topology (host)
    c->topo = hdg::build_topology(fine);
    const int nk = fine.n_cell, ne = c->topo.n_facet, nv = fine.n_vert;
    c->n_cell = nk;
    c->n_facet = ne;
    c->n_vert = nv;
    hipStream_t s = nullptr;

    // ---- per-cell assembly and condensation (device)
    std::vector<double> corners = hdg::cell_corners(fine);
    double *d_corners = dev_upload(c, corners);
    hdg::RefTables R = hdg::build_ref_tables(c->p);
    std::vector<double> ref;
    for (auto *v : {&R.M, &R.G, &R.E, &R.T, &R.F, &R.qx, &R.qw, &R.Phi}) ref.insert(ref.end(), v->begin(), v->end());
    double *d_ref = dev_upload(c, ref);
    c->ref = d_ref;
    int *d_err = dev_alloc<int>(c, 1);
    HDG_HIP_CHECK(hipMemset(d_err, 0, sizeof(int)));
    double *Sloc = dev_alloc<double>(c, (size_t)c->nt * c->nt * nk);
    c->Zr = dev_alloc<double>(c, (size_t)c->nt * hdg::cell_zw(c->p) * nk);
    c->Ar = dev_alloc<double>(c, (size_t)c->nc * c->nc * nk);
    c->Wr = dev_alloc<double>(c, (size_t)c->nc * c->nt * nk);
    hdg::CellParams cp{c->kappa, c->tau, c->dt, prm->f0, prm->omega, c->hscale, fine.geom};
    hdg::launch_cell_condense(c->p, c->nu, nk, d_corners, d_ref, cp, Sloc, c->Zr, c->Ar, c->Wr, d_err, s, nullptr,
                              nullptr);
    check_launch();
    HDG_HIP_CHECK(hipDeviceSynchronize());
    int herr = 0;
    HDG_HIP_CHECK(hipMemcpy(&herr, d_err, sizeof(int), hipMemcpyDeviceToHost));
    if (herr & 1) throw Error{HDG_EINVAL, "a cell has non-positive area (cells must be counter-clockwise)"};
    if (herr & 2) throw Error{HDG_EINVAL, "singular local cell matrix A_K"};

    // ---- facet block rows (device)
    std::vector<int32_t> cf_t((size_t)3 * nk);
    std::vector<int8_t> cr_t((size_t)3 * nk);
    for (int K = 0; K < nk; ++K)
        for (int i = 0; i < 3; ++i) {
            cf_t[(size_t)i * nk + K] = c->topo.cell_facet[3 * K + i];
            cr_t[(size_t)i * nk + K] = c->topo.cell_rev[3 * K + i];
        }
    c->cell_facet = dev_upload(c, cf_t);
    c->cell_rev = dev_upload(c, cr_t);
    int32_t *d_fcell = dev_upload(c, c->topo.facet_cell);
    int32_t *d_floc = dev_upload(c, c->topo.facet_loc);
    c->facet_vert = dev_upload(c, c->topo.facet_vert);
    const int m = c->m;
    c->nbr = dev_alloc<int32_t>(c, (size_t)4 * ne);
    c->prev = dev_alloc<int8_t>(c, (size_t)4 * ne);
    c->S64 = dev_alloc<double>(c, (size_t)hdg::wide_padded(5 * m * m, 2) * ne);
    c->T64 = dev_alloc<double>(c, (size_t)hdg::wide_padded(4 * m * m, 2) * ne);
    c->Dw64 = dev_alloc<double>(c, (size_t)hdg::wide_padded(m * m, 2) * ne);
    c->S32 = dev_alloc<float>(c, (size_t)hdg::wide_padded(5 * m * m, 4) * ne);
    c->T16 = dev_alloc<__hip_bfloat16>(c, (size_t)hdg::wide_padded(4 * m * m, 8) * ne);
    c->Dw32 = dev_alloc<float>(c, (size_t)hdg::wide_padded(m * m, 4) * ne);
    hdg::launch_facet_rows(c->p, c->nu, ne, nk, Sloc, d_fcell, d_floc, c->cell_facet, c->cell_rev, opt.omega, c->S64,
                           c->T64, c->Dw64, c->S32, c->T16, c->Dw32, c->nbr, c->prev, d_err, s);
    check_launch();
    HDG_HIP_CHECK(hipDeviceSynchronize());
    HDG_HIP_CHECK(hipMemcpy(&herr, d_err, sizeof(int), hipMemcpyDeviceToHost));
    if (herr & 4) throw Error{HDG_EINVAL, "singular facet diagonal block"};
    c->d_fcell = d_fcell;
    c->d_floc = d_floc;
    dev_release(c, Sloc, (size_t)c->nt * c->nt * nk * sizeof(double));
    c->corners = d_corners;   // kept for the explicit flux evaluation (hdg_dg_tendency)

    // ---- vertex -> facet-end CSR for the trace -> P1 restriction
    if (!lf) {
        std::vector<int32_t> cnt(nv + 1, 0);
        for (int e = 0; e < ne; ++e) {
            cnt[c->topo.facet_vert[2 * e] + 1]++;
            cnt[c->topo.facet_vert[2 * e + 1] + 1]++;
        }
        for (int v = 0; v < nv; ++v) cnt[v + 1] += cnt[v];
        std::vector<int32_t> col(cnt[nv]);
        std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
        for (int e = 0; e < ne; ++e)
            for (int end = 0; end < 2; ++end) col[fill[c->topo.facet_vert[2 * e + end]]++] = 2 * e + end;
        c->vf_row = dev_upload(c, cnt);
        c->vf_col = dev_upload(c, col);
    }

    HDG_REQUIRE(levels[nlev - 1].n_vert == nv, "the finest hierarchy level must be the HDG mesh");
    const int mr = opt.max_rhs;
    if (lf) {
        // ---- RT0 hierarchy: the finest level and every coarser one whose cells are fixed by their vertices
        int first = nlev - 1;
        while (first > 0 && levels[first - 1].n_vert >= 16 && hdg::cells_unique_by_vertices(levels[first - 1]))
            --first;
        const int nrt = nlev - first;
        std::vector<hdg::Rt0Host> H(nrt);
        for (int l = 0; l < nrt; ++l) H[l] = hdg::build_rt0_level(levels[first + l], c->kappa, l > 0);
        for (int l = 1; l < nrt; ++l) {
            HDG_REQUIRE(parents && parents[first + l], "parents[l] must be given for every level above the coarsest");
            hdg::rt0_transfer(levels[first + l], H[l], levels[first + l - 1], H[l - 1], parents[first + l]);
        }
        HDG_REQUIRE(H[0].ne <= 8192, "coarsest RT0 level must have at most 8192 facets");
        std::vector<double> dense = hdg::rt0_dense(H[0]);
        if (!hdg::spd_inverse(dense, H[0].ne)) throw Error{HDG_EINVAL, "coarsest RT0 operator is singular"};
        c->rt_coarse_inv = dev_upload(c, dense);
        c->rt.resize(nrt);
        int max_nv = 1;
        for (int l = 0; l < nrt; ++l) {
            const hdg::Rt0Host &h = H[l];
            hdg::Rt0LevelDev &L = c->rt[l];
            L.ne = h.ne;
            L.nv = h.nv;
            L.nbr = dev_upload(c, h.nbr);
            L.val = dev_upload(c, h.val);
            if (l > 0) {
                L.pf = dev_upload(c, h.pf);
                L.pinv = dev_upload(c, h.pinv);
                L.fs = dev_upload(c, h.fs);
                L.pc = dev_upload(c, h.pc);
                L.pw = dev_upload(c, h.pw);
                L.crow = dev_upload(c, h.crow);
                L.ccol = dev_upload(c, h.ccol);
                L.cw = dev_upload(c, h.cw);
                max_nv = std::max(max_nv, h.nv);
            }
            L.b = dev_alloc<double>(c, (size_t)h.ne * mr);
            L.x = dev_alloc<double>(c, (size_t)h.ne * mr);
            L.y = dev_alloc<double>(c, (size_t)h.ne * mr);
        }
        c->rt_corr = dev_alloc<double>(c, (size_t)max_nv * hdg::RT_PV * mr);
        // prolongation onto the trace and the CSR of its transpose (code 8 e + slot)
        const hdg::Rt0Host &F = H[nrt - 1];
        c->lf_pw = dev_upload(c, hdg::lf_prolongation_weights(fine, c->topo, c->p));
        std::vector<std::vector<int32_t>> users(ne);
        for (int e = 0; e < ne; ++e)
            for (int slot = 0; slot < 5; ++slot) {
                const int id = slot == 0 ? e : F.nbr[(size_t)(slot - 1) * ne + e];
                users[id].push_back(8 * e + slot);
            }
        std::vector<int32_t> rrow(ne + 1, 0), rcol;
        for (int e = 0; e < ne; ++e) {
            rcol.insert(rcol.end(), users[e].begin(), users[e].end());
            rrow[e + 1] = (int32_t)rcol.size();
        }
        c->lf_rrow = dev_upload(c, rrow);
        c->lf_rcol = dev_upload(c, rcol);
    }

    // ---- P1 hierarchy (upwind flux)
    c->lev.resize(lf ? 0 : nlev);
    std::vector<hdg::P1Host> galerkin;
    if (opt.p1_galerkin) {
        // S_c = pi^T S pi on the finest level, P^T A P below it (built on the host from the FP64 rows)
        std::vector<double> rows((size_t)hdg::wide_padded(5 * m * m, 2) * ne);
        std::vector<int32_t> nbr_h((size_t)4 * ne);
        HDG_HIP_CHECK(hipDeviceSynchronize());
        HDG_HIP_CHECK(hipMemcpy(rows.data(), c->S64, rows.size() * sizeof(double), hipMemcpyDeviceToHost));
        HDG_HIP_CHECK(hipMemcpy(nbr_h.data(), c->nbr, nbr_h.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
        galerkin.resize(nlev);
        galerkin[nlev - 1] = hdg::galerkin_from_rows(ne, m, nv, rows, nbr_h, c->topo.facet_vert);
        for (int l = nlev - 1; l > 0; --l) {
            HDG_REQUIRE(parents && parents[l], "parents[l] must be given for every level above the coarsest");
            galerkin[l - 1] = hdg::galerkin_coarsen(galerkin[l], parents[l], levels[l - 1].n_vert);
        }
    }
    std::vector<double> p1B;   // the P1 V-cycle as a matrix, for the persistent solve of small hierarchies
    if (!c->lev.empty()) {
        std::vector<hdg::P1Host> ops(c->lev.size());
        for (int l = 0; l < (int)c->lev.size(); ++l)
            ops[l] = opt.p1_galerkin ? galerkin[l] : hdg::assemble_p1(levels[l], c->kappa);
        hdg::build_p1_levels(c, levels, parents, ops, c->lev, &c->coarse_inv);
        if (opt.persistent && nv <= hdg::SMALL_P1_DENSE) p1B = hdg::p1_vcycle_matrix(ops, parents, opt.p1_nu, opt.p1_omega);
    }

    // ---- tail of the P1 hierarchy (levels small enough for one workgroup)
    // (one workgroup also reads the dense coarsest inverse: only for a small coarsest level)
    c->tail_top = -1;
    if (!c->lev.empty() && c->lev[0].n <= hdg::P1_TAIL_DENSE_MAX)   // (no P1 hierarchy with the LF flux)
        for (int l = 0; l < (int)c->lev.size() && l < hdg::P1_TAIL_LEVELS; ++l)
            if (c->lev[l].n <= opt.p1_tail_max) c->tail_top = l;
            else break;
    if (c->tail_top >= 0) {
        hdg::P1Tail &T = c->tail;
        T.top = c->tail_top;
        T.nu = opt.p1_nu;
        T.omega = opt.p1_omega;
        T.Ainv = c->coarse_inv;
        for (int l = 0; l <= c->tail_top; ++l) {
            const hdg::P1LevelDev &L = c->lev[l];
            T.lev[l] = hdg::P1Lev{L.n, L.w, L.col, L.val, L.diag, L.dinv, L.parents, L.crow, L.ccol, L.cw,
                                  L.b, L.x, L.y};
        }
    }

    // ---- work vectors
    const size_t vl = (size_t)ne * m * mr;
    c->vz0 = dev_alloc<double>(c, vl);
    c->vx = dev_alloc<double>(c, vl);
    c->vx2 = dev_alloc<double>(c, vl);
    c->vres = dev_alloc<double>(c, vl);
    c->vrc = dev_alloc<double>(c, vl);
    c->kr = dev_alloc<double>(c, vl);
    c->kz = dev_alloc<double>(c, vl);
    c->kp = dev_alloc<double>(c, vl);
    c->kw = dev_alloc<double>(c, vl);
    c->klam = dev_alloc<double>(c, vl);
    const int Rr = opt.restart;
    const bool need_gmres = !(opt.krylov == HDG_KRYLOV_PCG);
    if (need_gmres) {
        c->kV = dev_alloc<double>(c, vl * (Rr + 1));
        c->kZ = dev_alloc<double>(c, vl * Rr);
    }
    c->red_blocks = 2048;   // upper bound of red_grid() for any nrhs
    c->red = dev_alloc<double>(c, (size_t)c->red_blocks * (Rr + 1) * mr);
    c->scal = dev_alloc<double>(c, (size_t)SC_COUNT * mr);
    c->hcol = dev_alloc<double>(c, (size_t)(Rr + 1) * mr);
    c->gs_explicit = dev_alloc<int>(c, 1);
    c->gm = dev_alloc<double>(c, (size_t)((Rr + 1) * Rr + 2 * Rr + (Rr + 1)) * mr);
    c->hy = dev_alloc<double>(c, (size_t)Rr * mr);
    c->dbn = dev_alloc<double>(c, mr);
    c->loc = dev_alloc<double>(c, (size_t)c->nt * nk * mr);
    // learned smoother (zero weights until set: the untrained smoother is block-Jacobi)
    c->mlp_n1 = 64 * hdg::mlp_k1p(c->p);
    c->mlp_n2 = 16 * 64;
    {
        const size_t nw = c->mlp_n1 + c->mlp_n2;
        c->mlp_w = dev_alloc<float>(c, nw);
        c->mlp_m1 = dev_alloc<float>(c, nw);
        c->mlp_m2 = dev_alloc<float>(c, nw);
        c->mlp_g = dev_alloc<float>(c, nw);
        c->mlp_wb = dev_alloc<short>(c, nw);
        HDG_HIP_CHECK(hipMemset(c->mlp_w, 0, nw * sizeof(float)));
        HDG_HIP_CHECK(hipMemset(c->mlp_m1, 0, nw * sizeof(float)));
        HDG_HIP_CHECK(hipMemset(c->mlp_m2, 0, nw * sizeof(float)));
        HDG_HIP_CHECK(hipMemset(c->mlp_wb, 0, nw * sizeof(short)));
        const int nwv = hdg::mlp_grad_waves(ne, mr);
        c->mlp_pdW1 = dev_alloc<float>(c, (size_t)nwv * c->mlp_n1);
        c->mlp_pdW2 = dev_alloc<float>(c, (size_t)nwv * c->mlp_n2);
        c->mlp_ploss = dev_alloc<float>(c, (size_t)nwv);
        c->mlp_loss = dev_alloc<double>(c, 4096);
        c->p1_keep = dev_alloc<double>(c, (size_t)nv * mr);
        c->p1_acc = dev_alloc<double>(c, (size_t)nv * mr);
    }
    HDG_HIP_CHECK(hipHostMalloc((void **)&c->hscal, sizeof(double) * 64 * 4, hipHostMallocDefault));
    HDG_HIP_CHECK(hipHostMalloc((void **)&c->hlag, sizeof(double) * 64 * 4,
                                hipHostMallocMapped | hipHostMallocCoherent));
    HDG_HIP_CHECK(hipHostGetDevicePointer((void **)&c->dlag, c->hlag, 0));
    for (int i = 0; i < 2; ++i) HDG_HIP_CHECK(hipEventCreateWithFlags(&c->lag_ev[i], hipEventDisableTiming));
    c->hbn2.assign(mr, 0.0);
    c->stage_rhat = dev_alloc<double>(c, vl);

    // ---- persistent single-launch solve: every trace and P1 vector of one solve in one workgroup's LDS
    if (!lf && opt.persistent && (int)c->lev.size() <= hdg::P1_TAIL_LEVELS) {
        std::vector<hdg::P1Lev> lv;
        for (auto &L : c->lev) lv.push_back(hdg::P1Lev{L.n, L.w, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                                                        nullptr, nullptr, nullptr, nullptr, nullptr});
        int maxlds = 0;
        HDG_HIP_CHECK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device));
        // 2 KiB stay for the kernel's static LDS (level descriptors and tables)
        const size_t limit = (size_t)std::min(maxlds, 160 * 1024) - 2048;
        const int nB = p1B.empty() ? 0 : nv;
        const size_t with_ops = hdg::small_lds_bytes(ne, m, lv.data(), (int)lv.size(), true, nB);
        const size_t lds =
            with_ops <= limit ? with_ops : hdg::small_lds_bytes(ne, m, lv.data(), (int)lv.size(), false, nB);
        if (lds <= limit && hdg::small_prepare(c->p, lds) == hipSuccess) {
            c->small_ok = true;
            c->small_stage_ops = with_ops <= limit;
            c->small_lds = lds;
            if (nB) {
                // transposed: the kernel's lanes take consecutive rows
                std::vector<double> bt((size_t)nB * nB);
                for (int i = 0; i < nB; ++i)
                    for (int j = 0; j < nB; ++j) bt[(size_t)j * nB + i] = p1B[(size_t)i * nB + j];
                c->small_p1B = dev_upload(c, bt);
            }
            if (c->small_stage_ops) {
                // the operators packed once in the layout of their LDS copies
                const size_t bytes = hdg::small_image_bytes(ne, m, lv.data(), (int)lv.size(), nB);
                c->small_image = dev_alloc<char>(c, bytes);
                HDG_HIP_CHECK(hipDeviceSynchronize());   // every operator is complete
                hdg::small_image_walk(ne, m, lv.data(), (int)lv.size(), nB,
                                      [&](hdg::SmallPart part, int l, size_t off, size_t nbytes) {
                    const hdg::P1LevelDev &L = c->lev[l];
                    const void *src = nullptr;
                    switch (part) {
                    case hdg::SP_S: src = c->S64; break;
                    case hdg::SP_T: src = c->T64; break;
                    case hdg::SP_DW: src = c->Dw64; break;
                    case hdg::SP_NBR: src = c->nbr; break;
                    case hdg::SP_FVERT: src = c->facet_vert; break;
                    case hdg::SP_VF_ROW: src = c->vf_row; break;
                    case hdg::SP_VF_COL: src = c->vf_col; break;
                    case hdg::SP_B: src = c->small_p1B; break;
                    case hdg::SP_COL: src = L.col; break;
                    case hdg::SP_VAL: src = L.val; break;
                    case hdg::SP_DIAG: src = L.diag; break;
                    case hdg::SP_DINV: src = L.dinv; break;
                    case hdg::SP_PARENTS: src = L.parents; break;
                    case hdg::SP_CROW: src = L.crow; break;
                    case hdg::SP_CCOL: src = L.ccol; break;
                    case hdg::SP_CW: src = L.cw; break;
                    case hdg::SP_AINV: src = c->coarse_inv; break;
                    }
                    HDG_HIP_CHECK(hipMemcpy(c->small_image + off, src, nbytes, hipMemcpyDeviceToDevice));
                });
            }
            const size_t v1 = (size_t)ne * m;
            c->small_V = dev_alloc<double>(c, (size_t)mr * (hdg::SMALL_MAXR + 1) * v1);
            c->small_Z = dev_alloc<double>(c, (size_t)mr * hdg::SMALL_MAXR * v1);
            // the kernel writes each solve's record straight into host-mapped memory
            HDG_HIP_CHECK(hipHostMalloc((void **)&c->small_hinfo, sizeof(double) * 4 * mr,
                                        hipHostMallocMapped | hipHostMallocCoherent));
            HDG_HIP_CHECK(hipHostGetDevicePointer((void **)&c->small_info, c->small_hinfo, 0));
        }
    }
    HDG_HIP_CHECK(hipDeviceSynchronize());
    if (c->opt.smoother == HDG_SMOOTH_CHEBYSHEV) estimate_lambda_max(c);
}

void destroy_impl(hdg_ctx *c) {
    for (void *p : c->allocations) (void)hipFree(p);
    c->allocations.clear();
    for (auto &p : c->pending) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : c->event_pool) (void)hipEventDestroy(e);
    drop_graphs(c);
    if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
    if (c->hscal) (void)hipHostFree(c->hscal);
    if (c->hlag) (void)hipHostFree(c->hlag);
    if (c->small_hinfo) (void)hipHostFree(c->small_hinfo);
    for (int i = 0; i < 2; ++i)
        if (c->lag_ev[i]) (void)hipEventDestroy(c->lag_ev[i]);
}

}  // namespace

// ------------------------------------------------------------------ C ABI

// ------------------------------------------------------------------ P1 levels on the device
//
// Upload the P1 operators ops[l] (coarse to fine) as ELL rows with their
// diagonal and inverse diagonal, work vectors for max_rhs right-hand sides,
// the parent pairs and the children CSR of the linear-interpolation
// transfer, and the dense inverse of the coarsest operator.
void hdg::build_p1_levels(hdg_ctx *c, const hdg_mesh *levels, const int32_t *const *parents,
                          const std::vector<hdg::P1Host> &ops, std::vector<hdg::P1LevelDev> &lev,
                          double **coarse_inv) {
    lev.resize(ops.size());
    const int mr = c->opt.max_rhs;
    for (int l = 0; l < (int)lev.size(); ++l) {
        const hdg_mesh &lm = levels[l];
        const hdg::P1Host &P = ops[l];
        hdg::P1LevelDev &L = lev[l];
        L.n = lm.n_vert;
        std::vector<double> dinv(L.n);
        for (int v = 0; v < L.n; ++v) {
            HDG_REQUIRE(P.diag[v] > 0, "P1 operator has a non-positive diagonal");
            dinv[v] = 1.0 / P.diag[v];
        }
        {
            int W = 0;
            for (int vv = 0; vv < L.n; ++vv) W = std::max(W, P.rowptr[vv + 1] - P.rowptr[vv]);
            std::vector<int32_t> ec((size_t)std::max(W, 1) * L.n);
            std::vector<double> ev((size_t)std::max(W, 1) * L.n, 0.0);
            for (int vv = 0; vv < L.n; ++vv)
                for (int k = 0; k < W; ++k) {
                    const int q = P.rowptr[vv] + k;
                    const bool in = q < P.rowptr[vv + 1];
                    ec[(size_t)k * L.n + vv] = in ? P.col[q] : vv;
                    ev[(size_t)k * L.n + vv] = in ? P.val[q] : 0.0;
                }
            L.w = W;
            L.col = dev_upload(c, ec);
            L.val = dev_upload(c, ev);
        }
        L.diag = dev_upload(c, P.diag);
        L.dinv = dev_upload(c, dinv);
        L.b = dev_alloc<double>(c, (size_t)L.n * mr);
        L.x = dev_alloc<double>(c, (size_t)L.n * mr);
        L.y = dev_alloc<double>(c, (size_t)L.n * mr);
        if (l == 0) {
            HDG_REQUIRE(L.n <= 8192, "coarsest P1 level must have at most 8192 vertices");
            std::vector<double> dense((size_t)L.n * L.n, 0.0);
            for (int v = 0; v < L.n; ++v) {
                dense[(size_t)v * L.n + v] = P.diag[v];
                for (int k = P.rowptr[v]; k < P.rowptr[v + 1]; ++k) dense[(size_t)v * L.n + P.col[k]] += P.val[k];
            }
            if (!hdg::spd_inverse(dense, L.n)) throw Error{HDG_EINVAL, "coarsest P1 operator is singular"};   // pivoted inverse
            *coarse_inv = dev_upload(c, dense);
        } else {
            HDG_REQUIRE(parents && parents[l], "parents[l] must be given for every level above the coarsest");
            const int ncv = levels[l - 1].n_vert;
            std::vector<int32_t> par(parents[l], parents[l] + 2 * (size_t)L.n);
            std::vector<std::vector<std::pair<int, double>>> ch(ncv);
            for (int v = 0; v < L.n; ++v)
                for (int k = 0; k < 2; ++k) {
                    HDG_REQUIRE(par[2 * v + k] >= 0 && par[2 * v + k] < ncv, "parent id out of range");
                    ch[par[2 * v + k]].push_back({v, 0.5});
                }
            std::vector<int32_t> crow(ncv + 1, 0), ccol;
            std::vector<double> cw;
            for (int cv = 0; cv < ncv; ++cv) {
                for (auto &pr : ch[cv]) {
                    ccol.push_back(pr.first);
                    cw.push_back(pr.second);
                }
                crow[cv + 1] = (int)ccol.size();
            }
            L.parents = dev_upload(c, par);
            L.crow = dev_upload(c, crow);
            L.ccol = dev_upload(c, ccol);
            L.cw = dev_upload(c, cw);
        }
    }
}

void *hdg::ctx_alloc(hdg_ctx *c, size_t bytes) { return dev_alloc<char>(c, bytes); }
int hdg::guarded(const std::function<void()> &fn) { return guard(fn); }
void hdg::check_kernel_launch() { check_launch(); }
void hdg::check_abi(int rc) {
    if (rc < 0) throw Error{rc, hdg_last_error()};
}

extern "C" int hdg_default_options(hdg_options *o) {
    if (!o) return HDG_EINVAL;
    o->krylov = HDG_KRYLOV_AUTO;
    o->precision = HDG_FP64;
    o->smoother = HDG_SMOOTH_BJACOBI;
    o->p1_galerkin = 0;
    o->nu_pre = 2;
    o->nu_post = 2;
    o->omega = 0.7;
    o->p1_nu = 2;
    o->p1_omega = 2.0 / 3.0;
    o->rtol = 1e-8;
    o->maxit = 200;
    o->restart = 30;
    o->max_rhs = 1;
    o->use_graph = 1;
    o->fallback_ratio = 0.5;
    o->p1_tail_max = hdg::P1_TAIL_MAX;
    o->rt_nu = 1;
    o->rt_omega = 0.5;
    o->ir_inner_rtol = 1e-4;
    o->persistent = 1;
    return HDG_OK;
}

extern "C" int hdg_setup(const hdg_mesh *levels, int32_t n_levels, const int32_t *const *parents,
                         const hdg_params *prm, const hdg_options *opt, hdg_ctx **out) {
    if (!out) {
        hdg::set_error("out must not be NULL");
        return HDG_EINVAL;
    }
    *out = nullptr;
    hdg_ctx *c = new (std::nothrow) hdg_ctx();
    if (!c) {
        hdg::set_error("host allocation failed");
        return HDG_ENOMEM;
    }
    int rc = guard([&] { setup_impl(levels, n_levels, parents, prm, opt, c); });
    if (rc != HDG_OK) {
        destroy_impl(c);
        delete c;
        return rc;
    }
    *out = c;
    return HDG_OK;
}

extern "C" void hdg_destroy(hdg_ctx *c) {
    if (!c) return;
    destroy_impl(c);
    delete c;
}

extern "C" int hdg_get_sizes(const hdg_ctx *c, hdg_sizes *out) {
    if (!c || !out) {
        hdg::set_error("ctx and out must not be NULL");
        return HDG_EINVAL;
    }
    out->n_cell = c->n_cell;
    out->n_facet = c->n_facet;
    out->n_vert = c->n_vert;
    out->degree = c->p;
    out->n_loc = c->n;
    out->n_levels = (int)(c->flux == HDG_FLUX_LF ? c->rt.size() : c->lev.size());
    out->facet_dofs = c->m;
    out->flux = c->flux;
    out->device_bytes = c->device_bytes;
    out->kappa = c->kappa;
    out->lambda_max = c->cheb_lmax;
    out->persistent = c->small_ok ? 1 : 0;
    return HDG_OK;
}

extern "C" int hdg_get_topology(const hdg_ctx *c, int32_t *facet_cell, int32_t *facet_loc, int32_t *facet_vert) {
    if (!c) {
        hdg::set_error("ctx must not be NULL");
        return HDG_EINVAL;
    }
    const size_t n2 = (size_t)2 * c->n_facet;
    if (facet_cell) std::memcpy(facet_cell, c->topo.facet_cell.data(), n2 * sizeof(int32_t));
    if (facet_loc) std::memcpy(facet_loc, c->topo.facet_loc.data(), n2 * sizeof(int32_t));
    if (facet_vert) std::memcpy(facet_vert, c->topo.facet_vert.data(), n2 * sizeof(int32_t));
    return HDG_OK;
}

extern "C" int hdg_condense(hdg_ctx *c, int32_t nb, const double *r_cell, double *rhat, void *stream) {
    if (!c) return HDG_EINVAL;
    return guard([&] {
        check_nb(c, nb);
        HDG_REQUIRE(r_cell && rhat, "r_cell and rhat must not be NULL");
        hipStream_t s = as_stream(stream);
        Timed t(c, HDG_KERNEL_CONDENSE, HDG_FP64, s, nb);
        for (int rep = 0; rep < t.repeats(); ++rep)
            hdg::launch_condense(c->p, c->nu, c->n_cell, c->n_facet, nb, c->Zr, r_cell, c->loc, c->d_fcell, c->d_floc, rhat,
                                 s, c->cell_cells);
        check_launch();
    });
}

extern "C" int hdg_condense_noalloc(hdg_ctx *c, int32_t nb, const double *r_cell, double *rhat, void *stream) {
    if (!c) return HDG_EINVAL;
    return guard([&] {
        check_nb(c, nb);
        HDG_REQUIRE(r_cell && rhat, "r_cell and rhat must not be NULL");
        const size_t need = (size_t)c->nt * c->n_cell * nb;
        if (need > NOALLOC_SCRATCH_DOUBLES)
            throw Error{HDG_EINVAL, "hdg_condense_noalloc needs " + std::to_string(need) +
                                        " doubles of scratch (3 facet_dofs x n_cell x nrhs), the static scratch holds " +
                                        std::to_string(NOALLOC_SCRATCH_DOUBLES) + ": use hdg_condense"};
        HDG_REQUIRE(c->noalloc_scratch, "static scratch not resolved for this device");
        hdg::launch_condense(c->p, c->nu, c->n_cell, c->n_facet, nb, c->Zr, r_cell, c->noalloc_scratch, c->d_fcell,
                             c->d_floc, rhat, as_stream(stream), c->cell_cells);
        check_launch();
    });
}

extern "C" int hdg_trace_apply(hdg_ctx *c, int32_t nb, int32_t prec, const double *x, double *y, void *stream) {
    if (!c) return HDG_EINVAL;
    return guard([&] {
        check_nb(c, nb);
        check_prec(prec);
        HDG_REQUIRE(x && y && x != y, "x and y must be distinct non-NULL buffers");
        check_aligned(x, "x");
        check_aligned(y, "y");
        op_apply(c, nb, prec, x, nullptr, y, as_stream(stream), HDG_KERNEL_APPLY);
    });
}

extern "C" int hdg_mg_vcycle(hdg_ctx *c, int32_t nb, int32_t prec, const double *r, double *z, void *stream) {
    if (!c) return HDG_EINVAL;
    return guard([&] {
        check_nb(c, nb);
        check_prec(prec);
        HDG_REQUIRE(r && z && r != z, "r and z must be distinct non-NULL buffers");
        check_aligned(r, "r");
        check_aligned(z, "z");
        c->use_mlp_now = c->opt.smoother == HDG_SMOOTH_MLP;
        vcycle(c, nb, prec, r, z, as_stream(stream));
    });
}

namespace {
// Step 2 on the caller's stream (the argument checks are done by the callers)
int solve_impl(hdg_ctx *c, int nb, const double *rhat, double *lam, hdg_solve_info *info, hipStream_t s) {
    c->use_mlp_now = c->opt.smoother == HDG_SMOOTH_MLP;
    const int kry = krylov_kind(c);
    HDG_REQUIRE(!(kry == HDG_KRYLOV_PCG && c->use_mlp_now), "the learned smoother is nonlinear: use FGMRES");
    HDG_REQUIRE(c->opt.precision >= HDG_FP64 && c->opt.precision <= HDG_MIXED_IR, "unknown solve precision");
    if (kry == HDG_KRYLOV_FGMRES) HDG_REQUIRE(c->kV != nullptr, "FGMRES workspace was not allocated (krylov = PCG at setup)");
    if (kry == HDG_KRYLOV_PCG) HDG_REQUIRE(c->opt.precision == HDG_FP64, "PCG needs the FP64 (linear) preconditioner");
    if (use_small(c, kry)) return solve_small(c, nb, kry, false, rhat, nullptr, lam, nullptr, info, s);
    const double *h = dots_now(c, nb, rhat, rhat, scal(c, SC_BN2), s);
    hdg::launch_sqrt(nb, scal(c, SC_BN2), c->dbn, s);
    for (int r = 0; r < nb; ++r) c->hbn2[r] = h[r];
    if (kry == HDG_KRYLOV_PCG) return solve_pcg(c, nb, rhat, lam, info, s);
    if (c->opt.precision == HDG_MIXED_IR)
        return solve_fgmres(c, nb, HDG_MIXED, HDG_MIXED, c->opt.ir_inner_rtol, rhat, lam, info, s);
    return solve_fgmres(c, nb, c->opt.precision, HDG_FP64, 0.0, rhat, lam, info, s);
}
}  // namespace

extern "C" int hdg_solve(hdg_ctx *c, int32_t nb, const double *rhat, double *lam, hdg_solve_info *info,
                         void *stream) {
    if (!c) return HDG_EINVAL;
    int status = HDG_OK;
    int rc = guard([&] {
        check_nb(c, nb);
        HDG_REQUIRE(rhat && lam && rhat != lam, "rhat and lam must be distinct non-NULL buffers");
        check_aligned(rhat, "rhat");
        check_aligned(lam, "lam");
        status = solve_impl(c, nb, rhat, lam, info, as_stream(stream));
    });
    if (rc != HDG_OK) return rc;
    if (status == HDG_EBREAKDOWN) hdg::set_error("non-finite residual in the Krylov solve");
    return status;
}

extern "C" int hdg_stage_solve(hdg_ctx *c, int32_t nb, const double *r_cell, double *lam, double *q_cell,
                               hdg_solve_info *info, void *stream) {
    if (!c) return HDG_EINVAL;
    int status = HDG_OK;
    int rc = guard([&] {
        check_nb(c, nb);
        HDG_REQUIRE(r_cell && lam && q_cell, "r_cell, lam and q_cell must not be NULL");
        HDG_REQUIRE(r_cell != q_cell, "r_cell and q_cell must be distinct buffers");
        check_aligned(lam, "lam");
        hipStream_t s = as_stream(stream);
        const int kry = krylov_kind(c);
        if (use_small(c, kry)) {
            status = solve_small(c, nb, kry, true, nullptr, r_cell, lam, q_cell, info, s);
            return;
        }
        hdg::launch_condense(c->p, c->nu, c->n_cell, c->n_facet, nb, c->Zr, r_cell, c->loc, c->d_fcell, c->d_floc,
                             c->stage_rhat, s, c->cell_cells);
        check_launch();
        HDG_HIP_CHECK(hipMemsetAsync(lam, 0, sizeof(double) * (size_t)vec_len(c) * nb, s));
        status = solve_impl(c, nb, c->stage_rhat, lam, info, s);
        hdg::launch_recover(c->p, c->nu, c->n_cell, nb, c->Ar, c->Wr, c->cell_facet, c->cell_rev, r_cell, lam, q_cell,
                            s, c->cell_cells);
        check_launch();
        HDG_HIP_CHECK(hipStreamSynchronize(s));
    });
    if (rc != HDG_OK) return rc;
    if (status == HDG_EBREAKDOWN) hdg::set_error("non-finite residual in the Krylov solve");
    return status;
}

extern "C" int hdg_recover(hdg_ctx *c, int32_t nb, const double *r_cell, const double *lam, double *q_cell,
                           void *stream) {
    if (!c) return HDG_EINVAL;
    return guard([&] {
        check_nb(c, nb);
        HDG_REQUIRE(r_cell && lam && q_cell, "r_cell, lam and q_cell must not be NULL");
        check_aligned(lam, "lam");
        hipStream_t s = as_stream(stream);
        Timed t(c, HDG_KERNEL_RECOVER, HDG_FP64, s, nb);
        for (int rep = 0; rep < t.repeats(); ++rep)
            hdg::launch_recover(c->p, c->nu, c->n_cell, nb, c->Ar, c->Wr, c->cell_facet, c->cell_rev, r_cell, lam, q_cell,
                                s, c->cell_cells);
        check_launch();
    });
}

// ------------------------------------------------------------------ learned smoother

namespace {

void mlp_data_buffers(hdg_ctx *c) {
    if (c->mlp_E) return;
    const size_t vl = (size_t)vec_len(c) * c->opt.max_rhs;
    c->mlp_E = dev_alloc<double>(c, vl);
    c->mlp_R = dev_alloc<double>(c, vl);
    c->mlp_U = dev_alloc<double>(c, vl);
    c->mlp_T = dev_alloc<double>(c, vl);
}

// Training pair for the error e: r = S e, u = omega D^-1 r, and the target
// t = e - pi x_c - u, x_c = coarse_its stationary P1 V-cycles on
// S_c x_c = pi^T r from zero (the part of e the coarse correction leaves,
// minus the block-Jacobi step).  FP64 throughout.
void mlp_pair(hdg_ctx *c, int nb, int coarse_its, const double *e, double *r, double *u, double *t, hipStream_t s) {
    const int L = (int)c->lev.size() - 1;
    hdg::P1LevelDev &F = c->lev[L];
    const int64_t nv = (int64_t)F.n * nb;
    op_apply(c, nb, HDG_FP64, e, nullptr, r, s, HDG_KERNEL_APPLY);
    jacobi0(c, nb, HDG_FP64, r, nullptr, nullptr, nullptr, u, s);
    hdg::launch_restrict_trace(c->p, c->n_vert, nb, c->vf_row, c->vf_col, r, c->p1_keep, s);
    for (int k = 0; k < coarse_its; ++k) {
        if (k == 0)
            hdg::launch_copy(nv, c->p1_keep, F.b, s);
        else
            hdg::launch_p1_resid(F.n, F.w, nb, F.col, F.val, F.diag, c->p1_keep, c->p1_acc, F.b, s);
        const double *xl = p1_vcycle(c, L, nb, s, false);
        hdg::launch_lin3<double>(nv, 1.0, xl, k == 0 ? 0.0 : 1.0, k == 0 ? nullptr : c->p1_acc, 0.0, nullptr, c->p1_acc, s);
    }
    const int64_t n = vec_len(c) * nb;
    hdg::launch_lin3<double>(n, 1.0, e, -1.0, u, 0.0, nullptr, t, s);
    if (coarse_its > 0) {
        hdg::launch_lin3<double>(nv, -1.0, c->p1_acc, 0.0, nullptr, 0.0, nullptr, c->p1_acc, s);
        hdg::launch_prolong_trace(c->p, c->n_facet, nb, c->facet_vert, c->p1_acc, t, s);
    }
    check_launch();
}

void mlp_grad(hdg_ctx *c, int nb, const double *u, const double *t, double *loss, hipStream_t s) {
    hdg::launch_mlp_grad(c->p, c->n_facet, nb, u, t, c->nbr, c->prev, c->mlp_wb, c->mlp_wb + c->mlp_n1, c->mlp_pdW1,
                         c->mlp_pdW2, c->mlp_ploss, c->mlp_g, loss, s);
    check_launch();
}

// packed device layout [W1: 64 x K1P | W2: 16 x 64] <-> dense (64 x 5m), (m x 64);
// dense W1 column slot * m + node sits at packed column 4 slot + node
void mlp_pack(const hdg_ctx *c, const float *W1, const float *W2, std::vector<float> &buf) {
    const int m = c->p + 1, k1 = 5 * m, k1p = c->mlp_n1 / 64;
    buf.assign((size_t)c->mlp_n1 + c->mlp_n2, 0.f);
    for (int h = 0; h < 64; ++h)
        for (int k = 0; k < k1; ++k) buf[(size_t)h * k1p + 4 * (k / m) + k % m] = W1[(size_t)h * k1 + k];
    for (int o = 0; o < m; ++o)
        for (int h = 0; h < 64; ++h) buf[(size_t)c->mlp_n1 + o * 64 + h] = W2[(size_t)o * 64 + h];
}

void mlp_unpack(const hdg_ctx *c, const std::vector<float> &buf, float scale, float *W1, float *W2) {
    const int m = c->p + 1, k1 = 5 * m, k1p = c->mlp_n1 / 64;
    if (W1)
        for (int h = 0; h < 64; ++h)
            for (int k = 0; k < k1; ++k) W1[(size_t)h * k1 + k] = scale * buf[(size_t)h * k1p + 4 * (k / m) + k % m];
    if (W2)
        for (int o = 0; o < m; ++o)
            for (int h = 0; h < 64; ++h) W2[(size_t)o * 64 + h] = scale * buf[(size_t)c->mlp_n1 + o * 64 + h];
}

}  // namespace

extern "C" int hdg_mlp_set_weights(hdg_ctx *c, const float *W1, const float *W2) {
    if (!c) return HDG_EINVAL;
    return guard([&] {
        HDG_REQUIRE(c->flux == HDG_FLUX_UPWIND, "the learned smoother is built for the upwind flux only");
        HDG_REQUIRE(W1 && W2, "W1 and W2 must not be NULL");
        const int m = c->p + 1;
        for (size_t i = 0; i < (size_t)64 * 5 * m; ++i) HDG_REQUIRE(std::isfinite(W1[i]), "W1 has a non-finite entry");
        for (size_t i = 0; i < (size_t)m * 64; ++i) HDG_REQUIRE(std::isfinite(W2[i]), "W2 has a non-finite entry");
        std::vector<float> buf;
        mlp_pack(c, W1, W2, buf);
        const size_t nw = buf.size();
        HDG_HIP_CHECK(hipDeviceSynchronize());
        HDG_HIP_CHECK(hipMemcpy(c->mlp_w, buf.data(), nw * sizeof(float), hipMemcpyHostToDevice));
        HDG_HIP_CHECK(hipMemset(c->mlp_m1, 0, nw * sizeof(float)));
        HDG_HIP_CHECK(hipMemset(c->mlp_m2, 0, nw * sizeof(float)));
        hdg::launch_to_bf16((int)nw, c->mlp_w, c->mlp_wb, nullptr);
        check_launch();
        HDG_HIP_CHECK(hipDeviceSynchronize());
        c->mlp_step = 0;
    });
}

extern "C" int hdg_mlp_get_weights(hdg_ctx *c, float *W1, float *W2) {
    if (!c) return HDG_EINVAL;
    return guard([&] {
        HDG_REQUIRE(c->flux == HDG_FLUX_UPWIND, "the learned smoother is built for the upwind flux only");
        std::vector<float> buf((size_t)c->mlp_n1 + c->mlp_n2);
        HDG_HIP_CHECK(hipDeviceSynchronize());
        HDG_HIP_CHECK(hipMemcpy(buf.data(), c->mlp_w, buf.size() * sizeof(float), hipMemcpyDeviceToHost));
        mlp_unpack(c, buf, 1.f, W1, W2);
    });
}

extern "C" int hdg_mlp_make_data(hdg_ctx *c, int32_t nb, const double *e, double *u, double *t, int32_t coarse_its,
                                 void *stream) {
    if (!c) return HDG_EINVAL;
    return guard([&] {
        HDG_REQUIRE(c->flux == HDG_FLUX_UPWIND, "the learned smoother is built for the upwind flux only");
        check_nb(c, nb);
        HDG_REQUIRE(e && u && t && e != u && e != t && u != t, "e, u and t must be distinct non-NULL buffers");
        check_aligned(e, "e");
        check_aligned(u, "u");
        check_aligned(t, "t");
        HDG_REQUIRE(coarse_its >= 0 && coarse_its <= 64, "coarse_its must be in 0..64");
        hipStream_t s = as_stream(stream);
        mlp_data_buffers(c);
        mlp_pair(c, nb, coarse_its, e, c->mlp_R, u, t, s);
        HDG_HIP_CHECK(hipStreamSynchronize(s));
    });
}

extern "C" int hdg_mlp_loss_grad(hdg_ctx *c, int32_t nb, const double *u, const double *t, double *loss, float *dW1,
                                 float *dW2, void *stream) {
    if (!c) return HDG_EINVAL;
    return guard([&] {
        HDG_REQUIRE(c->flux == HDG_FLUX_UPWIND, "the learned smoother is built for the upwind flux only");
        check_nb(c, nb);
        HDG_REQUIRE(u && t, "u and t must not be NULL");
        check_aligned(u, "u");
        check_aligned(t, "t");
        hipStream_t s = as_stream(stream);
        mlp_grad(c, nb, u, t, c->mlp_loss, s);
        HDG_HIP_CHECK(hipStreamSynchronize(s));
        const double n = (double)c->n_facet * nb;
        std::vector<float> buf((size_t)c->mlp_n1 + c->mlp_n2);
        HDG_HIP_CHECK(hipMemcpy(buf.data(), c->mlp_g, buf.size() * sizeof(float), hipMemcpyDeviceToHost));
        mlp_unpack(c, buf, (float)(1.0 / n), dW1, dW2);
        if (loss) {
            double l = 0;
            HDG_HIP_CHECK(hipMemcpy(&l, c->mlp_loss, sizeof(double), hipMemcpyDeviceToHost));
            *loss = l / n;
        }
    });
}

extern "C" int hdg_mlp_train(hdg_ctx *c, int32_t nb, const double *e0, int32_t cycles, int32_t coarse_its,
                             int32_t epochs, double lr, double *loss_hist, void *stream) {
    if (!c) return HDG_EINVAL;
    return guard([&] {
        HDG_REQUIRE(c->flux == HDG_FLUX_UPWIND, "the learned smoother is built for the upwind flux only");
        check_nb(c, nb);
        HDG_REQUIRE(e0, "e0 must not be NULL");
        check_aligned(e0, "e0");
        HDG_REQUIRE(cycles >= 1 && epochs >= 1 && (int64_t)cycles * epochs <= 4096,
                    "need cycles, epochs >= 1 and cycles * epochs <= 4096");
        HDG_REQUIRE(coarse_its >= 0 && coarse_its <= 64, "coarse_its must be in 0..64");
        HDG_REQUIRE(lr > 0 && std::isfinite(lr), "lr must be positive");
        hipStream_t s = as_stream(stream);
        mlp_data_buffers(c);
        const int64_t n = vec_len(c) * nb;
        const float gscale = (float)(1.0 / ((double)c->n_facet * nb));
        const bool keep = c->use_mlp_now;
        c->use_mlp_now = false;   // the data come from the block-Jacobi cycle
        hdg::launch_copy(n, e0, c->mlp_E, s);
        int idx = 0;
        for (int k = 0; k < cycles; ++k) {
            mlp_pair(c, nb, coarse_its, c->mlp_E, c->mlp_R, c->mlp_U, c->mlp_T, s);
            for (int ep = 0; ep < epochs; ++ep, ++idx) {
                mlp_grad(c, nb, c->mlp_U, c->mlp_T, c->mlp_loss + idx, s);
                ++c->mlp_step;
                hdg::launch_adam(c->p, c->mlp_g, gscale, c->mlp_w, c->mlp_m1, c->mlp_m2, (float)lr, c->mlp_step,
                                 c->mlp_wb, s);
                check_launch();
            }
            if (k + 1 < cycles) {
                // next error: e <- e - V(S e) with the plain block-Jacobi cycle (r = S e is in mlp_R)
                vcycle_bj(c, nb, HDG_FP64, c->mlp_R, c->mlp_U, s);
                hdg::launch_lin3<double>(n, 1.0, c->mlp_E, -1.0, c->mlp_U, 0.0, nullptr, c->mlp_E, s);
                check_launch();
            }
        }
        c->use_mlp_now = keep;
        HDG_HIP_CHECK(hipStreamSynchronize(s));
        if (loss_hist) {
            std::vector<double> l(idx);
            HDG_HIP_CHECK(hipMemcpy(l.data(), c->mlp_loss, idx * sizeof(double), hipMemcpyDeviceToHost));
            for (int i = 0; i < idx; ++i) loss_hist[i] = l[i] * gscale;
        }
    });
}

// ------------------------------------------------------------------ launch tuning

namespace {

void check_tuning(const hdg_tuning &t) {
    const int v = t.mlp_samples_per_lane;
    HDG_REQUIRE(v == 1 || v == 2 || v == 4, "mlp_samples_per_lane must be 1, 2 or 4");
    HDG_REQUIRE(t.rhs_block == 1 || t.rhs_block == 4, "rhs_block must be 1 or 4");
    HDG_REQUIRE(t.cell_cells >= 0 && t.cell_cells <= 32, "cell_cells must be in 0..32");
}

// mean duration (ms) of `reps` launches of fn, after one untimed launch
template <typename F>
double time_launches(hipStream_t s, int reps, F &&fn) {
    hipEvent_t a, b;
    HDG_HIP_CHECK(hipEventCreate(&a));
    HDG_HIP_CHECK(hipEventCreate(&b));
    fn();
    HDG_HIP_CHECK(hipEventRecord(a, s));
    for (int i = 0; i < reps; ++i) fn();
    HDG_HIP_CHECK(hipEventRecord(b, s));
    HDG_HIP_CHECK(hipEventSynchronize(b));
    float ms = 0.f;
    HDG_HIP_CHECK(hipEventElapsedTime(&ms, a, b));
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    check_launch();
    return ms / reps;
}

}  // namespace

extern "C" int hdg_get_tuning(const hdg_ctx *c, hdg_tuning *out) {
    if (!c || !out) return HDG_EINVAL;
    out->mlp_samples_per_lane = c->mlp_spl;
    out->rhs_block = c->rhs_block;
    out->cell_cells = c->cell_cells;
    return HDG_OK;
}

extern "C" int hdg_set_tuning(hdg_ctx *c, const hdg_tuning *t) {
    if (!c) return HDG_EINVAL;
    return guard([&] {
        HDG_REQUIRE(t, "tuning must not be NULL");
        check_tuning(*t);
        HDG_HIP_CHECK(hipDeviceSynchronize());
        drop_graphs(c);
        c->mlp_spl = t->mlp_samples_per_lane;
        c->rhs_block = t->rhs_block;
        c->cell_cells = t->cell_cells;
    });
}

extern "C" int hdg_autotune(hdg_ctx *c, int32_t nb, hdg_tuning *chosen, void *stream) {
    if (!c) return HDG_EINVAL;
    return guard([&] {
        check_nb(c, nb);
        hipStream_t s = as_stream(stream);
        HDG_HIP_CHECK(hipDeviceSynchronize());
        drop_graphs(c);
        const size_t bytes = sizeof(double) * (size_t)vec_len(c) * nb;
        HDG_HIP_CHECK(hipMemsetAsync(c->vres, 0, bytes, s));
        HDG_HIP_CHECK(hipMemsetAsync(c->vx, 0, bytes, s));
        const short *W1b = c->mlp_wb, *W2b = c->mlp_wb + c->mlp_n1;
        double best = 1e300;
        int best_spl = c->mlp_spl;
        for (int spl : {1, 2, 4}) {
            if (c->opt.smoother != HDG_SMOOTH_MLP) break;   // no learned smoother to tune
            if (spl == 4 && nb % 4 != 0) continue;           // four right-hand sides per lane
            const double ms = time_launches(s, 10, [&] {
                hdg::launch_mlp_smooth(c->p, c->n_facet, nb, spl, c->vres, c->vx, nullptr, c->facet_vert, c->nbr,
                                       c->prev, W1b, W2b, c->vx2, s);
            });
            if (ms < best) {
                best = ms;
                best_spl = spl;
            }
        }
        c->mlp_spl = best_spl;
        // facet-row kernels: one thread per (facet, rhs) or RHS-blocked with LDS-staged rows
        HDG_HIP_CHECK(hipMemsetAsync(c->vx2, 0, bytes, s));
        best = 1e300;
        int best_rb = 1;
        for (int rb : {1, 4}) {
            c->rhs_block = rb;
            const double ms = time_launches(s, 10, [&] {
                op_apply(c, nb, HDG_FP64, c->vx, nullptr, c->vx2, s, HDG_KERNEL_APPLY);
                op_sweep(c, nb, HDG_MIXED, c->vx, c->vres, nullptr, c->vx2, s, bj_coef(c));
            });
            if (ms < best) {
                best = ms;
                best_rb = rb;
            }
        }
        c->rhs_block = best_rb;
        // batched cell kernels (condensation, recovery): the most cells per block
        // that fit, half or a quarter of them
        int best_cc = 0;
        if (nb >= 2) {
            const size_t cell_bytes = sizeof(double) * (size_t)c->n_cell * c->nc * nb;
            struct Scratch {   // freed on every way out, errors included
                double *p = nullptr;
                ~Scratch() {
                    if (p) (void)hipFree(p);
                }
            } rcb, qcb;
            HDG_HIP_CHECK(hipMalloc(&rcb.p, cell_bytes));
            HDG_HIP_CHECK(hipMalloc(&qcb.p, cell_bytes));
            double *const rc = rcb.p, *const qc = qcb.p;
            HDG_HIP_CHECK(hipMemsetAsync(rc, 0, cell_bytes, s));
            best = 1e300;
            for (int div : {1, 2, 4}) {
                const int mx = std::max(1, std::min(32, 256 / nb));   // upper bound; the launcher clamps further
                const int cc = div == 1 ? 0 : std::max(1, mx / div);
                const double ms = time_launches(s, 5, [&] {
                    hdg::launch_condense(c->p, c->nu, c->n_cell, c->n_facet, nb, c->Zr, rc, c->loc, c->d_fcell,
                                         c->d_floc, c->vres, s, cc);
                    hdg::launch_recover(c->p, c->nu, c->n_cell, nb, c->Ar, c->Wr, c->cell_facet, c->cell_rev, rc,
                                        c->vx, qc, s, cc);
                });
                if (ms < best) {
                    best = ms;
                    best_cc = cc;
                }
            }
            HDG_HIP_CHECK(hipStreamSynchronize(s));
        }
        c->cell_cells = best_cc;
        if (chosen) {
            chosen->mlp_samples_per_lane = best_spl;
            chosen->rhs_block = best_rb;
            chosen->cell_cells = best_cc;
        }
    });
}

extern "C" int hdg_set_timing(hdg_ctx *c, int32_t enable) {
    if (!c) return HDG_EINVAL;
    return guard([&] {
        HDG_REQUIRE(enable >= 0 && enable <= 64, "timing repeat count must be in 0..64");
        collect_timing(c);
        c->timing = enable != 0;
        c->timing_repeat = enable > 0 ? enable : 1;
        std::memset(c->t_ms, 0, sizeof(c->t_ms));
        std::memset(c->t_launches, 0, sizeof(c->t_launches));
        std::memset(c->t_bytes, 0, sizeof(c->t_bytes));
        std::memset(c->t_blaunch, 0, sizeof(c->t_blaunch));
    });
}

extern "C" int hdg_kernel_stats(hdg_ctx *c, int32_t kernel, int32_t prec, int64_t *launches, double *total_ms,
                                double *bytes_per_launch) {
    if (!c) return HDG_EINVAL;
    return guard([&] {
        HDG_REQUIRE(kernel >= 0 && kernel < HDG_KERNEL_COUNT, "unknown kernel id");
        check_prec(prec);
        collect_timing(c);
        if (launches) *launches = c->t_launches[prec][kernel];
        if (total_ms) *total_ms = c->t_ms[prec][kernel];
        if (bytes_per_launch) {
            // algorithmic bytes at the nrhs of the timed launches: every stored matrix entry
            // once, every vector entry read or written once, indices once
            const double m = c->m, ne = c->n_facet, nk = c->n_cell, nc = c->nc, nt = c->nt;
            const double nb = std::max(1, c->t_nb[prec][kernel]);
            const double sm = prec == HDG_MIXED ? 4.0 : 8.0, st = prec == HDG_MIXED ? 2.0 : 8.0;
            // vector entry sizes of the timed launches (FP32 vectors inside mixed solves)
            const double sx = c->t_sx[prec][kernel] ? c->t_sx[prec][kernel] : 8;
            const double sy = c->t_sy[prec][kernel] ? c->t_sy[prec][kernel] : 8;
            double b = 0;
            switch (kernel) {
            case HDG_KERNEL_APPLY: b = ne * (5 * m * m * sm + 4 * 4) + nb * ne * m * (sx + sy); break;
            case HDG_KERNEL_RESIDUAL: b = ne * (5 * m * m * sm + 4 * 4) + nb * ne * m * (sx + 2 * sy); break;
            case HDG_KERNEL_SWEEP: b = ne * (4 * m * m * st + 4 * 4) + nb * ne * 3 * m * sx; break;
            case HDG_KERNEL_CONDENSE: b = nk * nt * nc * 8 + nb * (nk * nc * 8 + ne * m * 8); break;
            case HDG_KERNEL_RECOVER: b = nk * (nc * nc + nc * nt) * 8 + nb * (nk * 2 * nc * 8 + ne * m * 8); break;
            case HDG_KERNEL_MLP: b = ne * (4 * 4 + 4) + nb * ne * 3 * m * sx; break;
            }
            // launches that stated their own bytes (operands that alias counted once, optional
            // terms only when present): their average
            const int64_t nl = c->t_launches[prec][kernel];
            if (nl > 0 && c->t_blaunch[prec][kernel] == nl) b = c->t_bytes[prec][kernel] / (double)nl;
            *bytes_per_launch = b;
        }
    });
}

extern "C" int hdg_copy(const double *src, double *dst, int64_t n, void *stream) {
    return guard([&] {
        HDG_REQUIRE(src && dst && n >= 0, "bad copy arguments");
        hdg::launch_copy(n, src, dst, as_stream(stream));
        check_launch();
    });
}
