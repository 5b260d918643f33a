// Learned facet-patch smoother: BF16 MFMA inference and training kernels.
//
// Per (facet e, right-hand side r) sample: features are the block-Jacobi
// corrections u = omega D^-1 r of the five facets of e's block row (slot 0 in
// e's direction, slots 1-4 counter-clockwise around the cell they come from),
// normalised by their RMS s; h = ReLU(W1 z) with 64 hidden units, y = W2 h;
// the smoother adds u_e + s y to the iterate.
//
// A wavefront handles 16 samples per tile with v_mfma_f32_16x16x16_bf16
// (lane l holds A[l%16][4(l/16)+v], B[4(l/16)+v][l%16], D[4(l/16)+v][l%16]).
// The first layer is computed transposed, H^T = W1 Z^T, so its accumulators
// are already in the B-operand layout the second layer Y^T = W2 H^T needs;
// in the backward pass dH^T = W2^T dY^T reuses the D layout of Y^T the same
// way.  Only the two weight-gradient products go through 16x16 LDS transposes.
#include "hdg_kernels.h"

namespace hdg {

typedef short s4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short bf_bits(float x) {
    return (short)__bfloat16_as_ushort(__float2bfloat16(x));
}
__device__ __forceinline__ float bf_float(short b) { return __uint_as_float(((unsigned)(unsigned short)b) << 16); }

__device__ __forceinline__ f4_t mfma16(s4_t a, s4_t b, f4_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// Feature k-index layout: slot s (0..4) occupies k = 4 s .. 4 s + 3, node
// j < M at k = 4 s + j (k-indices with j >= M and k >= 20 are zero), so a
// first-layer B operand lane (k = 16 kt + 4 grp + v) reads the nodes of one
// slot, s = 4 kt + grp.  The packed first-layer weights are [64][32] in this
// layout; K1 = 5 M real features enter the RMS.
constexpr int MLP_K1P = 32;

struct MlpWeights {
    s4_t a1[4][2];   // W1 A operands, [hidden tile][k tile]
    s4_t a2[4];      // W2 A operands, [hidden tile]
};

__device__ __forceinline__ void mlp_load_weights(MlpWeights &W, const short *__restrict__ W1b,
                                                 const short *__restrict__ W2b) {
    const int lane = threadIdx.x & 63, col = lane & 15, grp = lane >> 4;
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
            W.a1[mt][kt] = *reinterpret_cast<const s4_t *>(W1b + (16 * mt + col) * MLP_K1P + 16 * kt + 4 * grp);
        W.a2[mt] = *reinterpret_cast<const s4_t *>(W2b + col * 64 + 16 * mt + 4 * grp);
    }
}

template <int M>
struct MlpTile {
    static_assert(M >= 2 && M <= 4, "one slot must fit one 4-wide k group");
    s4_t zb[2];       // normalised features, B layout of the first layer
    f4_t pre[4];      // first-layer pre-activations, D layout
    s4_t hb[4];       // ReLU(pre) in bf16 = B layout of the second layer
    f4_t y;           // second-layer output, D layout (lanes 0-15 hold o = v)
    float s;          // RMS of the sample's features
    int e, r;
    bool valid;
};

// Forward pass of one tile of 16 samples (samp0 .. samp0 + 15).  The
// block-Jacobi corrections are u = y - xi (xi == nullptr: u = y).
template <int M>
__device__ void mlp_forward(MlpTile<M> &T, const MlpWeights &W, int samp0, int nsamp, int ne, int nb,
                            const double *__restrict__ y, const double *__restrict__ xi,
                            const int *__restrict__ nbr, const int8_t *__restrict__ prev) {
    const int lane = threadIdx.x & 63;
    const int col = lane & 15, grp = lane >> 4;
    const int samp = samp0 + col;
    T.valid = samp < nsamp;
    T.e = T.valid ? samp / nb : 0;
    T.r = T.valid ? samp - T.e * nb : 0;
    const size_t NE = (size_t)ne;
    float val[2][4];
    float ss = 0.f;
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) {
        const int slot = 4 * kt + grp;
#pragma unroll
        for (int v = 0; v < 4; ++v) val[kt][v] = 0.f;
        if (T.valid && slot < 5) {
            int id = T.e;
            bool rv = false;
            if (slot > 0) {
                id = nbr[(size_t)(slot - 1) * NE + T.e];
                rv = prev[(size_t)(slot - 1) * NE + T.e] != 0;
            }
            const size_t base = (size_t)id * M * nb + T.r;
            double d[M];
#pragma unroll
            for (int j = 0; j < M; ++j) {
                const size_t o = base + (size_t)j * nb;
                d[j] = xi ? y[o] - xi[o] : y[o];
            }
#pragma unroll
            for (int j = 0; j < M; ++j) {
                val[kt][j] = (float)(rv ? d[M - 1 - j] : d[j]);
                ss += val[kt][j] * val[kt][j];
            }
        }
    }
    ss += __shfl_xor(ss, 16, 64);
    ss += __shfl_xor(ss, 32, 64);
    T.s = sqrtf(ss / (float)(5 * M));
    const float inv = T.s > 0.f ? 1.f / T.s : 0.f;
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
#pragma unroll
        for (int v = 0; v < 4; ++v) T.zb[kt][v] = bf_bits(val[kt][v] * inv);
    // layer 1 (transposed): H^T[16 mt + i][sample] = sum_k W1[16 mt + i][k] z[sample][k]
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        f4_t acc = {0.f, 0.f, 0.f, 0.f};
        acc = mfma16(W.a1[mt][0], T.zb[0], acc);
        acc = mfma16(W.a1[mt][1], T.zb[1], acc);
        T.pre[mt] = acc;
#pragma unroll
        for (int v = 0; v < 4; ++v) T.hb[mt][v] = bf_bits(fmaxf(acc[v], 0.f));
    }
    // layer 2 (transposed): Y^T[o][sample] = sum_h W2[o][h] H^T[h][sample]
    f4_t out = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) out = mfma16(W.a2[mt], T.hb[mt], out);
    T.y = out;
}

// Learned smoothing step: xo = x' + u + s MLP(u-patch), u the block-Jacobi
// correction of the iterate x' = xi + pi qc (xi == nullptr: zero iterate;
// qc == nullptr: no prolongation term).
//
// Each lane gathers the patches of SPL samples itself (16-byte loads at
// nrhs = 1), normalises them and stages the BF16 features in LDS as
// [sample][k]; the wavefront then runs the 64 SPL / 16 tiles through the
// matrix cores with the weights held in registers, parks the outputs in the
// same LDS rows and every lane finishes its own samples.  Only wave-local LDS
// traffic, so no block barrier is needed beyond the wave's own ordering.
constexpr int MLP_ZROW = 40;   // LDS row stride of a sample's features (shorts): 80 B

template <int M, int SPL, bool HAS_X, bool NB1, typename VT>
__global__ __launch_bounds__(256) void k_mlp_smooth(int ne, int nb, const VT *__restrict__ u,
                                                    const VT *__restrict__ xi, const VT *__restrict__ qc,
                                                    const int *__restrict__ fvert, const int *__restrict__ nbr,
                                                    const int8_t *__restrict__ prev, const short *__restrict__ W1b,
                                                    const short *__restrict__ W2b, VT *__restrict__ xo) {
    constexpr int WS = 64 * SPL;   // samples per wavefront
    constexpr int P = M - 1;
    __shared__ short zs[4][WS * MLP_ZROW];
    const int nsamp = ne * nb;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wave = (xcd_block() * blockDim.x + threadIdx.x) >> 6;
    const int wbase = wave * WS;
    if (wbase >= nsamp) return;   // whole wavefront leaves together
    short *Z = zs[w];
    const size_t NE = (size_t)ne, MB = (size_t)M * (NB1 ? 1 : nb);
    float sc[SPL];
    double ue[SPL][M];
    // the iterate (and its prolongation term) is needed only at the end: issue those loads first
    double xe[SPL][M];
    if constexpr (HAS_X) {
#pragma unroll
        for (int q = 0; q < SPL; ++q) {
            const int samp = wbase + q * 64 + lane;
#pragma unroll
            for (int o = 0; o < M; ++o) xe[q][o] = 0.0;
            if (samp < nsamp) {
                const int e = NB1 ? samp : samp / nb, r = NB1 ? 0 : samp - e * nb;
                load_trace<M, NB1>(xi, e * MB + r, nb, xe[q]);
                if (qc) {
                    const double q0 = (double)qc[(size_t)fvert[2 * e] * nb + r];
                    const double q1 = (double)qc[(size_t)fvert[2 * e + 1] * nb + r];
#pragma unroll
                    for (int o = 0; o < M; ++o) xe[q][o] += p1_node<P>(o, q0, q1);
                }
            }
        }
    }
    // gather, normalise, stage
#pragma unroll
    for (int q = 0; q < SPL; ++q) {
        const int ls = q * 64 + lane, samp = wbase + ls;
        float f[5][M];
        float ss = 0.f;
        if (samp < nsamp) {
            const int e = NB1 ? samp : samp / nb, r = NB1 ? 0 : samp - e * nb;
            int id[5];
            bool rv[5];
            id[0] = e;
            rv[0] = false;
#pragma unroll
            for (int k = 1; k < 5; ++k) {
                id[k] = nbr[(size_t)(k - 1) * NE + e];
                rv[k] = prev[(size_t)(k - 1) * NE + e] != 0;
            }
            double d[5][M];
#pragma unroll
            for (int k = 0; k < 5; ++k) load_trace<M, NB1>(u, id[k] * MB + r, nb, d[k]);
#pragma unroll
            for (int j = 0; j < M; ++j) ue[q][j] = d[0][j];
#pragma unroll
            for (int k = 0; k < 5; ++k)
#pragma unroll
                for (int j = 0; j < M; ++j) {
                    f[k][j] = (float)(rv[k] ? d[k][M - 1 - j] : d[k][j]);
                    ss += f[k][j] * f[k][j];
                }
        } else {
#pragma unroll
            for (int k = 0; k < 5; ++k)
#pragma unroll
                for (int j = 0; j < M; ++j) f[k][j] = 0.f;
#pragma unroll
            for (int j = 0; j < M; ++j) ue[q][j] = 0.0;
        }
        const float s = sqrtf(ss / (float)(5 * M));
        const float inv = s > 0.f ? 1.f / s : 0.f;
        sc[q] = s;
        short *row = Z + ls * MLP_ZROW;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            s4_t v;
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = j < M ? bf_bits(f[k][j] * inv) : (short)0;
            *reinterpret_cast<s4_t *>(row + 4 * k) = v;
        }
        const s4_t zero = {0, 0, 0, 0};
#pragma unroll
        for (int k = 5; k < 8; ++k) *reinterpret_cast<s4_t *>(row + 4 * k) = zero;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // network on the matrix cores
    MlpWeights W;
    mlp_load_weights(W, W1b, W2b);
    const int col = lane & 15, grp = lane >> 4;
#pragma unroll
    for (int t = 0; t < WS / 16; ++t) {
        const short *zr = Z + (t * 16 + col) * MLP_ZROW + 4 * grp;
        const s4_t z0 = *reinterpret_cast<const s4_t *>(zr);
        const s4_t z1 = *reinterpret_cast<const s4_t *>(zr + 16);
        s4_t hb[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f4_t acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma16(W.a1[mt][0], z0, acc);
            acc = mfma16(W.a1[mt][1], z1, acc);
#pragma unroll
            for (int v = 0; v < 4; ++v) hb[mt][v] = bf_bits(fmaxf(acc[v], 0.f));
        }
        f4_t out = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) out = mfma16(W.a2[mt], hb[mt], out);
        // the outputs overwrite the first 16 bytes of the sample's own feature row, which
        // this tile has already read
        if (grp == 0) *reinterpret_cast<f4_t *>(Z + (t * 16 + col) * MLP_ZROW) = out;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // finish own samples: xo = x' + u + s out
#pragma unroll
    for (int q = 0; q < SPL; ++q) {
        const int ls = q * 64 + lane, samp = wbase + ls;
        if (samp >= nsamp) continue;
        const int e = NB1 ? samp : samp / nb, r = NB1 ? 0 : samp - e * nb;
        const f4_t out = *reinterpret_cast<const f4_t *>(Z + ls * MLP_ZROW);
        double res[M];
#pragma unroll
        for (int o = 0; o < M; ++o) res[o] = ue[q][o] + (double)(sc[q] * out[o]);
        if constexpr (HAS_X) {
#pragma unroll
            for (int o = 0; o < M; ++o) res[o] += xe[q][o];
        }
        store_trace<M, NB1>(xo, e * MB + r, nb, res);
    }
}

// Four consecutive right-hand sides of one facet per lane (nrhs a multiple
// of 4): the patch gathers become 16-byte (FP32) or 2 x 16-byte (FP64) loads
// of four samples at once.  A wavefront handles 256 samples (16 tiles); the
// per-sample arithmetic (features, RMS, network, combination) is that of
// k_mlp_smooth, so the results are bitwise equal.  128-thread blocks keep the
// staged features of two wavefronts (40 KiB) in LDS.
template <typename T>
__device__ __forceinline__ void load4(const T *__restrict__ p, double (&d)[4]) {
    if constexpr (std::is_same<T, float>::value) {
        const f4_t a = *reinterpret_cast<const f4_t *>(p);
        d[0] = a[0]; d[1] = a[1]; d[2] = a[2]; d[3] = a[3];
    } else {
        typedef double d2_t __attribute__((ext_vector_type(2)));
        const d2_t a = *reinterpret_cast<const d2_t *>(p), b = *reinterpret_cast<const d2_t *>(p + 2);
        d[0] = a.x; d[1] = a.y; d[2] = b.x; d[3] = b.y;
    }
}
template <typename T>
__device__ __forceinline__ void store4(T *__restrict__ p, const double (&d)[4]) {
    if constexpr (std::is_same<T, float>::value) {
        *reinterpret_cast<f4_t *>(p) = f4_t{(float)d[0], (float)d[1], (float)d[2], (float)d[3]};
    } else {
        typedef double d2_t __attribute__((ext_vector_type(2)));
        *reinterpret_cast<d2_t *>(p) = d2_t{d[0], d[1]};
        *reinterpret_cast<d2_t *>(p + 2) = d2_t{d[2], d[3]};
    }
}

template <int M, bool HAS_X, typename VT>
__global__ __launch_bounds__(128) void k_mlp_smooth_r4(int ne, int nb, const VT *__restrict__ u,
                                                       const VT *__restrict__ xi, const VT *__restrict__ qc,
                                                       const int *__restrict__ fvert, const int *__restrict__ nbr,
                                                       const int8_t *__restrict__ prev, const short *__restrict__ W1b,
                                                       const short *__restrict__ W2b, VT *__restrict__ xo) {
    constexpr int WS = 256;   // samples per wavefront
    constexpr int P = M - 1;
    __shared__ short zs[2][WS * MLP_ZROW];
    const int nsamp = ne * nb;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int wave = (xcd_block() * blockDim.x + threadIdx.x) >> 6;
    const int wbase = wave * WS;
    if (wbase >= nsamp) return;   // whole wavefront leaves together
    short *Z = zs[w];
    const size_t NE = (size_t)ne;
    const int s0 = wbase + 4 * lane;   // the lane's four samples s0 .. s0 + 3: one facet, rhs r0 .. r0 + 3
    const bool live = s0 < nsamp;
    const int e = live ? s0 / nb : 0, r0 = live ? s0 - e * nb : 0;
    float sc[4];
    double ue[4][M], xe[4][M];
    if constexpr (HAS_X) {
#pragma unroll
        for (int o = 0; o < M; ++o) {
            double v[4] = {0.0, 0.0, 0.0, 0.0};
            if (live) load4(xi + ((size_t)e * M + o) * nb + r0, v);
#pragma unroll
            for (int q = 0; q < 4; ++q) xe[q][o] = v[q];
        }
        if (qc && live) {
            double q0[4], q1[4];
            load4(qc + (size_t)fvert[2 * e] * nb + r0, q0);
            load4(qc + (size_t)fvert[2 * e + 1] * nb + r0, q1);
#pragma unroll
            for (int q = 0; q < 4; ++q)
#pragma unroll
                for (int o = 0; o < M; ++o) xe[q][o] += p1_node<P>(o, q0[q], q1[q]);
        }
    }
    // gather the patch of the four samples
    float f[4][5][M];
    if (live) {
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            const int id = k == 0 ? e : nbr[(size_t)(k - 1) * NE + e];
            const bool rv = k == 0 ? false : prev[(size_t)(k - 1) * NE + e] != 0;
#pragma unroll
            for (int j = 0; j < M; ++j) {
                double v[4];
                load4(u + ((size_t)id * M + j) * nb + r0, v);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    f[q][k][rv ? M - 1 - j : j] = (float)v[q];
                    if (k == 0) ue[q][j] = v[q];
                }
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
#pragma unroll
            for (int k = 0; k < 5; ++k)
#pragma unroll
                for (int j = 0; j < M; ++j) f[q][k][j] = 0.f;
#pragma unroll
            for (int j = 0; j < M; ++j) ue[q][j] = 0.0;
        }
    }
    // normalise and stage (same order of the RMS sum as k_mlp_smooth)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float ss = 0.f;
#pragma unroll
        for (int k = 0; k < 5; ++k)
#pragma unroll
            for (int j = 0; j < M; ++j) ss += f[q][k][j] * f[q][k][j];
        const float s = sqrtf(ss / (float)(5 * M));
        const float inv = s > 0.f ? 1.f / s : 0.f;
        sc[q] = s;
        short *row = Z + (4 * lane + q) * MLP_ZROW;
#pragma unroll
        for (int k = 0; k < 5; ++k) {
            s4_t v;
#pragma unroll
            for (int j = 0; j < 4; ++j) v[j] = j < M ? bf_bits(f[q][k][j] * inv) : (short)0;
            *reinterpret_cast<s4_t *>(row + 4 * k) = v;
        }
        const s4_t zero = {0, 0, 0, 0};
#pragma unroll
        for (int k = 5; k < 8; ++k) *reinterpret_cast<s4_t *>(row + 4 * k) = zero;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    MlpWeights W;
    mlp_load_weights(W, W1b, W2b);
    const int col = lane & 15, grp = lane >> 4;
#pragma unroll
    for (int t = 0; t < WS / 16; ++t) {
        const short *zr = Z + (t * 16 + col) * MLP_ZROW + 4 * grp;
        const s4_t z0 = *reinterpret_cast<const s4_t *>(zr);
        const s4_t z1 = *reinterpret_cast<const s4_t *>(zr + 16);
        s4_t hb[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            f4_t acc = {0.f, 0.f, 0.f, 0.f};
            acc = mfma16(W.a1[mt][0], z0, acc);
            acc = mfma16(W.a1[mt][1], z1, acc);
#pragma unroll
            for (int v = 0; v < 4; ++v) hb[mt][v] = bf_bits(fmaxf(acc[v], 0.f));
        }
        f4_t out = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) out = mfma16(W.a2[mt], hb[mt], out);
        if (grp == 0) *reinterpret_cast<f4_t *>(Z + (t * 16 + col) * MLP_ZROW) = out;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (!live) return;
    double res[M][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const f4_t out = *reinterpret_cast<const f4_t *>(Z + (4 * lane + q) * MLP_ZROW);
#pragma unroll
        for (int o = 0; o < M; ++o) {
            res[o][q] = ue[q][o] + (double)(sc[q] * out[o]);
            if constexpr (HAS_X) res[o][q] += xe[q][o];
        }
    }
#pragma unroll
    for (int o = 0; o < M; ++o) store4(xo + ((size_t)e * M + o) * nb + r0, res[o]);
}

// Loss and weight gradients over all (facet, rhs) samples of one data set.
// Targets t are normalised per sample by s.  Every block runs the same
// number of tile iterations (tiles past the end contribute nothing) so the
// block barriers around the LDS transposes are uniform.  Per-wave partial
// sums: dW1 [64][K1P], dW2 [16][64] (unscaled: d = 2 (y - t/s)), loss.
template <int M>
__global__ __launch_bounds__(256) void k_mlp_grad(int ne, int nb, const double *__restrict__ u,
                                                  const double *__restrict__ t, const int *__restrict__ nbr,
                                                  const int8_t *__restrict__ prev, const short *__restrict__ W1b,
                                                  const short *__restrict__ W2b, int iters,
                                                  float *__restrict__ pdW1, float *__restrict__ pdW2,
                                                  float *__restrict__ ploss) {
    constexpr int KT = 2, K1P = MLP_K1P;
    __shared__ unsigned short lds[4][4 + KT + 1 + 4][256];
    const int nsamp = ne * nb;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int col = lane & 15, grp = lane >> 4;
    const int wid = blockIdx.x * 4 + w;
    const int nwaves = gridDim.x * 4;
    unsigned short(*Tdh)[256] = &lds[w][0];
    unsigned short(*Tz)[256] = &lds[w][4];
    unsigned short *Tdy = lds[w][4 + KT];
    unsigned short(*Th)[256] = &lds[w][4 + KT + 1];

    f4_t g1[4][KT], g2[4];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
        g2[mt] = f4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kt = 0; kt < KT; ++kt) g1[mt][kt] = f4_t{0.f, 0.f, 0.f, 0.f};
    }
    float lsum = 0.f;
    MlpWeights W;
    mlp_load_weights(W, W1b, W2b);

    for (int it = 0; it < iters; ++it) {
        const int tile = wid + it * nwaves;
        MlpTile<M> T;
        mlp_forward<M>(T, W, tile * 16, nsamp, ne, nb, u, nullptr, nbr, prev);
        // d = 2 (y - t/s) on the M valid outputs (lanes 0-15 hold o = v)
        s4_t dyb;
        {
            const float inv = T.s > 0.f ? 1.f / T.s : 0.f;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                float d = 0.f;
                if (grp == 0 && v < M && T.valid) {
                    const float tau = (float)t[((size_t)T.e * M + v) * nb + T.r] * inv;
                    const float diff = T.y[v] - tau;
                    lsum += diff * diff;
                    d = 2.f * diff;
                }
                dyb[v] = bf_bits(d);
            }
        }
        // dH^T = W2^T dY^T, masked by ReLU'
        s4_t dhb[4];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            s4_t a;
#pragma unroll
            for (int v = 0; v < 4; ++v) a[v] = W2b[(size_t)(4 * grp + v) * 64 + 16 * mt + col];
            const f4_t dh = mfma16(a, dyb, f4_t{0.f, 0.f, 0.f, 0.f});
#pragma unroll
            for (int v = 0; v < 4; ++v) dhb[mt][v] = bf_bits(T.pre[mt][v] > 0.f ? dh[v] : 0.f);
        }
        // stage D-layout tiles (row = 4 grp + v, column = sample) for the transposes
        __syncthreads();
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int o = (4 * grp + v) * 16 + col;
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) {
                Tdh[mt][o] = (unsigned short)dhb[mt][v];
                Th[mt][o] = (unsigned short)T.hb[mt][v];
            }
#pragma unroll
            for (int kt = 0; kt < KT; ++kt) Tz[kt][o] = (unsigned short)T.zb[kt][v];
            Tdy[o] = (unsigned short)dyb[v];
        }
        __syncthreads();
        // read back as [row = lane % 16][sample = 4 grp + v]
        const int ib = col * 16 + 4 * grp;
        s4_t dyA;
#pragma unroll
        for (int v = 0; v < 4; ++v) dyA[v] = (short)Tdy[ib + v];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
            s4_t dhA, hB;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                dhA[v] = (short)Tdh[mt][ib + v];
                hB[v] = (short)Th[mt][ib + v];
            }
            // dW2[o][16 mt + h] += sum_s dY^T[o][s] H[s][h]
            g2[mt] = mfma16(dyA, hB, g2[mt]);
#pragma unroll
            for (int kt = 0; kt < KT; ++kt) {
                s4_t zB;
#pragma unroll
                for (int v = 0; v < 4; ++v) zB[v] = (short)Tz[kt][ib + v];
                // dW1[16 mt + h][16 kt + k] += sum_s dH^T[h][s] Z[s][k]
                g1[mt][kt] = mfma16(dhA, zB, g1[mt][kt]);
            }
        }
    }
    // per-wave partials
#pragma unroll
    for (int mt = 0; mt < 4; ++mt) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
#pragma unroll
            for (int kt = 0; kt < KT; ++kt)
                pdW1[(size_t)wid * 64 * K1P + (size_t)(16 * mt + 4 * grp + v) * K1P + 16 * kt + col] = g1[mt][kt][v];
            pdW2[(size_t)wid * 16 * 64 + (size_t)(4 * grp + v) * 64 + 16 * mt + col] = g2[mt][v];
        }
    }
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off, 64);
    if (lane == 0) ploss[wid] = lsum;
}

// Sum of the per-wave partials: g[i] for i < n1 + n2, and the loss (index
// n1 + n2).  A block reduces 64 consecutive entries with 16 thread rows, each
// row summing every 16th wave (coalesced over the 64 entries), then the 16
// row sums in a fixed order.
__global__ __launch_bounds__(1024) void k_mlp_reduce(int nwaves, int n1, int n2, const float *__restrict__ p1,
                                                     const float *__restrict__ p2, const float *__restrict__ pl,
                                                     float *__restrict__ g, double *__restrict__ loss) {
    __shared__ double part[16][64];
    const int i = blockIdx.x * 64 + threadIdx.x, row = threadIdx.y;
    double sum = 0.0;
    if (i < n1) {
        for (int w = row; w < nwaves; w += 16) sum += p1[(size_t)w * n1 + i];
    } else if (i < n1 + n2) {
        for (int w = row; w < nwaves; w += 16) sum += p2[(size_t)w * n2 + (i - n1)];
    } else if (i == n1 + n2) {
        for (int w = row; w < nwaves; w += 16) sum += pl[w];
    }
    part[row][threadIdx.x] = sum;
    __syncthreads();
    if (row == 0) {
        double t = 0.0;
        for (int r = 0; r < 16; ++r) t += part[r][threadIdx.x];
        if (i < n1 + n2) g[i] = (float)t;
        else if (i == n1 + n2) loss[0] = t;
    }
}

// Adam on the FP32 master weights [W1 (64 x K1P) | W2 (16 x 64)] with the
// gradient g scaled by gscale; entries outside the real (64 x 5m, m x 64)
// blocks stay zero.  Refreshes the BF16 copies.
__global__ void k_adam(int n1, int n2, int k1p, int m, const float *__restrict__ g, float gscale,
                       float *__restrict__ w, float *__restrict__ m1, float *__restrict__ m2, float lr, float b1,
                       float b2, float eps, float c1, float c2, short *__restrict__ wb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n1 + n2) return;
    bool live;
    if (i < n1) {
        const int k = i % k1p;   // slot-aligned feature layout: k = 4 slot + node
        live = k < 20 && (k & 3) < m;
    } else {
        live = ((i - n1) / 64) < m;
    }
    if (live) {
        const float gi = g[i] * gscale;
        const float a = b1 * m1[i] + (1.f - b1) * gi;
        const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
        m1[i] = a;
        m2[i] = b;
        w[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
    } else {
        w[i] = 0.f;
    }
    wb[i] = bf_bits(w[i]);
}

__global__ void k_to_bf16(int n, const float *__restrict__ w, short *__restrict__ wb) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) wb[i] = bf_bits(w[i]);
}

// x[e][k] += (1 - k/p) qc[v0] + (k/p) qc[v1]  (prolongation pi of a P1 vector)
template <int M>
__global__ void k_prolong_trace(int ne, int nb, const int *__restrict__ fvert, const double *__restrict__ qc,
                                double *__restrict__ x) {
    constexpr int P = M - 1;
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ne * nb) return;
    const int e = t / nb, r = t - e * nb;
    const double q0 = qc[(size_t)fvert[2 * e] * nb + r], q1 = qc[(size_t)fvert[2 * e + 1] * nb + r];
#pragma unroll
    for (int k = 0; k < M; ++k) x[((size_t)e * M + k) * nb + r] += p1_node<P>(k, q0, q1);
}

// out = a x + b y + c z (elementwise)
template <typename VT>
__global__ void k_lin3(int64_t n, double a, const VT *__restrict__ x, double b, const VT *__restrict__ y, double c,
                       const VT *__restrict__ z, VT *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = (VT)(a * (double)x[i] + (y ? b * (double)y[i] : 0.0) + (z ? c * (double)z[i] : 0.0));
}

#define GRIDL(n, b) dim3((unsigned)(((n) + (b) - 1) / (b))), dim3(b)

template <typename VT>
void launch_mlp_smooth(int p, int ne, int nb, int spl, const VT *u, const VT *xi, const double *qc,
                       const int *fvert, const int *nbr, const int8_t *prev, const short *W1b, const short *W2b,
                       VT *xo, hipStream_t s) {
    const VT *qv = reinterpret_cast<const VT *>(qc);   // P1 values in the smoother's vector type
    if (spl == 4 && nb % 4 == 0) {
        const int64_t waves = ((int64_t)ne * nb + 255) / 256;
        const dim3 grid((unsigned)(((waves + 1) / 2 + 7) / 8 * 8)), block(128);   // multiple of 8 for the XCD remap
#define MR(M, X) \
    hipLaunchKernelGGL((k_mlp_smooth_r4<M, X, VT>), grid, block, 0, s, ne, nb, u, xi, qv, fvert, nbr, prev, W1b, W2b, xo)
#define MR_X(M)                  \
    if (xi) MR(M, true);         \
    else MR(M, false);
        switch (p) { case 1: MR_X(2) break; case 2: MR_X(3) break; case 3: MR_X(4) break; }
#undef MR_X
#undef MR
        return;
    }
    spl = spl == 2 ? 2 : 1;   // 4 without a multiple of 4 right-hand sides: one sample per lane
    const int64_t waves = ((int64_t)ne * nb + 64 * spl - 1) / (64 * spl);
    const int64_t blocks = (waves + 3) / 4;
    const dim3 grid((unsigned)(((blocks + 7) / 8) * 8)), block(256);   // multiple of 8 for the XCD remap
    const bool hx = xi != nullptr, n1 = nb == 1;
#define MS(M, S, X, N) \
    hipLaunchKernelGGL((k_mlp_smooth<M, S, X, N, VT>), grid, block, 0, s, ne, nb, u, xi, qv, fvert, nbr, prev, W1b, W2b, xo)
#define MS_XN(M, S)                          \
    if (hx) {                                \
        if (n1) MS(M, S, true, true);        \
        else MS(M, S, true, false);          \
    } else {                                 \
        if (n1) MS(M, S, false, true);       \
        else MS(M, S, false, false);         \
    }
#define MS_P(S)                              \
    switch (p) {                             \
    case 1: MS_XN(2, S) break;               \
    case 2: MS_XN(3, S) break;               \
    case 3: MS_XN(4, S) break;               \
    }
    if (spl == 1) { MS_P(1) } else { MS_P(2) }
#undef MS_P
#undef MS_XN
#undef MS
}
template void launch_mlp_smooth<double>(int, int, int, int, const double *, const double *, const double *, const int *,
                                        const int *, const int8_t *, const short *, const short *, double *,
                                        hipStream_t);
template void launch_mlp_smooth<float>(int, int, int, int, const float *, const float *, const double *, const int *,
                                       const int *, const int8_t *, const short *, const short *, float *,
                                       hipStream_t);

int mlp_k1p(int) { return MLP_K1P; }

int mlp_grad_waves(int ne, int nb) {
    const int64_t tiles = ((int64_t)ne * nb + 15) / 16;
    int64_t blocks = (tiles + 3) / 4;
    if (blocks > 256) blocks = 256;
    return (int)blocks * 4;
}

void launch_mlp_grad(int p, int ne, int nb, const double *u, const double *t, const int *nbr, const int8_t *prev,
                     const short *W1b, const short *W2b, float *pdW1, float *pdW2, float *ploss, float *g,
                     double *loss, hipStream_t s) {
    const int nw = mlp_grad_waves(ne, nb);
    const int64_t tiles = ((int64_t)ne * nb + 15) / 16;
    const int iters = (int)((tiles + nw - 1) / nw);
    const dim3 grid(nw / 4), block(256);
    switch (p) {
    case 1: hipLaunchKernelGGL(k_mlp_grad<2>, grid, block, 0, s, ne, nb, u, t, nbr, prev, W1b, W2b, iters, pdW1, pdW2, ploss); break;
    case 2: hipLaunchKernelGGL(k_mlp_grad<3>, grid, block, 0, s, ne, nb, u, t, nbr, prev, W1b, W2b, iters, pdW1, pdW2, ploss); break;
    case 3: hipLaunchKernelGGL(k_mlp_grad<4>, grid, block, 0, s, ne, nb, u, t, nbr, prev, W1b, W2b, iters, pdW1, pdW2, ploss); break;
    }
    const int n1 = 64 * mlp_k1p(p), n2 = 16 * 64;
    hipLaunchKernelGGL(k_mlp_reduce, dim3((unsigned)((n1 + n2 + 1 + 63) / 64)), dim3(64, 16), 0, s, nw, n1, n2, pdW1,
                       pdW2, ploss, g, loss);
}

void launch_adam(int p, const float *g, float gscale, float *w, float *m1, float *m2, float lr, int step,
                 short *wb, hipStream_t s) {
    const int k1p = mlp_k1p(p), n1 = 64 * k1p, n2 = 16 * 64;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, GRIDL(n1 + n2, 256), 0, s, n1, n2, k1p, p + 1, g, gscale, w, m1, m2, lr,
                       b1, b2, 1e-8f, c1, c2, wb);
}

void launch_to_bf16(int n, const float *w, short *wb, hipStream_t s) {
    hipLaunchKernelGGL(k_to_bf16, GRIDL(n, 256), 0, s, n, w, wb);
}

void launch_prolong_trace(int p, int ne, int nb, const int *fvert, const double *qc, double *x, hipStream_t s) {
    switch (p) {
    case 1: hipLaunchKernelGGL(k_prolong_trace<2>, GRIDL(ne * nb, 256), 0, s, ne, nb, fvert, qc, x); break;
    case 2: hipLaunchKernelGGL(k_prolong_trace<3>, GRIDL(ne * nb, 256), 0, s, ne, nb, fvert, qc, x); break;
    case 3: hipLaunchKernelGGL(k_prolong_trace<4>, GRIDL(ne * nb, 256), 0, s, ne, nb, fvert, qc, x); break;
    }
}

template <typename VT>
void launch_lin3(int64_t n, double a, const VT *x, double b, const VT *y, double c, const VT *z, VT *out,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_lin3<VT>, GRIDL(n, 256), 0, s, n, a, x, b, y, c, z, out);
}
template void launch_lin3<double>(int64_t, double, const double *, double, const double *, double, const double *,
                                  double *, hipStream_t);
template void launch_lin3<float>(int64_t, double, const float *, double, const float *, double, const float *,
                                 float *, hipStream_t);

}  // namespace hdg
