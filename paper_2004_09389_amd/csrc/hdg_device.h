// Device helpers shared by the kernel sources (gfx950): storage of the
// facet-row matrices in 16-byte groups and the local trace numbering of a cell.
#pragma once

#include <type_traits>

#include "hdg_kernels.h"

namespace hdg {

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ double ldm(const double *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ldm(const float *p) { return __builtin_nontemporal_load(p); }
__device__ __forceinline__ float ldm(const __hip_bfloat16 *p) { return __bfloat162float(*p); }

template <typename MT> struct Acc { using type = float; };
template <> struct Acc<double> { using type = double; };

// Facet-row matrices are stored as [component / V][n_facet][V] with V the
// number of entries in 16 bytes (2 FP64, 4 FP32, 8 BF16), components padded
// with zeros to a multiple of V: a lane fetches V consecutive components of
// its facet with one 16-byte load and a wavefront reads 1 KiB contiguously.
__host__ __device__ constexpr int padded(int c, int v) { return (c + v - 1) / v * v; }
__device__ __forceinline__ size_t widx(int c, int e, size_t ne, int v) {
    return ((size_t)(c / v) * ne + e) * v + (c % v);
}


typedef double dbl2_t __attribute__((ext_vector_type(2)));
typedef float flt4_t __attribute__((ext_vector_type(4)));
typedef unsigned u32x4_t __attribute__((ext_vector_type(4)));

template <typename MT> struct Wide;
template <> struct Wide<double> {
    static constexpr int V = 2;
    __device__ static void load(const double *p, double (&o)[2]) {
        const dbl2_t v = __builtin_nontemporal_load(reinterpret_cast<const dbl2_t *>(p));
        o[0] = v.x; o[1] = v.y;
    }
};
template <> struct Wide<float> {
    static constexpr int V = 4;
    __device__ static void load(const float *p, float (&o)[4]) {
        const flt4_t v = __builtin_nontemporal_load(reinterpret_cast<const flt4_t *>(p));
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    }
};
template <> struct Wide<__hip_bfloat16> {
    static constexpr int V = 8;
    __device__ static void load(const __hip_bfloat16 *p, float (&o)[8]) {
        const u32x4_t v = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t *>(p));
        const unsigned w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            o[2 * i] = __uint_as_float(w[i] << 16);
            o[2 * i + 1] = __uint_as_float(w[i] & 0xffff0000u);
        }
    }
};

// Local trace index of trace unknown a (0 <= a < NU m: component a / m, node
// a % m in the facet's direction) of local facet i, for a cell that runs
// along (rev = 0) or against (rev = 1) the facet's direction.
template <int P, int NU>
__device__ __forceinline__ int loc_trace(int i, int a, int rev) {
    constexpr int m = P + 1;
    const int k = a % m;
    return i * NU * m + (a - k) + (rev ? P - k : k);
}

// Sum init + f(0) + ... + f(cnt - 1) in that order, U terms at a time: the U
// calls of a group are made first (index clamped into the list) so that their
// loads are in flight together, then the live ones are added.  For gathers
// whose row length is known only at run time.
template <int U, typename F>
__device__ __forceinline__ double acc_row(double init, int cnt, F &&f) {
    double s = init;
    for (int k0 = 0; k0 < cnt; k0 += U) {
        double t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) t[u] = f(min(k0 + u, cnt - 1));
#pragma unroll
        for (int u = 0; u < U; ++u) s = k0 + u < cnt ? s + t[u] : s;
    }
    return s;
}

}  // namespace hdg
