// Bandwidth probes for the measured side of the roofline: STREAM's triad
// a = b + s c and a read-only pass that sums its input by chunks.  They are
// not part of a solve.
//
// Each block owns one contiguous chunk of STREAM_CHUNK doubles.  A lane moves
// 16-byte double2 words and issues all of its STREAM_UNROLL loads per array
// before the first use, so a wave keeps 64 lanes x 4 x 16 B = 4 KiB per array
// in flight; consecutive lanes touch consecutive words (fully coalesced).  The
// last, ragged chunk falls back to scalar accesses.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hdg_internal.h"

namespace hdg {
namespace {

constexpr int STREAM_BLOCK = 256;
constexpr int STREAM_UNROLL = 4;
constexpr int64_t STREAM_CHUNK = (int64_t)STREAM_BLOCK * STREAM_UNROLL * 2;  // doubles per block

__global__ __launch_bounds__(STREAM_BLOCK) void k_stream_triad(int64_t n, const double *__restrict__ b,
                                                                 const double *__restrict__ c, double s,
                                                                 double *__restrict__ a) {
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * STREAM_CHUNK;
    if (base + STREAM_CHUNK <= n) {
        const double2 *b2 = reinterpret_cast<const double2 *>(b + base);
        const double2 *c2 = reinterpret_cast<const double2 *>(c + base);
        double2 *a2 = reinterpret_cast<double2 *>(a + base);
        double2 x[STREAM_UNROLL], y[STREAM_UNROLL];
#pragma unroll
        for (int u = 0; u < STREAM_UNROLL; ++u) {
            x[u] = b2[u * STREAM_BLOCK + tid];
            y[u] = c2[u * STREAM_BLOCK + tid];
        }
#pragma unroll
        for (int u = 0; u < STREAM_UNROLL; ++u)
            a2[u * STREAM_BLOCK + tid] = make_double2(x[u].x + s * y[u].x, x[u].y + s * y[u].y);
    } else {
        for (int64_t i = base + tid; i < n; i += STREAM_BLOCK) a[i] = b[i] + s * c[i];
    }
}

__global__ __launch_bounds__(STREAM_BLOCK) void k_stream_read(int64_t n, const double *__restrict__ src,
                                                                double *__restrict__ partial) {
    __shared__ double red[STREAM_BLOCK / 64];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * STREAM_CHUNK;
    double acc = 0.0;
    if (base + STREAM_CHUNK <= n) {
        const double2 *s2 = reinterpret_cast<const double2 *>(src + base);
        double2 x[STREAM_UNROLL];
#pragma unroll
        for (int u = 0; u < STREAM_UNROLL; ++u) x[u] = s2[u * STREAM_BLOCK + tid];
#pragma unroll
        for (int u = 0; u < STREAM_UNROLL; ++u) acc += x[u].x + x[u].y;
    } else {
        for (int64_t i = base + tid; i < n; i += STREAM_BLOCK) acc += src[i];
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_down(acc, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < STREAM_BLOCK / 64; ++w) t += red[w];
        partial[blockIdx.x] = t;
    }
}

int64_t read_blocks(int64_t n) { return n > 0 ? (n + STREAM_CHUNK - 1) / STREAM_CHUNK : 0; }

bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

bool overlap(const double *p, int64_t np, const double *q, int64_t nq) {
    return np > 0 && nq > 0 && p < q + nq && q < p + np;
}

}  // namespace
}  // namespace hdg

extern "C" int64_t hdg_stream_read_blocks(int64_t n) { return hdg::read_blocks(n); }

extern "C" int hdg_stream_triad(const double *b, const double *c, double s, double *a, int64_t n, void *stream) {
    return hdg::guarded([&] {
        HDG_REQUIRE(n >= 0, "n must be >= 0");
        if (n == 0) return;
        HDG_REQUIRE(a && b && c, "a, b and c must not be NULL");
        HDG_REQUIRE(hdg::aligned16(a) && hdg::aligned16(b) && hdg::aligned16(c), "arrays must be 16-byte aligned");
        HDG_REQUIRE(!hdg::overlap(a, n, b, n) && !hdg::overlap(a, n, c, n), "a must not overlap b or c");
        const int64_t blocks = hdg::read_blocks(n);
        HDG_REQUIRE(blocks <= 0x7fffffff, "n too large");
        hipLaunchKernelGGL(hdg::k_stream_triad, dim3((unsigned)blocks), dim3(hdg::STREAM_BLOCK), 0,
                           reinterpret_cast<hipStream_t>(stream), n, b, c, s, a);
        hdg::check_kernel_launch();
    });
}

extern "C" int hdg_stream_read(const double *src, int64_t n, double *partial, int64_t n_partial, void *stream) {
    return hdg::guarded([&] {
        HDG_REQUIRE(n >= 0, "n must be >= 0");
        if (n == 0) return;
        HDG_REQUIRE(src && partial, "src and partial must not be NULL");
        HDG_REQUIRE(hdg::aligned16(src), "src must be 16-byte aligned");
        const int64_t blocks = hdg::read_blocks(n);
        HDG_REQUIRE(n_partial >= blocks, "partial is shorter than hdg_stream_read_blocks(n)");
        HDG_REQUIRE(!hdg::overlap(src, n, partial, blocks), "partial must not overlap src");
        HDG_REQUIRE(blocks <= 0x7fffffff, "n too large");
        hipLaunchKernelGGL(hdg::k_stream_read, dim3((unsigned)blocks), dim3(hdg::STREAM_BLOCK), 0,
                           reinterpret_cast<hipStream_t>(stream), n, src, partial);
        hdg::check_kernel_launch();
    });
}
