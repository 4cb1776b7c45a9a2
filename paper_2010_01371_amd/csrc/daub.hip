// Orthonormal full-depth 2D Daubechies-4 transform (periodised), the other
// unitary U_DWT the wavelet preconditioner section names beside Haar, in place
// on [K][n][n] images.  Same layout as the Haar transform: at each level the
// block [0:m, 0:m] goes along rows, then along columns, down to 1 x 1; the
// inverse undoes the levels from the coarsest, columns then rows.
//
// One level along a line of even length m (power of two here):
//   lo_i = sum_k h_k x_{(2i+k) mod m},  hi_i = sum_k g_k x_{(2i+k) mod m},
// lo at i and hi at m/2 + i; the inverse x_j collects the two taps of each
// half that land on j.  h = (1 + r3, 3 + r3, 3 - r3, 1 - r3) / (4 r2),
// g_k = (-1)^k h_{3-k}.
//
// Levels with m > kCoarse run as two out-of-place launches each (rows into a
// scratch image, columns back), one thread per output; the levels from
// kCoarse down run in one workgroup per channel, entirely in LDS.  The work is
// L2/latency-bound: 8 bytes per coefficient per level pass.
#include <algorithm>
#include <cmath>

#include "internal.h"

namespace mbmd {

namespace {

constexpr int kThreads = 256;
constexpr int kCoarse = 64;                     // coarse levels: kCoarse^2 floats x 2 in LDS
constexpr int kCoarseThreads = 1024;

struct D4Filter {
    float h[4], g[4];
};

D4Filter d4_filter() {
    const double r3 = std::sqrt(3.0), s = 4.0 * std::sqrt(2.0);
    const double h[4] = {(1.0 + r3) / s, (3.0 + r3) / s, (3.0 - r3) / s, (1.0 - r3) / s};
    D4Filter f;
    for (int k = 0; k < 4; ++k) {
        f.h[k] = (float)h[k];
        f.g[k] = (float)((k & 1 ? -1.0 : 1.0) * h[3 - k]);
    }
    return f;
}

// Output t (t < m) of one level along a line whose m values are src[0..m) at
// the given stride: forward, lo_t for t < m/2 and hi_{t - m/2} above; inverse,
// x_t.
__device__ __forceinline__ float d4_line(const D4Filter& f, const float* src, int stride, int m, int t,
                                         bool inverse) {
    const int h = m >> 1;
    if (!inverse) {
        const bool hi = t >= h;
        const int i = hi ? t - h : t;
        float acc = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) acc = fmaf(hi ? f.g[k] : f.h[k], src[((2 * i + k) & (m - 1)) * stride], acc);
        return acc;
    }
    const int p = t & 1, i0 = t >> 1, i1 = (i0 + h - 1) & (h - 1);     // taps p and p + 2
    float acc = f.h[p] * src[i0 * stride];
    acc = fmaf(f.g[p], src[(h + i0) * stride], acc);
    acc = fmaf(f.h[p + 2], src[i1 * stride], acc);
    acc = fmaf(f.g[p + 2], src[(h + i1) * stride], acc);
    return acc;
}

// One pass of one level over block [0:m, 0:m] of every channel, out of place
// (src and dst [K][n][n], only the block is written): along rows or along
// columns, one thread per output, consecutive threads on consecutive columns.
__global__ __launch_bounds__(kThreads) void k_d4_pass(D4Filter f, int n, int m, int along_rows, int inverse,
                                                       const float* __restrict__ src, float* __restrict__ dst,
                                                       const long long* __restrict__ zd) {
    {                                                      // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        src = zadd(src, d);
        dst = zadd(dst, d);
    }
    const int t = blockIdx.x * kThreads + threadIdx.x;
    if (t >= m * m) return;
    const int r = t / m, c = t - r * m;
    const size_t base = (size_t)blockIdx.y * n * n;
    dst[base + (size_t)r * n + c] = along_rows ? d4_line(f, src + base + (size_t)r * n, 1, m, c, inverse != 0)
                                               : d4_line(f, src + base + c, n, m, r, inverse != 0);
}

// The levels m <= T of channel blockIdx.x (T = min(n, kCoarse)), in LDS:
// forward from m = T down to 2, inverse from 2 up to T.  Each level's first
// pass goes A -> B and its second B -> A, so a level ends in A; entries of B
// outside the current block are stale but never read.
__global__ __launch_bounds__(kCoarseThreads) void k_d4_coarse(D4Filter f, int n, int T, int inverse,
                                                             float* __restrict__ a,
                                                             const long long* __restrict__ zd) {
    __shared__ float A[kCoarse * kCoarse], B[kCoarse * kCoarse];
    a = zadd(a, zoff(zd, Z_BLOCK));                        // batched: this slice's buffer
    float* img = a + (size_t)blockIdx.x * n * n;
    for (int t = threadIdx.x; t < T * T; t += kCoarseThreads) A[t] = img[(size_t)(t / T) * n + t % T];
    __syncthreads();
    for (int m = inverse ? 2 : T; inverse ? m <= T : m >= 2; m = inverse ? 2 * m : m / 2) {
        for (int pass = 0; pass < 2; ++pass) {
            // forward: rows then columns; inverse: columns then rows
            const bool along_rows = (pass == 0) != (inverse != 0);
            const float* src = pass == 0 ? A : B;
            float* dst = pass == 0 ? B : A;
            for (int t = threadIdx.x; t < m * m; t += kCoarseThreads) {
                const int r = t / m, c = t - r * m;
                dst[r * T + c] = along_rows ? d4_line(f, src + r * T, 1, m, c, inverse != 0)
                                            : d4_line(f, src + c, T, m, r, inverse != 0);
            }
            __syncthreads();
        }
    }
    for (int t = threadIdx.x; t < T * T; t += kCoarseThreads) img[(size_t)(t / T) * n + t % T] = A[t];
}

void check(int n) {
    MBMD_REQUIRE(n >= 2 && (n & (n - 1)) == 0, MBMD_ERR_SHAPE,
                 "the Daubechies preconditioner needs a square power-of-two image");
}

// One level: forward rows x -> y, columns y -> x; inverse columns, then rows.
void level(const D4Filter& f, int K, int n, int m, bool inverse, float* x, float* y, hipStream_t s) {
    for (int pass = 0; pass < 2; ++pass) {
        const bool rows = (pass == 0) != inverse;
        KernelTimer kt_("k_d4_pass", s);
        hipLaunchKernelGGL(k_d4_pass, zgrid(dim3((m * m + kThreads - 1) / kThreads, K)), dim3(kThreads), 0, s, f, n,
                           m, rows ? 1 : 0, inverse ? 1 : 0, pass == 0 ? x : y, pass == 0 ? y : x, zarg());
        kt_.stop();
        MBMD_LAUNCHED();
    }
}

void coarse(const D4Filter& f, int K, int n, bool inverse, float* a, hipStream_t s) {
    {
        KernelTimer kt_("k_d4_coarse", s);
        hipLaunchKernelGGL(k_d4_coarse, zgrid(dim3(K)), dim3(kCoarseThreads), 0, s, f, n, std::min(n, kCoarse),
                           inverse ? 1 : 0, a, zarg());
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

}  // namespace

void launch_d4_forward(int K, int n, const float* in, const float* M, float* coef, float* scratch, hipStream_t s) {
    check(n);
    MBMD_REQUIRE(in != coef && scratch != coef && scratch != in, MBMD_ERR_ARG,
                 "the Daubechies transform needs distinct in, coef and scratch");
    const D4Filter f = d4_filter();
    if (M) launch_block_apply(n * n, K, M, in, coef, 1.0f, s);
    else launch_scale_copy(K * n * n, in, coef, 1.0f, s);
    for (int m = n; m > kCoarse; m /= 2) level(f, K, n, m, false, coef, scratch, s);
    coarse(f, K, n, false, coef, s);
}

void launch_d4_inverse(int K, int n, float* coef, const float* M, float* out, float out_sign, float* scratch,
                       hipStream_t s) {
    check(n);
    MBMD_REQUIRE(out != coef && scratch != coef, MBMD_ERR_ARG,
                 "the Daubechies inverse works in coef (with scratch), then writes out");
    const D4Filter f = d4_filter();
    coarse(f, K, n, true, coef, s);
    for (int m = 2 * std::min(n, kCoarse); m <= n; m *= 2) level(f, K, n, m, true, coef, scratch, s);
    if (M) launch_block_apply(n * n, K, M, coef, out, out_sign, s);
    else launch_scale_copy(K * n * n, coef, out, out_sign, s);
}

int launch_d4_apply(int K, int n, const float* in, const float* M, const float* Dinv, float* coef, float* out,
                    float out_sign, const float* g, double* partials, hipStream_t s) {
    launch_d4_forward(K, n, in, M, coef, out, s);            // out is written last: scratch until then
    launch_block_apply(n * n, K, Dinv, coef, coef, 1.0f, s);
    launch_d4_inverse(K, n, coef, M, out, out_sign, out, s);
    return partials ? launch_dot(K * n * n, g, out, partials, s) : 0;
}

}  // namespace mbmd
