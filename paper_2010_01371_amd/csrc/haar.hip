// Orthonormal full-depth 2D Haar transform (the U_DWT of the wavelet and
// cross-material wavelet sections) in the standard (Mallat) layout: each
// level transforms the current low-pass block along rows then columns, pairs
// (2i, 2i+1) -> ((a+b), (a-b)) / sqrt 2, lows first.
//
// Levels 1..log2(T) only involve pixels of one T x T tile (T = 32), so one
// workgroup per tile runs them in LDS and writes its detail coefficients
// straight to their global positions; the tiles' final low-pass values form
// an (n/T) x (n/T) coarse image whose remaining levels one workgroup
// finishes.  The inverse runs the same two stages backwards.
#include <cmath>

#include "internal.h"

namespace mbmd {

namespace {

constexpr int kThreads = 256;
constexpr int kTile = 32;
constexpr float kR2 = 0.70710678118654752440f;

__device__ __forceinline__ double block_sum(double v, double* sh) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[wv] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0) {
        const int nw = (blockDim.x + 63) >> 6;
        for (int i = 0; i < nw; ++i) t += sh[i];
    }
    return t;
}

// One forward level on cur[k][0:m][0:m] (row stride T); result back in cur.
__device__ void level_forward(float* cur, float* nxt, int K, int T, int m) {
    const int h = m >> 1;
    const int tot = K * m * h;
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int i = idx % h, r = (idx / h) % m, k = idx / (m * h);
        const float a = cur[(k * T + r) * T + 2 * i], b = cur[(k * T + r) * T + 2 * i + 1];
        nxt[(k * T + r) * T + i] = (a + b) * kR2;
        nxt[(k * T + r) * T + h + i] = (a - b) * kR2;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int c = idx % m, i = (idx / m) % h, k = idx / (m * h);
        const float a = nxt[(k * T + 2 * i) * T + c], b = nxt[(k * T + 2 * i + 1) * T + c];
        cur[(k * T + i) * T + c] = (a + b) * kR2;
        cur[(k * T + h + i) * T + c] = (a - b) * kR2;
    }
    __syncthreads();
}

// One inverse level producing cur[k][0:m][0:m] from its four quadrants.
__device__ void level_inverse(float* cur, float* nxt, int K, int T, int m) {
    const int h = m >> 1;
    const int tot = K * m * h;
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int c = idx % m, i = (idx / m) % h, k = idx / (m * h);
        const float lo = cur[(k * T + i) * T + c], hi = cur[(k * T + h + i) * T + c];
        nxt[(k * T + 2 * i) * T + c] = (lo + hi) * kR2;
        nxt[(k * T + 2 * i + 1) * T + c] = (lo - hi) * kR2;
    }
    __syncthreads();
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int i = idx % h, r = (idx / h) % m, k = idx / (m * h);
        const float lo = nxt[(k * T + r) * T + i], hi = nxt[(k * T + r) * T + h + i];
        cur[(k * T + r) * T + 2 * i] = (lo + hi) * kR2;
        cur[(k * T + r) * T + 2 * i + 1] = (lo - hi) * kR2;
    }
    __syncthreads();
}

// Global index of detail quadrant entries of tile (ty, tx) at a level whose
// tile-local band size is h (global band size nb = n h / T).
__device__ __forceinline__ size_t detail_index(int quad, int i, int jj, int ty, int tx, int h, int nb, int n) {
    const int gr = (quad >= 1 ? nb : 0) + ty * h + i;     // quad 0: (lo, hi), 1: (hi, lo), 2: (hi, hi)
    const int gc = (quad != 1 ? nb : 0) + tx * h + jj;
    return (size_t)gr * n + gc;
}

__global__ __launch_bounds__(kThreads) void k_haar_fwd_tile(int K, int n, int T, const float* __restrict__ in,
                                                            const float* __restrict__ M,
                                                            float* __restrict__ coef,
                                                            float* __restrict__ coarse,
                                                            const long long* __restrict__ zd) {
    extern __shared__ float lds[];
    {                                                      // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        in = zadd(in, d);
        M = zshift(M, d);
        coef = zadd(coef, d);
        coarse = zadd(coarse, d);
    }
    float* cur = lds;
    float* nxt = lds + K * T * T;
    const int tx = blockIdx.x, ty = blockIdx.y, nt = n / T;
    const int nj = n * n;
    for (int idx = threadIdx.x; idx < T * T; idx += blockDim.x) {
        const int r = idx / T, c = idx % T;
        const size_t j = (size_t)(ty * T + r) * n + tx * T + c;
        float a[kMaxMat];
        for (int k = 0; k < K; ++k) a[k] = in[(size_t)k * nj + j];
        for (int k = 0; k < K; ++k) {
            float v = a[k];
            if (M) {
                v = 0.0f;
                for (int l2 = 0; l2 < K; ++l2) v = fmaf(M[(size_t)packed_index(k, l2, K) * nj + j], a[l2], v);
            }
            cur[(k * T + r) * T + c] = v;
        }
    }
    __syncthreads();
    for (int m = T; m > 1; m >>= 1) {
        level_forward(cur, nxt, K, T, m);
        const int h = m >> 1, nb = n / T * h;
        for (int idx = threadIdx.x; idx < 3 * K * h * h; idx += blockDim.x) {
            const int jj = idx % h, i = (idx / h) % h, quad = (idx / (h * h)) % 3, k = idx / (3 * h * h);
            const int lr = (quad >= 1 ? h : 0) + i, lc = (quad != 1 ? h : 0) + jj;
            coef[(size_t)k * nj + detail_index(quad, i, jj, ty, tx, h, nb, n)] = cur[(k * T + lr) * T + lc];
        }
        __syncthreads();
    }
    if (threadIdx.x < K) coarse[(size_t)threadIdx.x * nt * nt + ty * nt + tx] = cur[threadIdx.x * T * T];
}

__global__ __launch_bounds__(kThreads) void k_haar_inv_tile(int K, int n, int T, const float* __restrict__ coef,
                                                            const float* __restrict__ coarse,
                                                            const float* __restrict__ M, float sign,
                                                            float* __restrict__ out,
                                                            const float* __restrict__ g,
                                                            double* __restrict__ partials,
                                                            const long long* __restrict__ zd) {
    extern __shared__ float lds[];
    __shared__ double sh[kThreads / 64];
    {                                                      // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        coef = zadd(coef, d);
        coarse = zadd(coarse, d);
        M = zshift(M, d);
        out = zadd(out, d);
        g = zshift(g, d);
        partials = zshift(partials, d);
    }
    float* cur = lds;
    float* nxt = lds + K * T * T;
    const int tx = blockIdx.x, ty = blockIdx.y, nt = n / T;
    const int nj = n * n;
    if (threadIdx.x < K) cur[threadIdx.x * T * T] = coarse[(size_t)threadIdx.x * nt * nt + ty * nt + tx];
    for (int m = 2; m <= T; m <<= 1) {
        const int h = m >> 1, nb = n / T * h;
        for (int idx = threadIdx.x; idx < 3 * K * h * h; idx += blockDim.x) {
            const int jj = idx % h, i = (idx / h) % h, quad = (idx / (h * h)) % 3, k = idx / (3 * h * h);
            const int lr = (quad >= 1 ? h : 0) + i, lc = (quad != 1 ? h : 0) + jj;
            cur[(k * T + lr) * T + lc] = coef[(size_t)k * nj + detail_index(quad, i, jj, ty, tx, h, nb, n)];
        }
        __syncthreads();
        level_inverse(cur, nxt, K, T, m);
    }
    double dot = 0.0;
    for (int idx = threadIdx.x; idx < T * T; idx += blockDim.x) {
        const int r = idx / T, c = idx % T;
        const size_t j = (size_t)(ty * T + r) * n + tx * T + c;
        float a[kMaxMat];
        for (int k = 0; k < K; ++k) a[k] = cur[(k * T + r) * T + c];
        for (int k = 0; k < K; ++k) {
            float v = a[k];
            if (M) {
                v = 0.0f;
                for (int l2 = 0; l2 < K; ++l2) v = fmaf(M[(size_t)packed_index(k, l2, K) * nj + j], a[l2], v);
            }
            v *= sign;
            out[(size_t)k * nj + j] = v;
            if (g) dot += (double)g[(size_t)k * nj + j] * (double)v;
        }
    }
    const double tot = block_sum(dot, sh);
    if (threadIdx.x == 0 && partials) partials[blockIdx.y * gridDim.x + blockIdx.x] = tot;
}

// Remaining levels on the nc x nc coarse image; its Mallat layout is the
// top-left nc x nc block of the global one.
__global__ __launch_bounds__(kThreads) void k_haar_coarse_fwd(int K, int n, int nc, const float* __restrict__ coarse,
                                                              float* __restrict__ coef,
                                                              const long long* __restrict__ zd) {
    extern __shared__ float lds[];
    {                                                      // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        coarse = zadd(coarse, d);
        coef = zadd(coef, d);
    }
    float* cur = lds;
    float* nxt = lds + K * nc * nc;
    const int nj = n * n;
    for (int idx = threadIdx.x; idx < K * nc * nc; idx += blockDim.x) cur[idx] = coarse[idx];
    __syncthreads();
    for (int m = nc; m > 1; m >>= 1) level_forward(cur, nxt, K, nc, m);
    for (int idx = threadIdx.x; idx < K * nc * nc; idx += blockDim.x) {
        const int k = idx / (nc * nc), r = (idx / nc) % nc, c = idx % nc;
        coef[(size_t)k * nj + (size_t)r * n + c] = cur[idx];
    }
}

__global__ __launch_bounds__(kThreads) void k_haar_coarse_inv(int K, int n, int nc, const float* __restrict__ coef,
                                                              float* __restrict__ coarse,
                                                              const long long* __restrict__ zd) {
    extern __shared__ float lds[];
    {                                                      // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        coef = zadd(coef, d);
        coarse = zadd(coarse, d);
    }
    float* cur = lds;
    float* nxt = lds + K * nc * nc;
    const int nj = n * n;
    for (int idx = threadIdx.x; idx < K * nc * nc; idx += blockDim.x) {
        const int k = idx / (nc * nc), r = (idx / nc) % nc, c = idx % nc;
        cur[idx] = coef[(size_t)k * nj + (size_t)r * n + c];
    }
    __syncthreads();
    for (int m = 2; m <= nc; m <<= 1) level_inverse(cur, nxt, K, nc, m);
    for (int idx = threadIdx.x; idx < K * nc * nc; idx += blockDim.x) coarse[idx] = cur[idx];
}

__global__ void k_coef_blocks(int K, int nj, int k_col, const float* __restrict__ coef, float* __restrict__ blocks) {
    const int f = blockIdx.x * kThreads + threadIdx.x;
    if (f >= nj) return;
    for (int kp = 0; kp < K; ++kp) {
        const float wgt = kp == k_col ? 1.0f : 0.5f;
        blocks[(size_t)packed_index(kp, k_col, K) * nj + f] += wgt * coef[(size_t)kp * nj + f];
    }
}

void check(int K, int n) {
    MBMD_REQUIRE(n >= 2 && (n & (n - 1)) == 0, MBMD_ERR_SHAPE, "the Haar preconditioner needs a square power-of-two image");
    const int nc = n / haar_tile(n);
    MBMD_REQUIRE((size_t)2 * K * nc * nc * sizeof(float) <= 65536, MBMD_ERR_SHAPE,
                 "image too large for the single-workgroup coarse Haar pass");
}

}  // namespace

int haar_tile(int n) { return n < kTile ? n : kTile; }

void launch_haar_forward(int K, int n, const float* in, const float* M, float* coef, float* coarse, hipStream_t s) {
    check(K, n);
    const int T = haar_tile(n), nt = n / T;
    {
        KernelTimer kt_("k_haar_fwd_tile", s);
        hipLaunchKernelGGL(k_haar_fwd_tile, zgrid(dim3(nt, nt)), dim3(kThreads), sizeof(float) * 2 * K * T * T, s, K, n,
                           T, in, M, coef, coarse, zarg());
        kt_.stop();
    }
    MBMD_LAUNCHED();
    {
        KernelTimer kt_("k_haar_coarse_fwd", s);
        hipLaunchKernelGGL(k_haar_coarse_fwd, zgrid(dim3(1)), dim3(kThreads), sizeof(float) * 2 * K * nt * nt, s, K, n,
                           nt, coarse, coef, zarg());
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

void launch_haar_inverse(int K, int n, const float* coef, float* coarse, const float* M, float* out, float out_sign,
                         hipStream_t s) {
    check(K, n);
    const int T = haar_tile(n), nt = n / T;
    {
        KernelTimer kt_("k_haar_coarse_inv", s);
        hipLaunchKernelGGL(k_haar_coarse_inv, zgrid(dim3(1)), dim3(kThreads), sizeof(float) * 2 * K * nt * nt, s, K, n,
                           nt, coef, coarse, zarg());
        kt_.stop();
    }
    MBMD_LAUNCHED();
    {
        KernelTimer kt_("k_haar_inv_tile", s);
        hipLaunchKernelGGL(k_haar_inv_tile, zgrid(dim3(nt, nt)), dim3(kThreads), sizeof(float) * 2 * K * T * T, s, K, n,
                           T, coef, (const float*)coarse, M, out_sign, out, (const float*)nullptr, (double*)nullptr,
                           zarg());
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

int launch_haar_apply(int K, int n, const float* in, const float* M, const float* Kinv, float* coef, float* coarse,
                      float* out, float out_sign, const float* g, double* partials, hipStream_t s) {
    check(K, n);
    const int T = haar_tile(n), nt = n / T;
    MBMD_REQUIRE(nt * nt <= kMaxPartials, MBMD_ERR_SHAPE, "too many Haar tiles for the partial-sum buffer");
    launch_haar_forward(K, n, in, M, coef, coarse, s);
    launch_block_apply(n * n, K, Kinv, coef, coef, 1.0f, s);
    {
        KernelTimer kt_("k_haar_coarse_inv", s);
        hipLaunchKernelGGL(k_haar_coarse_inv, zgrid(dim3(1)), dim3(kThreads), sizeof(float) * 2 * K * nt * nt, s, K, n,
                           nt, coef, coarse, zarg());
        kt_.stop();
    }
    MBMD_LAUNCHED();
    {
        KernelTimer kt_("k_haar_inv_tile", s);
        hipLaunchKernelGGL(k_haar_inv_tile, zgrid(dim3(nt, nt)), dim3(kThreads), sizeof(float) * 2 * K * T * T, s, K, n,
                           T, coef, (const float*)coarse, M, out_sign, out, g, partials, zarg());
        kt_.stop();
    }
    MBMD_LAUNCHED();
    return nt * nt;
}

void launch_coef_blocks(int K, int n, int k_col, const float* coef, float* blocks, hipStream_t s) {
    const int nj = n * n;
    {
        KernelTimer kt_("k_coef_blocks", s);
        hipLaunchKernelGGL(k_coef_blocks, dim3((nj + kThreads - 1) / kThreads), dim3(kThreads), 0, s, K, nj, k_col, coef,
                       blocks);
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

}  // namespace mbmd
