// LDS-resident 2D FFT for the Fourier preconditioners.
//
// The unitary DFT U of the Fourier and cross-material Fourier sections
// applied to every material image: M M^T v = M0 U^H L^-1 U M0 v, so one
// iteration needs one forward and one inverse 2D transform per material.
// Three passes:
//   rows   : one workgroup per image row (all materials); optional packed
//            per-pixel blocks applied on load (M0) and a circular shift
//            (used by the impulse-response build); radix-2 decimation in
//            time in LDS from bit-reversed loads.
//   columns: a group of columns per workgroup; forward DIT, then (apply
//            only) the per-frequency N_k x N_k filter and an inverse
//            decimation-in-frequency transform in the same LDS buffer, so the
//            spectrum makes one round trip through memory.
//   rows^-1: inverse DIT per row, real part, 1/(nx ny), packed blocks (M0)
//            on store, sign, and per-block FP64 partials of g . out.
// Twiddles exp(-2 pi i k / N) are computed in FP64 on the host.
#include <cmath>
#include <vector>

#include "internal.h"

namespace mbmd {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ int bitrev(int x, int logn) { return (int)(__brev((unsigned)x) >> (32 - logn)); }

// In-place radix-2 DIT over nbuf contiguous transforms of length N (input in
// bit-reversed order, output natural).  INV conjugates the twiddles.
template <bool INV>
__device__ void fft_dit(float2* buf, int nbuf, int N, int logN, const float2* __restrict__ tw) {
    const int halfN = N >> 1;
    const int total = nbuf * halfN;
    for (int s = 1; s <= logN; ++s) {
        const int half = 1 << (s - 1);
        const int tstride = N >> s;
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
            const int bidx = t >> (logN - 1);
            const int bi = t & (halfN - 1);
            const int grp = bi >> (s - 1);
            const int pos = bi & (half - 1);
            const int i0 = bidx * N + grp * 2 * half + pos;
            const int i1 = i0 + half;
            float2 w = tw[pos * tstride];
            if (INV) w.y = -w.y;
            const float2 a = buf[i0];
            const float2 bw = cmul(buf[i1], w);
            buf[i0] = make_float2(a.x + bw.x, a.y + bw.y);
            buf[i1] = make_float2(a.x - bw.x, a.y - bw.y);
        }
        __syncthreads();
    }
}

// In-place radix-2 DIF (natural input, bit-reversed output).
template <bool INV>
__device__ void fft_dif(float2* buf, int nbuf, int N, int logN, const float2* __restrict__ tw) {
    const int halfN = N >> 1;
    const int total = nbuf * halfN;
    for (int s = logN; s >= 1; --s) {
        const int half = 1 << (s - 1);
        const int tstride = N >> s;
        for (int t = threadIdx.x; t < total; t += blockDim.x) {
            const int bidx = t >> (logN - 1);
            const int bi = t & (halfN - 1);
            const int grp = bi >> (s - 1);
            const int pos = bi & (half - 1);
            const int i0 = bidx * N + grp * 2 * half + pos;
            const int i1 = i0 + half;
            float2 w = tw[pos * tstride];
            if (INV) w.y = -w.y;
            const float2 a = buf[i0], b = buf[i1];
            buf[i0] = make_float2(a.x + b.x, a.y + b.y);
            buf[i1] = cmul(make_float2(a.x - b.x, a.y - b.y), w);
        }
        __syncthreads();
    }
}

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

__global__ __launch_bounds__(kThreads) void k_fft_rows_fwd(int K, int nx, int ny, int logx,
                                                           const float* __restrict__ in,
                                                           const float* __restrict__ M, int sy, int sx,
                                                           float2* __restrict__ spec,
                                                           const float2* __restrict__ tw) {
    extern __shared__ float2 buf[];
    const int y = blockIdx.x;
    const int nj = nx * ny;
    const int ys = (y + sy) % ny;
    for (int xx = threadIdx.x; xx < nx; xx += blockDim.x) {
        const int j = ys * nx + (xx + sx) % nx;
        float a[kMaxMat];
        for (int k = 0; k < K; ++k) a[k] = in[(size_t)k * nj + j];
        const int br = bitrev(xx, logx);
        for (int k = 0; k < K; ++k) {
            float v = a[k];
            if (M) {
                v = 0.0f;
                for (int l2 = 0; l2 < K; ++l2) v = fmaf(M[(size_t)packed_index(k, l2, K) * nj + j], a[l2], v);
            }
            buf[k * nx + br] = make_float2(v, 0.0f);
        }
    }
    __syncthreads();
    fft_dit<false>(buf, K, nx, logx, tw);
    for (int idx = threadIdx.x; idx < K * nx; idx += blockDim.x) {
        const int k = idx / nx, xx = idx - k * nx;
        spec[(size_t)k * nj + (size_t)y * nx + xx] = buf[idx];
    }
}

__global__ __launch_bounds__(kThreads) void k_fft_cols(int K, int nx, int ny, int logy, int C,
                                                       float2* __restrict__ spec,
                                                       const float* __restrict__ filt,
                                                       const float2* __restrict__ tw) {
    extern __shared__ float2 buf[];
    const int x0 = blockIdx.x * C;
    const int nj = nx * ny;
    const int tot = K * C * ny;
    for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
        const int c = idx % C;
        const int rest = idx / C;
        const int yy = rest % ny, k = rest / ny;
        buf[(k * C + c) * ny + bitrev(yy, logy)] = spec[(size_t)k * nj + (size_t)yy * nx + x0 + c];
    }
    __syncthreads();
    fft_dit<false>(buf, K * C, ny, logy, tw);
    if (filt) {
        for (int idx = threadIdx.x; idx < C * ny; idx += blockDim.x) {
            const int c = idx % C, yy = idx / C;
            const size_t f = (size_t)yy * nx + x0 + c;
            float2 a[kMaxMat];
            for (int k = 0; k < K; ++k) a[k] = buf[(k * C + c) * ny + yy];
            for (int k = 0; k < K; ++k) {
                float re = 0.0f, im = 0.0f;
                for (int l2 = 0; l2 < K; ++l2) {
                    const float m = filt[(size_t)packed_index(k, l2, K) * nj + f];
                    re = fmaf(m, a[l2].x, re);
                    im = fmaf(m, a[l2].y, im);
                }
                buf[(k * C + c) * ny + yy] = make_float2(re, im);
            }
        }
        __syncthreads();
        fft_dif<true>(buf, K * C, ny, logy, tw);
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
            const int c = idx % C;
            const int rest = idx / C;
            const int yy = rest % ny, k = rest / ny;
            spec[(size_t)k * nj + (size_t)yy * nx + x0 + c] = buf[(k * C + c) * ny + bitrev(yy, logy)];
        }
    } else {
        for (int idx = threadIdx.x; idx < tot; idx += blockDim.x) {
            const int c = idx % C;
            const int rest = idx / C;
            const int yy = rest % ny, k = rest / ny;
            spec[(size_t)k * nj + (size_t)yy * nx + x0 + c] = buf[(k * C + c) * ny + yy];
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_fft_rows_inv(int K, int nx, int ny, int logx,
                                                           const float2* __restrict__ spec,
                                                           const float* __restrict__ M, float scale,
                                                           float* __restrict__ out,
                                                           const float* __restrict__ g,
                                                           double* __restrict__ partials,
                                                           const float2* __restrict__ tw) {
    extern __shared__ float2 buf[];
    __shared__ double sh[kThreads / 64];
    const int y = blockIdx.x;
    const int nj = nx * ny;
    for (int idx = threadIdx.x; idx < K * nx; idx += blockDim.x) {
        const int k = idx / nx, xx = idx - k * nx;
        buf[k * nx + bitrev(xx, logx)] = spec[(size_t)k * nj + (size_t)y * nx + xx];
    }
    __syncthreads();
    fft_dit<true>(buf, K, nx, logx, tw);
    double dot = 0.0;
    for (int xx = threadIdx.x; xx < nx; xx += blockDim.x) {
        const int j = y * nx + xx;
        float a[kMaxMat];
        for (int k = 0; k < K; ++k) a[k] = buf[k * nx + xx].x * scale;
        for (int k = 0; k < K; ++k) {
            float v = a[k];
            if (M) {
                v = 0.0f;
                for (int l2 = 0; l2 < K; ++l2) v = fmaf(M[(size_t)packed_index(k, l2, K) * nj + j], a[l2], v);
            }
            out[(size_t)k * nj + j] = v;
            if (g) dot += (double)g[(size_t)k * nj + j] * (double)v;
        }
    }
    const double tot = block_sum(dot, sh);
    if (threadIdx.x == 0 && partials) partials[blockIdx.x] = tot;
}

__global__ void k_spectrum_real_to_blocks(int K, int nj, int k_col, const float2* __restrict__ spec,
                                          float* __restrict__ blocks) {
    const int f = blockIdx.x * kThreads + threadIdx.x;
    if (f >= nj) return;
    for (int kp = 0; kp < K; ++kp) {
        const float wgt = kp == k_col ? 1.0f : 0.5f;
        blocks[(size_t)packed_index(kp, k_col, K) * nj + f] += wgt * spec[(size_t)kp * nj + f].x;
    }
}

int ilog2(int n) {
    int l = 0;
    while ((1 << l) < n) ++l;
    return l;
}

int col_group(int K, int nx, int ny) {
    int C = 8;
    while (C > 1 && (size_t)K * C * ny * sizeof(float2) > 32768) C >>= 1;
    while (C > 1 && nx / C < 256) C >>= 1;
    while (C > nx) C >>= 1;
    return C;
}

void check_sizes(int K, int nx, int ny) {
    MBMD_REQUIRE(nx >= 2 && ny >= 2 && (nx & (nx - 1)) == 0 && (ny & (ny - 1)) == 0, MBMD_ERR_SHAPE,
                 "the Fourier preconditioner needs power-of-two image sizes");
    MBMD_REQUIRE((size_t)K * nx * sizeof(float2) <= 65536 && (size_t)K * ny * sizeof(float2) <= 65536,
                 MBMD_ERR_SHAPE, "image too large for the LDS-resident FFT");
}

}  // namespace

void fill_twiddles(float2* tw, int n, hipStream_t s) {
    std::vector<float2> h(n / 2 > 0 ? n / 2 : 1);
    for (int k = 0; k < n / 2; ++k) {
        const double a = -2.0 * M_PI * (double)k / (double)n;
        h[k] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    MBMD_HIP(hipMemcpyAsync(tw, h.data(), sizeof(float2) * h.size(), hipMemcpyHostToDevice, s));
    MBMD_HIP(hipStreamSynchronize(s));
}

void launch_fft2_forward(int K, int nx, int ny, const float* in, const float* M, int sy, int sx, float2* spec,
                         const float2* twx, const float2* twy, hipStream_t s) {
    check_sizes(K, nx, ny);
    {
        KernelTimer kt_("k_fft_rows_fwd", s);
        hipLaunchKernelGGL(k_fft_rows_fwd, dim3(ny), dim3(kThreads), sizeof(float2) * K * nx, s, K, nx, ny,
                       ilog2(nx), in, M, sy, sx, spec, twx);
        kt_.stop();
    }
    MBMD_LAUNCHED();
    const int C = col_group(K, nx, ny);
    {
        KernelTimer kt_("k_fft_cols", s);
        hipLaunchKernelGGL(k_fft_cols, dim3(nx / C), dim3(kThreads), sizeof(float2) * K * C * ny, s, K, nx, ny,
                       ilog2(ny), C, spec, (const float*)nullptr, twy);
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

int launch_fourier_apply(int K, int nx, int ny, const float* in, const float* M, const float* Filt, float2* spec,
                         const float2* twx, const float2* twy, float* out, float out_sign, const float* g,
                         double* partials, hipStream_t s) {
    check_sizes(K, nx, ny);
    MBMD_REQUIRE(ny <= kMaxPartials, MBMD_ERR_SHAPE, "too many rows for the partial-sum buffer");
    {
        KernelTimer kt_("k_fft_rows_fwd", s);
        hipLaunchKernelGGL(k_fft_rows_fwd, dim3(ny), dim3(kThreads), sizeof(float2) * K * nx, s, K, nx, ny,
                       ilog2(nx), in, M, 0, 0, spec, twx);
        kt_.stop();
    }
    MBMD_LAUNCHED();
    const int C = col_group(K, nx, ny);
    {
        KernelTimer kt_("k_fft_cols", s);
        hipLaunchKernelGGL(k_fft_cols, dim3(nx / C), dim3(kThreads), sizeof(float2) * K * C * ny, s, K, nx, ny,
                       ilog2(ny), C, spec, Filt, twy);
        kt_.stop();
    }
    MBMD_LAUNCHED();
    {
        KernelTimer kt_("k_fft_rows_inv", s);
        hipLaunchKernelGGL(k_fft_rows_inv, dim3(ny), dim3(kThreads), sizeof(float2) * K * nx, s, K, nx, ny,
                       ilog2(nx), spec, M, out_sign / (float)((double)nx * ny), out, g, partials, twx);
        kt_.stop();
    }
    MBMD_LAUNCHED();
    return ny;
}

void launch_spectrum_real_to_blocks(int K, int nj, int k_col, const float2* spec, float* blocks, hipStream_t s) {
    {
        KernelTimer kt_("k_spectrum_real_to_blocks", s);
        hipLaunchKernelGGL(k_spectrum_real_to_blocks, dim3((nj + kThreads - 1) / kThreads), dim3(kThreads), 0, s, K,
                       nj, k_col, spec, blocks);
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

}  // namespace mbmd
