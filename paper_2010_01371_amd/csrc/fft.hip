// LDS-resident 2D FFT for the Fourier preconditioners.
//
// The unitary DFT U of the Fourier and cross-material Fourier sections
// applied to every material image: M M^T v = M0 U^H L^-1 U M0 v, so one
// iteration needs one forward and one inverse 2D transform per material.
// Three passes:
//   rows   : a few image rows per workgroup (all materials); optional packed
//            per-pixel blocks applied on load (M0) and a circular shift
//            (used by the impulse-response build).
//   columns: a few columns per workgroup; forward transform, then (apply
//            only) the per-frequency N_k x N_k filter and the inverse
//            transform in the same LDS buffer, so the spectrum makes one
//            round trip through memory.
//   rows^-1: inverse transform per row, real part, 1/(nx ny), packed blocks
//            (M0) on store, sign, and per-block FP64 partials of g . out.
// Each 1D transform is a mixed-radix Stockham autosort FFT (radix 8, then 4 or
// 2 for the last pass): natural order in and out, so no bit reversal; N/8
// threads per transform, each holding eight values in registers per pass, with
// one read phase and one write phase through LDS per pass.  For N = 512 that
// is three passes (the first without twiddles) instead of nine radix-2 stages.
// Twiddles exp(-2 pi i m / N), m < N, are computed in FP64 on the host.
#include <cmath>
#include <vector>

#include "internal.h"

namespace mbmd {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// z times -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 z) {
    return INV ? make_float2(-z.y, z.x) : make_float2(z.y, -z.x);
}

// 4-point DFT in place, natural order in and out.
template <bool INV>
__device__ __forceinline__ void dft4(float2& v0, float2& v1, float2& v2, float2& v3) {
    const float2 b0 = cadd(v0, v2), b1 = cadd(v1, v3), b2 = csub(v0, v2), b3 = mul_mi<INV>(csub(v1, v3));
    v0 = cadd(b0, b1);
    v1 = cadd(b2, b3);
    v2 = csub(b0, b1);
    v3 = csub(b2, b3);
}

// 8-point DFT in place: one radix-2 split into even and odd outputs, then two
// 4-point DFTs.
template <bool INV>
__device__ __forceinline__ void dft8(float2* v) {
    const float h = 0.70710678118654752f;
    const float2 w1 = make_float2(h, INV ? h : -h), w3 = make_float2(-h, INV ? h : -h);
    float2 a0 = cadd(v[0], v[4]), a1 = cadd(v[1], v[5]), a2 = cadd(v[2], v[6]), a3 = cadd(v[3], v[7]);
    float2 o0 = csub(v[0], v[4]), o1 = cmul(csub(v[1], v[5]), w1), o2 = mul_mi<INV>(csub(v[2], v[6])),
           o3 = cmul(csub(v[3], v[7]), w3);
    dft4<INV>(a0, a1, a2, a3);
    dft4<INV>(o0, o1, o2, o3);
    v[0] = a0;
    v[1] = o0;
    v[2] = a1;
    v[3] = o1;
    v[4] = a2;
    v[5] = o2;
    v[6] = a3;
    v[7] = o3;
}

template <bool INV, int R>
__device__ __forceinline__ void dftR(float2* v) {
    if constexpr (R == 8) {
        dft8<INV>(v);
    } else if constexpr (R == 4) {
        dft4<INV>(v[0], v[1], v[2], v[3]);
    } else {
        const float2 a = v[0], b = v[1];
        v[0] = cadd(a, b);
        v[1] = csub(a, b);
    }
}

__host__ __device__ inline int fft_threads(int N) { return N >= 8 ? N / 8 : 1; }
// LDS position of element i of a transform: one pad slot after every eight
// elements, which keeps the strided write phases of the radix-8 passes (stride 8
// in the first, 64 apart in groups of 8 in the second) at most 2-way bank
// conflicted; a transform of length N takes lds_len(N) slots, an odd number, so
// that the same element of neighbouring transforms falls in different banks.
__host__ __device__ constexpr int pad(int i) { return i + (i >> 3); }
__host__ __device__ constexpr int lds_len(int N) { return (N + (N >> 3)) | 1; }

// One Stockham pass of radix R over a length-N transform held in LDS (buf),
// after Ns points have been combined: butterfly j reads buf[j + r N/R],
// multiplies by W_{Ns R}^{r (j mod Ns)}, takes the R-point DFT and writes
// buf[(j / Ns) Ns R + (j mod Ns) + q Ns].  t in [0, T) is the thread's index in
// its transform; all threads of the block read before any writes (barrier).
template <bool INV, int R>
__device__ __forceinline__ void stockham_pass(float2* buf, int N, int Ns, int t, int T, bool active,
                                              const float2* __restrict__ tw) {
    constexpr int NB = 8 / R;                  // butterflies per thread (T = N / 8 for N >= 8)
    const int nbf = N / R;
    const int step = N / (Ns * R);             // twiddle table stride
    float2 v[NB][R];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * T;
        if (active && j < nbf) {
            const int k = j & (Ns - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                v[b][r] = buf[pad(j + r * nbf)];
                if (r > 0 && Ns > 1) {
                    float2 w = tw[r * k * step];
                    if (INV) w.y = -w.y;
                    v[b][r] = cmul(v[b][r], w);
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * T;
        if (active && j < nbf) {
            dftR<INV, R>(v[b]);
            const int k = j & (Ns - 1);
            const int d = (j - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) buf[pad(d + q * Ns)] = v[b][q];
        }
    }
    __syncthreads();
}

// Full length-N transform (N a power of two) of the block's transforms; each
// thread owns index t of the transform at buf (inactive threads only join the
// barriers).  The pass sequence depends on N alone, so it is uniform.
template <bool INV>
__device__ __forceinline__ void fft_lds(float2* buf, int N, int t, int T, bool active,
                                        const float2* __restrict__ tw) {
    int Ns = 1;
    while (Ns < N) {
        const int rem = N / Ns;
        if (rem % 8 == 0) {
            stockham_pass<INV, 8>(buf, N, Ns, t, T, active, tw);
            Ns *= 8;
        } else if (rem == 4) {
            stockham_pass<INV, 4>(buf, N, Ns, t, T, active, tw);
            Ns *= 4;
        } else {
            stockham_pass<INV, 2>(buf, N, Ns, t, T, active, tw);
            Ns *= 2;
        }
    }
}

// The same transform with N (and so the pass sequence, the thread count N/8 and
// every LDS offset) fixed at compile time.
template <bool INV, int R, int N, int NS>
__device__ __forceinline__ void stockham_pass_ct(float2* buf, int t, bool active, const float2* __restrict__ tw) {
    constexpr int T = N >= 8 ? N / 8 : 1;
    constexpr int NB = 8 / R;
    constexpr int nbf = N / R;
    constexpr int step = N / (NS * R);
    float2 v[NB][R];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * T;
        if (active && j < nbf) {
            const int k = j & (NS - 1);
#pragma unroll
            for (int r = 0; r < R; ++r) {
                v[b][r] = buf[pad(j + r * nbf)];
                if (r > 0 && NS > 1) {
                    float2 w = tw[r * k * step];
                    if (INV) w.y = -w.y;
                    v[b][r] = cmul(v[b][r], w);
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + b * T;
        if (active && j < nbf) {
            dftR<INV, R>(v[b]);
            const int k = j & (NS - 1);
            const int d = (j - k) * R + k;
#pragma unroll
            for (int q = 0; q < R; ++q) buf[pad(d + q * NS)] = v[b][q];
        }
    }
    __syncthreads();
}

template <bool INV, int N, int NS>
__device__ __forceinline__ void fft_passes_ct(float2* buf, int t, bool active, const float2* __restrict__ tw) {
    if constexpr (NS < N) {
        constexpr int rem = N / NS;
        constexpr int R = rem % 8 == 0 ? 8 : rem;            // radix 8, then the last 4 or 2
        stockham_pass_ct<INV, R, N, NS>(buf, t, active, tw);
        fft_passes_ct<INV, N, NS * R>(buf, t, active, tw);
    }
}

// Transform of length NT (compile time) or N (run time, NT = 0).
template <bool INV, int NT>
__device__ __forceinline__ void fft_any(float2* buf, int N, int t, int T, bool active, const float2* __restrict__ tw) {
    if constexpr (NT > 0) {
        fft_passes_ct<INV, NT, 1>(buf, t, active, tw);
    } else {
        fft_lds<INV>(buf, N, t, T, active, tw);
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

// RB rows per block: transform (rr, k) of row y0 + rr lives at buf[(rr K + k) nx].
template <int NT>
__global__ __launch_bounds__(kThreads) void k_fft_rows_fwd(int K, int nx_rt, int ny, int RB,
                                                           const float* __restrict__ in,
                                                           const float* __restrict__ M, int sy, int sx,
                                                           float2* __restrict__ spec,
                                                           const float2* __restrict__ tw,
                                                           const long long* __restrict__ zd) {
    extern __shared__ float2 buf[];
    if (zd) {                                              // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        in = zshift(in, d);
        M = zshift(M, d);
        spec = zshift(spec, d);
        tw = zshift(tw, d);
    }
    const int nx = NT ? NT : nx_rt;                        // transform length (a constant when NT > 0)
    const int PN = lds_len(nx);
    float2* twl = buf + (size_t)RB * K * PN;               // twiddle table staged in LDS
    const int y0 = blockIdx.x * RB;
    const int nj = nx * ny;
    const int lx = __builtin_ctz(nx);                     // sizes are powers of two
    for (int idx = threadIdx.x; idx < nx; idx += blockDim.x) twl[idx] = tw[idx];
    for (int idx = threadIdx.x; idx < RB * nx; idx += blockDim.x) {
        const int rr = idx >> lx, xx = idx & (nx - 1);
        if (y0 + rr >= ny) continue;
        const int j = ((y0 + rr + sy) & (ny - 1)) * nx + ((xx + sx) & (nx - 1));
        float a[kMaxMat];                                  // static indices: registers
#pragma unroll
        for (int k = 0; k < kMaxMat; ++k) a[k] = k < K ? in[(size_t)k * nj + j] : 0.0f;
#pragma unroll
        for (int k = 0; k < kMaxMat; ++k) {
            if (k >= K) break;
            float v = a[k];
            if (M) {
                v = 0.0f;
#pragma unroll
                for (int l2 = 0; l2 < kMaxMat; ++l2)
                    if (l2 < K) v = fmaf(M[(size_t)packed_index(k, l2, K) * nj + j], a[l2], v);
            }
            buf[(rr * K + k) * PN + pad(xx)] = make_float2(v, 0.0f);
        }
    }
    __syncthreads();
    const int T = fft_threads(nx);
    const int tr = threadIdx.x / T;                        // transform index rr K + k
    const bool active = tr < RB * K && y0 + tr / K < ny;
    fft_any<false, NT>(buf + (size_t)(active ? tr : 0) * PN, nx, threadIdx.x - tr * T, T, active, twl);
    for (int idx = threadIdx.x; idx < RB * K * nx; idx += blockDim.x) {
        const int trn = idx >> lx, xx = idx & (nx - 1);
        const int rr = trn / K, k = trn - rr * K;
        if (y0 + rr < ny) spec[(size_t)k * nj + (size_t)(y0 + rr) * nx + xx] = buf[trn * PN + pad(xx)];
    }
}

// C columns per block: transform (c, k) of column x0 + c lives at buf[(c K + k) ny];
// the block's filter blocks are staged at fl[(p ny + yy) C + c].  All global
// reads of the block (spectrum, twiddles, filter) are issued in batches before
// any is waited for.
constexpr int kBatch = 8;
template <int NT>
__global__ __launch_bounds__(kThreads) void k_fft_cols(int K, int nx, int ny_rt, int C, float2* __restrict__ spec,
                                                       const float* __restrict__ filt,
                                                       const float2* __restrict__ tw,
                                                       const long long* __restrict__ zd) {
    extern __shared__ float2 buf[];
    if (zd) {                                              // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        spec = zshift(spec, d);
        filt = zshift(filt, d);
        tw = zshift(tw, d);
    }
    const int ny = NT ? NT : ny_rt;                        // transform length (a constant when NT > 0)
    const int PN = lds_len(ny);
    float2* twl = buf + (size_t)K * C * PN;                // twiddle table staged in LDS
    float* fl = reinterpret_cast<float*>(twl + ny);        // filter blocks staged in LDS
    const int x0 = blockIdx.x * C;
    const int nj = nx * ny;
    const int npk = K * (K + 1) / 2;
    const int tot = K * C * ny, fl_tot = filt ? npk * C * ny : 0;
    const int lc = __builtin_ctz(C), ly = __builtin_ctz(ny);   // powers of two
    for (int idx = threadIdx.x; idx < ny; idx += kThreads) twl[idx] = tw[idx];
    for (int base = threadIdx.x; base < tot || base < fl_tot; base += kThreads * kBatch) {
        float2 v[kBatch];
        float fv[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int idx = base + u * kThreads;
            const int c = idx & (C - 1), rest = idx >> lc;       // c fastest: neighbouring columns
            const int yy = rest & (ny - 1), k = rest >> ly;
            if (idx < tot) v[u] = spec[(size_t)k * nj + (size_t)yy * nx + x0 + c];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int idx = base + u * kThreads;
            const int c = idx & (C - 1), rest = idx >> lc;
            const int yy = rest & (ny - 1), p = rest >> ly;
            if (idx < fl_tot) fv[u] = filt[(size_t)p * nj + (size_t)yy * nx + x0 + c];
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
            const int idx = base + u * kThreads;
            const int c = idx & (C - 1), rest = idx >> lc;
            const int yy = rest & (ny - 1), k = rest >> ly;
            if (idx < tot) buf[(c * K + k) * PN + pad(yy)] = v[u];
            if (idx < fl_tot) fl[idx] = fv[u];
        }
    }
    __syncthreads();
    const int T = fft_threads(ny);
    const int tr = threadIdx.x / T;
    const bool active = tr < C * K;
    float2* mine = buf + (size_t)(active ? tr : 0) * PN;
    const int t = threadIdx.x - tr * T;
    fft_any<false, NT>(mine, ny, t, T, active, twl);
    if (filt) {
        for (int idx = threadIdx.x; idx < C * ny; idx += kThreads) {
            const int c = idx & (C - 1), yy = idx >> lc;
            float2 a[kMaxMat];                             // static indices: registers
#pragma unroll
            for (int k = 0; k < kMaxMat; ++k) a[k] = k < K ? buf[(c * K + k) * PN + pad(yy)] : make_float2(0.0f, 0.0f);
#pragma unroll
            for (int k = 0; k < kMaxMat; ++k) {
                if (k >= K) break;
                float re = 0.0f, im = 0.0f;
#pragma unroll
                for (int l2 = 0; l2 < kMaxMat; ++l2) {
                    if (l2 >= K) break;
                    const float m = fl[(packed_index(k, l2, K) * ny + yy) * C + c];
                    re = fmaf(m, a[l2].x, re);
                    im = fmaf(m, a[l2].y, im);
                }
                buf[(c * K + k) * PN + pad(yy)] = make_float2(re, im);
            }
        }
        __syncthreads();
        fft_any<true, NT>(mine, ny, t, T, active, twl);
    }
    for (int idx = threadIdx.x; idx < tot; idx += kThreads) {
        const int c = idx & (C - 1);
        const int rest = idx >> lc;
        const int yy = rest & (ny - 1), k = rest >> ly;
        spec[(size_t)k * nj + (size_t)yy * nx + x0 + c] = buf[(c * K + k) * PN + pad(yy)];
    }
}

template <int NT>
__global__ __launch_bounds__(kThreads) void k_fft_rows_inv(int K, int nx_rt, int ny, int RB,
                                                           const float2* __restrict__ spec,
                                                           const float* __restrict__ M, float scale,
                                                           float* __restrict__ out,
                                                           const float* __restrict__ g,
                                                           double* __restrict__ partials,
                                                           const float2* __restrict__ tw,
                                                           const long long* __restrict__ zd) {
    extern __shared__ float2 buf[];
    __shared__ double sh[kThreads / 64];
    if (zd) {                                              // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        spec = zshift(spec, d);
        M = zshift(M, d);
        out = zshift(out, d);
        g = zshift(g, d);
        partials = zshift(partials, d);
        tw = zshift(tw, d);
    }
    const int nx = NT ? NT : nx_rt;                        // transform length (a constant when NT > 0)
    const int PN = lds_len(nx);
    float2* twl = buf + (size_t)RB * K * PN;               // twiddle table staged in LDS
    const int y0 = blockIdx.x * RB;
    const int nj = nx * ny;
    const int lx = __builtin_ctz(nx);                     // sizes are powers of two
    for (int idx = threadIdx.x; idx < nx; idx += blockDim.x) twl[idx] = tw[idx];
    for (int idx = threadIdx.x; idx < RB * K * nx; idx += blockDim.x) {
        const int trn = idx >> lx, xx = idx & (nx - 1);
        const int rr = trn / K, k = trn - rr * K;
        if (y0 + rr < ny) buf[trn * PN + pad(xx)] = spec[(size_t)k * nj + (size_t)(y0 + rr) * nx + xx];
    }
    __syncthreads();
    const int T = fft_threads(nx);
    const int tr = threadIdx.x / T;
    const bool active = tr < RB * K && y0 + tr / K < ny;
    fft_any<true, NT>(buf + (size_t)(active ? tr : 0) * PN, nx, threadIdx.x - tr * T, T, active, twl);
    double dot = 0.0;
    for (int idx = threadIdx.x; idx < RB * nx; idx += blockDim.x) {
        const int rr = idx >> lx, xx = idx & (nx - 1);
        if (y0 + rr >= ny) continue;
        const int j = (y0 + rr) * nx + xx;
        float a[kMaxMat];                                  // static indices: registers
#pragma unroll
        for (int k = 0; k < kMaxMat; ++k) a[k] = k < K ? buf[(rr * K + k) * PN + pad(xx)].x * scale : 0.0f;
#pragma unroll
        for (int k = 0; k < kMaxMat; ++k) {
            if (k >= K) break;
            float v = a[k];
            if (M) {
                v = 0.0f;
#pragma unroll
                for (int l2 = 0; l2 < kMaxMat; ++l2)
                    if (l2 < K) v = fmaf(M[(size_t)packed_index(k, l2, K) * nj + j], a[l2], v);
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

// Rows per block of the row passes: enough transforms for about one wavefront of
// FFT threads.  Blocks always have kThreads threads, so that the loads and stores
// of a block are spread over all of them (few in flight per thread); threads
// beyond the transforms only join the barriers.
int rows_per_block(int K, int nx, int ny) {
    int RB = 1;
    while (RB * 2 * K * fft_threads(nx) <= 64 && RB * 2 <= ny) RB *= 2;
    return RB;
}

// Columns per block of the column pass: as many as keep every thread of the
// block in a transform, at most 8 (C-column row segments per load).
int col_group(int K, int nx, int ny) {
    int C = 1;
    while (C < 8 && C * 2 * K * fft_threads(ny) <= kThreads && C * 2 <= nx) C *= 2;
    return C;
}

size_t cols_lds(int K, int C, int ny, bool filt) {
    return sizeof(float2) * ((size_t)K * C * lds_len(ny) + ny) +
           (filt ? sizeof(float) * (size_t)(K * (K + 1) / 2) * C * ny : 0);
}

size_t rows_lds(int K, int RB, int nx) { return sizeof(float2) * ((size_t)RB * K * lds_len(nx) + nx); }

void check_sizes(int K, int nx, int ny) {
    MBMD_REQUIRE(nx >= 2 && ny >= 2 && (nx & (nx - 1)) == 0 && (ny & (ny - 1)) == 0, MBMD_ERR_SHAPE,
                 "the Fourier preconditioner needs power-of-two image sizes");
    MBMD_REQUIRE(K * fft_threads(nx) <= kThreads && K * fft_threads(ny) <= kThreads &&
                     rows_lds(K, 1, nx) <= 65536 && cols_lds(K, 1, ny, true) <= 65536,
                 MBMD_ERR_SHAPE, "image too large for the LDS-resident FFT");
}

// Transform lengths compiled as constants (the pass sequence and the LDS
// offsets fold into immediates); other powers of two take the general form.
#define MBMD_FFT_DISPATCH(N, LAUNCH)                  \
    do {                                              \
        switch (N) {                                  \
            case 64: LAUNCH(64); break;               \
            case 128: LAUNCH(128); break;             \
            case 256: LAUNCH(256); break;             \
            case 512: LAUNCH(512); break;             \
            case 1024: LAUNCH(1024); break;           \
            default: LAUNCH(0); break;                \
        }                                             \
    } while (0)

}  // namespace

void fill_twiddles(float2* tw, int n, hipStream_t s) {
    std::vector<float2> h(n);
    for (int k = 0; k < n; ++k) {
        const double a = -2.0 * M_PI * (double)k / (double)n;
        h[k] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    MBMD_HIP(hipMemcpyAsync(tw, h.data(), sizeof(float2) * h.size(), hipMemcpyHostToDevice, s));
    MBMD_HIP(hipStreamSynchronize(s));
}

void launch_fft2_forward(int K, int nx, int ny, const float* in, const float* M, int sy, int sx, float2* spec,
                         const float2* twx, const float2* twy, hipStream_t s) {
    check_sizes(K, nx, ny);
    const int RB = rows_per_block(K, nx, ny);
    {
        KernelTimer kt_("k_fft_rows_fwd", s);
#define L_(NT) hipLaunchKernelGGL((k_fft_rows_fwd<NT>), zgrid(dim3((ny + RB - 1) / RB)), dim3(kThreads),                 \
                               rows_lds(K, RB, nx), s, K, nx, ny, RB, in, M, sy, sx, spec, twx, zarg())
        MBMD_FFT_DISPATCH(nx, L_);
#undef L_
        kt_.stop();
    }
    MBMD_LAUNCHED();
    const int C = col_group(K, nx, ny);
    {
        KernelTimer kt_("k_fft_cols", s);
#define L_(NT) hipLaunchKernelGGL((k_fft_cols<NT>), zgrid(dim3(nx / C)), dim3(kThreads), cols_lds(K, C, ny, false), s, K, \
                               nx, ny, C, spec, (const float*)nullptr, twy, zarg())
        MBMD_FFT_DISPATCH(ny, L_);
#undef L_
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

int launch_fourier_apply(int K, int nx, int ny, const float* in, const float* M, const float* Filt, float2* spec,
                         const float2* twx, const float2* twy, float* out, float out_sign, const float* g,
                         double* partials, hipStream_t s) {
    check_sizes(K, nx, ny);
    const int RB = rows_per_block(K, nx, ny);
    const int nblk = (ny + RB - 1) / RB;
    MBMD_REQUIRE(nblk <= kMaxPartials, MBMD_ERR_SHAPE, "too many rows for the partial-sum buffer");
    {
        KernelTimer kt_("k_fft_rows_fwd", s);
#define L_(NT) hipLaunchKernelGGL((k_fft_rows_fwd<NT>), zgrid(dim3(nblk)), dim3(kThreads), rows_lds(K, RB, nx), s, K, nx, \
                               ny, RB, in, M, 0, 0, spec, twx, zarg())
        MBMD_FFT_DISPATCH(nx, L_);
#undef L_
        kt_.stop();
    }
    MBMD_LAUNCHED();
    const int C = col_group(K, nx, ny);
    MBMD_REQUIRE(cols_lds(K, C, ny, true) <= 65536, MBMD_ERR_SHAPE, "image too large for the LDS-resident FFT");
    {
        KernelTimer kt_("k_fft_cols", s);
#define L_(NT) hipLaunchKernelGGL((k_fft_cols<NT>), zgrid(dim3(nx / C)), dim3(kThreads), cols_lds(K, C, ny, true), s, K, \
                               nx, ny, C, spec, Filt, twy, zarg())
        MBMD_FFT_DISPATCH(ny, L_);
#undef L_
        kt_.stop();
    }
    MBMD_LAUNCHED();
    {
        KernelTimer kt_("k_fft_rows_inv", s);
#define L_(NT) hipLaunchKernelGGL((k_fft_rows_inv<NT>), zgrid(dim3(nblk)), dim3(kThreads), rows_lds(K, RB, nx), s, K, nx, \
                               ny, RB, spec, M, out_sign / (float)((double)nx * ny), out, g, partials, twx, zarg())
        MBMD_FFT_DISPATCH(nx, L_);
#undef L_
        kt_.stop();
    }
    MBMD_LAUNCHED();
    return nblk;
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
