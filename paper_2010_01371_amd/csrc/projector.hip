// Distance-driven forward and back projection for gfx950.
//
// Forward (ray-driven, "branchless" distance-driven): for each sweep frame the
// image lines are integrated once per call into exclusive prefix sums
// F[k] = sum_{p<k} img[p] (FP64 accumulation, stored FP32 next to img[k] as
// a float2).  The integral of the piecewise-constant line over the footprint
// [lo, hi] is then F(hi) - F(lo) with F linear inside a pixel, so each
// (ray, line) costs two interpolated lookups whatever the footprint width.
// One thread per (view, bin); a wavefront covers 64 consecutive bins of one
// view, so the lookups on a line are nearly contiguous and the sinogram row
// is written coalesced.
//
// Back projection (pixel-driven gather, same boundary table): one thread per
// pixel of the sweep frame loops over the views of that frame, maps the
// pixel's two edges to fractional bin indices, and for each bin in range adds
// overlap / footprint * path * sino.  Sums over views use Kahan compensation.
// No atomics, so results are bitwise reproducible.  Views that sweep rows and
// views that sweep columns run as two launches; the second adds into the
// first's output.
#include <cmath>

#include "internal.h"

namespace mbmd {

namespace {

constexpr int kFwdThreads = 256;
constexpr int kBackX = 64;
constexpr int kBackY = 4;
constexpr int kScanThreads = 256;

// Exclusive prefix sums of every sweep line of n_mat images for one frame.
// Line q of frame 0 is image row q; of frame 1 image column q.
__global__ __launch_bounds__(kScanThreads) void k_line_prefix(const float* __restrict__ img,
                                                               float2* __restrict__ out, int nx,
                                                               int ny, int frame) {
    const int q = blockIdx.x;
    const int m = blockIdx.y;
    const int Nq = frame ? nx : ny;
    const int Np = frame ? ny : nx;
    if (q >= Nq) return;
    const float* src = img + (size_t)m * nx * ny;
    const size_t elem_stride = frame ? (size_t)nx : 1;
    const size_t line_off = frame ? (size_t)q : (size_t)q * nx;
    float2* dst = out + ((size_t)m * Nq + q) * Np;

    __shared__ double part[kScanThreads];
    const int per = (Np + kScanThreads - 1) / kScanThreads;
    const int p0 = threadIdx.x * per;
    double s = 0.0;
    for (int i = 0; i < per; ++i) {
        const int p = p0 + i;
        if (p < Np) s += (double)src[line_off + (size_t)p * elem_stride];
    }
    part[threadIdx.x] = s;
    __syncthreads();
    // Hillis-Steele inclusive scan of the per-thread totals (FP64)
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const double add = threadIdx.x >= off ? part[threadIdx.x - off] : 0.0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    double run = threadIdx.x ? part[threadIdx.x - 1] : 0.0;
    for (int i = 0; i < per; ++i) {
        const int p = p0 + i;
        if (p < Np) {
            const float val = src[line_off + (size_t)p * elem_stride];
            dst[p] = make_float2((float)run, val);
            run += (double)val;
        }
    }
}

// Interpolated cumulative integral at along position K (pixels, centred).
__device__ __forceinline__ void interp_index(float K, float half, int Np, int& k, float& f) {
    K = fminf(fmaxf(K, -half), half);
    k = (int)floorf(K + half);
    k = min(max(k, 0), Np - 1);
    f = K - ((float)k - half);
}

template <int NK>
__global__ __launch_bounds__(kFwdThreads) void k_dd_forward(const ViewParams* __restrict__ view,
                                                            const float2* __restrict__ bound,
                                                            const float* __restrict__ path,
                                                            const float2* __restrict__ pre_rows,
                                                            const float2* __restrict__ pre_cols,
                                                            int nx, int ny, int V, int B,
                                                            float* __restrict__ sino) {
    const int v = blockIdx.y;
    const int b = blockIdx.x * kFwdThreads + threadIdx.x;
    if (b >= B) return;
    const int frame = view[v].frame;
    const int Nq = frame ? nx : ny;
    const int Np = frame ? ny : nx;
    const float2* pre = frame ? pre_cols : pre_rows;
    const size_t mat_stride = (size_t)Nq * Np;
    const float2 b0 = bound[(size_t)v * (B + 1) + b];
    const float2 b1 = bound[(size_t)v * (B + 1) + b + 1];
    const float half = 0.5f * (float)Np;
    const float qc = 0.5f * (float)(Nq - 1);
    float acc[NK];
#pragma unroll
    for (int m = 0; m < NK; ++m) acc[m] = 0.0f;
    for (int q = 0; q < Nq; ++q) {
        const float qq = (float)q - qc;
        const float ka = fmaf(b0.y, qq, b0.x);
        const float kb = fmaf(b1.y, qq, b1.x);
        const float lo = fminf(ka, kb), hi = fmaxf(ka, kb);
        if (hi <= -half || lo >= half) continue;     // footprint off the image on this line
        const float inv_w = 1.0f / (hi - lo);
        int klo, khi;
        float flo, fhi;
        interp_index(lo, half, Np, klo, flo);
        interp_index(hi, half, Np, khi, fhi);
        const float2* line = pre + (size_t)q * Np;
#pragma unroll
        for (int m = 0; m < NK; ++m) {
            const float2 a = line[m * mat_stride + klo];
            const float2 c = line[m * mat_stride + khi];
            const float fa = fmaf(flo, a.y, a.x);
            const float fc = fmaf(fhi, c.y, c.x);
            acc[m] = fmaf(fc - fa, inv_w, acc[m]);
        }
    }
    const float L = path[(size_t)v * B + b];
#pragma unroll
    for (int m = 0; m < NK; ++m) sino[((size_t)m * V + v) * B + b] = acc[m] * L;
}

template <int NCH>
__global__ __launch_bounds__(kBackX* kBackY) void k_dd_back(
    const ViewParams* __restrict__ view, const float2* __restrict__ bound,
    const float* __restrict__ path, const int* __restrict__ frame_views, int n_frame_views,
    int frame, int nx, int ny, int V, int B, const float* __restrict__ sino, float* __restrict__ x,
    int accumulate) {
    const int Nq = frame ? nx : ny;
    const int Np = frame ? ny : nx;
    const int p = blockIdx.x * kBackX + threadIdx.x;
    const int q = blockIdx.y * kBackY + threadIdx.y;
    if (p >= Np || q >= Nq) return;
    const float half = 0.5f * (float)Np;
    const float qq = (float)q - 0.5f * (float)(Nq - 1);
    const float K0 = (float)p - half;
    const float K1 = K0 + 1.0f;
    float acc[NCH], comp[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] = comp[c] = 0.0f;
    const size_t ch_stride = (size_t)V * B;
    for (int iv = 0; iv < n_frame_views; ++iv) {
        const int v = frame_views[iv];
        const ViewParams vp = view[v];
        const float nb = fmaf(vp.nq, qq, vp.n0);
        const float db = fmaf(vp.dq, qq, vp.d0);
        const float beta0 = fmaf(vp.nK, K0, nb) / fmaf(vp.dK, K0, db);
        const float beta1 = fmaf(vp.nK, K1, nb) / fmaf(vp.dK, K1, db);
        int bmin = (int)floorf(fminf(beta0, beta1) - 0.01f);
        int bmax = (int)floorf(fmaxf(beta0, beta1) + 0.01f);
        bmin = max(bmin, 0);
        bmax = min(bmax, B - 1);
        float part[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) part[c] = 0.0f;
        const float2* bd = bound + (size_t)v * (B + 1);
        const float* pa = path + (size_t)v * B;
        const float* sv = sino + (size_t)v * B;
        for (int b = bmin; b <= bmax; ++b) {
            const float2 c0 = bd[b];
            const float2 c1 = bd[b + 1];
            const float ka = fmaf(c0.y, qq, c0.x);
            const float kb = fmaf(c1.y, qq, c1.x);
            const float lo = fminf(ka, kb), hi = fmaxf(ka, kb);
            const float ov = fminf(hi, K1) - fmaxf(lo, K0);
            if (ov > 0.0f) {
                const float wgt = ov / (hi - lo) * pa[b];
#pragma unroll
                for (int c = 0; c < NCH; ++c) part[c] = fmaf(wgt, sv[c * ch_stride + b], part[c]);
            }
        }
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const float yk = part[c] - comp[c];
            const float t = acc[c] + yk;
            comp[c] = (t - acc[c]) - yk;
            acc[c] = t;
        }
    }
    const size_t pix = frame ? (size_t)p * nx + q : (size_t)q * nx + p;
    const size_t img_stride = (size_t)nx * ny;
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        float* dst = x + c * img_stride + pix;
        *dst = accumulate ? *dst + acc[c] : acc[c];
    }
}

// Number of (ray, pixel) pairs with a positive footprint overlap, i.e. the
// nonzeros of A, from the same boundary table the projector uses.
__global__ __launch_bounds__(kFwdThreads) void k_dd_count(const ViewParams* __restrict__ view,
                                                          const float2* __restrict__ bound, int nx, int ny,
                                                          int V, int B, unsigned long long* __restrict__ nnz) {
    __shared__ unsigned long long sh[kFwdThreads];
    const int v = blockIdx.y;
    const int b = blockIdx.x * kFwdThreads + threadIdx.x;
    unsigned long long cnt = 0;
    if (b < B) {
        const int frame = view[v].frame;
        const int Nq = frame ? nx : ny;
        const int Np = frame ? ny : nx;
        const float2 b0 = bound[(size_t)v * (B + 1) + b];
        const float2 b1 = bound[(size_t)v * (B + 1) + b + 1];
        const float half = 0.5f * (float)Np;
        const float qc = 0.5f * (float)(Nq - 1);
        for (int q = 0; q < Nq; ++q) {
            const float qq = (float)q - qc;
            const float ka = fmaf(b0.y, qq, b0.x), kb = fmaf(b1.y, qq, b1.x);
            const float lo = fmaxf(fminf(ka, kb), -half), hi = fminf(fmaxf(ka, kb), half);
            if (hi <= lo) continue;
            const int k0 = (int)floorf(lo + half);
            const int k1 = (int)ceilf(hi + half) - 1;
            cnt += (unsigned long long)max(0, min(k1, Np - 1) - max(k0, 0) + 1);
        }
    }
    sh[threadIdx.x] = cnt;
    __syncthreads();
    for (int off = kFwdThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(nnz, sh[0]);
}

template <int NK>
void fwd_launch(const GeomTables& t, float* sino, hipStream_t s) {
    dim3 grid((t.B + kFwdThreads - 1) / kFwdThreads, t.V);
    const size_t nj = (size_t)t.nx * t.ny;
    const float2* rows = t.prefix;
    const float2* cols = t.prefix + nj * t.prefix_mat;
    {
        KernelTimer kt_("k_dd_forward", s);
        hipLaunchKernelGGL(k_dd_forward<NK>, grid, dim3(kFwdThreads), 0, s, t.view, t.bound, t.path, rows,
                       cols, t.nx, t.ny, t.V, t.B, sino);
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

template <int NCH>
void back_launch(const GeomTables& t, const float* sino, float* x, hipStream_t s) {
    for (int frame = 0; frame < 2; ++frame) {
        const int Nq = frame ? t.nx : t.ny;
        const int Np = frame ? t.ny : t.nx;
        dim3 grid((Np + kBackX - 1) / kBackX, (Nq + kBackY - 1) / kBackY);
        const int* fv = t.frame_views + (frame ? t.n_frame_views[0] : 0);
        {
            KernelTimer kt_("k_dd_back", s);
            hipLaunchKernelGGL(k_dd_back<NCH>, grid, dim3(kBackX, kBackY), 0, s, t.view, t.bound, t.path,
                           fv, t.n_frame_views[frame], frame, t.nx, t.ny, t.V, t.B, sino, x,
                           frame);
            kt_.stop();
        }
        MBMD_LAUNCHED();
    }
}

}  // namespace

void launch_project(const GeomTables& t, const float* x, float* sino, int n_mat, hipStream_t s) {
    MBMD_REQUIRE(n_mat >= 1 && n_mat <= kMaxMat, MBMD_ERR_SHAPE, "n_mat must be in 1..4");
    MBMD_REQUIRE(t.prefix != nullptr && t.prefix_mat >= n_mat, MBMD_ERR_ARG,
                 "projector prefix scratch too small");
    const size_t nj = (size_t)t.nx * t.ny;
    for (int frame = 0; frame < 2; ++frame) {
        if (t.n_frame_views[frame] == 0) continue;
        const int Nq = frame ? t.nx : t.ny;
        float2* out = t.prefix + (frame ? nj * t.prefix_mat : 0);
        {
            KernelTimer kt_("k_line_prefix", s);
            hipLaunchKernelGGL(k_line_prefix, dim3(Nq, n_mat), dim3(kScanThreads), 0, s, x, out, t.nx,
                           t.ny, frame);
            kt_.stop();
        }
        MBMD_LAUNCHED();
    }
    switch (n_mat) {
        case 1: fwd_launch<1>(t, sino, s); break;
        case 2: fwd_launch<2>(t, sino, s); break;
        case 3: fwd_launch<3>(t, sino, s); break;
        default: fwd_launch<4>(t, sino, s); break;
    }
}

long long count_nonzeros(const GeomTables& t, hipStream_t s) {
    unsigned long long* d = nullptr;
    MBMD_HIP(hipMalloc(&d, sizeof(unsigned long long)));
    unsigned long long h = 0;
    try {
        MBMD_HIP(hipMemcpyAsync(d, &h, sizeof(h), hipMemcpyHostToDevice, s));
        dim3 grid((t.B + kFwdThreads - 1) / kFwdThreads, t.V);
        hipLaunchKernelGGL(k_dd_count, grid, dim3(kFwdThreads), 0, s, t.view, t.bound, t.nx, t.ny, t.V, t.B, d);
        MBMD_LAUNCHED();
        MBMD_HIP(hipMemcpyAsync(&h, d, sizeof(h), hipMemcpyDeviceToHost, s));
        MBMD_HIP(hipStreamSynchronize(s));
    } catch (...) {
        (void)hipFree(d);
        throw;
    }
    MBMD_HIP(hipFree(d));
    return (long long)h;
}

void launch_backproject(const GeomTables& t, const float* sino, float* x, int n_ch, hipStream_t s) {
    MBMD_REQUIRE(n_ch >= 1 && n_ch <= kMaxBackCh, MBMD_ERR_SHAPE, "back projection channels must be in 1..10");
    switch (n_ch) {
        case 1: back_launch<1>(t, sino, x, s); break;
        case 2: back_launch<2>(t, sino, x, s); break;
        case 3: back_launch<3>(t, sino, x, s); break;
        case 4: back_launch<4>(t, sino, x, s); break;
        case 5: back_launch<5>(t, sino, x, s); break;
        case 6: back_launch<6>(t, sino, x, s); break;
        case 7: back_launch<7>(t, sino, x, s); break;
        case 8: back_launch<8>(t, sino, x, s); break;
        case 9: back_launch<9>(t, sino, x, s); break;
        default: back_launch<10>(t, sino, x, s); break;
    }
}

}  // namespace mbmd
