// Distance-driven forward and back projection for gfx950.
//
// Both directions use cumulative integrals, so that the work per
// (ray, line) or (pixel, view) is a constant handful of instructions whatever
// the footprint width, with no divergent inner loop.
//
// Forward (ray-driven): each image line of each sweep frame is integrated once
// per call into exclusive prefix sums F[k] = sum_{p<k} img[p] (FP64
// accumulation, stored FP32 next to img[k]).  F is linear inside a pixel, so
// the integral of the line over a footprint [K_b, K_b+1] is F(K_b+1) - F(K_b).
// One lane per bin BOUNDARY: a wavefront evaluates F at 64 consecutive
// boundaries and takes its right-hand neighbour's value with a wave shuffle,
// giving 63 bins per wavefront.  The sign of (F(K_b+1) - F(K_b)) / (K_b+1 -
// K_b) does not depend on the orientation of the view.
//
// Back projection (pixel-driven gather): per call and view the sinogram times
// the per-line path length is integrated over the detector in FP64,
// C_v[b] = sum_{b'<b} sino * path.  The back projected detector signal on a
// sweep line is piecewise constant in the along-line position K, with
// cumulative integral H(K) = C[b] + (C[b+1] - C[b]) (K - K_b)/(K_b+1 - K_b)
// for K in bin b, so a pixel [K, K+1] receives H(K+1) - H(K); the view's
// orientation sign is folded into C.  One lane per pixel EDGE: 63 pixels per wavefront, the
// right edge taken from the neighbour lane.  The bin holding an edge comes
// from the rational map K -> fractional bin index; the fraction inside the
// bin is clamped to [0, 1], which keeps H continuous when that map is off by
// rounding near a boundary.  H and the sums over views are FP64 (full rate on
// CDNA); no atomics, so results are bitwise reproducible.
//
// Table reads go through buffer loads (32-bit offsets from a base held in
// scalar registers; out-of-range offsets read zero), neighbour exchanges are
// DPP wave shifts, and the line / view loops are unrolled so that several
// loads are in flight per wavefront.
//
// Views sweeping rows and views sweeping columns are interleaved in one launch
// with an XCD-aware block order: blocks are dispatched round-robin to the 8
// XCDs, and blocks landing on XCDs 0-3 take row-sweep work, 4-7 column-sweep
// work, so each XCD's L2 holds one frame's prefix arrays.  The column-sweep
// part of a back projection is written in its own (transposed) layout and
// added by a tiled transpose.
#include <cmath>

#include "internal.h"

namespace mbmd {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kPerWave = 63;                 // bins (forward) or pixels (back) per wavefront
constexpr int kScanThreads = 256;
constexpr int kBufferWord3 = 0x00020000;     // raw buffer resource, gfx9 family

__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Value held by lane + 1 (DPP wave shift left by one lane; lane 63 reads 0 and
// its result is never stored).
__device__ __forceinline__ float next_lane(float v) {
    const int i = __builtin_bit_cast(int, v);
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(i, 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ double next_lane(double v) {
    const long long i = __builtin_bit_cast(long long, v);
    const int nlo = __builtin_amdgcn_mov_dpp((int)(i & 0xffffffffll), 0x130, 0xf, 0xf, true);
    const int nhi = __builtin_amdgcn_mov_dpp((int)(i >> 32), 0x130, 0xf, 0xf, true);
    return __builtin_bit_cast(double, ((long long)nhi << 32) | (unsigned int)nlo);
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* base, size_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes, kBufferWord3);
}
__device__ __forceinline__ float2 load_f2(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
__device__ __forceinline__ float4 load_f4(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
__device__ __forceinline__ double2 load_d2(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}

// Exclusive prefix sums of every sweep line of n_mat images for one frame, with
// the line total appended (entry Np).  Line q of frame 0 is image row q; of
// frame 1 image column q.
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
    float2* dst = out + ((size_t)m * Nq + q) * (Np + 1);

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
    if (threadIdx.x == kScanThreads - 1) dst[Np] = make_float2((float)part[kScanThreads - 1], 0.0f);
}

// Per slot and channel: C[b] = orient * sum_{b'<b} sino[b'] path[b'] (FP64),
// b = 0..B; the view's orientation sign makes H(K+1) - H(K) the pixel value.
__global__ __launch_bounds__(kScanThreads) void k_detector_prefix(const float* __restrict__ sino,
                                                                   const float* __restrict__ path,
                                                                   const ViewParams* __restrict__ view, int V,
                                                                   int B, double* __restrict__ C) {
    const int slot = blockIdx.x, ch = blockIdx.y;
    const double orient = (double)view[slot].orient;
    const float* s = sino + ((size_t)ch * V + vp_view(view[slot])) * B;
    const float* pa = path + (size_t)slot * B;
    double* dst = C + ((size_t)ch * V + slot) * (B + 1);
    __shared__ double part[kScanThreads];
    const int per = (B + kScanThreads - 1) / kScanThreads;
    const int b0 = threadIdx.x * per;
    double acc = 0.0;
    for (int i = 0; i < per; ++i) {
        const int b = b0 + i;
        if (b < B) acc += orient * ((double)s[b] * (double)pa[b]);
    }
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        const double add = threadIdx.x >= off ? part[threadIdx.x - off] : 0.0;
        __syncthreads();
        part[threadIdx.x] += add;
        __syncthreads();
    }
    double run = threadIdx.x ? part[threadIdx.x - 1] : 0.0;
    for (int i = 0; i < per; ++i) {
        const int b = b0 + i;
        if (b < B) {
            dst[b] = run;
            run += orient * ((double)s[b] * (double)pa[b]);
        }
    }
    if (threadIdx.x == kScanThreads - 1) dst[B] = part[kScanThreads - 1];
}

// Work of the two sweep frames of one launch.
struct FrameSplit {
    int n_items[2];
};

// XCD-aware decode: block id -> (frame, item); false for padding blocks.
__device__ __forceinline__ bool decode_block(const FrameSplit& fs, int& frame, int& item) {
    const int id = blockIdx.x;
    const int xcd = id & 7;
    frame = xcd >> 2;
    item = (id >> 3) * 4 + (xcd & 3);
    return item < fs.n_items[frame];
}

template <int NK>
__global__ __launch_bounds__(kThreads) void k_dd_forward(const ViewParams* __restrict__ view,
                                                         const float2* __restrict__ bound,
                                                         const float* __restrict__ path,
                                                         const float2* __restrict__ pre_rows,
                                                         const float2* __restrict__ pre_cols, int nv0,
                                                         FrameSplit fs, int chunks, int nx, int ny, int V, int B,
                                                         float* __restrict__ sino) {
    int frame, item;
    if (!decode_block(fs, frame, item)) return;
    const int slot = (frame ? nv0 : 0) + item / chunks;
    const int chunk = item % chunks;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int edge = (chunk * kWaves + wave) * kPerWave + lane;   // boundary index; valid ones are 0..B
    const int Nq = frame ? nx : ny;
    const int Np = frame ? ny : nx;
    const int Lp = Np + 1;
    const __amdgpu_buffer_rsrc_t pre =
        rsrc(frame ? pre_cols : pre_rows, sizeof(float2) * (size_t)NK * Nq * Lp);
    const float2 bd = bound[(size_t)slot * (B + 1) + min(edge, B)];
    const float half = 0.5f * (float)Np;
    float qq = -0.5f * (float)(Nq - 1);
    float acc[NK];
#pragma unroll
    for (int m = 0; m < NK; ++m) acc[m] = 0.0f;
    // one sweep line: F at this lane's boundary, the neighbour's from lane + 1
    auto line_step = [&](int q) {
        const float K = fmaf(bd.y, qq, bd.x);
        qq += 1.0f;
        const float Kc = fminf(fmaxf(K, -half), half);
        const int k = (int)(Kc + half);                          // >= 0, so truncation is floor
        const float f = Kc - ((float)k - half);
        const float inv_w = fast_rcp(next_lane(K) - K);
        const int voff = k * (int)sizeof(float2);
#pragma unroll
        for (int m = 0; m < NK; ++m) {
            const float2 e = load_f2(pre, voff, (m * Nq + q) * Lp * (int)sizeof(float2));
            const float F = fmaf(f, e.y, e.x);
            acc[m] = fmaf(next_lane(F) - F, inv_w, acc[m]);
        }
    };
    int q = 0;
    for (; q + 4 <= Nq; q += 4) {     // trip counts are uniform over the wavefront
        line_step(q);
        line_step(q + 1);
        line_step(q + 2);
        line_step(q + 3);
    }
    for (; q < Nq; ++q) line_step(q);
    if (lane < kPerWave && edge < B) {
        const int v = vp_view(view[slot]);
        const float L = path[(size_t)slot * B + edge];
#pragma unroll
        for (int m = 0; m < NK; ++m) sino[((size_t)m * V + v) * B + edge] = acc[m] * L;
    }
}

template <int NCH>
__global__ __launch_bounds__(kThreads) void k_dd_back(const ViewParams* __restrict__ view,
                                                      const float2* __restrict__ bound, int nv0, int nv1,
                                                      FrameSplit fs, int nx, int ny, int V, int B,
                                                      const double* __restrict__ C, float* __restrict__ x,
                                                      float* __restrict__ xt) {
    int frame, item;
    if (!decode_block(fs, frame, item)) return;
    const int Nq = frame ? nx : ny;
    const int Np = frame ? ny : nx;
    const int segs = (Np + kPerWave - 1) / kPerWave;
    const int seg = item % segs;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int q = (item / segs) * kWaves + wave;
    if (q >= Nq) return;                           // whole wavefront (one line) outside the image
    const int pe = seg * kPerWave + lane;          // edge index; lanes past Np repeat edge Np
    const float half = 0.5f * (float)Np;
    const float qq = (float)q - 0.5f * (float)(Nq - 1);
    const float K = (float)min(pe, Np) - half;
    const int nv = frame ? nv1 : nv0;
    const int slot0 = frame ? nv0 : 0;
    const int row = (B + 1) * (int)sizeof(float2);
    const __amdgpu_buffer_rsrc_t tb = rsrc(bound, sizeof(float2) * (size_t)V * (B + 1));
    const __amdgpu_buffer_rsrc_t tc = rsrc(C, sizeof(double) * (size_t)NCH * V * (B + 1));
    const int crow = (B + 1) * (int)sizeof(double);
    double acc[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) acc[c] = 0.0;
    auto view_step = [&](int is) {
        const int slot = slot0 + is;
        const ViewParams vp = view[slot];
        const float num = fmaf(vp.nK, K, fmaf(vp.nq, qq, vp.n0));
        const float den = fmaf(vp.dK, K, fmaf(vp.dq, qq, vp.d0));
        const int b = min((int)fmaxf(num * fast_rcp(den), 0.0f), B - 1);   // >= 0: truncation is floor
        const float4 cb = load_f4(tb, b * (int)sizeof(float2), slot * row);    // boundaries b, b+1
        const float kb = fmaf(cb.y, qq, cb.x);
        const float kb1 = fmaf(cb.w, qq, cb.z);
        const float fr = fminf(fmaxf((K - kb) * fast_rcp(kb1 - kb), 0.0f), 1.0f);
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            const double2 h = load_d2(tc, b * (int)sizeof(double), (c * V + slot) * crow);
            const double H = fma(h.y - h.x, (double)fr, h.x);
            acc[c] += next_lane(H) - H;
        }
    };
    int is = 0;
    for (; is + 2 <= nv; is += 2) {   // trip counts are uniform over the wavefront
        view_step(is);
        view_step(is + 1);
    }
    for (; is < nv; ++is) view_step(is);
    if (lane < kPerWave && pe < Np) {
        const size_t img_stride = (size_t)nx * ny;
        const size_t pix = (size_t)q * Np + pe;    // frame layout [q][p]
        float* dst = frame ? xt : x;
#pragma unroll
        for (int c = 0; c < NCH; ++c) dst[c * img_stride + pix] = (float)acc[c];
    }
}

// x[c][iy][ix] += xt[c][ix][iy]  (32 x 32 tiles through LDS)
__global__ __launch_bounds__(kThreads) void k_add_transposed(const float* __restrict__ xt, float* __restrict__ x,
                                                             int nx, int ny) {
    __shared__ float tile[32][33];
    const size_t off = (size_t)blockIdx.z * nx * ny;
    const int bx = blockIdx.x * 32, by = blockIdx.y * 32;    // image tile origin (ix, iy)
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8 threads
    for (int r = ty; r < 32; r += 8) {
        const int ix = bx + r, iy = by + tx;                  // xt[ix][iy], coalesced along iy
        if (ix < nx && iy < ny) tile[r][tx] = xt[off + (size_t)ix * ny + iy];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int iy = by + r, ix = bx + tx;
        if (ix < nx && iy < ny) x[off + (size_t)iy * nx + ix] += tile[tx][r];
    }
}

FrameSplit split(int items0, int items1) {
    FrameSplit fs;
    fs.n_items[0] = items0;
    fs.n_items[1] = items1;
    return fs;
}

// 8 blocks per slot of the dispatch order, 4 for each frame.
int grid_blocks(const FrameSplit& fs) {
    const int most = fs.n_items[0] > fs.n_items[1] ? fs.n_items[0] : fs.n_items[1];
    return ((most + 3) / 4) * 8;
}

template <int NK>
void fwd_launch(const GeomTables& t, float* sino, hipStream_t s) {
    const int chunks = (t.B + 1 + kWaves * kPerWave - 1) / (kWaves * kPerWave);
    const FrameSplit fs = split(t.n_frame_views[0] * chunks, t.n_frame_views[1] * chunks);
    const float2* rows = t.prefix;
    const float2* cols = t.prefix + (size_t)t.prefix_mat * t.ny * (t.nx + 1);
    {
        KernelTimer kt_("k_dd_forward", s);
        hipLaunchKernelGGL(k_dd_forward<NK>, dim3(grid_blocks(fs)), dim3(kThreads), 0, s, t.view, t.bound, t.path,
                           rows, cols, t.n_frame_views[0], fs, chunks, t.nx, t.ny, t.V, t.B, sino);
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

template <int NCH>
void back_launch(const GeomTables& t, const float* sino, float* x, hipStream_t s) {
    {
        KernelTimer kt_("k_detector_prefix", s);
        hipLaunchKernelGGL(k_detector_prefix, dim3(t.V, NCH), dim3(kScanThreads), 0, s, sino, t.path,
                           t.view, t.V, t.B, t.det_prefix);
        kt_.stop();
    }
    MBMD_LAUNCHED();
    const int segs0 = (t.nx + kPerWave - 1) / kPerWave, segs1 = (t.ny + kPerWave - 1) / kPerWave;
    const int groups0 = (t.ny + kWaves - 1) / kWaves, groups1 = (t.nx + kWaves - 1) / kWaves;
    const FrameSplit fs = split(t.n_frame_views[0] ? segs0 * groups0 : 0, t.n_frame_views[1] ? segs1 * groups1 : 0);
    if (!t.n_frame_views[0]) launch_fill(NCH * t.nx * t.ny, x, 0.0f, s);
    {
        KernelTimer kt_("k_dd_back", s);
        hipLaunchKernelGGL(k_dd_back<NCH>, dim3(grid_blocks(fs)), dim3(kThreads), 0, s, t.view, t.bound,
                           t.n_frame_views[0], t.n_frame_views[1], fs, t.nx, t.ny, t.V, t.B, t.det_prefix, x,
                           t.back_tmp);
        kt_.stop();
    }
    MBMD_LAUNCHED();
    if (t.n_frame_views[1]) {
        KernelTimer kt_("k_add_transposed", s);
        hipLaunchKernelGGL(k_add_transposed, dim3((t.nx + 31) / 32, (t.ny + 31) / 32, NCH), dim3(kThreads), 0, s,
                           t.back_tmp, x, t.nx, t.ny);
        kt_.stop();
        MBMD_LAUNCHED();
    }
}

// Number of (ray, pixel) pairs with a positive footprint overlap, i.e. the
// nonzeros of A, from the same boundary table the projector uses.
__global__ __launch_bounds__(kThreads) void k_dd_count(const ViewParams* __restrict__ view,
                                                       const float2* __restrict__ bound, int nx, int ny,
                                                       int V, int B, unsigned long long* __restrict__ nnz) {
    __shared__ unsigned long long sh[kThreads];
    const int slot = blockIdx.y;
    const int b = blockIdx.x * kThreads + threadIdx.x;
    unsigned long long cnt = 0;
    if (b < B) {
        const int frame = vp_frame(view[slot]);
        const int Nq = frame ? nx : ny;
        const int Np = frame ? ny : nx;
        const float2 b0 = bound[(size_t)slot * (B + 1) + b];
        const float2 b1 = bound[(size_t)slot * (B + 1) + b + 1];
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
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(nnz, sh[0]);
}

}  // namespace

void launch_project(const GeomTables& t, const float* x, float* sino, int n_mat, hipStream_t s) {
    MBMD_REQUIRE(n_mat >= 1 && n_mat <= kMaxMat, MBMD_ERR_SHAPE, "n_mat must be in 1..4");
    MBMD_REQUIRE(t.prefix != nullptr && t.prefix_mat >= n_mat, MBMD_ERR_ARG, "projector prefix scratch too small");
    for (int frame = 0; frame < 2; ++frame) {
        if (t.n_frame_views[frame] == 0) continue;
        const int Nq = frame ? t.nx : t.ny;
        float2* out = t.prefix + (frame ? (size_t)t.prefix_mat * t.ny * (t.nx + 1) : 0);
        {
            KernelTimer kt_("k_line_prefix", s);
            hipLaunchKernelGGL(k_line_prefix, dim3(Nq, n_mat), dim3(kScanThreads), 0, s, x, out, t.nx, t.ny, frame);
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

void launch_backproject(const GeomTables& t, const float* sino, float* x, int n_ch, hipStream_t s) {
    MBMD_REQUIRE(n_ch >= 1 && n_ch <= kMaxBackCh, MBMD_ERR_SHAPE, "back projection channels must be in 1..10");
    MBMD_REQUIRE(t.det_prefix != nullptr && t.back_ch >= n_ch, MBMD_ERR_ARG, "back projection scratch too small");
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

long long count_nonzeros(const GeomTables& t, hipStream_t s) {
    unsigned long long* d = nullptr;
    MBMD_HIP(hipMalloc(&d, sizeof(unsigned long long)));
    unsigned long long h = 0;
    try {
        MBMD_HIP(hipMemcpyAsync(d, &h, sizeof(h), hipMemcpyHostToDevice, s));
        dim3 grid((t.B + kThreads - 1) / kThreads, t.V);
        hipLaunchKernelGGL(k_dd_count, grid, dim3(kThreads), 0, s, t.view, t.bound, t.nx, t.ny, t.V, t.B, d);
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

}  // namespace mbmd
