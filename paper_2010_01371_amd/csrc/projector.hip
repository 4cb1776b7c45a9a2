// Distance-driven forward and back projection for gfx950.
//
// Both directions use cumulative integrals, so that the work per
// (ray, line) or (pixel, view) is a constant handful of instructions whatever
// the footprint width, with no divergent inner loop.
//
// Forward (ray-driven): each image line of each sweep frame is integrated once
// per call into exclusive prefix sums F[k] = sum_{p<k} img[p] (FP64
// accumulation, stored FP32).  F is linear inside a pixel, so the integral of
// the line over a footprint [K_b, K_b+1] is F(K_b+1) - F(K_b).  Each lane owns
// two neighbouring bin BOUNDARIES and takes the next lane's first one with a
// wave shift, giving 127 bins per wavefront; one 16-byte read of F[k..k+3]
// serves both boundaries when no bin is wider than two pixels.  The footprint
// width is the difference of the same two FP32 boundary positions that F is
// evaluated at, so position rounding cancels to first order in the ratio (the
// exact width would not); signs cancel too, whatever the orientation of the
// view.  Each wavefront's active lines are split into two work items added
// atomically onto the cleared output (two additions onto zero commute), taken
// heaviest first.
//
// Back projection (pixel-driven gather): per call and view the sinogram times
// the per-line path length is integrated over the detector in FP64, C[b] =
// sum_{b'<b} w[b'], in increasing-K order (the rows of views whose bins run
// along -K are stored from the last bin, with the map of the reversed index).
// The back projected detector signal on a sweep line is piecewise constant in
// the along-line position K, with cumulative integral H(K) = C[b] + w[b] (K -
// K_b)/(K_b+1 - K_b) for K in bin b, so a pixel [K, K+1] receives H(K+1) -
// H(K).  Lanes own pixel EDGES (one or two per lane: 63 or 127 pixels per
// wavefront), sum H over the views and take pixel values as differences of
// neighbouring edges' sums.  The bin holding an edge and the fraction
// (K - K_b)/(K_b+1 - K_b) come from the projective map K -> fractional bin
// index restricted to the sweep line, whose per-line coefficients are read
// with scalar loads; the only per-lane table read is a 16-byte detector entry
// {C[b+1], w[b], w[b+1]}, which serves both edges of a lane.  The fractions are
// clamped to [0, 1], which keeps H continuous when the bin index is off by
// rounding near a boundary.  Sums over views of C are FP64 (full rate on
// CDNA), the in-bin parts (within one bin width) FP32.  Every pixel is the sum
// of two halves of its views, added onto zero, which two wavefronts may do with
// atomics (they commute exactly): results are bitwise reproducible whatever
// the tile shape.
//
// Table reads go through buffer loads (32-bit offsets from a base held in
// scalar registers; out-of-range offsets read zero), neighbour exchanges are
// DPP wave shifts, and the line / view loops are unrolled so that several
// loads are in flight per wavefront.
//
// Views sweeping rows and views sweeping columns are interleaved in one launch
// with an XCD-aware block order: blocks are dispatched round-robin to the 8
// XCDs, and blocks landing on XCDs 0-3 take row-sweep work, 4-7 column-sweep
// work, so each XCD's L2 holds one frame's tables.  The column-sweep part of a
// back projection is written in image layout to a buffer of its own and added
// by the caller (the iteration does it in the penalty pass).
#include <cmath>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <type_traits>

#include "back_rows.h"
#include "internal.h"

namespace mbmd {

namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
// Pixels per wavefront of the back projection's main path: 63 with one pixel
// edge per lane, 127 with two.
__host__ __device__ constexpr int back_ppw(int epl) { return epl == 2 ? 127 : 63; }

// Back projection tiling of a sweep line of Np pixels (Np + 1 edges): full
// segments of ppw pixels, then the pixels left over (Np mod ppw) as a tail of
// tail_edges edges, packed tail_lines lines per wavefront -- one wavefront per
// line there would spend a whole wavefront's time on a handful of lanes.  A
// tail that would not fit two lines per wavefront is an ordinary partial
// segment instead (counted in full; lanes past the last edge repeat it).
struct BackTiling {
    int full, tail_edges, tail_lines;
};
__host__ __device__ inline BackTiling back_tiling(int Np, int ppw) {
    BackTiling b{Np / ppw, 0, 0};
    const int rem = Np - b.full * ppw;
    if (rem > 0) {
        b.tail_edges = rem + 1;
        b.tail_lines = 64 / b.tail_edges;
        if (b.tail_lines < 2) b = BackTiling{b.full + 1, 0, 0};
    }
    return b;
}
// Blocks (kWaves wavefronts) of one sweep frame: the tail, then segments x line groups.
__host__ __device__ inline int back_main_items(int Np, int Nq, int lpw, int ppw) {
    return back_tiling(Np, ppw).full * ((Nq + kWaves * lpw - 1) / (kWaves * lpw));
}
// Tail blocks: each tail wavefront's views are split into two halves (items
// 2 i and 2 i + 1), whose pixel values are added onto the cleared tail pixels.
__host__ __device__ inline int back_tail_items(int Np, int Nq, int ppw) {
    const BackTiling b = back_tiling(Np, ppw);
    if (!b.tail_lines) return 0;
    const int waves = (Nq + b.tail_lines - 1) / b.tail_lines;
    return 2 * ((waves + kWaves - 1) / kWaves);
}
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
// One detector entry as loaded: C[b+1] and the widths of bins b and b + 1.  A word
// that the reader does not use is kept live until the entry is consumed (see
// keep()), since otherwise the compiler reuses its register as a temporary and
// must wait for the load.
struct DetValue {
    double c;
    float d;
    float dn;
};
__device__ __forceinline__ DetValue load_det(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(DetValue, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
}
// Marks a register as read here (an empty instruction string: no code).
__device__ __forceinline__ void keep(float v) { asm volatile("" ::"v"(v)); }

// One view's detector values at a lane's edge for NCH channels (see
// kPackFrom): two 16-byte gathers per triple of channels (planes A and B), one
// per remaining channel, all at the same entry offset.
template <int NCH>
struct DetView {
    static constexpr int T = NCH >= kPackFrom ? NCH / 3 : 0;     // triples
    static constexpr int L = NCH - 3 * T;                        // channels with rows of their own
    float4 a[T ? T : 1], b[T ? T : 1];
    DetValue e[L ? L : 1];
};
// The values at entry offset off (bytes) of a view whose row starts soff bytes
// into the first set of rows; vstride: the distance between sets of rows (V
// rows, bytes).  Triple t takes sets 2 t and 2 t + 1, the remaining channels
// one set each after the triples.
template <int NCH>
__device__ __forceinline__ void load_view(__amdgpu_buffer_rsrc_t r, int off, int soff, int vstride,
                                          DetView<NCH>& v) {
    constexpr int T = DetView<NCH>::T;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        v.a[t] = load_f4(r, off, soff + 2 * t * vstride);
        v.b[t] = load_f4(r, off, soff + (2 * t + 1) * vstride);
    }
#pragma unroll
    for (int j = 0; j < DetView<NCH>::L; ++j) v.e[j] = load_det(r, off, soff + (2 * T + j) * vstride);
}
// Adds one view: per channel the FP64 sum of C[b+1] (a triple's q 2^-s with the
// row scale sc[c], an exact product, so the one rounding is the sum's, as for
// an entry of its own) and the FP32 sum of (fr - 1) w[b].
template <int NCH>
__device__ __forceinline__ void add_view(const DetView<NCH>& v, float fr, const double* sc, double* acc,
                                         float* accw) {
#pragma unroll
    for (int t = 0; t < DetView<NCH>::T; ++t) {
        const int hi[3] = {__float_as_int(v.a[t].x), __float_as_int(v.a[t].y), __float_as_int(v.a[t].z)};
        const unsigned l01 = __float_as_uint(v.a[t].w);
        const unsigned lo[3] = {l01 & 0xffffu, l01 >> 16, __float_as_uint(v.b[t].w)};
        const float w[3] = {v.b[t].x, v.b[t].y, v.b[t].z};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const int c = 3 * t + k;
            const double q = __builtin_fma((double)hi[k], 65536.0, (double)lo[k]);   // exact: |q| < 2^47
            acc[c] = __builtin_fma(q, sc[c], acc[c]);
            accw[c] = fmaf(fr, w[k], accw[c] - w[k]);
        }
    }
#pragma unroll
    for (int j = 0; j < DetView<NCH>::L; ++j) {
        const int c = 3 * DetView<NCH>::T + j;
        acc[c] += v.e[j].c;                                      // C[b+1]
        accw[c] = fmaf(fr, v.e[j].d, accw[c] - v.e[j].d);        // + (fr - 1) w[b]
        keep(v.e[j].dn);
    }
}

// Exclusive prefix sums F[p] = sum_{p'<p} img[p'] (FP64 accumulation, stored
// FP32) of every sweep line of n_mat images, entries Np .. Np+3 holding the line
// total.  One block per line: blocks [0, ny) take the rows (frame 0), blocks
// [ny, ny+nx) the columns (frame 1); a frame without views is skipped by the
// caller's grid.
__global__ __launch_bounds__(kScanThreads) void k_line_prefix(const float* __restrict__ img,
                                                               float* __restrict__ rows, float* __restrict__ cols,
                                                               int nx, int ny, int line0,
                                                               float* __restrict__ zero_out, int zero_n,
                                                               const long long* __restrict__ zd, int img_is_x) {
    if (zd) {                                                  // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        img = zshift(img, img_is_x ? zoff(zd, Z_IMAGE) : d);
        rows = zshift(rows, d);
        cols = zshift(cols, d);
        zero_out = zshift(zero_out, d);
    }
    // side job: clear the projection's output, which the forward adds into
    for (int i = (blockIdx.y * gridDim.x + blockIdx.x) * kScanThreads + threadIdx.x; i < zero_n;
         i += gridDim.x * gridDim.y * kScanThreads)
        zero_out[i] = 0.0f;
    const int line = line0 + blockIdx.x;
    const int m = blockIdx.y;
    const int frame = line >= ny ? 1 : 0;
    const int q = frame ? line - ny : line;
    const int Nq = frame ? nx : ny;
    const int Np = frame ? ny : nx;
    const float* src = img + (size_t)m * nx * ny;
    const size_t elem_stride = frame ? (size_t)nx : 1;
    const size_t line_off = frame ? (size_t)q : (size_t)q * nx;
    float* dst = (frame ? cols : rows) + ((size_t)m * Nq + q) * prefix_row(Np);

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
            dst[p] = (float)run;
            run += (double)src[line_off + (size_t)p * elem_stride];
        }
    }
    if (threadIdx.x < 4) dst[Np + threadIdx.x] = (float)part[kScanThreads - 1];
}

// Per slot, the detector rows (see build_detector_row, and build_triple_rows
// for the channels in triples) of the widths w[b] = sino[b'] path[b'] of the
// bins in increasing-K order (b' = b, or B - 1 - b for views with orient < 0).
// One workgroup per (slot, triple) and per (slot, channel outside triples):
// blockIdx.y < T takes triple blockIdx.y, the others channel 3 T + blockIdx.y -
// T.  Every workgroup also clears its share of the pixels the back projection
// kernel adds into.
constexpr int kPrefixThreads = kRowThreads;
__global__ __launch_bounds__(kPrefixThreads) void k_detector_prefix(const float* __restrict__ sino,
                                                                     const float* __restrict__ path,
                                                                     const ViewParams* __restrict__ view, int V,
                                                                     int B, int nch, DetEntry* __restrict__ C,
                                                                     BackClear tc, const long long* __restrict__ zd) {
    if (zd) {                                                  // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        sino = zshift(sino, d);
        path = zshift(path, d);
        view = zshift(view, d);
        C = zshift(C, d);
        tc.x = zshift(tc.x, d);
        tc.part = zshift(tc.part, d);
    }
    clear_back_pixels(tc, blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);   // side job
    const int slot = blockIdx.x, set = blockIdx.y;
    const bool rev = view[slot].orient < 0.0f;
    const float* pa = path + (size_t)slot * B;
    const int vw = vp_view(view[slot]);
    __shared__ double lds[12 * kPrefixThreads / 64];
    char* rows = reinterpret_cast<char*>(C);
    const int T = det_triples(nch);
    if (set < T) {                                                // uniform
        const float* s = sino + ((size_t)(3 * set) * V + vw) * B;
        const size_t cs = (size_t)V * B;                          // channel stride of sino
        build_triple_rows(
            [&](int k, int b) {                                   // b in row order, < B
                const int i = rev ? B - 1 - b : b;
                return (float)((double)s[k * cs + i] * (double)pa[i]);
            },
            B, C + ((size_t)2 * set * V + slot) * det_row(B), (size_t)V * det_row(B),
            reinterpret_cast<double*>(rows + det_scales(nch, V, B)) + (size_t)slot * 3 * T + 3 * set, lds);
    } else {
        const int ch = 3 * T + (set - T);
        const float* s = sino + ((size_t)ch * V + vw) * B;
        DetEntry* single = reinterpret_cast<DetEntry*>(rows + det_single_base(nch, V, B));
        build_detector_row(
            [&](int b) {                                          // b in row order, < B
                const int i = rev ? B - 1 - b : b;
                return (float)((double)s[i] * (double)pa[i]);
            },
            B, single + ((size_t)(set - T) * V + slot) * det_row(B), lds);
    }
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
    return item < (frame ? fs.n_items[1] : fs.n_items[0]);   // no dynamic index into the by-value array
}

template <int NK>
__global__ __launch_bounds__(kFwdWaves * 64) void k_dd_forward(const ViewParams* __restrict__ view,
                                                         const float2* __restrict__ bound,
                                                         const float* __restrict__ path,
                                                         const float* __restrict__ pre_rows,
                                                         const float* __restrict__ pre_cols, int nv0,
                                                         FrameSplit fs, const int* __restrict__ order, int chunks,
                                                         int nx, int ny, int V, int B, float* __restrict__ sino,
                                                         const long long* __restrict__ zd) {
    if (zd) {                                                  // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        view = zshift(view, d);
        bound = zshift(bound, d);
        path = zshift(path, d);
        pre_rows = zshift(pre_rows, d);
        pre_cols = zshift(pre_cols, d);
        order = zshift(order, d);
        sino = zshift(sino, d);
    }
    int frame, item;
    if (!decode_block(fs, frame, item)) return;
    item = order[(frame ? fs.n_items[0] : 0) + item];             // heaviest items first
    const int half = item & 1;                                    // which half of the active lines
    item >>= 1;
    const int slot = (frame ? nv0 : 0) + item / chunks;
    const int chunk = item % chunks;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int e0 = (chunk * kFwdWaves + wave) * kFwdBinsPerWave;  // first boundary of the wavefront
    if (e0 >= B) return;                                          // whole wavefront: no bins
    const int Nq = frame ? nx : ny;
    const int Np = frame ? ny : nx;
    const int Lp = prefix_row(Np);
    const __amdgpu_buffer_rsrc_t pre = rsrc(frame ? pre_cols : pre_rows, sizeof(float) * (size_t)NK * Nq * Lp);
    // boundaries ea (bin ea = [ea, eb] in this lane) and eb (bin eb = [eb, next lane's ea])
    const int ea = min(e0 + 2 * lane, B), eb = min(e0 + 2 * lane + 1, B);
    const float2* brow = bound + (size_t)slot * (B + 1);
    const float2 ba = brow[ea], bb = brow[eb];
    const float Npf = (float)Np;
    float acc_a[NK], acc_b[NK];
#pragma unroll
    for (int m = 0; m < NK; ++m) acc_a[m] = acc_b[m] = 0.0f;
    // Only lines on which some boundary of this wavefront lies inside the image
    // contribute: elsewhere every lane's position clamps to the same end of the
    // line, F is equal across lanes and the differences are exactly zero.
    int q_lo = 0, q_hi = -1;
    active_lines(brow[e0], brow[min(e0 + kFwdBinsPerWave, B)], Np, Nq, q_lo, q_hi);
    // Two wavefronts share these lines, one half each, and add their sums into
    // the cleared output: the heavy wavefronts (bins that cross the image on
    // every line) are then twice as many and half as long.  Two additions onto
    // zero give the same result in either order.
    {
        const int q_mid = (q_lo + q_hi + 1) >> 1;
        if (half) q_lo = q_mid;
        else q_hi = q_mid - 1;
    }
    // The in-lane bin width is affine in q, so its largest value over the active
    // lines is at an end: at most two pixels everywhere means X_b lies in the
    // four-entry window that starts at floor(X_a).
    float wmax = 0.0f;
    if (q_lo <= q_hi) {
        const float w0 = fabsf(fmaf(bb.y - ba.y, (float)q_lo, bb.x - ba.x));
        const float w1 = fabsf(fmaf(bb.y - ba.y, (float)q_hi, bb.x - ba.x));
        wmax = fmaxf(w0, w1);
        for (int off = 32; off > 0; off >>= 1) wmax = fmaxf(wmax, __shfl_xor(wmax, off, 64));
    }
    const bool narrow = wmax < 1.99f;                             // uniform over the wavefront
    // one sweep line at boundary positions Xa, Xb; NARROW: both boundaries' F
    // from one 16-byte read of F[k..k+3], else one 8-byte read of F[k], F[k+1]
    // per boundary
    auto line_step = [&](int q, float Xa, float Xb, auto narrow_tag) {
        constexpr bool NARROW = decltype(narrow_tag)::value;
        const float Xca = __builtin_amdgcn_fmed3f(Xa, 0.0f, Npf), Xcb = __builtin_amdgcn_fmed3f(Xb, 0.0f, Npf);
        const float sa = fast_rcp(Xb - Xa);                        // in-lane bin width
        const float sb = fast_rcp(next_lane(Xa) - Xb);             // bin across to the next lane
        const float kf = floorf(Xca);
        const int k = (int)kf;
        const float da = Xca - kf;
#pragma unroll
        for (int m = 0; m < NK; ++m) {
            const int row = (m * Nq + q) * Lp * (int)sizeof(float);
            float Fa, Fb;
            if constexpr (NARROW) {
                // F is piecewise linear on [k, k+3]: its value at k + db is
                // F[k] plus the clamped parts of db in each pixel times the pixel
                const float db = Xcb - kf;                         // in [da, 3)
                const float4 e = load_f4(pre, k * (int)sizeof(float), row);
                const float d0 = e.y - e.x;
                Fa = fmaf(da, d0, e.x);
                const float c0 = fminf(db, 1.0f);
                const float c1 = __builtin_amdgcn_fmed3f(db - 1.0f, 0.0f, 1.0f);
                const float c2 = __builtin_amdgcn_fmed3f(db - 2.0f, 0.0f, 1.0f);   // db < 3
                Fb = fmaf(c2, e.w - e.z, fmaf(c1, e.z - e.y, fmaf(c0, d0, e.x)));
            } else {
                const float2 ea2 = load_f2(pre, k * (int)sizeof(float), row);
                const float2 eb2 = load_f2(pre, (int)Xcb * (int)sizeof(float), row);
                Fa = fmaf(da, ea2.y - ea2.x, ea2.x);
                Fb = fmaf(__builtin_amdgcn_fractf(Xcb), eb2.y - eb2.x, eb2.x);
            }
            acc_a[m] = fmaf(Fb - Fa, sa, acc_a[m]);
            acc_b[m] = fmaf(next_lane(Fa) - Fb, sb, acc_b[m]);
        }
    };
    // Positions are affine in q: one FMA from the line index per group of four
    // lines, then steps of the slope with inline-constant multipliers.
    auto sweep = [&](auto narrow_tag) {
        int q = q_lo;
        for (; q + 4 <= q_hi + 1; q += 4) {   // trip counts are uniform over the wavefront
            const float qf = (float)q;
            const float Xa0 = fmaf(ba.y, qf, ba.x), Xb0 = fmaf(bb.y, qf, bb.x);
            const float Xa1 = Xa0 + ba.y, Xb1 = Xb0 + bb.y;
            line_step(q, Xa0, Xb0, narrow_tag);
            line_step(q + 1, Xa1, Xb1, narrow_tag);
            line_step(q + 2, fmaf(ba.y, 2.0f, Xa0), fmaf(bb.y, 2.0f, Xb0), narrow_tag);
            line_step(q + 3, fmaf(ba.y, 2.0f, Xa1), fmaf(bb.y, 2.0f, Xb1), narrow_tag);
        }
        for (; q <= q_hi; ++q) {
            const float qf = (float)q;
            line_step(q, fmaf(ba.y, qf, ba.x), fmaf(bb.y, qf, bb.x), narrow_tag);
        }
    };
    if (narrow)
        sweep(std::true_type{});
    else
        sweep(std::false_type{});
    // bins in table order; views stored reversed map bin i to B - 1 - i
    const bool rev = view[slot].orient < 0.0f;
    const int v = vp_view(view[slot]);
    const int bin_a = ea, bin_b = eb;
    if (bin_a < B && bin_a < e0 + kFwdBinsPerWave) {
        const int o = rev ? B - 1 - bin_a : bin_a;
        const float L = path[(size_t)slot * B + o];
#pragma unroll
        for (int m = 0; m < NK; ++m) unsafeAtomicAdd(&sino[((size_t)m * V + v) * B + o], acc_a[m] * L);
    }
    if (lane < 63 && bin_b < B && bin_b < e0 + kFwdBinsPerWave) {
        const int o = rev ? B - 1 - bin_b : bin_b;
        const float L = path[(size_t)slot * B + o];
#pragma unroll
        for (int m = 0; m < NK; ++m) unsafeAtomicAdd(&sino[((size_t)m * V + v) * B + o], acc_b[m] * L);
    }
}

// One (sweep line, view) at along-line position K: byte offset of the edge's
// detector entry and the fraction of its bin.  m = {n, m, c, a}, g: the line's
// map coefficients; span = back_shift(B) (the clamp, symmetric about the
// detector centre), origin = span entries in bytes.
__device__ __forceinline__ void back_locate(const float4& m, float g, float K, float span, int origin, int& off,
                                            float& fr) {
    const float den = fmaf(m.z, K, 1.0f);
    const float num = fmaf(m.y, K, m.x);
    const float bf = __builtin_amdgcn_fmed3f(floorf(num * fast_rcp(den)), -span, span);
    off = (int)bf * (int)sizeof(DetEntry) + origin;          // entry in [0, B + 1]
    fr = __builtin_amdgcn_fmed3f(fmaf(-bf, den, num) * fmaf(-g, bf, m.w), 0.0f, 1.0f);
}

// Both edges of a lane on one (sweep line, view): edge A at K, edge B at K + 1.
// The map increases with K, so edge B's bin is at least edge A's bin b0, and
//   H(A) = C[b0+1] + (frA - 1) w[b0],
//   H(B) = C[b0+1] + (f0 - 1) w[b0] + f1 w[b0+1]
// with f0, f1 the clamped fractions of bins b0 and b0 + 1 covered up to edge B
// (the projective fraction formula holds for any bin, so no second division);
// one entry (C[b0+1], w[b0], w[b0+1]) serves both edges, and both FP32 parts
// stay within one bin width.  When edge B lies past bin b0 + 1 (f1 reaches 1),
// it is wide and takes its own entry.
struct EdgePair {
    int off;            // byte offset of the entry of b0
    float frA, f0, f1;
};
__device__ __forceinline__ EdgePair back_pair(const float4& m, float g, float K, float span, int origin) {
    EdgePair e;
    const float den = fmaf(m.z, K, 1.0f);
    const float num = fmaf(m.y, K, m.x);
    // -b0 (the clamp is symmetric), so that every use below is a plain FMA
    const float nbf = __builtin_amdgcn_fmed3f(-floorf(num * fast_rcp(den)), -span, span);
    e.off = (int)(-nbf) * (int)sizeof(DetEntry) + origin;
    const float qa = fmaf(g, nbf, m.w);                         // bin b0's scale
    e.frA = __builtin_amdgcn_fmed3f(fmaf(nbf, den, num) * qa, 0.0f, 1.0f);
    const float denB = den + m.z, numB = num + m.y;             // at K + 1
    const float n0 = fmaf(nbf, denB, numB);
    e.f0 = __builtin_amdgcn_fmed3f(n0 * qa, 0.0f, 1.0f);
    e.f1 = __builtin_amdgcn_fmed3f((n0 - denB) * (qa - g), 0.0f, 1.0f);
    return e;
}

// The tail of every sweep line (see back_tiling): lane l of tail wavefront tw
// takes edge full*ppw + l mod E of line tw*LT + l / E, so each lane reads
// its own line's coefficients (vector loads: LT distinct addresses per
// wavefront).  Views [is0, is1) go in groups of UT with the next group's
// coefficients in flight while this group's detector entries arrive, summed in
// view order; the pixel values (FP64 differences of the lanes' sums, then FP32)
// are added onto the tail pixels, which the detector-prefix launch clears: the
// two halves of the views add once each, which gives the same result in either
// order.
template <int NCH>
__device__ __forceinline__ void back_tail(const float4* __restrict__ line_tab, int tw, int is0, int is1, int slot0,
                                          int Np, int Nq, int V, int B, int frame, int nx, int ny, int ppw,
                                          const __amdgpu_buffer_rsrc_t& tc, int row, const double* __restrict__ sct,
                                          float* __restrict__ dst) {
    constexpr int UT = NCH <= 2 ? 4 : 2;   // keeps the tail within the main path's registers
    if (is0 >= is1) return;                // no views in this half (uniform)
    const BackTiling bt = back_tiling(Np, ppw);
    const int E = bt.tail_edges, LT = bt.tail_lines;
    const int lane = threadIdx.x & 63;
    const int ql = lane / E, el = lane - ql * E;
    const int q = tw * LT + ql;
    const bool lane_ok = ql < LT && q < Nq;
    const int pe = min(bt.full * ppw + el, Np);
    const float K = (float)pe - 0.5f * (float)Np;
    const float4* lt = line_tab + (size_t)min(q, Nq - 1) * V * 2;
    const float* ltf = reinterpret_cast<const float*>(lt);
    const int shift = back_shift(B);
    const float span = (float)shift;
    const int origin = shift * (int)sizeof(DetEntry);
    double acc[NCH];
    float accw[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
        acc[c] = 0.0;
        accw[c] = 0.0f;
    }
    float4 tm[UT];
    float tg[UT];
    auto fetch = [&](int is) {
#pragma unroll
        for (int u = 0; u < UT; ++u) {
            const int slot = slot0 + min(is + u, is1 - 1);
            tm[u] = lt[2 * slot];
            tg[u] = ltf[4 * (2 * slot + 1)];
        }
    };
    fetch(is0);
    for (int is = is0; is < is1; is += UT) {                   // uniform
        int off[UT];
        float fr[UT];
#pragma unroll
        for (int u = 0; u < UT; ++u) back_locate(tm[u], tg[u], K, span, origin, off[u], fr[u]);
        DetView<NCH> h[UT];
#pragma unroll
        for (int u = 0; u < UT; ++u)
            load_view<NCH>(tc, off[u], (slot0 + min(is + u, is1 - 1)) * row, V * row, h[u]);
        fetch(is + UT);
        constexpr int NT = 3 * DetView<NCH>::T;                // triple channels: their rows' scales
        double sc[UT][NT ? NT : 1];
#pragma unroll
        for (int u = 0; u < UT; ++u)
#pragma unroll
            for (int c = 0; c < NT; ++c) sc[u][c] = sct[(size_t)(slot0 + min(is + u, is1 - 1)) * NT + c];
#pragma unroll
        for (int u = 0; u < UT; ++u) {
            if (is + u >= is1) break;                          // uniform
            add_view<NCH>(h[u], fr[u], sc[u], acc, accw);
        }
    }
    const size_t img_stride = (size_t)nx * ny;
    float val[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c)
        val[c] = (float)((next_lane(acc[c]) - acc[c]) + (double)(next_lane(accw[c]) - accw[c]));
    if (lane_ok && el < E - 1) {                               // pixel pe, whose right edge is the next lane
        const size_t pix = frame ? (size_t)pe * nx + q : (size_t)q * nx + pe;
#pragma unroll
        for (int c = 0; c < NCH; ++c) unsafeAtomicAdd(&dst[c * img_stride + pix], val[c]);
    }
}

// One block: kWaves wavefronts x LPW adjacent sweep lines each, one segment of
// back_ppw(EPL) pixels (EPL edges per lane); every wavefront walks all views of
// its frame, or one half of them.  Several lines per wavefront give each wave
// LPW independent load chains per view, which is what hides the memory
// latency.  EPL = 1: per lane, line and channel, the FP64 sum over views of
// C[b+1] and the FP32 sum of (fr - 1) w[b] at the lane's edge; the pixel is the
// difference of the next lane's sums and its own.  EPL = 2: the FP64 sum over
// views of C[b0+1] and the FP32 sums of H(A) - C[b0+1] and H(B) - C[b0+1]; the
// pixel between the lane's edges is the difference of the two FP32 sums, the
// pixel after edge B takes the next lane's sums.  Two edges per lane halve the
// gathers and the locate work of edge B; one edge per lane gives twice the
// wavefronts and fewer registers, which small images with several channels
// need.  Row sweeps write x; column sweeps write their partial image to part in
// the image's own layout (scattered 4-byte stores, once per pixel), which the
// caller adds -- the iteration does it inside the penalty kernel.
template <int NCH, int LPW, int U, int EPL>
__global__ __launch_bounds__(kThreads) void k_dd_back(const float4* __restrict__ line_tab, int nv0, int nv1,
                                                      FrameSplit fs, int nx, int ny, int V, int B,
                                                      const DetEntry* __restrict__ C, float* __restrict__ x,
                                                      float* __restrict__ part, int vsplit,
                                                      const long long* __restrict__ zd) {
    {                                                          // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        line_tab = zadd(line_tab, d);
        C = zadd(C, d);
        x = zadd(x, d);
        part = zshift(part, d);
    }
    int frame, item;
    if (!decode_block(fs, frame, item)) return;
    const int Nq = frame ? nx : ny;
    const int Np = frame ? ny : nx;
    const int nv = frame ? nv1 : nv0;
    const int slot0 = frame ? nv0 : 0;
    const int row = det_row(B) * (int)sizeof(DetEntry);
    const __amdgpu_buffer_rsrc_t tc = rsrc(C, det_scales(NCH, V, B));
    // the triples' scales [slot][3 T]
    const double* sct = reinterpret_cast<const double*>(reinterpret_cast<const char*>(C) + det_scales(NCH, V, B));
    constexpr int NT = 3 * DetView<NCH>::T;
    // the tail items come first: their wavefronts are the longest, so they are
    // dispatched before the main ones fill the machine
    constexpr int PPW = back_ppw(EPL);
    const int tail_items = back_tail_items(Np, Nq, PPW);
    if (item < tail_items) {
        const int tw = (item >> 1) * kWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        if (tw * back_tiling(Np, PPW).tail_lines >= Nq) return;      // whole wavefront past the last line
        const int mid = nv >> 1;
        back_tail<NCH>(line_tab, tw, (item & 1) ? mid : 0, (item & 1) ? nv : mid, slot0, Np, Nq, V, B, frame, nx,
                       ny, PPW, tc, row, sct, frame ? part : x);
        return;
    }
    item -= tail_items;
    // Every pixel value is the sum of two half values, views [0, nv/2) and
    // [nv/2, nv), added onto zero in that order: with split views items 2 i and
    // 2 i + 1 each add one half onto the cleared image (two additions onto zero
    // give the same result in either order); unsplit, a wavefront does both
    // halves itself.  Both schedules give the same bits.
    const int half = vsplit == 2 ? item & 1 : 0;
    if (vsplit == 2) item >>= 1;
    const int segs = back_tiling(Np, PPW).full;
    const int seg = item % segs;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int q0 = ((item / segs) * kWaves + wave) * LPW;
    if (q0 >= Nq) return;                          // whole wavefront outside the image
    const int pe = seg * PPW + EPL * lane;         // (first) edge; lanes past Np repeat edge Np
    const float K = (float)min(pe, Np) - 0.5f * (float)Np;
    // first table entry of each line, kept in scalar registers
    int lt0[LPW];
#pragma unroll
    for (int j = 0; j < LPW; ++j) lt0[j] = __builtin_amdgcn_readfirstlane(min(q0 + j, Nq - 1) * V * 2);
    const int shift = back_shift(B);
    const float span = (float)shift;               // bin index clamp, symmetric about the centre
    const int origin = shift * (int)sizeof(DetEntry);
    const size_t img_stride = (size_t)nx * ny;
    float* dst = frame ? part : x;
    // pixel values summed over the halves taken (EPL = 2: pixels pe and pe + 1)
    float outa[LPW][NCH], outb[LPW][NCH];
#pragma unroll
    for (int j = 0; j < LPW; ++j)
#pragma unroll
        for (int c = 0; c < NCH; ++c) outa[j][c] = outb[j][c] = 0.0f;
    int sl0 = 0, nvh = 0;                          // first slot and number of views of the half
    // Software pipeline over groups of U views: the per-line tables of the next
    // group are requested (scalar loads) only after this group's values are in
    // registers -- scalar loads complete out of order, so a wait for one waits
    // for all -- and land while this group's detector gathers are in flight.
    float4 tm[U][LPW];
    float tg[U][LPW];
    // Each line's entries of the half start at lp[j]; a group's entries lie at
    // constant offsets from its first view's, so the scalar loads take immediate
    // offsets from one base per line (one 64-bit add per line and group).  The
    // prefetch after the last full group reads up to 2 U - 2 entries past the
    // half's views: they are never used, and the table is padded at its end.
    static_assert(U <= kBackMaxU, "the per-line table is padded for kBackMaxU views in flight");
    const float4* lp[LPW];
    auto fetch = [&](int is) {
#pragma unroll
        for (int j = 0; j < LPW; ++j) {
            const float4* grp = lp[j] + 2 * is;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                tm[u][j] = grp[2 * u];                                               // {n, m, c, a}
                tg[u][j] = reinterpret_cast<const float*>(grp + 2 * u + 1)[0];       // g
            }
        }
    };
    for (int h = half; h < (vsplit == 2 ? half + 1 : 2); ++h) {   // uniform
        const int iv0 = h ? nv >> 1 : 0, iv1 = h ? nv : nv >> 1;
        if (iv0 >= iv1) continue;                  // no views in this half: it adds zero
        sl0 = slot0 + iv0;
        nvh = iv1 - iv0;
#pragma unroll
        for (int j = 0; j < LPW; ++j) lp[j] = line_tab + lt0[j] + 2 * sl0;
        const int nfull = nvh - nvh % U;
        if constexpr (EPL == 1) {
            double acc[LPW][NCH];                   // sum over views of C[b+1]
            float accw[LPW][NCH];                   // sum over views of (fr - 1) w[b]
#pragma unroll
            for (int j = 0; j < LPW; ++j)
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    acc[j][c] = 0.0;
                    accw[j][c] = 0.0f;
                }
            const double* scp = sct + (size_t)sl0 * NT;      // the half's triple scales
            fetch(0);
            for (int is = 0; is < nfull; is += U) {   // trip counts are uniform over the wavefront
                int off[U][LPW];
                float frs[U][LPW];
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int j = 0; j < LPW; ++j)
                        back_locate(tm[u][j], tg[u][j], K, span, origin, off[u][j], frs[u][j]);
                DetView<NCH> hv[U][LPW];
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int j = 0; j < LPW; ++j)
                        load_view<NCH>(tc, off[u][j], (sl0 + is + u) * row, V * row, hv[u][j]);
                // the scales of this group's triple rows arrive with the next group's tables
                double sc[U][NT ? NT : 1];
                __builtin_amdgcn_sched_barrier(0);
                fetch(is + U);
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int c = 0; c < NT; ++c) sc[u][c] = scp[(is + u) * NT + c];
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int j = 0; j < LPW; ++j) add_view<NCH>(hv[u][j], frs[u][j], sc[u], acc[j], accw[j]);
            }
            // the remaining views (fewer than U); their tables were fetched into slots 0..
#pragma unroll
            for (int u = 0; u < U - 1; ++u) {
                if (nfull + u >= nvh) break;   // uniform
                double sc[NT ? NT : 1];
#pragma unroll
                for (int c = 0; c < NT; ++c) sc[c] = scp[(nfull + u) * NT + c];
#pragma unroll
                for (int j = 0; j < LPW; ++j) {
                    int o;
                    float fr;
                    back_locate(tm[u][j], tg[u][j], K, span, origin, o, fr);
                    DetView<NCH> hr;
                    load_view<NCH>(tc, o, (sl0 + nfull + u) * row, V * row, hr);
                    add_view<NCH>(hr, fr, sc, acc[j], accw[j]);   // as in the main loop
                }
            }
#pragma unroll
            for (int j = 0; j < LPW; ++j)
#pragma unroll
                for (int c = 0; c < NCH; ++c)
                    outa[j][c] += (float)((next_lane(acc[j][c]) - acc[j][c]) +
                                          (double)(next_lane(accw[j][c]) - accw[j][c]));
        } else {
            static_assert(NCH < kPackFrom, "two edges per lane read unpacked rows (one or two channels)");
            double acc[LPW][NCH];                   // sum over views of C[b0+1]
            float wa[LPW][NCH], wb[LPW][NCH];       // sums over views of H(A) - C[b0+1], H(B) - C[b0+1]
            double accw64[LPW][NCH];                // the part of the latter from wide lanes' C[bB+1] - C[b0+1]
#pragma unroll
            for (int j = 0; j < LPW; ++j)
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    acc[j][c] = 0.0;
                    accw64[j][c] = 0.0;
                    wa[j][c] = 0.0f;
                    wb[j][c] = 0.0f;
                }
            // One view's contribution from its edge pair, the entry hp of b0 and,
            // for a wide lane, edge B's own entry hw (of bin bB) and fraction frw:
            // H(B) - C[b0+1] is then (C[bB+1] - C[b0+1]) + (frw - 1) w[bB] instead
            // of the two pieces, the difference of cumulative values summed in
            // FP64 on its own.  any_wide (uniform) skips the correction in
            // wavefronts without wide lanes.
            auto add_view = [&](int j, int c, const EdgePair& e, const DetValue& hp, bool any_wide, bool wide,
                                const DetValue& hw, float frw) {
                acc[j][c] += hp.c;
                wa[j][c] = fmaf(e.frA, hp.d, wa[j][c] - hp.d);
                float tb = fmaf(e.f1, hp.dn, fmaf(e.f0, hp.d, -hp.d));
                if (any_wide) {
                    if (wide) {
                        tb = fmaf(frw, hw.d, -hw.d);
                        accw64[j][c] += hw.c - hp.c;
                    }
                    keep(hw.dn);
                }
                wb[j][c] += tb;
            };
            fetch(0);
            for (int is = 0; is < nfull; is += U) {   // trip counts are uniform over the wavefront
                EdgePair ep[U][LPW];
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int j = 0; j < LPW; ++j) ep[u][j] = back_pair(tm[u][j], tg[u][j], K, span, origin);
                DetValue hv[U][LPW][NCH];
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int j = 0; j < LPW; ++j)
#pragma unroll
                        for (int c = 0; c < NCH; ++c)
                            hv[u][j][c] = load_det(tc, ep[u][j].off, (c * V + sl0 + is + u) * row);
                // wide lanes: edge B's own bin, entry and fraction (skipped by wavefronts without any)
                bool wide[U][LPW], any_wide[U][LPW];
                DetValue hw[U][LPW][NCH];
                float frw[U][LPW];
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int j = 0; j < LPW; ++j) {
                        wide[u][j] = ep[u][j].f1 >= 1.0f;
                        any_wide[u][j] = __builtin_amdgcn_ballot_w64(wide[u][j]) != 0;
                        if (wide[u][j]) {                  // frw is read only where set
                            int o;
                            back_locate(tm[u][j], tg[u][j], K + 1.0f, span, origin, o, frw[u][j]);
#pragma unroll
                            for (int c = 0; c < NCH; ++c)
                                hw[u][j][c] = load_det(tc, o, (c * V + sl0 + is + u) * row);
                        }
                    }
                __builtin_amdgcn_sched_barrier(0);
                fetch(is + U);
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int j = 0; j < LPW; ++j)
#pragma unroll
                        for (int c = 0; c < NCH; ++c)
                            add_view(j, c, ep[u][j], hv[u][j][c], any_wide[u][j], wide[u][j], hw[u][j][c],
                                     frw[u][j]);
            }
            // the remaining views (fewer than U); their tables were fetched into slots 0..
#pragma unroll
            for (int u = 0; u < U - 1; ++u) {
                if (nfull + u >= nvh) break;       // uniform
#pragma unroll
                for (int j = 0; j < LPW; ++j) {
                    const EdgePair e = back_pair(tm[u][j], tg[u][j], K, span, origin);
                    const bool wd = e.f1 >= 1.0f;
                    int o = 0;
                    float frw = 0.0f;
                    if (wd) back_locate(tm[u][j], tg[u][j], K + 1.0f, span, origin, o, frw);
#pragma unroll
                    for (int c = 0; c < NCH; ++c) {
                        const int rc = (c * V + sl0 + nfull + u) * row;
                        const DetValue hp = load_det(tc, e.off, rc);
                        DetValue hw = hp;
                        if (wd) hw = load_det(tc, o, rc);
                        add_view(j, c, e, hp, true, wd, hw, frw);
                    }
                }
            }
#pragma unroll
            for (int j = 0; j < LPW; ++j)
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    outa[j][c] += (float)(accw64[j][c] + (double)(wb[j][c] - wa[j][c]));
                    outb[j][c] += (float)(((next_lane(acc[j][c]) - acc[j][c]) - accw64[j][c]) +
                                          (double)(next_lane(wa[j][c]) - wb[j][c]));
                }
        }
    }
    // image layout: rows sweep (iy = q, ix = p), columns sweep (iy = p, ix = q)
    const size_t step = frame ? (size_t)nx : 1;
#pragma unroll
    for (int j = 0; j < LPW; ++j) {
        if (q0 + j >= Nq) break;                   // uniform
        const size_t pix = frame ? (size_t)pe * nx + (q0 + j) : (size_t)(q0 + j) * nx + pe;
        // EPL = 1: pixel pe from lanes 0..62; EPL = 2: pixels pe and pe + 1
        const bool va_ok = EPL == 1 ? lane < 63 && pe < Np : pe < Np;
        const bool vb_ok = EPL == 2 && lane < 63 && pe + 1 < Np;
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
            if (vsplit == 2) {                     // onto the cleared image (uniform)
                if (va_ok) unsafeAtomicAdd(&dst[c * img_stride + pix], outa[j][c]);
                if (vb_ok) unsafeAtomicAdd(&dst[c * img_stride + pix + step], outb[j][c]);
            } else {
                if (va_ok) dst[c * img_stride + pix] = outa[j][c];
                if (vb_ok) dst[c * img_stride + pix + step] = outb[j][c];
            }
        }
    }
}

// x = (accumulate ? x : 0) + part, elementwise over n floats.
__global__ __launch_bounds__(kThreads) void k_add_part(int n, const float* __restrict__ part, int accumulate,
                                                       float* __restrict__ x, const long long* __restrict__ zd) {
    if (zd) {                                                  // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        part = zshift(part, d);
        x = zshift(x, d);
    }
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) x[i] = accumulate ? x[i] + part[i] : part[i];
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
    const int chunks = fwd_chunks(t.B);
    const FrameSplit fs = split(t.n_frame_views[0] * chunks * 2, t.n_frame_views[1] * chunks * 2);   // two halves
    const float* rows = t.prefix;
    const float* cols = t.prefix + (size_t)t.prefix_mat * t.ny * prefix_row(t.nx);
    {
        KernelTimer kt_("k_dd_forward", s);
        hipLaunchKernelGGL(k_dd_forward<NK>, zgrid(dim3(grid_blocks(fs))), dim3(kFwdWaves * 64), 0, s, t.view,
                           t.bound, t.path, rows, cols, t.n_frame_views[0], fs, t.fwd_order, chunks, t.nx, t.ny, t.V,
                           t.B, sino, zarg());
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

// Wavefronts of k_dd_back<NCH, LPW, 2, EPL> resident on the whole device at once.
template <int NCH, int LPW, int EPL>
int back_waves_per_round() {
    static int cached[kMaxGpus] = {};
    int dev = 0;
    MBMD_HIP(hipGetDevice(&dev));
    MBMD_REQUIRE(dev >= 0 && dev < kMaxGpus, MBMD_ERR_ARG, "device index out of range");
    if (!cached[dev]) {
        int cus = 0, occ = 0;
        MBMD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        MBMD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k_dd_back<NCH, LPW, 2, EPL>, kThreads, 0));
        cached[dev] = (cus > 0 ? cus : 1) * (occ > 0 ? occ : 1) * kWaves;
    }
    return cached[dev];
}

// Run-time tuning of tile shapes; MBMD_AUTOTUNE=0 in the environment turns it
// off (the cost model then decides).
bool autotune_enabled() {
    static const bool on = [] {
        const char* e = std::getenv("MBMD_AUTOTUNE");
        return !(e && e[0] == '0');
    }();
    return on;
}

// Shapes chosen by the tuner, by device, geometry and channel count, so that
// problems of one geometry (the slices of a batch, repeated problems) time the
// candidates once per process.  Every shape gives the same bits, so sharing
// the choice only saves the timing runs.
std::string tuned_key(const GeomTables& t, int nch) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    const mbmd_geometry& g = t.g;
    const double f[] = {(double)dev, (double)nch, (double)g.kind, (double)g.nx, (double)g.ny, g.dx, g.dy,
                        (double)g.n_views, g.theta0, g.dtheta, (double)g.n_bins, g.du, g.u_offset, g.dso, g.dsd};
    return std::string(reinterpret_cast<const char*>(f), sizeof(f));
}
std::mutex g_tuned_mu;
std::map<std::string, int> g_tuned;
int tuned_lookup(const GeomTables& t, int nch) {
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    const auto it = g_tuned.find(tuned_key(t, nch));
    return it == g_tuned.end() ? -1 : it->second;
}
void tuned_store(const GeomTables& t, int nch, int v) {
    std::lock_guard<std::mutex> lock(g_tuned_mu);
    g_tuned[tuned_key(t, nch)] = v;
}

// Relative time of a back projection launch with LPW lines per wavefront:
// rounds of resident waves, each lasting the longer of the per-view latency
// of one wavefront (~900 cycles with two views in flight) and the VALU time of
// the waves sharing a SIMD (~76 cycles per line and view), both measured on
// gfx950 at the fan-beam workloads.
double back_cost(long long waves, int per_round, int lpw, int simds) {
    double t = 0.0;
    for (long long left = waves; left > 0; left -= per_round) {
        const long long w = left < per_round ? left : per_round;
        const double per_simd = (double)w / simds;
        const double valu = per_simd * lpw * 76.0;
        t += valu > 900.0 ? valu : 900.0;
    }
    return t;
}

template <int NCH, int LPW, int U, int EPL>
void back_kernel_launch(const GeomTables& t, float* x, hipStream_t s, int vsplit) {
    const int nv0 = t.n_frame_views[0], nv1 = t.n_frame_views[1];
    constexpr int ppw = back_ppw(EPL);
    const int u0 = nv0 ? vsplit * back_main_items(t.nx, t.ny, LPW, ppw) + back_tail_items(t.nx, t.ny, ppw) : 0;
    const int u1 = nv1 ? vsplit * back_main_items(t.ny, t.nx, LPW, ppw) + back_tail_items(t.ny, t.nx, ppw) : 0;
    const FrameSplit fs = split(u0, u1);
    KernelTimer kt_("k_dd_back", s);
    hipLaunchKernelGGL((k_dd_back<NCH, LPW, U, EPL>), zgrid(dim3(grid_blocks(fs))), dim3(kThreads), 0, s,
                       t.back_line, nv0, nv1, fs, t.nx, t.ny, t.V, t.B, t.det_prefix, x, t.back_part, vsplit, zarg());
    kt_.stop();
}

// Tile shape.  The pixel edges per lane are fixed by the problem: two for one
// or two channels when every swept line is at least one wavefront segment long
// (two edges per lane halve the gathers, but with more channels their
// registers, and on shorter lines their idle lanes, cost more), else one.
// Within that choice the shapes -- lines per wavefront x views in flight, views
// split over two wavefronts or not -- give bit-identical results: every pixel
// is the sum of the same two halves, each summing its views in the same order.
using BackLaunch = void (*)(const GeomTables&, float*, hipStream_t, int);
struct BackShape {
    BackLaunch fn;
    int vsplit, ppw;
};
template <int NCH>
int back_shapes(const GeomTables& t, BackShape* cand, bool& two_edges) {
    const int nv0 = t.n_frame_views[0], nv1 = t.n_frame_views[1];
    const int np_min = std::min(nv0 ? t.nx : 1 << 30, nv1 ? t.ny : 1 << 30);
    int n = 0;
    two_edges = false;
    if constexpr (NCH <= 2) {
        if (np_min >= back_ppw(2)) {
            two_edges = true;
            const BackShape c[5] = {
                {back_kernel_launch<NCH, 1, 2, 2>, 1, 127}, {back_kernel_launch<NCH, 1, 4, 2>, 1, 127},
                {back_kernel_launch<NCH, 2, 2, 2>, 1, 127}, {back_kernel_launch<NCH, 1, 2, 2>, 2, 127},
                {back_kernel_launch<NCH, 1, 4, 2>, 2, 127}};
            for (const BackShape& e : c) cand[n++] = e;
        }
    }
    if (!two_edges) {
        const BackShape c[4] = {{back_kernel_launch<NCH, 1, 2, 1>, 1, 63}, {back_kernel_launch<NCH, 1, 4, 1>, 1, 63},
                                {back_kernel_launch<NCH, 1, 2, 1>, 2, 63}, {back_kernel_launch<NCH, 1, 4, 1>, 2, 63}};
        for (const BackShape& e : c) cand[n++] = e;
    }
    return n;
}
constexpr int kMaxBackShapes = 5;

// The pixels a back projection in shape sh adds into (the tail's, or all with
// split views), which its detector rows' launch clears.
BackClear back_clear(const GeomTables& t, float* x, int nch, const BackShape& sh) {
    const int nv0 = t.n_frame_views[0], nv1 = t.n_frame_views[1];
    const BackTiling b0 = back_tiling(t.nx, sh.ppw), b1 = back_tiling(t.ny, sh.ppw);
    const int w0 = !nv0 ? 0 : sh.vsplit == 2 ? t.nx : b0.tail_lines ? t.nx - b0.full * sh.ppw : 0;
    const int h1 = !nv1 ? 0 : sh.vsplit == 2 ? t.ny : b1.tail_lines ? t.ny - b1.full * sh.ppw : 0;
    return BackClear{x, t.back_part, t.nx, t.ny, w0, h1, nch};
}

// The shape in use for NCH channels: forced by the testing hook, else the
// tuned one; -1 when none is chosen yet.
template <int NCH>
int back_chosen(const GeomTables& t) {
    BackShape cand[kMaxBackShapes];
    bool two_edges;
    const int n = back_shapes<NCH>(t, cand, two_edges);
    const int forced = t.forced_back;
    if (forced >= 0 && forced < n) return forced;
    return t.back_variant[NCH];
}

// Writes the row-sweep part of A^T sino to x (zero when no view sweeps rows) and
// returns the column-sweep part, in image layout, or nullptr when there is none.
template <int NCH>
const float* back_launch(const GeomTables& t, const float* sino, float* x, hipStream_t s) {
    const int nv0 = t.n_frame_views[0], nv1 = t.n_frame_views[1];
    BackShape cand[kMaxBackShapes];
    bool two_edges;
    const int n_cand = back_shapes<NCH>(t, cand, two_edges);
    // The detector prefix, which also clears the pixels the kernel adds into,
    // precedes every back projection kernel (the tuner's too).
    auto prefix = [&](const BackShape& sh) {
        KernelTimer kt_("k_detector_prefix", s);
        constexpr int sets = NCH - 2 * (NCH >= kPackFrom ? NCH / 3 : 0);   // triples and single rows
        hipLaunchKernelGGL(k_detector_prefix, zgrid(dim3(t.V, sets)), dim3(kPrefixThreads), 0, s, sino, t.path,
                           t.view, t.V, t.B, NCH, t.det_prefix, back_clear(t, x, NCH, sh), zarg());
        kt_.stop();
        MBMD_LAUNCHED();
    };
    if (!nv0) launch_fill(NCH * t.nx * t.ny, x, 0.0f, s);
    // The first back projection of a geometry and channel count outside graph
    // capture times the shapes on its own inputs and keeps the fastest; under
    // capture, or when tuning is switched off, a cost model of resident rounds
    // picks between unsplit shapes.
    auto run = [&](int v) {
        prefix(cand[v]);
        cand[v].fn(t, x, s, cand[v].vsplit);
        MBMD_LAUNCHED();
    };
    int& choice = t.back_variant[NCH];
    const int forced = t.forced_back;
    if (forced >= 0 && forced < n_cand) {           // testing hook: no tuning, nothing cached
        run(forced);
        return nv1 ? t.back_part : nullptr;
    }
    if (choice < 0) {
        hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
        MBMD_HIP(hipStreamIsCapturing(s, &cap));
        const int known = autotune_enabled() ? tuned_lookup(t, NCH) : -1;
        if (known >= 0 && known < n_cand) {
            choice = known;                            // timed before for this geometry
        } else if (cap == hipStreamCaptureStatusNone && autotune_enabled()) {
            hipEvent_t ev[2];
            MBMD_HIP(hipEventCreate(&ev[0]));
            MBMD_HIP(hipEventCreate(&ev[1]));
            // Candidates interleaved over several rounds, each keeping its best
            // round: the shapes are often within a few per cent of each other,
            // closer than the spread of back-to-back launches, and the first
            // back projection of a process often meets the device still
            // raising its clocks (two warm-up passes).
            float best[5] = {1e30f, 1e30f, 1e30f, 1e30f, 1e30f};
            for (int pass = 0; pass < 2; ++pass)
                for (int v = 0; v < n_cand; ++v) run(v);  // warm-up
            for (int round = 0; round < 6; ++round)
                for (int v = 0; v < n_cand; ++v) {
                    MBMD_HIP(hipEventRecord(ev[0], s));
                    for (int r = 0; r < 2; ++r) run(v);  // the prefix is the same for every candidate
                    MBMD_HIP(hipEventRecord(ev[1], s));
                    MBMD_HIP(hipEventSynchronize(ev[1]));
                    float ms = 0.0f;
                    MBMD_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
                    if (ms < best[v]) best[v] = ms;
                }
            choice = 0;
            for (int v = 1; v < n_cand; ++v)
                if (best[v] < best[choice]) choice = v;
            (void)hipEventDestroy(ev[0]);
            (void)hipEventDestroy(ev[1]);
            tuned_store(t, NCH, choice);
        } else {
            int cus = 0, dev = 0;
            MBMD_HIP(hipGetDevice(&dev));
            MBMD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
            const int simds = 4 * (cus > 0 ? cus : 1);
            auto waves = [&](int lpw) {
                const long long u0 =
                    nv0 ? (long long)back_main_items(t.nx, t.ny, lpw, 127) + back_tail_items(t.nx, t.ny, 127) : 0;
                const long long u1 =
                    nv1 ? (long long)back_main_items(t.ny, t.nx, lpw, 127) + back_tail_items(t.ny, t.nx, 127) : 0;
                return (u0 + u1) * kWaves;
            };
            // two edges: one line per wavefront (shape 0) or two (shape 2); one edge: shape 0
            constexpr int N2 = NCH <= 2 ? NCH : 1;     // two edges per lane: one or two channels only
            const int per1 = two_edges ? back_waves_per_round<N2, 1, 2>() : back_waves_per_round<NCH, 1, 1>();
            const double c1 = back_cost(waves(1), per1, 1, simds);
            const double c2 = two_edges ? back_cost(waves(2), back_waves_per_round<N2, 2, 2>(), 2, simds) : 1e300;
            const int pick = c2 < c1 ? 2 : 0;
            if (cap != hipStreamCaptureStatusNone) {
                run(pick);                             // not cached: tune on a later uncaptured call
                return nv1 ? t.back_part : nullptr;
            }
            choice = pick;
        }
    }
    run(choice);
    return nv1 ? t.back_part : nullptr;
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
        for (int q = 0; q < Nq; ++q) {
            const float xa = fmaf(b0.y, (float)q, b0.x), xb = fmaf(b1.y, (float)q, b1.x);
            const float lo = fmaxf(fminf(xa, xb), 0.0f), hi = fminf(fmaxf(xa, xb), (float)Np);
            if (hi <= lo) continue;
            const int k0 = (int)floorf(lo);
            const int k1 = (int)ceilf(hi) - 1;
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
    {
        // lines [line0, line1): rows then columns, only the frames that have views
        const int line0 = t.n_frame_views[0] ? 0 : t.ny;
        const int line1 = t.n_frame_views[1] ? t.ny + t.nx : t.ny;
        float* cols = t.prefix + (size_t)t.prefix_mat * t.ny * prefix_row(t.nx);
        KernelTimer kt_("k_line_prefix", s);
        hipLaunchKernelGGL(k_line_prefix, zgrid(dim3(line1 - line0, n_mat)), dim3(kScanThreads), 0, s, x, t.prefix,
                           cols, t.nx, t.ny, line0, sino, n_mat * t.V * t.B, zarg(),
                           (int)(zarg() && x == zbatch().x0));
        kt_.stop();
    }
    MBMD_LAUNCHED();
    switch (n_mat) {
        case 1: fwd_launch<1>(t, sino, s); break;
        case 2: fwd_launch<2>(t, sino, s); break;
        case 3: fwd_launch<3>(t, sino, s); break;
        default: fwd_launch<4>(t, sino, s); break;
    }
}

const float* launch_backproject_parts(const GeomTables& t, const float* sino, float* x, int n_ch, hipStream_t s) {
    MBMD_REQUIRE(n_ch >= 1 && n_ch <= kMaxBackCh, MBMD_ERR_SHAPE, "back projection channels must be in 1..10");
    MBMD_REQUIRE(t.det_prefix != nullptr && t.back_ch >= n_ch, MBMD_ERR_ARG, "back projection scratch too small");
    switch (n_ch) {
        case 1: return back_launch<1>(t, sino, x, s);
        case 2: return back_launch<2>(t, sino, x, s);
        case 3: return back_launch<3>(t, sino, x, s);
        case 4: return back_launch<4>(t, sino, x, s);
        case 5: return back_launch<5>(t, sino, x, s);
        case 6: return back_launch<6>(t, sino, x, s);
        case 7: return back_launch<7>(t, sino, x, s);
        case 8: return back_launch<8>(t, sino, x, s);
        case 9: return back_launch<9>(t, sino, x, s);
        default: return back_launch<10>(t, sino, x, s);
    }
}

namespace {
template <int NCH>
BackRows back_rows_n(const GeomTables& t, float* x) {
    BackRows r{};
    const int v = back_chosen<NCH>(t);
    if (v < 0) return r;                          // ok = false
    BackShape cand[kMaxBackShapes];
    bool two_edges;
    back_shapes<NCH>(t, cand, two_edges);
    r.ok = true;
    r.rows = t.det_prefix;
    r.view = t.view;
    r.path = t.path;
    r.V = t.V;
    r.B = t.B;
    r.clr = back_clear(t, x, NCH, cand[v]);
    return r;
}
template <int NCH>
const float* back_kernel_n(const GeomTables& t, float* x, hipStream_t s) {
    const int v = back_chosen<NCH>(t);
    MBMD_REQUIRE(v >= 0, MBMD_ERR_ARG, "back projection shape not chosen yet");
    BackShape cand[kMaxBackShapes];
    bool two_edges;
    back_shapes<NCH>(t, cand, two_edges);
    if (!t.n_frame_views[0]) launch_fill(NCH * t.nx * t.ny, x, 0.0f, s);
    cand[v].fn(t, x, s, cand[v].vsplit);
    MBMD_LAUNCHED();
    return t.n_frame_views[1] ? t.back_part : nullptr;
}
}  // namespace

BackRows back_rows(const GeomTables& t, float* x, int n_ch) {
    MBMD_REQUIRE(n_ch >= 1 && n_ch <= kMaxBackCh, MBMD_ERR_SHAPE, "back projection channels must be in 1..10");
    MBMD_REQUIRE(t.det_prefix != nullptr && t.back_ch >= n_ch, MBMD_ERR_ARG, "back projection scratch too small");
    static_assert(kPackFrom == 3, "producers write the unpacked rows of one or two channels");
    switch (n_ch) {
        case 1: return back_rows_n<1>(t, x);
        case 2: return back_rows_n<2>(t, x);
        default: return BackRows{};               // packed rows: the detector-prefix path
    }
}

const float* launch_back_kernel(const GeomTables& t, float* x, int n_ch, hipStream_t s) {
    switch (n_ch) {
        case 1: return back_kernel_n<1>(t, x, s);
        case 2: return back_kernel_n<2>(t, x, s);
        default: MBMD_REQUIRE(false, MBMD_ERR_ARG, "detector rows are written by the caller for 1 or 2 channels only");
    }
    return nullptr;
}

void launch_backproject(const GeomTables& t, const float* sino, float* x, int n_ch, hipStream_t s) {
    const float* part = launch_backproject_parts(t, sino, x, n_ch, s);
    if (part) {
        const int n = n_ch * t.nx * t.ny;
        KernelTimer kt_("k_add_part", s);
        hipLaunchKernelGGL(k_add_part, zgrid(dim3((n + kThreads - 1) / kThreads)), dim3(kThreads), 0, s, n, part, 1,
                           x, zarg());
        kt_.stop();
        MBMD_LAUNCHED();
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
