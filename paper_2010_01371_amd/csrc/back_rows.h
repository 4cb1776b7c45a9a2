// Device helpers for the back projector's detector rows, shared by the
// detector-prefix launch and by the ray gradient launch that builds the rows of
// its own output (so that both give the same bits).
#pragma once

#include <cfloat>

#include "internal.h"

namespace mbmd {

// Threads of a workgroup that builds detector rows (one row per workgroup).
constexpr int kRowThreads = 256;

// Clears the pixels a back projection adds into (see BackClear): a grid-stride
// side job of every block of a launch, block bid of nblk.
__device__ __forceinline__ void clear_back_pixels(const BackClear& tc, int bid, int nblk) {
    const int n0 = tc.nch * tc.ny * tc.w0, n1 = tc.nch * tc.h1 * tc.nx, nj = tc.nx * tc.ny;
    for (int i = bid * kRowThreads + threadIdx.x; i < n0 + n1; i += nblk * kRowThreads) {
        if (i < n0) {                                      // row sweeps: columns [nx - w0, nx) of x
            const int c = i / (tc.ny * tc.w0), r = i - c * tc.ny * tc.w0;
            const int iy = r / tc.w0, ix = tc.nx - tc.w0 + (r - iy * tc.w0);
            tc.x[(size_t)c * nj + (size_t)iy * tc.nx + ix] = 0.0f;
        } else {                                           // column sweeps: rows [ny - h1, ny) of part
            const int k = i - n0;
            const int c = k / (tc.h1 * tc.nx), r = k - c * tc.h1 * tc.nx;
            tc.part[(size_t)c * nj + (size_t)(tc.ny - tc.h1) * tc.nx + r] = 0.0f;
        }
    }
}

// One detector row (DetEntry, det_row(B) entries) from the widths w[b] of its
// bins in row order, width(b) for b < B: entry b holds C[b+1], w[b] and w[b+1]
// with C[b] = sum_{b'<b} w[b'] (FP64 sums of the FP32 widths, so that
// C[b+1] - w[b] gives C[b] up to FP64 rounding), w[B] = 0; entries B and B+1
// hold the total with zero widths.  Called by all kRowThreads threads of the
// workgroup (one barrier; wave_total: kRowThreads / 64 doubles of LDS of its
// own).  Each thread takes a contiguous run of bins, an FP64 shuffle scan
// combines the lanes of a wavefront and the barrier the wavefronts.
template <class Width>
__device__ __forceinline__ void build_detector_row(Width width, int B, DetEntry* __restrict__ dst,
                                                   double* wave_total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int per = (B + kRowThreads - 1) / kRowThreads;
    const int b0 = threadIdx.x * per;
    double acc = 0.0;
    for (int i = 0; i < per; ++i) {
        const int b = b0 + i;
        if (b < B) acc += (double)width(b);
    }
    double inc = acc;                                             // inclusive scan over the wavefront
    for (int off = 1; off < 64; off <<= 1) {
        const double t = __shfl_up(inc, off, 64);
        if (lane >= off) inc += t;
    }
    if (lane == 63) wave_total[wave] = inc;
    __syncthreads();
    double run = inc - acc;
    for (int w = 0; w < wave; ++w) run += wave_total[w];          // fixed order
    float d = b0 < B ? width(b0) : 0.0f;
    for (int i = 0; i < per; ++i) {
        const int b = b0 + i;
        if (b < B) {
            const float dn = b + 1 < B ? width(b + 1) : 0.0f;
            run += (double)d;
            dst[b] = DetEntry{run, d, dn};
            d = dn;
        }
    }
    if (threadIdx.x == kRowThreads - 1) {                         // holds the total after its run
        dst[B] = DetEntry{run, 0.0f, 0.0f};
        dst[B + 1] = DetEntry{run, 0.0f, 0.0f};
    }
}

// One triple row (see kPackFrom) from the widths width(k, b) of its three
// channels k: entry b of planes A (at dst) and B (at dst + plane bytes) holds,
// per channel, q = round((C[b+1] - c0) 2^s) (hi, lo) and w[b], with C the FP64
// prefix sums of the widths as in
// build_detector_row; entries B and B+1 hold the totals with zero widths, and
// scale[k] = 2^-s.  Per channel, c0 is the middle of the row's range of C and
// s puts the half-range into [2^46, 2^47) (up to the rounding of the range,
// which the scan takes from partial sums: the largest q is clamped to 48 bits),
// so a decoded value q 2^-s, an exact FP64 number, is within 2^-47 of that
// half-range of C[b+1] - c0: for a row of B bins about 2^-47 B/2 of a typical
// width, against the 2^-24 of each FP32 width.  Both edges of a pixel read one
// row per view, so c0 drops out of every pixel exactly.  A channel with a
// non-finite C stores q = 0 and a NaN scale, so every pixel its view reaches
// becomes NaN (the other two channels are unaffected).  Called by all
// kRowThreads threads of the workgroup (one barrier; lds: 12 kRowThreads / 64
// doubles of LDS of its own).  Each thread takes a contiguous run of bins for
// all three channels (independent chains), an FP64 shuffle scan combines the
// lanes of a wavefront, the barrier the wavefronts.
template <class Width>
__device__ __forceinline__ void build_triple_rows(Width width, int B, DetEntry* __restrict__ dst, size_t plane,
                                                  double* __restrict__ scale, double* lds) {
    constexpr int NW = kRowThreads / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int per = (B + kRowThreads - 1) / kRowThreads;
    const int b0 = threadIdx.x * per;
    // per channel: the thread's sum and the range of its partial sums
    double acc[3] = {0.0, 0.0, 0.0}, phi[3], plo[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        phi[k] = -INFINITY;
        plo[k] = INFINITY;
    }
    for (int i = 0; i < per; ++i) {
        const int b = b0 + i;
        if (b < B) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                acc[k] += (double)width(k, b);
                phi[k] = fmax(phi[k], acc[k]);
                plo[k] = fmin(plo[k], acc[k]);
            }
        }
    }
    double start[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const bool bad = !(fabs(acc[k]) <= DBL_MAX);             // a sum of finite FP32 widths is finite
        double inc = acc[k];                                      // inclusive scan over the wavefront
        for (int off = 1; off < 64; off <<= 1) {
            const double t = __shfl_up(inc, off, 64);
            if (lane >= off) inc += t;
        }
        start[k] = inc - acc[k];
        // range relative to the wavefront's start
        double h = start[k] + phi[k], l = start[k] + plo[k];
        for (int off = 32; off > 0; off >>= 1) {
            h = fmax(h, __shfl_xor(h, off, 64));
            l = fmin(l, __shfl_xor(l, off, 64));
        }
        const bool any_bad = __builtin_amdgcn_ballot_w64(bad) != 0;
        if (lane == 63) lds[k * NW + wave] = inc;
        if (lane == 0) {
            lds[(3 + k) * NW + wave] = h;
            lds[(6 + k) * NW + wave] = l;
            lds[(9 + k) * NW + wave] = any_bad ? 1.0 : 0.0;
        }
    }
    __syncthreads();
    double c0[3], up[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        double pre = 0.0, h = -INFINITY, l = INFINITY;
        bool bad = false;
        for (int w = 0; w < NW; ++w) {                            // fixed order
            if (w == wave) start[k] += pre;
            h = fmax(h, pre + lds[(3 + k) * NW + w]);
            l = fmin(l, pre + lds[(6 + k) * NW + w]);
            bad |= lds[(9 + k) * NW + w] != 0.0;
            pre += lds[k * NW + w];
        }
        const bool finite = !bad && h <= DBL_MAX && l >= -DBL_MAX;
        c0[k] = finite ? 0.5 * h + 0.5 * l : 0.0;
        const double half = finite ? 0.5 * h - 0.5 * l : 0.0;
        // nonzero half-ranges of sums of FP32 widths lie in [2^-150, 2^159): s within [-112, 196]
        const int s = half > 0.0 ? 46 - ilogb(half) : 0;
        up[k] = finite ? ldexp(1.0, s) : 0.0;
        if (threadIdx.x == 0) scale[k] = finite ? ldexp(1.0, -s) : __builtin_nan("");
    }
    auto put = [&](int b, const double* c, const float* w) {
        constexpr double kMax = 140737488355327.0;                // 2^47 - 1
        long long q[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) q[k] = (long long)fmin(fmax(rint((c[k] - c0[k]) * up[k]), -kMax), kMax);
        const unsigned lo01 = (unsigned)(q[0] & 0xffff) | (unsigned)(q[1] & 0xffff) << 16;
        float4* a = reinterpret_cast<float4*>(dst + b);
        float4* e = reinterpret_cast<float4*>(dst + plane + b);
        *a = make_float4(__int_as_float((int)(q[0] >> 16)), __int_as_float((int)(q[1] >> 16)),
                         __int_as_float((int)(q[2] >> 16)), __uint_as_float(lo01));   // hi: floor(q / 2^16)
        *e = make_float4(w[0], w[1], w[2], __uint_as_float((unsigned)(q[2] & 0xffff)));
    };
    double run[3] = {start[0], start[1], start[2]};
    for (int i = 0; i < per; ++i) {
        const int b = b0 + i;
        if (b < B) {
            float w[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                w[k] = width(k, b);
                run[k] += (double)w[k];
            }
            put(b, run, w);
        }
    }
    if (threadIdx.x == kRowThreads - 1) {                         // holds the totals after its run
        const float z[3] = {0.0f, 0.0f, 0.0f};
        put(B, run, z);
        put(B + 1, run, z);
    }
}

}  // namespace mbmd
