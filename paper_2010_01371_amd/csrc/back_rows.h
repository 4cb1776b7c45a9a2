// Device helpers for the back projector's detector rows, shared by the
// detector-prefix launch and by the ray gradient launch that builds the rows of
// its own output (so that both give the same bits).
#pragma once

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

}  // namespace mbmd
