// Device helpers shared by the image-space and per-ray kernels: FP64 block
// sums, the Huber weight, the penalty's curvature along a direction for one
// pixel, and the final reduction of the partial-sum regions into the objective
// and the step size.
#pragma once

#include "internal.h"

namespace mbmd {
namespace dev {

// Sum over the block (any multiple of 64 threads), valid in thread 0.
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

__device__ __forceinline__ float huber_omega(float t, float d) {
    const float a = fabsf(t);
    return a <= d ? 1.0f : d / a;
}

__device__ __forceinline__ float huber_dpsi(float t, float d) { return fminf(fmaxf(t, -d), d); }
__device__ __forceinline__ double huber_psi(double t, double d) {
    const double a = fabs(t);
    return a <= d ? 0.5 * t * t : d * a - 0.5 * d * d;
}

// Pixel j of the penalty: its gradient gr[k] per material, its separable SPS
// curvature cur[k] (when cur is not NULL) and the share of R(x) charged to it
// (the pairs (j, right) and (j, down)), which it returns.  Quadratic:
// R = 1/2 x^T (beta (x) Gamma) x, curvature sum_k' |beta_kk'| 2 |N_j|; Huber (one
// material): R = beta sum_pairs psi(x_j - x_j'), gradient beta sum psi'(.),
// curvature 2 beta sum omega(.).
__device__ __forceinline__ double penalty_grad_at(const PenaltyArgs& a, const float* __restrict__ x, int j,
                                                  float* gr, float* cur) {
    const int nj = a.nx * a.ny;
    const int iy = j / a.nx, ix = j - iy * a.nx;
    const bool L = ix > 0, R = ix + 1 < a.nx, U = iy > 0, D = iy + 1 < a.ny;
    double phi = 0.0;
    if (a.kind == MBMD_PENALTY_HUBER) {
        const float xc = x[j];
        float g = 0.0f, om = 0.0f;
        if (L) { const float t = xc - x[j - 1]; g += huber_dpsi(t, a.delta); om += huber_omega(t, a.delta); }
        if (R) { const float t = xc - x[j + 1]; g += huber_dpsi(t, a.delta); om += huber_omega(t, a.delta);
                 phi += huber_psi((double)t, (double)a.delta); }
        if (U) { const float t = xc - x[j - a.nx]; g += huber_dpsi(t, a.delta); om += huber_omega(t, a.delta); }
        if (D) { const float t = xc - x[j + a.nx]; g += huber_dpsi(t, a.delta); om += huber_omega(t, a.delta);
                 phi += huber_psi((double)t, (double)a.delta); }
        const float b = a.beta[0];
        gr[0] = b * g;
        if (cur) cur[0] = 2.0f * b * om;
        return phi * (double)b;
    }
    const float nn = (float)(L + R + U + D);
    float lap[kMaxMat];
#pragma unroll
    for (int k = 0; k < kMaxMat; ++k) {
        if (k >= a.K) break;
        const float* xk = x + (size_t)k * nj;
        float s = nn * xk[j];
        if (L) s -= xk[j - 1];
        if (R) s -= xk[j + 1];
        if (U) s -= xk[j - a.nx];
        if (D) s -= xk[j + a.nx];
        lap[k] = s;
    }
#pragma unroll
    for (int k = 0; k < kMaxMat; ++k) {
        if (k >= a.K) break;
        float g = 0.0f, ab = 0.0f;
#pragma unroll
        for (int l2 = 0; l2 < kMaxMat; ++l2) {
            if (l2 >= a.K) break;
            g = fmaf(a.beta[k * a.K + l2], lap[l2], g);
            ab += fabsf(a.beta[k * a.K + l2]);
        }
        gr[k] = g;
        if (cur) cur[k] = ab * 2.0f * nn;
        phi += 0.5 * (double)x[(size_t)k * nj + j] * (double)g;
    }
    return phi;
}

// Pixel j's share of p^T R''(x) p: the pairs (j, right) and (j, down).  Huber
// (one material): beta sum omega(x_j - x_j') (p_j - p_j')^2; quadratic:
// sum_kl beta_kl (p_k,j - p_k,j')(p_l,j - p_l,j').
__device__ __forceinline__ double penalty_quadform_at(const PenaltyArgs& a, const float* __restrict__ x,
                                                      const float* __restrict__ p, int j) {
    const int nj = a.nx * a.ny;
    const int iy = j / a.nx, ix = j - iy * a.nx;
    const bool R = ix + 1 < a.nx, D = iy + 1 < a.ny;
    double acc = 0.0;
    if (a.kind == MBMD_PENALTY_HUBER) {
        float s = 0.0f;
        if (R) { const float dp = p[j] - p[j + 1]; s += huber_omega(x[j] - x[j + 1], a.delta) * dp * dp; }
        if (D) { const float dp = p[j] - p[j + a.nx]; s += huber_omega(x[j] - x[j + a.nx], a.delta) * dp * dp; }
        acc = (double)a.beta[0] * (double)s;
    } else {
        for (int k = 0; k < a.K; ++k)
            for (int l2 = 0; l2 < a.K; ++l2) {
                const float* pk = p + (size_t)k * nj;
                const float* pl = p + (size_t)l2 * nj;
                float s = 0.0f;
                if (R) s += (pk[j] - pk[j + 1]) * (pl[j] - pl[j + 1]);
                if (D) s += (pk[j] - pk[j + a.nx]) * (pl[j] - pl[j + a.nx]);
                acc += (double)a.beta[k * a.K + l2] * (double)s;
            }
    }
    return acc;
}

struct Counts {
    int c[kRegions];
};

// Threads of a block that sums the regions: two wavefronts per region.
constexpr int kReduceThreads = 128 * kRegions;

// Sums every partial-sum region (region r at partials + r kMaxPartials, counts.c[r]
// entries): two wavefronts per region, each lane adding a strided share with
// eight loads in flight, in a fixed order.  Block of kReduceThreads threads; on
// return (after a barrier) region r's sum is sh[2 r] + sh[2 r + 1].
__device__ __forceinline__ void region_sums(const double* partials, const Counts& counts, double* sh) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int r = wave >> 1, t = (wave & 1) * 64 + lane;
    const double* pr = partials + (size_t)r * kMaxPartials;
    const int n = counts.c[r];
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int i = t; i < n; i += 128 * 8) {
#pragma unroll
        for (int u = 0; u < 8; ++u)
            if (i + 128 * u < n) acc[u] += pr[i + 128 * u];
    }
    double v = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) sh[wave] = v;
    __syncthreads();
}

// The scalars formed from the region sums (sh as left by region_sums):
// phi = PHI_L + PHI_R and, with mode RED_STEP, the step alpha = -GP / (CQ2 + PRP)
// (0 when the denominator is not positive or alpha is not finite).  With write,
// stores them to scal (and phi to trace_slot) and raises numeric flags in
// flags[0]: MBMD_FLAG_NONFINITE when phi or alpha is not finite,
// MBMD_FLAG_NO_CURVATURE when the denominator is not positive for a nonzero
// g^T p, MBMD_FLAG_ASCENT when alpha < 0 (g^T p > 0: M M^T not positive
// semi-definite), and with mode RED_MONOTONE MBMD_FLAG_INCREASE when phi
// exceeds the previous objective of the run (scal[S_PHI_PREV], NaN at its
// start) by more than kIncreaseTol relative; phi then replaces it.  Returns
// alpha (0 without RED_STEP).
__device__ __forceinline__ double form_scalars(const double* sh, int mode, double* scal, double* trace_slot,
                                               int* flags, bool write) {
    double sums[kRegions];
    for (int k = 0; k < kRegions; ++k) sums[k] = sh[2 * k] + sh[2 * k + 1];
    const double phi = sums[R_PHI_L] + sums[R_PHI_R];
    int bits = isfinite(phi) ? 0 : MBMD_FLAG_NONFINITE;
    double alpha_out = 0.0;
    if (mode & RED_STEP) {
        const double gp = sums[R_GP];
        const double den = sums[R_CQ2] + sums[R_PRP];
        const double alpha = den > 0.0 ? -gp / den : 0.0;
        alpha_out = isfinite(alpha) ? alpha : 0.0;
        if (!isfinite(alpha) || !isfinite(gp) || !isfinite(den)) bits |= MBMD_FLAG_NONFINITE;
        else if (!(den > 0.0) && gp != 0.0) bits |= MBMD_FLAG_NO_CURVATURE;
        else if (alpha < 0.0) bits |= MBMD_FLAG_ASCENT;
        if (write) {
            scal[S_GP] = gp;
            scal[S_DEN] = den;
            scal[S_ALPHA] = alpha_out;
        }
    }
    if (write) {
        if (mode & RED_MONOTONE) {
            const double prev = scal[S_PHI_PREV];
            if (isfinite(prev) && phi > prev + kIncreaseTol * fabs(prev)) bits |= MBMD_FLAG_INCREASE;
            scal[S_PHI_PREV] = phi;
        }
        scal[S_PHI] = phi;
        if (trace_slot) *trace_slot = phi;
        if (bits && flags) flags[0] |= bits;
    }
    return alpha_out;
}

}  // namespace dev
}  // namespace mbmd
