// Per-ray (per detector element) passes of the polyenergetic model.
//
// One thread per ray.  The energy loop recomputes t_E = exp(-sum_k Q_Ek l_k)
// instead of storing a ray x energy tensor: the first pass forms the channel
// means ybar_c and the weighted residuals r_c = w_c (ybar_c - y_c); the second
// pass forms, per energy (SPS section, with rho read as S^T W (ybar - y) -
// eta t):
//   s_E    = sum_c S_cE r_c
//   eta_E  = sum_c S_cE w_c sum_E' S_cE'
//   hdot_E = -t_E s_E                      (dL/dl_E)
//   c_E    = max(2 eta_E + s_E - eta_E t_E, 0)   (maximum curvature on l >= 0)
// and accumulates u_k = sum_E Q_Ek hdot_E and v_k = sum_E Q_Ek gamma_E c_E
// with gamma_E = (A 1)_i sum_k Q_Ek.  With a projection-domain blur B (BB =
// B S) the residual couples neighbouring bins, and the pass splits in three
// launches: the unblurred means ybar0 = S t, then r = W (B ybar0 - y) with the
// objective, then the energy pass with B^T r in place of r and B^T W B 1 in
// place of w in eta.  The spectral model Q, S is read with
// wave-uniform indices (scalar loads).  Objective partial sums are FP64 and
// reduced per block in a fixed order.
#include <cmath>

#include "back_rows.h"
#include "device_common.h"
#include "internal.h"

namespace mbmd {

namespace {

constexpr int kRayThreads = 256;

using dev::block_sum;

struct RayModel {
    int K, E, C;
    const float *Q, *S, *rowS, *Qsum;
};

// The model of slice d of a batched launch (its tables lie d bytes further).
__device__ __forceinline__ RayModel zshift_model(RayModel m, long long d) {
    m.Q = zshift(m.Q, d);
    m.S = zshift(m.S, d);
    m.rowS = zshift(m.rowS, d);
    m.Qsum = zshift(m.Qsum, d);
    return m;
}

// t = exp(-le) with the hardware base-2 exponential (one multiply and one
// v_exp_f32, where expf takes about ten VALU for its range reduction): the
// rounding of le log2(e) gives a relative error of about 1.2e-7 (1 + |le|
// log2 e), 2e-6 at le = 20 (transmission 2e-9), and the result flushes to
// zero below 2^-126, where it no longer moves any mean.
__device__ __forceinline__ float transmission(float le) { return __expf(-le); }

// Spectral tables staged in LDS once per block, per energy contiguous:
// Q[e][k], S[e][c] (transposed from [c][e]) and Qsum[e]; every lane reads the
// same entry, which LDS broadcasts.  KT / CT > 0 fix N_k / N_c at compile time
// (the loops over materials and channels unroll into registers); 0 reads them
// from the model.
struct SharedModel {
    float Q[kMaxEnergy * kMaxMat];
    float S[kMaxEnergy * kMaxChan];
    float Qsum[kMaxEnergy];
};

template <int KT, int CT>
__device__ __forceinline__ void stage_model(const RayModel& m, SharedModel& sm) {
    const int K = KT ? KT : m.K, C = CT ? CT : m.C;
    for (int i = threadIdx.x; i < m.E * K; i += blockDim.x) sm.Q[i] = m.Q[i];
    for (int i = threadIdx.x; i < m.E * C; i += blockDim.x) {
        const int e = i / C, c = i - e * C;
        sm.S[i] = m.S[c * m.E + e];
    }
    for (int i = threadIdx.x; i < m.E; i += blockDim.x) sm.Qsum[i] = m.Qsum ? m.Qsum[i] : 0.0f;
    __syncthreads();
}

// Pass 1: ybar_c for the ray with line integrals lk.
template <int KT, int CT>
__device__ __forceinline__ void channel_means(const RayModel& m, const SharedModel& sm, const float* lk,
                                              float* ybar) {
    const int K = KT ? KT : m.K, C = CT ? CT : m.C;
    for (int c = 0; c < C; ++c) ybar[c] = 0.0f;
#pragma unroll 2
    for (int e = 0; e < m.E; ++e) {
        float le = 0.0f;
        for (int k = 0; k < K; ++k) le = fmaf(sm.Q[e * K + k], lk[k], le);
        const float t = transmission(le);
        for (int c = 0; c < C; ++c) ybar[c] = fmaf(sm.S[e * C + c], t, ybar[c]);
    }
}

// Ray i's line integrals, after applying the pending step to them (l += a q,
// a = the step size, 0 for none).
template <int KT>
__device__ __forceinline__ void ray_line_integrals(const RayModel& m, int ni, int i, const float* __restrict__ l,
                                                   const StepUpdate& up, float a, float* lk) {
    const int K = KT ? KT : m.K;
    if (a != 0.0f) {                                       // l += alpha q, then use it
        for (int k = 0; k < K; ++k) {
            lk[k] = fmaf(a, up.q[(size_t)k * ni + i], up.l[(size_t)k * ni + i]);
            up.l[(size_t)k * ni + i] = lk[k];
        }
    } else {
        for (int k = 0; k < K; ++k) lk[k] = l[(size_t)k * ni + i];
    }
}

// Pass 2 of a ray from its line integrals lk, the residual terms rc[c] (the
// channel's share of BB^T W (ybar - y)) and sig[c] (its share of eta per unit
// S_cE): uk[k], and vk[k] when want_v.
template <int KT, int CT>
__device__ __forceinline__ void ray_pass2(const RayModel& m, const SharedModel& sm, const float* lk,
                                          const float* rc, const float* sig, float gA, bool want_v, float* uk,
                                          float* vk) {
    const int K = KT ? KT : m.K, C = CT ? CT : m.C;
    for (int k = 0; k < K; ++k) uk[k] = vk[k] = 0.0f;
#pragma unroll 2
    for (int e = 0; e < m.E; ++e) {
        float le = 0.0f;
        for (int k = 0; k < K; ++k) le = fmaf(sm.Q[e * K + k], lk[k], le);
        const float t = transmission(le);
        float s = 0.0f, eta = 0.0f;
        for (int c = 0; c < C; ++c) {
            const float sce = sm.S[e * C + c];
            s = fmaf(sce, rc[c], s);
            eta = fmaf(sce, sig[c], eta);
        }
        const float hdot = -t * s;
        for (int k = 0; k < K; ++k) uk[k] = fmaf(sm.Q[e * K + k], hdot, uk[k]);
        if (want_v) {
            const float ce = fmaxf(2.0f * eta + s - eta * t, 0.0f);
            const float gc = gA * sm.Qsum[e] * ce;
            for (int k = 0; k < K; ++k) vk[k] = fmaf(sm.Q[e * K + k], gc, vk[k]);
        }
    }
}

// Ray i of the gradient pass: applies the pending step to its line integrals,
// and returns its share of the data term of Phi, with uk[k] (and vk[k] when
// want_v) of the ray and the residuals r_c stored to r_out (when not NULL).
template <int KT, int CT>
__device__ __forceinline__ double ray_grad_at(const RayModel& m, const SharedModel& sm, int ni, int i,
                                              const float* __restrict__ l, const float* __restrict__ y,
                                              const float* __restrict__ w, const float* __restrict__ gammaA,
                                              float* __restrict__ r_out, const StepUpdate& up, float a,
                                              bool want_v, float* uk, float* vk) {
    const int C = CT ? CT : m.C;
    float lk[kMaxMat], ybar[kMaxChan], rc[kMaxChan], sig[kMaxChan];
    ray_line_integrals<KT>(m, ni, i, l, up, a, lk);
    channel_means<KT, CT>(m, sm, lk, ybar);
    double phi = 0.0;
    for (int c = 0; c < C; ++c) {
        const float yc = y[(size_t)c * ni + i], wc = w[(size_t)c * ni + i];
        const float dv = ybar[c] - yc;
        rc[c] = wc * dv;
        sig[c] = wc * m.rowS[c];
        phi += 0.5 * (double)wc * (double)dv * (double)dv;
        if (r_out) r_out[(size_t)c * ni + i] = rc[c];
    }
    ray_pass2<KT, CT>(m, sm, lk, rc, sig, gammaA ? gammaA[i] : 1.0f, want_v, uk, vk);
    return phi;
}

// The blur of channel c at ray i = view * b.B + bin, on a channel's rays z:
// (B z)_bin = sum_d taps[d + h] z_{bin+d}, or (B^T z)_bin = sum_d taps[d + h]
// z_{bin-d}, bins beyond the detector dropped.
__device__ __forceinline__ float blur_at(const BlurArgs& b, const float* __restrict__ z, int i, int c,
                                         bool transpose) {
    const int bin = i % b.B, row0 = i - bin;
    float s = 0.0f;
    for (int d = -b.h; d <= b.h; ++d) {
        const int bb = transpose ? bin - d : bin + d;
        if (bb >= 0 && bb < b.B) s = fmaf(b.taps[c][d + b.h], z[row0 + bb], s);
    }
    return s;
}

// Blurred model, pass 1: the pending step (as k_ray_grad) and the unblurred
// channel means ybar0_c = sum_E S_cE t_E of every ray.
template <int KT, int CT>
__global__ __launch_bounds__(kRayThreads) void k_ray_means(RayModel m, int ni, const float* __restrict__ l,
                                                           float* __restrict__ ybar0, StepUpdate up, int nb_ray,
                                                           const long long* __restrict__ zd) {
    __shared__ SharedModel sm;
    if (zd) {                                              // batched: this slice's buffers and image
        const long long d = zoff(zd, Z_BLOCK);
        m = zshift_model(m, d);
        l = zshift(l, d);
        ybar0 = zshift(ybar0, d);
        up.alpha = zshift(up.alpha, d);
        up.q = zshift(up.q, d);
        up.l = zshift(up.l, d);
        up.p = zshift(up.p, d);
        up.x = zshift(up.x, zoff(zd, Z_IMAGE));
    }
    if (up.alpha && (int)blockIdx.x >= nb_ray) {           // the image part of the step: x += alpha p
        const float a = (float)*up.alpha;
        const int i = ((int)blockIdx.x - nb_ray) * kRayThreads + threadIdx.x;
        if (a != 0.0f && i < up.n_img) up.x[i] = fmaf(a, up.p[i], up.x[i]);
        return;
    }
    stage_model<KT, CT>(m, sm);
    const int C = CT ? CT : m.C;
    const int i = blockIdx.x * kRayThreads + threadIdx.x;
    if (i >= ni) return;
    float lk[kMaxMat], ybar[kMaxChan];
    ray_line_integrals<KT>(m, ni, i, l, up, up.alpha ? (float)*up.alpha : 0.0f, lk);
    channel_means<KT, CT>(m, sm, lk, ybar);
    for (int c = 0; c < C; ++c) ybar0[(size_t)c * ni + i] = ybar[c];
}

// Blurred model, pass 2: ybar = B ybar0, the weighted residuals
// rres_c = w_c (ybar_c - y_c) and the rays' shares of the data term of Phi
// (partials per block, when not NULL).
__global__ __launch_bounds__(kRayThreads) void k_blur_resid(BlurArgs b, int ni, int C,
                                                            const float* __restrict__ ybar0,
                                                            const float* __restrict__ y,
                                                            const float* __restrict__ w,
                                                            float* __restrict__ rres,
                                                            double* __restrict__ partials,
                                                            const long long* __restrict__ zd) {
    __shared__ double sh[kRayThreads / 64];
    if (zd) {                                              // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        ybar0 = zshift(ybar0, d);
        y = zshift(y, d);
        w = zshift(w, d);
        rres = zshift(rres, d);
        partials = zshift(partials, d);
    }
    const int i = blockIdx.x * kRayThreads + threadIdx.x;
    double phi = 0.0;
    if (i < ni) {
        for (int c = 0; c < C; ++c) {
            const float yb = blur_at(b, ybar0 + (size_t)c * ni, i, c, false);
            const float wc = w[(size_t)c * ni + i];
            const float dv = yb - y[(size_t)c * ni + i];
            rres[(size_t)c * ni + i] = wc * dv;
            phi += 0.5 * (double)wc * (double)dv * (double)dv;
        }
    }
    const double tot = block_sum(phi, sh);
    if (threadIdx.x == 0 && partials) partials[blockIdx.x] = tot;
}

// Blurred model, pass 3: r_c = (B^T rres_c)_i (stored to r_out when not NULL)
// and the energy pass with it and sig_c = wb_c rowS_c (eta = S^T B^T W B S 1).
template <int KT, int CT>
__global__ __launch_bounds__(kRayThreads) void k_ray_grad_r(RayModel m, int ni, const float* __restrict__ l,
                                                            const float* __restrict__ rres,
                                                            const float* __restrict__ wb,
                                                            const float* __restrict__ gammaA, BlurArgs b,
                                                            float* __restrict__ u, float* __restrict__ v,
                                                            float* __restrict__ r_out,
                                                            const long long* __restrict__ zd) {
    __shared__ SharedModel sm;
    if (zd) {                                              // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        m = zshift_model(m, d);
        l = zshift(l, d);
        rres = zshift(rres, d);
        wb = zshift(wb, d);
        gammaA = zshift(gammaA, d);
        u = zshift(u, d);
        v = zshift(v, d);
        r_out = zshift(r_out, d);
    }
    stage_model<KT, CT>(m, sm);
    const int K = KT ? KT : m.K, C = CT ? CT : m.C;
    const int i = blockIdx.x * kRayThreads + threadIdx.x;
    if (i >= ni) return;
    float lk[kMaxMat], rc[kMaxChan], sig[kMaxChan], uk[kMaxMat], vk[kMaxMat];
    for (int k = 0; k < K; ++k) lk[k] = l[(size_t)k * ni + i];
    for (int c = 0; c < C; ++c) {
        rc[c] = blur_at(b, rres + (size_t)c * ni, i, c, true);
        sig[c] = wb[(size_t)c * ni + i] * m.rowS[c];
        if (r_out) r_out[(size_t)c * ni + i] = rc[c];
    }
    ray_pass2<KT, CT>(m, sm, lk, rc, sig, gammaA ? gammaA[i] : 1.0f, v != nullptr, uk, vk);
    for (int k = 0; k < K; ++k) {
        u[(size_t)k * ni + i] = uk[k];
        if (v) v[(size_t)k * ni + i] = vk[k];
    }
}

// out_c = wt_c (B z_c) (or B^T z_c), one channel per grid row.
__global__ __launch_bounds__(kRayThreads) void k_blur(BlurArgs b, int ni, const float* __restrict__ in,
                                                      const float* __restrict__ wt, float* __restrict__ out,
                                                      int transpose) {
    const int i = blockIdx.x * kRayThreads + threadIdx.x, c = blockIdx.y;
    if (i >= ni) return;
    float s = blur_at(b, in + (size_t)c * ni, i, c, transpose != 0);
    if (wt) s *= wt[(size_t)c * ni + i];
    out[(size_t)c * ni + i] = s;
}

// Per ray with J [C][K][ni]: out_c = sum_k J_ck in_k, or transposed
// out_k = sum_c J_ck in_c.
__global__ __launch_bounds__(kRayThreads) void k_jmix(int ni, int K, int C, const float* __restrict__ J,
                                                      const float* __restrict__ in, float* __restrict__ out,
                                                      int transpose) {
    const int i = blockIdx.x * kRayThreads + threadIdx.x;
    if (i >= ni) return;
    if (!transpose) {
        for (int c = 0; c < C; ++c) {
            float s = 0.0f;
            for (int k = 0; k < K; ++k) s = fmaf(J[((size_t)c * K + k) * ni + i], in[(size_t)k * ni + i], s);
            out[(size_t)c * ni + i] = s;
        }
    } else {
        for (int k = 0; k < K; ++k) {
            float s = 0.0f;
            for (int c = 0; c < C; ++c) s = fmaf(J[((size_t)c * K + k) * ni + i], in[(size_t)c * ni + i], s);
            out[(size_t)k * ni + i] = s;
        }
    }
}

template <int KT, int CT>
__global__ __launch_bounds__(kRayThreads) void k_ray_grad(RayModel m, int ni, const float* __restrict__ l,
                                                          const float* __restrict__ y,
                                                          const float* __restrict__ w,
                                                          const float* __restrict__ gammaA,
                                                          float* __restrict__ u, float* __restrict__ v,
                                                          float* __restrict__ r_out,
                                                          double* __restrict__ partials, StepUpdate up, int nb_ray,
                                                          const long long* __restrict__ zd) {
    __shared__ double sh[kRayThreads / 64];
    __shared__ SharedModel sm;
    if (zd) {                                              // batched: this slice's buffers and image
        const long long d = zoff(zd, Z_BLOCK);
        m = zshift_model(m, d);
        l = zshift(l, d);
        y = zshift(y, d);
        w = zshift(w, d);
        gammaA = zshift(gammaA, d);
        u = zshift(u, d);
        v = zshift(v, d);
        r_out = zshift(r_out, d);
        partials = zshift(partials, d);
        up.alpha = zshift(up.alpha, d);
        up.q = zshift(up.q, d);
        up.l = zshift(up.l, d);
        up.p = zshift(up.p, d);
        up.x = zshift(up.x, zoff(zd, Z_IMAGE));
    }
    if (up.alpha && (int)blockIdx.x >= nb_ray) {           // the image part of the step: x += alpha p
        const float a = (float)*up.alpha;
        const int i = ((int)blockIdx.x - nb_ray) * kRayThreads + threadIdx.x;
        if (a != 0.0f && i < up.n_img) up.x[i] = fmaf(a, up.p[i], up.x[i]);
        return;
    }
    stage_model<KT, CT>(m, sm);
    const int K = KT ? KT : m.K;
    const int i = blockIdx.x * kRayThreads + threadIdx.x;
    double phi = 0.0;
    if (i < ni) {
        const float a = up.alpha ? (float)*up.alpha : 0.0f;
        float uk[kMaxMat], vk[kMaxMat];
        phi = ray_grad_at<KT, CT>(m, sm, ni, i, l, y, w, gammaA, r_out, up, a, v != nullptr, uk, vk);
        for (int k = 0; k < K; ++k) {
            u[(size_t)k * ni + i] = uk[k];
            if (v) v[(size_t)k * ni + i] = vk[k];
        }
    }
    const double tot = block_sum(phi, sh);
    if (threadIdx.x == 0 && partials) partials[blockIdx.x] = tot;
}

// The gradient pass fused with the back projector's detector rows of u: block
// slot < br.V takes the rays of that view slot (bins in row order, strided over
// the threads), keeps u times the path length in LDS and builds the rows from
// there -- the same values and arithmetic as storing u and running the
// detector prefix; blocks from br.V on apply the image part of the step.  Every
// block clears its share of br.clr.  Objective partials: one per view slot.
template <int KT, int CT>
__global__ __launch_bounds__(kRayThreads) void k_ray_grad_rows(RayModel m, int ni, const float* __restrict__ l,
                                                               const float* __restrict__ y,
                                                               const float* __restrict__ w,
                                                               float* __restrict__ r_out,
                                                               double* __restrict__ partials, StepUpdate up,
                                                               BackRows br) {
    extern __shared__ float wl[];                          // [K][B] widths of the slot's rows
    __shared__ double sh[kRayThreads / 64];
    __shared__ double wave_total[kMaxMat][kRayThreads / 64];
    __shared__ SharedModel sm;
    clear_back_pixels(br.clr, blockIdx.x, gridDim.x);      // side job
    if ((int)blockIdx.x >= br.V) {                         // the image part of the step: x += alpha p
        const float a = up.alpha ? (float)*up.alpha : 0.0f;
        const int i = ((int)blockIdx.x - br.V) * kRayThreads + threadIdx.x;
        if (a != 0.0f && i < up.n_img) up.x[i] = fmaf(a, up.p[i], up.x[i]);
        return;
    }
    stage_model<KT, CT>(m, sm);
    const int K = KT ? KT : m.K;
    const int slot = blockIdx.x, B = br.B;
    const ViewParams vp = br.view[slot];
    const bool rev = vp.orient < 0.0f;
    const int view = vp_view(vp);
    const float* pa = br.path + (size_t)slot * B;
    const float a = up.alpha ? (float)*up.alpha : 0.0f;
    double phi = 0.0;
    for (int pos = threadIdx.x; pos < B; pos += kRayThreads) {
        const int bin = rev ? B - 1 - pos : pos;           // row order runs along +K
        float uk[kMaxMat], vk[kMaxMat];
        phi += ray_grad_at<KT, CT>(m, sm, ni, view * B + bin, l, y, w, nullptr, r_out, up, a, false, uk, vk);
        const double L = (double)pa[bin];
        for (int k = 0; k < K; ++k) wl[k * B + pos] = (float)((double)uk[k] * L);
    }
    const double tot = block_sum(phi, sh);                 // its barriers also publish wl
    if (threadIdx.x == 0 && partials) partials[slot] = tot;
    __syncthreads();
    for (int k = 0; k < K; ++k)
        build_detector_row([&](int b) { return wl[k * B + b]; }, B,
                           br.rows + ((size_t)k * br.V + slot) * det_row(B), wave_total[k]);
}

// Ray i's share of sum_iE c_iE q_iE^2 with q_iE = sum_k Q_Ek q_ik, c recomputed
// from l and r.
template <int KT, int CT>
__device__ __forceinline__ double ray_curv_at(const RayModel& m, const SharedModel& sm, int ni,
                                              const float* __restrict__ l, const float* __restrict__ r,
                                              const float* __restrict__ w, const float* __restrict__ q, int i) {
    const int K = KT ? KT : m.K, C = CT ? CT : m.C;
    float lk[kMaxMat], qk[kMaxMat], rc[kMaxChan], sig[kMaxChan];
    for (int k = 0; k < K; ++k) {
        lk[k] = l[(size_t)k * ni + i];
        qk[k] = q[(size_t)k * ni + i];
    }
    for (int c = 0; c < C; ++c) {
        rc[c] = r[(size_t)c * ni + i];
        sig[c] = w[(size_t)c * ni + i] * m.rowS[c];
    }
    float a = 0.0f;
#pragma unroll 2
    for (int e = 0; e < m.E; ++e) {
        float le = 0.0f, qe = 0.0f;
        for (int k = 0; k < K; ++k) {
            const float qek = sm.Q[e * K + k];
            le = fmaf(qek, lk[k], le);
            qe = fmaf(qek, qk[k], qe);
        }
        const float t = transmission(le);
        float s = 0.0f, eta = 0.0f;
        for (int c = 0; c < C; ++c) {
            const float sce = sm.S[e * C + c];
            s = fmaf(sce, rc[c], s);
            eta = fmaf(sce, sig[c], eta);
        }
        const float ce = fmaxf(2.0f * eta + s - eta * t, 0.0f);
        a = fmaf(ce * qe, qe, a);
    }
    return (double)a;
}

template <int KT, int CT>
__global__ __launch_bounds__(kRayThreads) void k_ray_curv(RayModel m, int ni, const float* __restrict__ l,
                                                          const float* __restrict__ r,
                                                          const float* __restrict__ w,
                                                          const float* __restrict__ q,
                                                          double* __restrict__ partials) {
    __shared__ double sh[kRayThreads / 64];
    __shared__ SharedModel sm;
    stage_model<KT, CT>(m, sm);
    const int i = blockIdx.x * kRayThreads + threadIdx.x;
    const double acc = i < ni ? ray_curv_at<KT, CT>(m, sm, ni, l, r, w, q, i) : 0.0;
    const double tot = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// The curvature of the objective along the direction in one launch: blocks
// [0, nb_ray) write the rays' partial sums of c q^2 (region CQ2), blocks
// [nb_ray, nb_ray + nb_pen) the penalty's partial sums of p^T R''(x) p (region
// PRP).  (A last-block reduction in the same launch was tried: the per-block
// device-scope release and the single-address ticket cost far more than the
// separate reduction launch on a GPU whose L2s are per XCD.)
template <int KT, int CT>
__global__ __launch_bounds__(kRayThreads) void k_curvature(RayModel m, int ni, const float* __restrict__ l,
                                                           const float* __restrict__ r,
                                                           const float* __restrict__ w,
                                                           const float* __restrict__ q, int nb_ray,
                                                           PenaltyArgs pa, const float* __restrict__ x,
                                                           const float* __restrict__ p,
                                                           double* __restrict__ partials,
                                                           const long long* __restrict__ zd) {
    __shared__ double sh[kRayThreads / 64];
    __shared__ SharedModel sm;
    if (zd) {                                              // batched: this slice's buffers and image
        const long long d = zoff(zd, Z_BLOCK);
        m = zshift_model(m, d);
        l = zshift(l, d);
        r = zshift(r, d);
        w = zshift(w, d);
        q = zshift(q, d);
        pa.beta = zshift(pa.beta, d);
        x = zshift(x, zoff(zd, Z_IMAGE));
        p = zshift(p, d);
        partials = zshift(partials, d);
    }
    const int b = blockIdx.x;
    double acc = 0.0;
    if (b < nb_ray) {                                      // uniform over the block
        stage_model<KT, CT>(m, sm);
        const int i = b * kRayThreads + threadIdx.x;
        if (i < ni) acc = ray_curv_at<KT, CT>(m, sm, ni, l, r, w, q, i);
    } else {
        const int j = (b - nb_ray) * kRayThreads + threadIdx.x;
        if (j < pa.nx * pa.ny) acc = dev::penalty_quadform_at(pa, x, p, j);
    }
    const double tot = block_sum(acc, sh);
    if (threadIdx.x == 0)
        partials[b < nb_ray ? (size_t)R_CQ2 * kMaxPartials + b : (size_t)R_PRP * kMaxPartials + (b - nb_ray)] = tot;
}

template <int KT, int CT>
__global__ __launch_bounds__(kRayThreads) void k_forward_model(RayModel m, int ni, const float* __restrict__ l,
                                                               float* __restrict__ ybar_out) {
    __shared__ SharedModel sm;
    stage_model<KT, CT>(m, sm);
    const int K = KT ? KT : m.K, C = CT ? CT : m.C;
    const int i = blockIdx.x * kRayThreads + threadIdx.x;
    if (i >= ni) return;
    float lk[kMaxMat], ybar[kMaxChan];
    for (int k = 0; k < K; ++k) lk[k] = l[(size_t)k * ni + i];
    channel_means<KT, CT>(m, sm, lk, ybar);
    for (int c = 0; c < C; ++c) ybar_out[(size_t)c * ni + i] = ybar[c];
}

// s_k = sum_E Q_Ek (-t_E) sum_c S_cE gbar_c
template <int KT, int CT>
__global__ __launch_bounds__(kRayThreads) void k_forward_vjp(RayModel m, int ni, const float* __restrict__ l,
                                                             const float* __restrict__ gbar,
                                                             float* __restrict__ sk) {
    __shared__ SharedModel sm;
    stage_model<KT, CT>(m, sm);
    const int K = KT ? KT : m.K, C = CT ? CT : m.C;
    const int i = blockIdx.x * kRayThreads + threadIdx.x;
    if (i >= ni) return;
    float lk[kMaxMat], gc[kMaxChan], acc[kMaxMat];
    for (int k = 0; k < K; ++k) {
        lk[k] = l[(size_t)k * ni + i];
        acc[k] = 0.0f;
    }
    for (int c = 0; c < C; ++c) gc[c] = gbar[(size_t)c * ni + i];
#pragma unroll 2
    for (int e = 0; e < m.E; ++e) {
        float le = 0.0f;
        for (int k = 0; k < K; ++k) le = fmaf(sm.Q[e * K + k], lk[k], le);
        const float t = transmission(le);
        float s = 0.0f;
        for (int c = 0; c < C; ++c) s = fmaf(sm.S[e * C + c], gc[c], s);
        const float f = -t * s;
        for (int k = 0; k < K; ++k) acc[k] = fmaf(sm.Q[e * K + k], f, acc[k]);
    }
    for (int k = 0; k < K; ++k) sk[(size_t)k * ni + i] = acc[k];
}

// Fisher weights W_i = J^T diag(w) J (and J itself to Jout when not NULL),
// J[c,k] = -sum_E S_cE D_E Q_Ek, with D
// the transmission exp(-sum_k Q_Ek lref_k) at reference line integrals lref
// [K][ni] when given, else the data-based D: y / I0 for one energy and
// channel, else exp(-mu_w(E) l_w) from a 10-step Gauss-Newton water-only
// estimate (material 0 is water).
__global__ __launch_bounds__(kRayThreads) void k_fisher(RayModel m, int ni, const float* __restrict__ y,
                                                        const float* __restrict__ w,
                                                        const float* __restrict__ lref,
                                                        float* __restrict__ W, float* __restrict__ Jout) {
    const int i = blockIdx.x * kRayThreads + threadIdx.x;
    if (i >= ni) return;
    const int npk = m.K * (m.K + 1) / 2;
    double yc[kMaxChan], wc[kMaxChan];
    for (int c = 0; c < m.C; ++c) {
        yc[c] = y[(size_t)c * ni + i];
        wc[c] = w[(size_t)c * ni + i];
    }
    double J[kMaxChan][kMaxMat];
    if (lref) {
        double lk[kMaxMat];
        for (int k = 0; k < m.K; ++k) lk[k] = lref[(size_t)k * ni + i];
        for (int c = 0; c < m.C; ++c)
            for (int k = 0; k < m.K; ++k) J[c][k] = 0.0;
        for (int e = 0; e < m.E; ++e) {
            double le = 0.0;
            for (int k = 0; k < m.K; ++k) le += (double)m.Q[e * m.K + k] * lk[k];
            const double D = exp(-le);
            for (int c = 0; c < m.C; ++c) {
                const double sd = (double)m.S[c * m.E + e] * D;
                for (int k = 0; k < m.K; ++k) J[c][k] -= sd * (double)m.Q[e * m.K + k];
            }
        }
    } else if (m.E == 1 && m.C == 1) {
        const double D = yc[0] / (double)m.S[0];
        for (int k = 0; k < m.K; ++k) J[0][k] = -(double)m.S[0] * D * (double)m.Q[k];
    } else {
        double lw = 0.0;
        for (int it = 0; it < 10; ++it) {
            double res[kMaxChan], jac[kMaxChan];
            for (int c = 0; c < m.C; ++c) res[c] = jac[c] = 0.0;
            for (int e = 0; e < m.E; ++e) {
                const double mu = m.Q[e * m.K];
                const double ex = exp(-mu * lw);
                for (int c = 0; c < m.C; ++c) {
                    const double sce = m.S[c * m.E + e];
                    res[c] += sce * ex;
                    jac[c] -= sce * mu * ex;
                }
            }
            double num = 0.0, den = 0.0;
            for (int c = 0; c < m.C; ++c) {
                num += wc[c] * jac[c] * (res[c] - yc[c]);
                den += wc[c] * jac[c] * jac[c];
            }
            const double step = den > 0.0 ? num / den : 0.0;
            lw = fmax(lw - step, 0.0);
        }
        for (int c = 0; c < m.C; ++c)
            for (int k = 0; k < m.K; ++k) J[c][k] = 0.0;
        for (int e = 0; e < m.E; ++e) {
            const double D = exp(-(double)m.Q[e * m.K] * lw);
            for (int c = 0; c < m.C; ++c) {
                const double sd = (double)m.S[c * m.E + e] * D;
                for (int k = 0; k < m.K; ++k) J[c][k] -= sd * (double)m.Q[e * m.K + k];
            }
        }
    }
    for (int k = 0; k < m.K; ++k)
        for (int l2 = k; l2 < m.K; ++l2) {
            double s = 0.0;
            for (int c = 0; c < m.C; ++c) s += wc[c] * J[c][k] * J[c][l2];
            W[(size_t)packed_index(k, l2, m.K) * ni + i] = (float)s;
        }
    if (Jout)
        for (int c = 0; c < m.C; ++c)
            for (int k = 0; k < m.K; ++k) Jout[((size_t)c * m.K + k) * ni + i] = (float)J[c][k];
    (void)npk;
}

__global__ __launch_bounds__(kRayThreads) void k_fisher_mix(int ni, int K, const float* __restrict__ W,
                                                            const float* __restrict__ in,
                                                            float* __restrict__ out) {
    const int i = blockIdx.x * kRayThreads + threadIdx.x;
    if (i >= ni) return;
    float a[kMaxMat];
    for (int k = 0; k < K; ++k) a[k] = in[(size_t)k * ni + i];
    for (int k = 0; k < K; ++k) {
        float s = 0.0f;
        for (int l2 = 0; l2 < K; ++l2) s = fmaf(W[(size_t)packed_index(k, l2, K) * ni + i], a[l2], s);
        out[(size_t)k * ni + i] = s;
    }
}

// Whole iteration of the identity geometry without a penalty: every ray is an
// independent N_k-unknown problem, so all n_iter iterations run in registers.
// precond 0: plain SPS, x -= g / d.  precond 3: p = -M0 M0 g, per-ray alpha
// from the 1D majoriser.  Objective partials of iteration it go to
// partials[it * stride + block], the final one to partials[n_iter * stride + block].
template <int KT, int CT>
__global__ __launch_bounds__(kRayThreads) void k_identity_iterate(RayModel m, int ni, float* __restrict__ x,
                                                                  const float* __restrict__ y,
                                                                  const float* __restrict__ w,
                                                                  const float* __restrict__ M0,
                                                                  int precond, int n_iter,
                                                                  double* __restrict__ partials,
                                                                  int stride) {
    __shared__ double sh[kRayThreads / 64];
    __shared__ SharedModel sm;
    stage_model<KT, CT>(m, sm);
    const int K = KT ? KT : m.K, C = CT ? CT : m.C;
    const int i = blockIdx.x * kRayThreads + threadIdx.x;
    const bool act = i < ni;
    float xk[kMaxMat], yc[kMaxChan], wc[kMaxChan], sig[kMaxChan], Mb[kMaxPacked];
    const int npk = K * (K + 1) / 2;
    if (act) {
        for (int k = 0; k < K; ++k) xk[k] = x[(size_t)k * ni + i];
        for (int c = 0; c < C; ++c) {
            yc[c] = y[(size_t)c * ni + i];
            wc[c] = w[(size_t)c * ni + i];
            sig[c] = wc[c] * m.rowS[c];
        }
        if (precond == MBMD_PRECOND_BLOCKDIAG)
            for (int t = 0; t < npk; ++t) Mb[t] = M0[(size_t)t * ni + i];
    }
    for (int it = 0; it <= n_iter; ++it) {
        double phi = 0.0;
        float rc[kMaxChan], ybar[kMaxChan];
        if (act) {
            channel_means<KT, CT>(m, sm, xk, ybar);
            for (int c = 0; c < C; ++c) {
                const float dv = ybar[c] - yc[c];
                rc[c] = wc[c] * dv;
                phi += 0.5 * (double)wc[c] * (double)dv * (double)dv;
            }
        }
        const double tot = block_sum(phi, sh);
        if (threadIdx.x == 0) partials[(size_t)it * stride + blockIdx.x] = tot;
        if (it == n_iter || !act) continue;
        float gk[kMaxMat], dk[kMaxMat];
        for (int k = 0; k < K; ++k) gk[k] = dk[k] = 0.0f;
#pragma unroll 2
        for (int e = 0; e < m.E; ++e) {
            float le = 0.0f;
            for (int k = 0; k < K; ++k) le = fmaf(sm.Q[e * K + k], xk[k], le);
            const float t = transmission(le);
            float s = 0.0f, eta = 0.0f;
            for (int c = 0; c < C; ++c) {
                const float sce = sm.S[e * C + c];
                s = fmaf(sce, rc[c], s);
                eta = fmaf(sce, sig[c], eta);
            }
            const float hdot = -t * s;
            const float ce = fmaxf(2.0f * eta + s - eta * t, 0.0f);
            const float gc = sm.Qsum[e] * ce;
            for (int k = 0; k < K; ++k) {
                gk[k] = fmaf(sm.Q[e * K + k], hdot, gk[k]);
                dk[k] = fmaf(sm.Q[e * K + k], gc, dk[k]);
            }
        }
        if (precond != MBMD_PRECOND_BLOCKDIAG) {
            for (int k = 0; k < K; ++k) xk[k] -= gk[k] / fmaxf(dk[k], 1e-30f);
            continue;
        }
        float h[kMaxMat], p[kMaxMat];
        for (int k = 0; k < K; ++k) {
            float s = 0.0f;
            for (int l2 = 0; l2 < K; ++l2) s = fmaf(Mb[packed_index(k, l2, K)], gk[l2], s);
            h[k] = s;
        }
        float num = 0.0f;
        for (int k = 0; k < K; ++k) {
            float s = 0.0f;
            for (int l2 = 0; l2 < K; ++l2) s = fmaf(Mb[packed_index(k, l2, K)], h[l2], s);
            p[k] = -s;
            num = fmaf(-gk[k], p[k], num);
        }
        float den = 0.0f;
#pragma unroll 2
        for (int e = 0; e < m.E; ++e) {
            float le = 0.0f, qe = 0.0f;
            for (int k = 0; k < K; ++k) {
                le = fmaf(sm.Q[e * K + k], xk[k], le);
                qe = fmaf(sm.Q[e * K + k], p[k], qe);
            }
            const float t = transmission(le);
            float s = 0.0f, eta = 0.0f;
            for (int c = 0; c < C; ++c) {
                const float sce = sm.S[e * C + c];
                s = fmaf(sce, rc[c], s);
                eta = fmaf(sce, sig[c], eta);
            }
            const float ce = fmaxf(2.0f * eta + s - eta * t, 0.0f);
            den = fmaf(ce * qe, qe, den);
        }
        const float alpha = den > 0.0f ? num / den : 0.0f;
        for (int k = 0; k < K; ++k) xk[k] = fmaf(alpha, p[k], xk[k]);
    }
    if (act)
        for (int k = 0; k < K; ++k) x[(size_t)k * ni + i] = xk[k];
}

RayModel model_of(const RayArgs& a) { return RayModel{a.K, a.E, a.C, a.Q, a.S, a.rowS, a.Qsum}; }

int blocks_for(int n) { return (n + kRayThreads - 1) / kRayThreads; }

// Compile-time (N_k, N_c) for the shapes in use; anything else runs the generic form.
#define MBMD_RAY_DISPATCH(K, C, LAUNCH)                \
    do {                                                \
        if ((K) == 1 && (C) == 1) { LAUNCH(1, 1); }     \
        else if ((K) == 2 && (C) == 2) { LAUNCH(2, 2); } \
        else if ((K) == 3 && (C) == 4) { LAUNCH(3, 4); } \
        else { LAUNCH(0, 0); }                          \
    } while (0)



}  // namespace

int launch_ray_grad(const RayArgs& a, const float* l, float* u, float* v, float* r, double* phi_partials,
                    hipStream_t s, const StepUpdate* up) {
    const int nb = blocks_for(a.ni);
    MBMD_REQUIRE(nb <= kMaxPartials, MBMD_ERR_SHAPE, "too many rays for the partial-sum buffer");
    const StepUpdate upd = up ? *up : StepUpdate{nullptr, nullptr, nullptr, nullptr, nullptr, 0};
    MBMD_REQUIRE(!up || up->l == l, MBMD_ERR_ARG, "the step update must update the l it reads");
    const int nb_img = up ? blocks_for(up->n_img) : 0;
    if (a.blur.h > 0) {                                    // three passes (the residual couples bins)
        MBMD_REQUIRE(a.tmp0 && a.tmp1 && a.wb && a.blur.B > 0 && a.ni % a.blur.B == 0, MBMD_ERR_ARG,
                     "blurred ray pass without its buffers");
        {
            KernelTimer kt_("k_ray_means", s);
#define L_(KT, CT) hipLaunchKernelGGL((k_ray_means<KT, CT>), zgrid(dim3(nb + nb_img)), dim3(kRayThreads), 0, s, \
                                   model_of(a), a.ni, l, a.tmp0, upd, nb, zarg())
            MBMD_RAY_DISPATCH(a.K, a.C, L_);
#undef L_
            kt_.stop();
        }
        MBMD_LAUNCHED();
        {
            KernelTimer kt_("k_blur_resid", s);
            hipLaunchKernelGGL(k_blur_resid, zgrid(dim3(nb)), dim3(kRayThreads), 0, s, a.blur, a.ni, a.C, a.tmp0,
                               a.y, a.w, a.tmp1, phi_partials, zarg());
            kt_.stop();
        }
        MBMD_LAUNCHED();
        {
            KernelTimer kt_("k_ray_grad_r", s);
#define L_(KT, CT) hipLaunchKernelGGL((k_ray_grad_r<KT, CT>), zgrid(dim3(nb)), dim3(kRayThreads), 0, s, \
                                   model_of(a), a.ni, l, a.tmp1, a.wb, a.gammaA, a.blur, u, v, r, zarg())
            MBMD_RAY_DISPATCH(a.K, a.C, L_);
#undef L_
            kt_.stop();
        }
        MBMD_LAUNCHED();
        return nb;
    }
    {
        KernelTimer kt_("k_ray_grad", s);
#define L_(KT, CT) hipLaunchKernelGGL((k_ray_grad<KT, CT>), zgrid(dim3(nb + nb_img)), dim3(kRayThreads), 0, s,     \
                                   model_of(a), a.ni, l, a.y, a.w, a.gammaA, u, v, r, phi_partials, upd, nb, zarg())
        MBMD_RAY_DISPATCH(a.K, a.C, L_);
#undef L_
        kt_.stop();
    }
    MBMD_LAUNCHED();
    return nb;
}

int launch_ray_grad_rows(const RayArgs& a, const float* l, float* r, double* phi_partials, hipStream_t s,
                         const StepUpdate& up, const BackRows& br) {
    MBMD_REQUIRE(br.ok && br.V * br.B == a.ni, MBMD_ERR_ARG, "detector rows do not match the rays");
    MBMD_REQUIRE(a.blur.h == 0, MBMD_ERR_ARG, "the fused gradient rows take no blur");
    MBMD_REQUIRE(br.V <= kMaxPartials, MBMD_ERR_SHAPE, "too many views for the partial-sum buffer");
    MBMD_REQUIRE(up.l == l, MBMD_ERR_ARG, "the step update must update the l it reads");
    const size_t lds = sizeof(float) * (size_t)a.K * br.B;
    if (lds > 32768) return -1;                            // with the static LDS, over the per-block budget
    const int nb_img = up.alpha ? blocks_for(up.n_img) : 0;
    {
        KernelTimer kt_("k_ray_grad_rows", s);
#define L_(KT, CT) hipLaunchKernelGGL((k_ray_grad_rows<KT, CT>), dim3(br.V + nb_img), dim3(kRayThreads), lds, s, \
                                   model_of(a), a.ni, l, a.y, a.w, r, phi_partials, up, br)
        MBMD_RAY_DISPATCH(a.K, a.C, L_);
#undef L_
        kt_.stop();
    }
    MBMD_LAUNCHED();
    return br.V;
}

int launch_ray_curv(const RayArgs& a, const float* l, const float* r, const float* q, double* partials,
                    hipStream_t s) {
    const int nb = blocks_for(a.ni);
    MBMD_REQUIRE(nb <= kMaxPartials, MBMD_ERR_SHAPE, "too many rays for the partial-sum buffer");
    {
        KernelTimer kt_("k_ray_curv", s);
#define L_(KT, CT) hipLaunchKernelGGL((k_ray_curv<KT, CT>), dim3(nb), dim3(kRayThreads), 0, s, model_of(a), a.ni, \
                                   l, r, a.wb, q, partials)
        MBMD_RAY_DISPATCH(a.K, a.C, L_);
#undef L_
        kt_.stop();
    }
    MBMD_LAUNCHED();
    return nb;
}

void launch_curvature(const RayArgs& a, const float* l, const float* r, const float* q, const PenaltyArgs* pen,
                      const float* x, const float* p, double* partials, int* counts, hipStream_t s) {
    const int nb_ray = blocks_for(a.ni);
    const int nb_pen = pen ? (pen->nx * pen->ny + kRayThreads - 1) / kRayThreads : 0;
    MBMD_REQUIRE(nb_ray <= kMaxPartials && nb_pen <= kMaxPartials, MBMD_ERR_SHAPE,
                 "too many rays or pixels for the partial-sum buffer");
    const PenaltyArgs pa = pen ? *pen : PenaltyArgs{1, 0, 0, 0, nullptr, 0.0f};
    {
        KernelTimer kt_("k_curvature", s);
#define L_(KT, CT) hipLaunchKernelGGL((k_curvature<KT, CT>), zgrid(dim3(nb_ray + nb_pen)), dim3(kRayThreads), 0, s, \
                                   model_of(a), a.ni, l, r, a.wb, q, nb_ray, pa, x, p, partials, zarg())
        MBMD_RAY_DISPATCH(a.K, a.C, L_);
#undef L_
        kt_.stop();
    }
    MBMD_LAUNCHED();
    counts[R_CQ2] = nb_ray;
    counts[R_PRP] = nb_pen;
}

void launch_forward_model(const RayArgs& a, const float* l, float* ybar, hipStream_t s) {
    float* out = a.blur.h > 0 ? a.tmp0 : ybar;             // the unblurred means, then B
    MBMD_REQUIRE(out != nullptr, MBMD_ERR_ARG, "blurred forward model without its buffers");
    {
        KernelTimer kt_("k_forward_model", s);
#define L_(KT, CT) hipLaunchKernelGGL((k_forward_model<KT, CT>), dim3(blocks_for(a.ni)), dim3(kRayThreads), 0, s, \
                                   model_of(a), a.ni, l, out)
        MBMD_RAY_DISPATCH(a.K, a.C, L_);
#undef L_
        kt_.stop();
    }
    MBMD_LAUNCHED();
    if (a.blur.h > 0) launch_blur(a.blur, a.ni, a.C, out, nullptr, ybar, false, s);
}

void launch_forward_vjp(const RayArgs& a, const float* l, const float* gbar, float* sk, hipStream_t s) {
    if (a.blur.h > 0) {                                    // B^T gbar first
        MBMD_REQUIRE(a.tmp0 != nullptr, MBMD_ERR_ARG, "blurred VJP without its buffers");
        launch_blur(a.blur, a.ni, a.C, gbar, nullptr, a.tmp0, true, s);
        gbar = a.tmp0;
    }
    {
        KernelTimer kt_("k_forward_vjp", s);
#define L_(KT, CT) hipLaunchKernelGGL((k_forward_vjp<KT, CT>), dim3(blocks_for(a.ni)), dim3(kRayThreads), 0, s, \
                                   model_of(a), a.ni, l, gbar, sk)
        MBMD_RAY_DISPATCH(a.K, a.C, L_);
#undef L_
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

void launch_fisher(const RayArgs& a, float* W, hipStream_t s, const float* lref, float* J) {
    {
        KernelTimer kt_("k_fisher", s);
        hipLaunchKernelGGL(k_fisher, dim3(blocks_for(a.ni)), dim3(kRayThreads), 0, s, model_of(a), a.ni, a.y,
                       a.w, lref, W, J);
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

void launch_blur(const BlurArgs& b, int ni, int C, const float* in, const float* wt, float* out, bool transpose,
                 hipStream_t s) {
    MBMD_REQUIRE(b.h > 0 && b.h <= kMaxBlurHalf && b.B > 0 && ni % b.B == 0 && C <= kMaxChan && in != out,
                 MBMD_ERR_ARG, "bad blur launch");
    {
        KernelTimer kt_("k_blur", s);
        hipLaunchKernelGGL(k_blur, dim3(blocks_for(ni), C), dim3(kRayThreads), 0, s, b, ni, in, wt, out,
                           transpose ? 1 : 0);
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

void launch_jmix(int ni, int K, int C, const float* J, const float* in, float* out, bool transpose, hipStream_t s) {
    MBMD_REQUIRE(in != out, MBMD_ERR_ARG, "k_jmix works out of place");
    {
        KernelTimer kt_("k_jmix", s);
        hipLaunchKernelGGL(k_jmix, dim3(blocks_for(ni)), dim3(kRayThreads), 0, s, ni, K, C, J, in, out,
                           transpose ? 1 : 0);
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

void launch_fisher_mix(int ni, int K, const float* W, const float* in, float* out, hipStream_t s) {
    {
        KernelTimer kt_("k_fisher_mix", s);
        hipLaunchKernelGGL(k_fisher_mix, dim3(blocks_for(ni)), dim3(kRayThreads), 0, s, ni, K, W, in, out);
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

int launch_identity_iterate(const RayArgs& a, float* x, const float* M0, int precond, int n_iter,
                            double* partials_per_iter, int stride, hipStream_t s) {
    const int nb = blocks_for(a.ni);
    MBMD_REQUIRE(nb <= stride, MBMD_ERR_SHAPE, "too many rays for the partial-sum buffer");
    {
        KernelTimer kt_("k_identity_iterate", s);
#define L_(KT, CT) hipLaunchKernelGGL((k_identity_iterate<KT, CT>), dim3(nb), dim3(kRayThreads), 0, s, model_of(a), \
                                   a.ni, x, a.y, a.w, M0, precond, n_iter, partials_per_iter, stride)
        MBMD_RAY_DISPATCH(a.K, a.C, L_);
#undef L_
        kt_.stop();
    }
    MBMD_LAUNCHED();
    return nb;
}

}  // namespace mbmd
