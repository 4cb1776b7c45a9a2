// Image-space kernels: roughness penalties, SPS updates, per-pixel material
// blocks and the final FP64 reductions.
//
// Penalties (eq:quadraticSmoothess, quadReg_summation): Gamma is the
// 4-neighbour graph Laplacian with out-of-image neighbours dropped;
// R = 1/2 x^T (beta (x) Gamma) x, with separable SPS curvature
// sum_k' |beta_kk'| 2 |N_j|.  Huber (one material): R = beta sum_pairs
// psi(x_j - x_j'), gradient beta sum psi'(.), separable curvature
// 2 beta sum omega(.) with omega(t) = psi'(t)/t (De Pierro split of Huber's
// quadratic majoriser).  Each unordered pair is charged to its left / upper
// pixel when a value is summed.
//
// Block operations: per-pixel (or per-frequency) symmetric N_k x N_k
// matrices are stored packed, component-major ([npk][n]) so that loads
// coalesce.  Inverse square roots use FP64 cyclic Jacobi (N_k <= 4).
#include <algorithm>
#include <cfloat>
#include <cmath>

#include "device_common.h"
#include "internal.h"

namespace mbmd {

namespace {

constexpr int kThreads = 256;

using dev::block_sum;
using dev::huber_omega;
using dev::Counts;


// g = gL (+ gL2) + dR/dx, d = dL + d_R (d may be NULL), partials of R(x).
// gL may alias g and dL may alias d (each element is read before it is written);
// gL2, when given, is a second addend (the column-sweep part of a back projection).
__global__ __launch_bounds__(kThreads) void k_penalty_grad(PenaltyArgs a, const float* __restrict__ x,
                                                           const float* gL, const float* dL, float* g, float* d,
                                                           double* __restrict__ partials,
                                                           const float* __restrict__ gL2,
                                                           const long long* __restrict__ zd) {
    __shared__ double sh[kThreads / 64];
    if (zd) {                                              // batched: this slice's buffers and image
        const long long dz = zoff(zd, Z_BLOCK);
        a.beta = zshift(a.beta, dz);
        x = zshift(x, zoff(zd, Z_IMAGE));
        gL = zshift(gL, dz);
        dL = zshift(dL, dz);
        g = zshift(g, dz);
        d = zshift(d, dz);
        partials = zshift(partials, dz);
        gL2 = zshift(gL2, dz);
    }
    const int nj = a.nx * a.ny;
    const int j = blockIdx.x * kThreads + threadIdx.x;
    double phi = 0.0;
    if (j < nj) {
        float gr[kMaxMat], cur[kMaxMat];
        phi = dev::penalty_grad_at(a, x, j, gr, d ? cur : nullptr);
        const int K = a.kind == MBMD_PENALTY_HUBER ? 1 : a.K;
#pragma unroll
        for (int k = 0; k < kMaxMat; ++k) {
            if (k >= K) break;
            const size_t jk = (size_t)k * nj + j;
            g[jk] = (gL2 ? gL[jk] + gL2[jk] : gL[jk]) + gr[k];
            if (d) d[jk] = dL[jk] + cur[k];
        }
    }
    const double tot = block_sum(phi, sh);
    if (threadIdx.x == 0 && partials) partials[blockIdx.x] = tot;
}

// p^T R'' p: quadratic p^T (beta (x) Gamma) p; Huber beta sum_pairs omega(x_j - x_j') (p_j - p_j')^2.
__global__ __launch_bounds__(kThreads) void k_penalty_quadform(PenaltyArgs a, const float* __restrict__ x,
                                                               const float* __restrict__ p,
                                                               double* __restrict__ partials) {
    __shared__ double sh[kThreads / 64];
    const int j = blockIdx.x * kThreads + threadIdx.x;
    const double acc = j < a.nx * a.ny ? dev::penalty_quadform_at(a, x, p, j) : 0.0;
    const double tot = block_sum(acc, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// out += (beta (x) Gamma) v (the quadratic Hessian; Huber builds use it too).
__global__ __launch_bounds__(kThreads) void k_penalty_hess_add(PenaltyArgs a, const float* __restrict__ v,
                                                               float* __restrict__ out) {
    const int nj = a.nx * a.ny;
    const int j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= nj) return;
    const int iy = j / a.nx, ix = j - iy * a.nx;
    const bool L = ix > 0, R = ix + 1 < a.nx, U = iy > 0, D = iy + 1 < a.ny;
    const float nn = (float)(L + R + U + D);
    float lap[kMaxMat];
    for (int k = 0; k < a.K; ++k) {
        const float* vk = v + (size_t)k * nj;
        float s = nn * vk[j];
        if (L) s -= vk[j - 1];
        if (R) s -= vk[j + 1];
        if (U) s -= vk[j - a.nx];
        if (D) s -= vk[j + a.nx];
        lap[k] = s;
    }
    for (int k = 0; k < a.K; ++k) {
        float gr = 0.0f;
        for (int l2 = 0; l2 < a.K; ++l2) gr = fmaf(a.beta[k * a.K + l2], lap[l2], gr);
        out[(size_t)k * nj + j] += gr;
    }
}

__global__ void k_plain_update(int n, float* __restrict__ x, const float* __restrict__ g,
                               const float* __restrict__ d, const long long* __restrict__ zd) {
    if (zd) {                                              // batched: this slice's buffers and image
        x = zshift(x, zoff(zd, Z_IMAGE));
        g = zshift(g, zoff(zd, Z_BLOCK));
        d = zshift(d, zoff(zd, Z_BLOCK));
    }
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) x[i] -= g[i] / fmaxf(d[i], 1e-30f);
}

__global__ void k_axpy_alpha(int n, float* __restrict__ x, const float* __restrict__ p,
                             const double* __restrict__ alpha) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) x[i] = fmaf((float)*alpha, p[i], x[i]);
}

__global__ void k_axpy2_alpha(int n1, float* __restrict__ x1, const float* __restrict__ p1, int n2,
                              float* __restrict__ x2, const float* __restrict__ p2,
                              const double* __restrict__ alpha, const long long* __restrict__ zd) {
    if (zd) {                                              // batched: x1 is the slice's image
        const long long d = zoff(zd, Z_BLOCK);
        x1 = zshift(x1, zoff(zd, Z_IMAGE));
        p1 = zshift(p1, d);
        x2 = zshift(x2, d);
        p2 = zshift(p2, d);
        alpha = zshift(alpha, d);
    }
    const int i = blockIdx.x * kThreads + threadIdx.x;
    const float a = (float)*alpha;
    if (i < n1) x1[i] = fmaf(a, p1[i], x1[i]);
    else if (i - n1 < n2) x2[i - n1] = fmaf(a, p2[i - n1], x2[i - n1]);
}

__global__ void k_fill(int n, float* __restrict__ x, float value, const long long* __restrict__ zd, int x_is_image) {
    if (zd) x = zshift(x, zoff(zd, x_is_image ? Z_IMAGE : Z_BLOCK));   // batched: this slice's buffer
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) x[i] = value;
}

__global__ void k_scale_copy(int n, const float* __restrict__ in, float* __restrict__ out, float scale,
                             const long long* __restrict__ zd) {
    {                                                      // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        in = zadd(in, d);
        out = zadd(out, d);
    }
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) out[i] = scale * in[i];
}

// Adds material column k_col of per-pixel blocks (col [K][nj]: entry (k2, k_col)
// at channel k2) to the packed symmetric blocks: the diagonal entry whole, the
// others half each (the other half comes from column k2), which gives the
// symmetric part of blocks that are not exactly symmetric.
__global__ void k_block_add_column(int nj, int K, int k_col, const float* __restrict__ col,
                                   float* __restrict__ packed) {
    const int j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= nj) return;
    for (int k2 = 0; k2 < K; ++k2) {
        const float wgt = k2 == k_col ? 1.0f : 0.5f;
        packed[(size_t)packed_index(k2, k_col, K) * nj + j] += wgt * col[(size_t)k2 * nj + j];
    }
}

__global__ __launch_bounds__(kThreads) void k_dot(int n, const float* __restrict__ a,
                                                  const float* __restrict__ b,
                                                  double* __restrict__ partials,
                                                  const long long* __restrict__ zd) {
    __shared__ double sh[kThreads / 64];
    if (zd) {                                              // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        a = zshift(a, d);
        b = zshift(b, d);
        partials = zshift(partials, d);
    }
    // one element per thread up to kMaxPartials blocks; longer vectors (several
    // materials at the largest images) add further elements in a fixed order
    double v = 0.0;
    for (long long i = (long long)blockIdx.x * kThreads + threadIdx.x; i < n; i += (long long)gridDim.x * kThreads)
        v += (double)a[i] * (double)b[i];
    const double tot = block_sum(v, sh);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// out_k = scale * sum_l M_kl in_l per pixel; M packed component-major.  in may alias out.
__global__ void k_block_apply(int nj, int K, const float* __restrict__ M, const float* in, float* out,
                              float scale, const long long* __restrict__ zd) {
    if (zd) {                                              // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        M = zshift(M, d);
        in = zshift(in, d);
        out = zshift(out, d);
    }
    const int j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= nj) return;
    float a[kMaxMat];
    for (int k = 0; k < K; ++k) a[k] = in[(size_t)k * nj + j];
    for (int k = 0; k < K; ++k) {
        float s = 0.0f;
        for (int l2 = 0; l2 < K; ++l2) s = fmaf(M[(size_t)packed_index(k, l2, K) * nj + j], a[l2], s);
        out[(size_t)k * nj + j] = scale * s;
    }
}

// Symmetric eigen-decomposition of a K x K matrix (K <= 4) by cyclic Jacobi.
__device__ void jacobi_eig(int K, double A[kMaxMat][kMaxMat], double V[kMaxMat][kMaxMat], double* lam) {
    for (int i = 0; i < K; ++i)
        for (int j = 0; j < K; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 16; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int i = 0; i < K; ++i)
            for (int j = 0; j < K; ++j) {
                tot += A[i][j] * A[i][j];
                if (i != j) off += A[i][j] * A[i][j];
            }
        if (off <= 1e-30 * tot || off == 0.0) break;
        for (int p = 0; p < K - 1; ++p)
            for (int q = p + 1; q < K; ++q) {
                if (A[p][q] == 0.0) continue;
                const double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                const double t = (theta >= 0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                for (int k = 0; k < K; ++k) {
                    const double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - s * akq;
                    A[k][q] = s * akp + c * akq;
                }
                for (int k = 0; k < K; ++k) {
                    const double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - s * aqk;
                    A[q][k] = s * apk + c * aqk;
                }
                for (int k = 0; k < K; ++k) {
                    const double vkp = V[k][p], vkq = V[k][q];
                    V[k][p] = c * vkp - s * vkq;
                    V[k][q] = s * vkp + c * vkq;
                }
            }
    }
    for (int i = 0; i < K; ++i) lam[i] = A[i][i];
}

__device__ void load_block(int K, const float* __restrict__ in, int n, int j, double A[kMaxMat][kMaxMat]) {
    for (int k = 0; k < K; ++k)
        for (int l2 = 0; l2 < K; ++l2) A[k][l2] = (double)in[(size_t)packed_index(k, l2, K) * n + j];
}

// out = V diag(max(lam, floor)^power) V^T.  floor = floor_rel * lambda_max of
// the block (blocks with lambda_max <= 0 map to 0) unless floor_abs is given,
// in which case floor = eps * (*floor_abs) for every block.
__global__ void k_block_invsqrt(int n, int K, const float* __restrict__ in, float* __restrict__ out,
                                double power, double floor_rel, const double* __restrict__ floor_abs,
                                double eps, int* __restrict__ n_floored) {
    const int j = blockIdx.x * kThreads + threadIdx.x;
    if (j >= n) return;
    double A[kMaxMat][kMaxMat], V[kMaxMat][kMaxMat], lam[kMaxMat];
    load_block(K, in, n, j, A);
    jacobi_eig(K, A, V, lam);
    double lmax = -DBL_MAX;
    for (int k = 0; k < K; ++k) lmax = fmax(lmax, lam[k]);
    double floor;
    bool zero = false;
    if (floor_abs) {
        floor = eps * (*floor_abs);
    } else {
        floor = floor_rel * lmax;
        zero = !(lmax > 0.0);
    }
    int nf = 0;
    double f[kMaxMat];
    for (int k = 0; k < K; ++k) {
        double l2 = lam[k];
        if (l2 < floor) { l2 = floor; ++nf; }
        f[k] = (zero || !(l2 > 0.0)) ? 0.0 : pow(l2, power);
    }
    for (int k = 0; k < K; ++k)
        for (int l2 = k; l2 < K; ++l2) {
            double s = 0.0;
            for (int m = 0; m < K; ++m) s += V[k][m] * f[m] * V[l2][m];
            out[(size_t)packed_index(k, l2, K) * n + j] = (float)s;
        }
    if (nf && n_floored) atomicAdd(n_floored, nf);
}

__device__ void atomic_max_double(double* addr, double val) {
    unsigned long long* a = reinterpret_cast<unsigned long long*>(addr);
    unsigned long long old = *a;
    while (__longlong_as_double(old) < val) {
        const unsigned long long prev = atomicCAS(a, old, __double_as_longlong(val));
        if (prev == old) break;
        old = prev;
    }
}

__global__ __launch_bounds__(kThreads) void k_block_lmax(int n, int K, const float* __restrict__ in,
                                                         double* __restrict__ lmax_out) {
    __shared__ double sh[kThreads];
    const int j = blockIdx.x * kThreads + threadIdx.x;
    double lm = -DBL_MAX;
    if (j < n) {
        double A[kMaxMat][kMaxMat], V[kMaxMat][kMaxMat], lam[kMaxMat];
        load_block(K, in, n, j, A);
        jacobi_eig(K, A, V, lam);
        for (int k = 0; k < K; ++k) lm = fmax(lm, lam[k]);
    }
    sh[threadIdx.x] = lm;
    __syncthreads();
    for (int off = kThreads / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomic_max_double(lmax_out, sh[0]);
}

__global__ void k_inv_var(int n, const float* __restrict__ y, float* __restrict__ w) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) w[i] = 1.0f / fmaxf(y[i], 1.0f);
}

// out[c][i] = in[c][i] * vec[i] for c < nch
__global__ void k_scale_by_vec(int n, int nch, const float* __restrict__ in, const float* __restrict__ vec,
                               float* __restrict__ out) {
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const float s = vec ? vec[i] : 1.0f;
    for (int c = 0; c < nch; ++c) out[(size_t)c * n + i] = in[(size_t)c * n + i] * s;
}

__global__ void k_fill_double(int n, double* __restrict__ x, double value, const long long* __restrict__ zd) {
    if (zd) x = zshift(x, zoff(zd, Z_BLOCK));             // batched: this slice's buffer
    const int i = blockIdx.x * kThreads + threadIdx.x;
    if (i < n) x[i] = value;
}


// Sums of the partial-sum regions and the scalars formed from them, in an
// order fixed by the block size: the result does not depend on timing.
__global__ __launch_bounds__(dev::kReduceThreads) void k_reduce_final(const double* __restrict__ partials,
                                                                      Counts counts, double* __restrict__ scal,
                                                                      double* __restrict__ trace_slot, int mode,
                                                                      int* __restrict__ flags,
                                                                      const long long* __restrict__ zd) {
    __shared__ double sh[2 * kRegions];
    {                                                      // batched: this slice's buffers
        const long long d = zoff(zd, Z_BLOCK);
        partials = zadd(partials, d);
        scal = zadd(scal, d);
        trace_slot = zshift(trace_slot, d);
        flags = zadd(flags, d);
    }
    dev::region_sums(partials, counts, sh);
    if (threadIdx.x == 0) dev::form_scalars(sh, mode, scal, trace_slot, flags, true);
}

int nblk(int n) { return (n + kThreads - 1) / kThreads; }

}  // namespace

void launch_inv_var(int n, const float* y, float* w, hipStream_t s) {
    {
        KernelTimer kt_("k_inv_var", s);
        hipLaunchKernelGGL(k_inv_var, dim3(nblk(n)), dim3(kThreads), 0, s, n, y, w);
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

void launch_scale_by_vec(int n, int nch, const float* in, const float* vec, float* out, hipStream_t s) {
    {
        KernelTimer kt_("k_scale_by_vec", s);
        hipLaunchKernelGGL(k_scale_by_vec, dim3(nblk(n)), dim3(kThreads), 0, s, n, nch, in, vec, out);
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

void launch_fill_double(int n, double* x, double value, hipStream_t s) {
    {
        KernelTimer kt_("k_fill_double", s);
        hipLaunchKernelGGL(k_fill_double, zgrid(dim3(nblk(n))), dim3(kThreads), 0, s, n, x, value, zarg());
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

int launch_penalty_grad(const PenaltyArgs& a, const float* x, const float* gL, const float* dL, float* g,
                        float* d, double* phi_partials, hipStream_t s, const float* gL2) {
    const int nb = nblk(a.nx * a.ny);
    MBMD_REQUIRE(nb <= kMaxPartials, MBMD_ERR_SHAPE, "image too large for the partial-sum buffer");
    {
        KernelTimer kt_("k_penalty_grad", s);
        hipLaunchKernelGGL(k_penalty_grad, zgrid(dim3(nb)), dim3(kThreads), 0, s, a, x, gL, dL, g, d, phi_partials, gL2,
                           zarg());
        kt_.stop();
    }
    MBMD_LAUNCHED();
    return nb;
}

int launch_penalty_quadform(const PenaltyArgs& a, const float* x, const float* p, double* partials,
                            hipStream_t s) {
    const int nb = nblk(a.nx * a.ny);
    {
        KernelTimer kt_("k_penalty_quadform", s);
        hipLaunchKernelGGL(k_penalty_quadform, dim3(nb), dim3(kThreads), 0, s, a, x, p, partials);
        kt_.stop();
    }
    MBMD_LAUNCHED();
    return nb;
}

void launch_penalty_hess_add(const PenaltyArgs& a, const float* v, float* out, hipStream_t s) {
    {
        KernelTimer kt_("k_penalty_hess_add", s);
        hipLaunchKernelGGL(k_penalty_hess_add, dim3(nblk(a.nx * a.ny)), dim3(kThreads), 0, s, a, v, out);
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

void launch_plain_update(int n, float* x, const float* g, const float* d, hipStream_t s) {
    {
        KernelTimer kt_("k_plain_update", s);
        hipLaunchKernelGGL(k_plain_update, zgrid(dim3(nblk(n))), dim3(kThreads), 0, s, n, x, g, d, zarg());
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

void launch_axpy_alpha(int n, float* x, const float* p, const double* alpha, hipStream_t s) {
    {
        KernelTimer kt_("k_axpy_alpha", s);
        hipLaunchKernelGGL(k_axpy_alpha, dim3(nblk(n)), dim3(kThreads), 0, s, n, x, p, alpha);
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

void launch_axpy2_alpha(int n1, float* x1, const float* p1, int n2, float* x2, const float* p2,
                        const double* alpha, hipStream_t s) {
    {
        KernelTimer kt_("k_axpy2_alpha", s);
        hipLaunchKernelGGL(k_axpy2_alpha, zgrid(dim3(nblk(n1 + n2))), dim3(kThreads), 0, s, n1, x1, p1, n2, x2, p2,
                           alpha, zarg());
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

void launch_fill(int n, float* x, float value, hipStream_t s) {
    {
        KernelTimer kt_("k_fill", s);
        hipLaunchKernelGGL(k_fill, zgrid(dim3(nblk(n))), dim3(kThreads), 0, s, n, x, value, zarg(),
                           (int)(zarg() && x == zbatch().x0));
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

void launch_block_add_column(int nj, int K, int k_col, const float* col, float* packed, hipStream_t s) {
    {
        KernelTimer kt_("k_block_add_column", s);
        hipLaunchKernelGGL(k_block_add_column, dim3(nblk(nj)), dim3(kThreads), 0, s, nj, K, k_col, col, packed);
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

void launch_scale_copy(int n, const float* in, float* out, float scale, hipStream_t s) {
    {
        KernelTimer kt_("k_scale_copy", s);
        hipLaunchKernelGGL(k_scale_copy, zgrid(dim3(nblk(n))), dim3(kThreads), 0, s, n, in, out, scale, zarg());
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

int launch_dot(int n, const float* a, const float* b, double* partials, hipStream_t s) {
    const int nb = std::min(nblk(n), kMaxPartials);
    {
        KernelTimer kt_("k_dot", s);
        hipLaunchKernelGGL(k_dot, zgrid(dim3(nb)), dim3(kThreads), 0, s, n, a, b, partials, zarg());
        kt_.stop();
    }
    MBMD_LAUNCHED();
    return nb;
}

void launch_block_apply(int nj, int K, const float* M, const float* in, float* out, float scale, hipStream_t s) {
    {
        KernelTimer kt_("k_block_apply", s);
        hipLaunchKernelGGL(k_block_apply, zgrid(dim3(nblk(nj))), dim3(kThreads), 0, s, nj, K, M, in, out, scale,
                           zarg());
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

void launch_block_invsqrt(int n, int K, const float* in_packed, float* out_packed, double power,
                          double floor_rel, const double* floor_abs_scaled, double eps, int* n_floored,
                          hipStream_t s) {
    {
        KernelTimer kt_("k_block_invsqrt", s);
        hipLaunchKernelGGL(k_block_invsqrt, dim3(nblk(n)), dim3(kThreads), 0, s, n, K, in_packed, out_packed,
                       power, floor_rel, floor_abs_scaled, eps, n_floored);
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

void launch_block_lmax(int n, int K, const float* in_packed, double* lmax, hipStream_t s) {
    {
        KernelTimer kt_("k_block_lmax", s);
        hipLaunchKernelGGL(k_block_lmax, dim3(nblk(n)), dim3(kThreads), 0, s, n, K, in_packed, lmax);
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

void launch_reduce_final(double* partials, const int* counts, double* scal, double* trace_slot, int mode,
                         int* flags, hipStream_t s) {
    Counts c;
    for (int r = 0; r < kRegions; ++r) {
        MBMD_REQUIRE(counts[r] >= 0 && counts[r] <= kMaxPartials, MBMD_ERR_SHAPE, "bad partial count");
        c.c[r] = counts[r];
    }
    {
        KernelTimer kt_("k_reduce_final", s);
        hipLaunchKernelGGL(k_reduce_final, zgrid(dim3(1)), dim3(dev::kReduceThreads), 0, s, partials, c, scal,
                           trace_slot, mode, flags, zarg());
        kt_.stop();
    }
    MBMD_LAUNCHED();
}

}  // namespace mbmd
