// C-ABI of the library (include/mbmd.h): problem state, preconditioner
// builds, and the schedules of the plain and preconditioned SPS iterations.
//
// Every device step of the iteration runs in the kernels of this library; the
// host only enqueues launches on the caller's stream.  Per-block FP64 partial
// sums are reduced by one final kernel that also forms the step size alpha on
// the device, so an iteration has no host synchronisation and can be captured
// in a hipGraph (batched form).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <memory>
#include <string>
#include <vector>

#include "internal.h"

struct mbmd_problem : public mbmd::Problem {};

// Problems whose launch parameters are identical form a class (same geometry,
// sizes and block layout): each kernel of their iteration runs once for the
// whole class, blockIdx.z selecting the slice (see ZBatch), so a batch of 24
// slices in three sizes issues the launches of three iterations per
// iteration.  The classes (and the problems left alone) are dealt round-robin
// onto library-owned streams (at most kBatchStreams) forked from and joined
// back into the caller's stream -- or, captured, onto parallel branches of one
// graph per iteration.  The per-slice offsets of every class live in the
// batch's device table zdev: [n][2] int64, a class's rows contiguous.
constexpr int kBatchStreams = 4;
struct mbmd_batch {
    std::vector<mbmd_problem*> probs;
    std::vector<std::vector<int>> units;   // classes (members in order) and lone problems
    std::vector<int> unit_first;           // first row of each unit in the offset table
    std::vector<int> lane;                 // branch stream of each unit
    int n_lanes = 0;
    bool shared = true;                    // shared launches within classes (else one unit per problem)
    long long* zdev = nullptr;             // device offset table [n][2]
    std::vector<long long> zhost;          // its host copy (kept alive for the asynchronous upload)
    std::vector<float*> zx;                // images the table was filled for
    std::vector<int> zversions;            // each problem's launch_version when the units were formed
    int zprecond = -1;                     // preconditioner the units were formed for
    bool owns_z = false;
    std::vector<float*> xs;
    std::vector<int> versions;             // each problem's launch_version when captured
    int precond = -1;
    hipGraph_t graph[2] = {nullptr, nullptr};
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    bool captured = false;
    hipStream_t stream = nullptr;          // caller stream the graphs were last launched on
    hipStream_t capture = nullptr;         // library-owned stream used only for capture
    hipStream_t branch[kBatchStreams] = {};
    hipEvent_t fork = nullptr;
    hipEvent_t join[kBatchStreams] = {};
};

namespace mbmd {

namespace {
thread_local std::string g_last_error;
constexpr int kTraceCap = 4096;
constexpr double kM0Floor = 1e-6;
constexpr double kEpsFourier = 1e-2;
constexpr double kEpsHaar = 1e-2;
}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

void Arena::reserve(size_t bytes) {
    MBMD_HIP(hipMalloc(&base, bytes));
    size = bytes;
    used = 0;
    owned = true;
}

void Arena::adopt(void* mem, size_t bytes) {
    MBMD_REQUIRE((reinterpret_cast<uintptr_t>(mem) & 255) == 0, MBMD_ERR_ARG, "workspace must be 256-byte aligned");
    base = static_cast<char*>(mem);
    size = bytes;
    used = 0;
    owned = false;
}

void Arena::release() {
    if (base && owned) (void)hipFree(base);
    base = nullptr;
    size = used = 0;
    owned = false;
}

namespace {

template <class F>
int guarded(F&& f) {
    (void)hipGetLastError();   // do not attribute an earlier, unrelated failure to this call
    try {
        f();
        return MBMD_OK;
    } catch (const Error& e) {
        set_error(e.msg);
        return e.status;
    } catch (const std::exception& e) {
        set_error(e.what());
        return MBMD_ERR_HIP;
    } catch (...) {
        set_error("unknown error");
        return MBMD_ERR_HIP;
    }
}

bool is_pow2(int n) { return n >= 2 && (n & (n - 1)) == 0; }

RayArgs ray_args(const Problem& P) {
    return RayArgs{P.ni, P.K, P.E, P.C, P.Q, P.S, P.rowS, P.Qsum, P.y, P.w, P.identity ? nullptr : P.gammaA,
                   P.blur.h ? P.wb : P.w, P.blur, P.btmp0, P.btmp1};
}

PenaltyArgs pen_args(const Problem& P) {
    return PenaltyArgs{P.K, P.nx, P.ny, P.pen_kind, P.beta_d, (float)P.delta};
}

void project(Problem& P, const float* x, float* sino, int nmat, hipStream_t s) {
    if (P.identity) {
        MBMD_HIP(hipMemcpyAsync(sino, x, sizeof(float) * (size_t)nmat * P.ni, hipMemcpyDeviceToDevice, s));
        return;
    }
    launch_project(*P.geom, x, sino, nmat, s);
}

void backproject(Problem& P, const float* sino, float* img, int nch, hipStream_t s) {
    if (P.identity) {
        MBMD_HIP(hipMemcpyAsync(img, sino, sizeof(float) * (size_t)nch * P.nj, hipMemcpyDeviceToDevice, s));
        return;
    }
    launch_backproject(*P.geom, sino, img, nch, s);
}

// A^T sino with the column-sweep part left separate (see launch_backproject_parts).
const float* backproject_parts(Problem& P, const float* sino, float* img, int nch, hipStream_t s) {
    if (P.identity) {
        MBMD_HIP(hipMemcpyAsync(img, sino, sizeof(float) * (size_t)nch * P.nj, hipMemcpyDeviceToDevice, s));
        return nullptr;
    }
    return launch_backproject_parts(*P.geom, sino, img, nch, s);
}

double* region(Problem& P, int r) { return P.partials + (size_t)r * kMaxPartials; }

// The projection-domain blur's buffers, from arena A.
void carve_blur(Problem& P, Arena& A) {
    const size_t ni = P.ni, C = P.C, K = P.K;
    P.wb = A.take<float>(C * ni);
    P.J = A.take<float>(C * K * ni);
    P.btmp0 = A.take<float>(C * ni);
    P.btmp1 = A.take<float>(C * ni);
}

// Back projection channels a problem's geometry is sized for.
int problem_back_ch(const Problem& P) { return std::max(P.npk, 2 * P.K); }

// Sizes every buffer; called twice (sizing pass with a null arena base, then for real).
void carve(Problem& P) {
    Arena& A = P.arena;
    const size_t nj = P.nj, ni = P.ni, K = P.K, C = P.C, E = P.E, npk = P.npk;
    P.geom_mem = P.identity ? nullptr : A.take<char>(P.geom_bytes);
    P.Q = A.take<float>(E * K);
    P.S = A.take<float>(C * E);
    P.rowS = A.take<float>(C);
    P.Qsum = A.take<float>(E);
    P.beta_d = A.take<float>(K * K);
    P.y = A.take<float>(C * ni);
    P.w = A.take<float>(C * ni);
    P.gammaA = A.take<float>(ni);
    P.l = A.take<float>(K * ni);
    P.q = A.take<float>(K * ni);
    P.u = A.take<float>(2 * K * ni);         // u then v, contiguous for one fused back projection
    P.v = P.u ? P.u + K * ni : nullptr;
    P.r = A.take<float>(C * ni);
    const size_t tmp_ch = npk > 2 * K ? npk : 2 * K;
    P.sino_tmp = A.take<float>(tmp_ch * ni);
    P.W = A.take<float>(npk * ni);
    P.g_img = A.take<float>(2 * K * nj);     // g then d, contiguous
    P.d_img = P.g_img ? P.g_img + K * nj : nullptr;
    P.p_img = A.take<float>(K * nj);
    P.t_img = A.take<float>(npk > K ? npk * nj : K * nj);
    P.t2_img = A.take<float>(K * nj);
    P.dL_const = A.take<float>(K * nj);
    P.M0 = A.take<float>(npk * nj);
    if (!P.identity && is_pow2(P.nx) && is_pow2(P.ny)) {
        P.spec = A.take<float2>(K * nj);
        P.Linv = A.take<float>(npk * nj);
        P.tw_x = A.take<float2>(P.nx);
        P.tw_y = A.take<float2>(P.ny);
        if (P.nx == P.ny) {
            const int T = haar_tile(P.nx), nt = P.nx / T;
            P.coef = A.take<float>(K * nj);
            P.coarse = A.take<float>(K * (size_t)nt * nt);
            P.Kinv = A.take<float>(npk * nj);
            P.Dinv = A.take<float>(npk * nj);
        }
    }
    P.partials = A.take<double>((size_t)kRegions * kMaxPartials);
    P.scal = A.take<double>(kScalars);
    P.trace = A.take<double>(kTraceCap + 1);
    P.trace_cap = kTraceCap;
    P.flags = A.take<int>(4);
    if (P.ws_flags & MBMD_WORKSPACE_BLUR) carve_blur(P, A);
}

// Sizes of a problem from its descriptors (everything carve needs).
void size_problem(Problem& P, const mbmd_geometry& g, const mbmd_spectral& sp, int flags) {
    validate_geometry(g);
    MBMD_REQUIRE(sp.n_mat >= 1 && sp.n_mat <= kMaxMat && sp.n_chan >= 1 && sp.n_chan <= kMaxChan &&
                     sp.n_energy >= 1 && sp.n_energy <= kMaxEnergy,
                 MBMD_ERR_SHAPE, "spectral sizes out of range (n_mat<=4, n_chan<=8, n_energy<=256)");
    MBMD_REQUIRE((flags & ~MBMD_WORKSPACE_BLUR) == 0, MBMD_ERR_ARG, "unknown workspace flag");
    P.g = g;
    P.identity = g.kind == MBMD_GEOM_IDENTITY;
    P.K = sp.n_mat;
    P.E = sp.n_energy;
    P.C = sp.n_chan;
    P.npk = P.K * (P.K + 1) / 2;
    P.nx = g.nx;
    P.ny = g.ny;
    P.V = g.n_views;
    P.B = g.n_bins;
    P.nj = g.nx * g.ny;
    P.ni = g.n_views * g.n_bins;
    P.ws_flags = flags;
    MBMD_REQUIRE(P.ni <= 256 * kMaxPartials && P.nj <= 256 * kMaxPartials, MBMD_ERR_SHAPE,
                 "problem too large for the partial-sum buffer");
    P.geom_bytes = P.identity ? 0 : geometry_bytes(g, P.K, problem_back_ch(P));
}

// Bytes of the device state of a problem sized by size_problem.
size_t problem_bytes(Problem& P) {
    P.arena = Arena{};
    carve(P);                                     // sizing pass
    const size_t bytes = P.arena.used;
    P.arena = Arena{};
    return bytes;
}

// The data part of the Fisher information on line integrals in [K][ni] ->
// out [K][ni] (distinct buffers): W_i in_i per ray, or with a blur
// J^T B^T W B J in (J per ray, the blur coupling the bins of a view).
void fisher_sino_apply(Problem& P, const float* in, float* out, hipStream_t s) {
    if (P.blur.h == 0) {
        launch_fisher_mix(P.ni, P.K, P.W, in, out, s);
        return;
    }
    launch_jmix(P.ni, P.K, P.C, P.J, in, P.btmp0, false, s);
    launch_blur(P.blur, P.ni, P.C, P.btmp0, P.w, P.btmp1, false, s);
    launch_blur(P.blur, P.ni, P.C, P.btmp1, nullptr, P.btmp0, true, s);
    launch_jmix(P.ni, P.K, P.C, P.J, P.btmp0, out, true, s);
}

// r = M0 H M0 v (or H v when M0 is NULL), H = A^T F_data A + beta Gamma (quadratic).
void hessian_apply(Problem& P, const float* v, float* out, const float* M0, hipStream_t s) {
    const float* src = v;
    if (M0) {
        launch_block_apply(P.nj, P.K, M0, v, P.p_img, 1.0f, s);
        src = P.p_img;
    }
    project(P, src, P.q, P.K, s);
    fisher_sino_apply(P, P.q, P.sino_tmp, s);
    backproject(P, P.sino_tmp, out, P.K, s);
    if (P.has_penalty) launch_penalty_hess_add(pen_args(P), src, out, s);
    if (M0) launch_block_apply(P.nj, P.K, M0, out, out, 1.0f, s);
}

// The Fisher weights W (from the data, or at reference line integrals lref) and
// M0: modified, M0_j = Htilde_j^-1/2 from the material columns; else M0 = I.
// state (see Problem::m0_state) records what they are; a new state, or any
// rebuild from a reference image, voids the preconditioners built on the old
// ones.
void build_fisher_m0(Problem& P, int state, const float* lref, bool modified, hipStream_t s) {
    launch_fisher(ray_args(P), P.W, s, lref, P.blur.h ? P.J : nullptr);
    if (!modified) {
        launch_fill(P.npk * P.nj, P.M0, 0.0f, s);
        for (int k = 0; k < P.K; ++k) launch_fill(P.nj, P.M0 + (size_t)packed_index(k, k, P.K) * P.nj, 1.0f, s);
    } else if (P.blur.h) {
        // Column k of Htilde = A^T F_data (gamma_A e_k), one material column at a
        // time.  The blur makes the off-diagonal blocks of F non-symmetric across
        // pixels, so their row sums (column k) and column sums (column k2)
        // differ: keep the symmetric part, as the eigen-solve does.
        launch_fill(P.npk * P.nj, P.t_img, 0.0f, s);
        for (int k = 0; k < P.K; ++k) {
            launch_fill(P.K * P.ni, P.q, 0.0f, s);
            launch_scale_copy(P.ni, P.gammaA, P.q + (size_t)k * P.ni, 1.0f, s);
            fisher_sino_apply(P, P.q, P.sino_tmp, s);
            backproject(P, P.sino_tmp, P.g_img, P.K, s);
            launch_block_add_column(P.nj, P.K, k, P.g_img, P.t_img, s);
        }
        launch_block_invsqrt(P.nj, P.K, P.t_img, P.M0, -0.5, kM0Floor, nullptr, 0.0, P.flags + 1, s);
    } else {
        // Htilde_j = column blocks of (F + R) 1_k = A^T (gamma_A W_kk')  (Gamma 1 = 0)
        if (P.identity) {
            launch_scale_copy(P.npk * P.ni, P.W, P.t_img, 1.0f, s);
        } else {
            launch_scale_by_vec(P.ni, P.npk, P.W, P.gammaA, P.sino_tmp, s);
            backproject(P, P.sino_tmp, P.t_img, P.npk, s);
        }
        launch_block_invsqrt(P.nj, P.K, P.t_img, P.M0, -0.5, kM0Floor, nullptr, 0.0, P.flags + 1, s);
    }
    for (int k = 0; k < kPreconds; ++k) P.built[k] = 0;
    P.m0_state = state;
}

// The data-based, modified weights and M0 (built once).
void ensure_fisher_m0(Problem& P, hipStream_t s) {
    if (P.m0_state != 1) build_fisher_m0(P, 1, nullptr, true, s);
}

void finish_filter(Problem& P, const float* blocks, float* out, double eps, hipStream_t s) {
    double* lmax = P.scal + S_LMAX;
    launch_fill_double(1, lmax, -1e300, s);
    launch_block_lmax(P.nj, P.K, blocks, lmax, s);
    launch_block_invsqrt(P.nj, P.K, blocks, out, -1.0, 0.0, lmax, eps, P.flags + 2, s);
}

void build_fourier(Problem& P, hipStream_t s) {
    MBMD_REQUIRE(P.spec != nullptr, MBMD_ERR_SHAPE, "the Fourier preconditioner needs power-of-two image sizes");
    const int jy = P.ny / 2, jx = P.nx / 2;
    float* blocks = P.t_img;                                // [npk][nj], zeroed
    launch_fill(P.npk * P.nj, blocks, 0.0f, s);
    for (int k = 0; k < P.K; ++k) {
        launch_fill(P.K * P.nj, P.t2_img, 0.0f, s);
        launch_fill(1, P.t2_img + (size_t)k * P.nj + (size_t)jy * P.nx + jx, 1.0f, s);
        hessian_apply(P, P.t2_img, P.g_img, P.M0, s);       // r_k = M0 H M0 delta_k
        launch_fft2_forward(P.K, P.nx, P.ny, P.g_img, nullptr, jy, jx, P.spec, P.tw_x, P.tw_y, s);
        launch_spectrum_real_to_blocks(P.K, P.nj, k, P.spec, blocks, s);
    }
    finish_filter(P, blocks, P.Linv, kEpsFourier, s);
}

void build_haar(Problem& P, hipStream_t s) {
    MBMD_REQUIRE(P.coef != nullptr, MBMD_ERR_SHAPE, "the Haar preconditioner needs a square power-of-two image");
    const int n = P.nx;
    // Delta x = U^T 1 (one material), kept in d_img
    launch_fill(P.nj, P.coef, 1.0f, s);
    launch_haar_inverse(1, n, P.coef, P.coarse, nullptr, P.d_img, 1.0f, s);
    float* blocks = P.t_img;
    launch_fill(P.npk * P.nj, blocks, 0.0f, s);
    for (int k = 0; k < P.K; ++k) {
        launch_fill(P.K * P.nj, P.t2_img, 0.0f, s);
        launch_scale_copy(P.nj, P.d_img, P.t2_img + (size_t)k * P.nj, 1.0f, s);
        hessian_apply(P, P.t2_img, P.g_img, P.M0, s);
        launch_haar_forward(P.K, n, P.g_img, nullptr, P.coef, P.coarse, s);
        launch_coef_blocks(P.K, n, k, P.coef, blocks, s);
    }
    finish_filter(P, blocks, P.Kinv, kEpsHaar, s);
}

// The same build with the Daubechies-4 transform (the other unitary wavelet).
void build_daub4(Problem& P, hipStream_t s) {
    MBMD_REQUIRE(P.coef != nullptr, MBMD_ERR_SHAPE, "the Daubechies preconditioner needs a square power-of-two image");
    const int n = P.nx;
    launch_fill(P.nj, P.coef, 1.0f, s);                     // Delta x = U^T 1 (one material), in d_img
    launch_d4_inverse(1, n, P.coef, nullptr, P.d_img, 1.0f, P.d_img, s);
    float* blocks = P.t_img;
    launch_fill(P.npk * P.nj, blocks, 0.0f, s);
    for (int k = 0; k < P.K; ++k) {
        launch_fill(P.K * P.nj, P.t2_img, 0.0f, s);
        launch_scale_copy(P.nj, P.d_img, P.t2_img + (size_t)k * P.nj, 1.0f, s);
        hessian_apply(P, P.t2_img, P.g_img, P.M0, s);
        launch_d4_forward(P.K, n, P.g_img, nullptr, P.coef, P.t2_img, s);
        launch_coef_blocks(P.K, n, k, P.coef, blocks, s);
    }
    finish_filter(P, blocks, P.Dinv, kEpsHaar, s);
}

// out = sign * M M^T g, with partials of g.out into `partials` when non-NULL.
int apply_direction(Problem& P, int kind, const float* g, float* out, float sign, double* partials,
                    hipStream_t s) {
    switch (kind) {
        case MBMD_PRECOND_BLOCKDIAG:
            launch_block_apply(P.nj, P.K, P.M0, g, P.t2_img, 1.0f, s);
            launch_block_apply(P.nj, P.K, P.M0, P.t2_img, out, sign, s);
            return partials ? launch_dot(P.K * P.nj, g, out, partials, s) : 0;
        case MBMD_PRECOND_FOURIER:
            return launch_fourier_apply(P.K, P.nx, P.ny, g, P.M0, P.Linv, P.spec, P.tw_x, P.tw_y, out, sign, g,
                                        partials, s);
        case MBMD_PRECOND_HAAR:
            return launch_haar_apply(P.K, P.nx, g, P.M0, P.Kinv, P.coef, P.coarse, out, sign, g, partials, s);
        case MBMD_PRECOND_DAUB4:
            return launch_d4_apply(P.K, P.nx, g, P.M0, P.Dinv, P.coef, out, sign, g, partials, s);
        default:
            launch_scale_copy(P.K * P.nj, g, out, sign, s);
            return partials ? launch_dot(P.K * P.nj, g, out, partials, s) : 0;
    }
}

// One energy and channel without a blur: the SPS curvature does not depend on x.
bool single_energy(const Problem& P) { return P.E == 1 && P.C == 1 && P.blur.h == 0; }

void ensure_dL_const(Problem& P, hipStream_t s) {
    if (P.dL_valid || !single_energy(P)) return;
    // c does not depend on x for one energy: evaluate at any line integrals
    launch_fill(P.K * P.ni, P.l, 0.0f, s);
    launch_ray_grad(ray_args(P), P.l, P.u, P.v, nullptr, nullptr, s);
    backproject(P, P.v, P.dL_const, P.K, s);
    P.dL_valid = 1;
}

// Phi(x) into *slot (device), recomputing A x.
void objective_at(Problem& P, const float* x, double* slot, hipStream_t s) {
    int counts[kRegions] = {0};
    project(P, x, P.l, P.K, s);
    counts[R_PHI_L] = launch_ray_grad(ray_args(P), P.l, P.u, nullptr, nullptr, region(P, R_PHI_L), s);
    counts[R_PHI_R] = launch_penalty_grad(pen_args(P), x, P.t2_img, nullptr, P.t2_img, nullptr,
                                          region(P, R_PHI_R), s);
    launch_reduce_final(P.partials, counts, P.scal, slot, RED_MONOTONE, P.flags, s);
}

// One plain SPS iteration: x <- x - (g + dR)/(d + d_R).
void plain_iteration(Problem& P, float* x, double* trace_slot, hipStream_t s) {
    int counts[kRegions] = {0};
    const bool cconst = single_energy(P);
    project(P, x, P.l, P.K, s);
    counts[R_PHI_L] = launch_ray_grad(ray_args(P), P.l, P.u, cconst ? nullptr : P.v, nullptr,
                                      region(P, R_PHI_L), s);
    backproject(P, P.u, P.g_img, cconst ? P.K : 2 * P.K, s);
    counts[R_PHI_R] = launch_penalty_grad(pen_args(P), x, P.g_img, cconst ? P.dL_const : P.d_img, P.g_img,
                                          P.d_img, region(P, R_PHI_R), s);
    launch_plain_update(P.K * P.nj, x, P.g_img, P.d_img, s);
    launch_reduce_final(P.partials, counts, P.scal, trace_slot, RED_MONOTONE, P.flags, s);
}

// One preconditioned iteration.  On entry l = A x up to the step the previous
// iteration left pending in alpha (zero when none), which this one applies first;
// on exit its own step is pending.
void precond_iteration(Problem& P, float* x, int kind, double* trace_slot, hipStream_t s) {
    int counts[kRegions] = {0};
    // the previous iteration's step (x += alpha p, l += alpha q) is applied by this launch
    const StepUpdate up{P.scal + S_ALPHA, P.q, P.l, x, P.p_img, P.K * P.nj};
    // Once the back projector's shape is chosen for K channels, the gradient
    // launch of a single-energy problem writes its detector rows itself (the
    // same bits as storing u and running the detector prefix), and only the
    // back projection kernel follows.  With many energies per ray the fused
    // launch, one workgroup per view, has too few threads for the ray work.
    const float* part = nullptr;                                       // summed by the penalty pass
    const bool fuse = !P.identity && P.E == 1 && P.blur.h == 0 && P.fuse_rows && !zarg();
    const BackRows br = fuse ? back_rows(*P.geom, P.g_img, P.K) : BackRows{};
    const int n_rows = br.ok ? launch_ray_grad_rows(ray_args(P), P.l, P.r, region(P, R_PHI_L), s, up, br) : -1;
    if (n_rows >= 0) {
        counts[R_PHI_L] = n_rows;
        part = launch_back_kernel(*P.geom, P.g_img, P.K, s);
    } else {
        counts[R_PHI_L] = launch_ray_grad(ray_args(P), P.l, P.u, nullptr, P.r, region(P, R_PHI_L), s, &up);
        part = backproject_parts(P, P.u, P.g_img, P.K, s);
    }
    counts[R_PHI_R] = launch_penalty_grad(pen_args(P), x, P.g_img, nullptr, P.g_img, nullptr,
                                          region(P, R_PHI_R), s, part);
    counts[R_GP] = apply_direction(P, kind, P.g_img, P.p_img, -1.0f, region(P, R_GP), s);
    project(P, P.p_img, P.q, P.K, s);
    const PenaltyArgs pa = pen_args(P);
    launch_curvature(ray_args(P), P.l, P.r, P.q, P.has_penalty ? &pa : nullptr, x, P.p_img, P.partials, counts, s);
    launch_reduce_final(P.partials, counts, P.scal, trace_slot, RED_STEP | RED_MONOTONE, P.flags, s);   // alpha: applied next
}

// Applies a pending preconditioned step (x += alpha p, l += alpha q) and clears
// alpha, which makes the next iteration's application a no-op; every run of
// preconditioned iterations ends with this, and so does every refresh of l.
void flush_step(Problem& P, float* x, hipStream_t s) {
    launch_axpy2_alpha(P.K * P.nj, x, P.p_img, P.K * P.ni, P.l, P.q, P.scal + S_ALPHA, s);
    launch_fill_double(1, P.scal + S_ALPHA, 0.0, s);
}

void check_precond_ready(Problem& P, int precond) {
    MBMD_REQUIRE(precond >= 0 && precond < kPreconds, MBMD_ERR_ARG, "unknown preconditioner");
    if (P.identity) {
        MBMD_REQUIRE(!P.has_penalty, MBMD_ERR_UNSUPPORTED,
                     "identity geometry iterations need a zero penalty (the problem separates by ray)");
        MBMD_REQUIRE(precond == MBMD_PRECOND_NONE || precond == MBMD_PRECOND_BLOCKDIAG, MBMD_ERR_UNSUPPORTED,
                     "identity geometry supports the plain and block-diagonal iterations");
    }
    if (precond != MBMD_PRECOND_NONE) MBMD_REQUIRE(P.built[precond], MBMD_ERR_NOT_BUILT, "preconditioner not built");
}

// Waits for s, returns the numeric flags raised since they were last read
// (in *out when not NULL) and clears them; throws MBMD_ERR_NUMERIC when one of
// the error bits is among them.
void read_flags(Problem& P, hipStream_t s, int* out = nullptr) {
    int f[4];
    MBMD_HIP(hipMemcpyAsync(f, P.flags, sizeof(f), hipMemcpyDeviceToHost, s));
    MBMD_HIP(hipStreamSynchronize(s));
    if (out) *out = f[0];
    if (f[0]) {
        launch_fill(1, reinterpret_cast<float*>(P.flags), 0.0f, s);
        MBMD_HIP(hipStreamSynchronize(s));
    }
    if (f[0] & kFlagErrors) {
        std::string what;
        if (f[0] & MBMD_FLAG_NONFINITE) what += " non-finite objective or step size;";
        if (f[0] & MBMD_FLAG_NO_CURVATURE) what += " no positive curvature along a nonzero direction;";
        if (f[0] & MBMD_FLAG_ASCENT) what += " the direction was not a descent direction (g^T p > 0);";
        throw Error{MBMD_ERR_NUMERIC, "numeric failure:" + what};
    }
}

// Starts a run of iterations: the first objective of the run is checked against nothing.
void begin_run(Problem& P, hipStream_t s) {
    launch_fill_double(1, P.scal + S_PHI_PREV, std::nan(""), s);
}

void identity_iterate(Problem& P, float* x, int precond, int n_iter, double* trace_host, hipStream_t s) {
    const int nb = (P.ni + 255) / 256;
    const int total_slots = kRegions * kMaxPartials;
    // A chunk of n iterations writes n + 1 rows of nb partials and, traced, n + 1
    // trace slots (the device trace holds trace_cap + 1).
    int chunk_max = total_slots / nb - 1;
    if (trace_host) chunk_max = std::min(chunk_max, P.trace_cap);
    MBMD_REQUIRE(chunk_max >= 1, MBMD_ERR_SHAPE, "too many rays for the partial-sum buffer");
    int done = 0;
    do {
        const int n = std::min(chunk_max, n_iter - done);
        launch_identity_iterate(ray_args(P), x, P.M0, precond, n, P.partials, nb, s);
        if (trace_host) {
            for (int it = 0; it <= n; ++it) {
                if (it == n && done + n < n_iter) break;      // next chunk starts from this point
                int counts[kRegions] = {0};
                counts[R_PHI_L] = nb;
                launch_reduce_final(P.partials + (size_t)it * nb, counts, P.scal, P.trace + it, RED_MONOTONE,
                                    P.flags, s);
            }
            const int nvals = (done + n < n_iter) ? n : n + 1;
            MBMD_HIP(hipMemcpyAsync(trace_host + done, P.trace, sizeof(double) * nvals, hipMemcpyDeviceToHost, s));
            MBMD_HIP(hipStreamSynchronize(s));
        } else if (done + n == n_iter) {
            // the objective after the last iteration, for the numeric flags only
            int counts[kRegions] = {0};
            counts[R_PHI_L] = nb;
            launch_reduce_final(P.partials + (size_t)n * nb, counts, P.scal, nullptr, RED_MONOTONE, P.flags, s);
        }
        done += n;
    } while (done < n_iter);
}

void sps_run(Problem& P, float* x, int precond, int n_iter, double* trace_host, hipStream_t s) {
    check_precond_ready(P, precond);
    P.last_stream = s;
    begin_run(P, s);
    if (P.identity) {
        identity_iterate(P, x, precond, n_iter, trace_host, s);
        if (trace_host) read_flags(P, s);
        return;
    }
    if (precond == MBMD_PRECOND_NONE) ensure_dL_const(P, s);
    int base = 0;   // trace index of slot 0 of the device trace buffer
    for (int n = 0; n < n_iter; ++n) {
        if (trace_host && n - base == P.trace_cap) {
            MBMD_HIP(hipMemcpyAsync(trace_host + base, P.trace, sizeof(double) * P.trace_cap,
                                    hipMemcpyDeviceToHost, s));
            MBMD_HIP(hipStreamSynchronize(s));
            base = n;
        }
        double* slot = trace_host ? P.trace + (n - base) : nullptr;
        if (precond == MBMD_PRECOND_NONE) {
            plain_iteration(P, x, slot, s);
        } else {
            if (n % kRefreshEvery == 0) {
                flush_step(P, x, s);
                project(P, x, P.l, P.K, s);
            }
            precond_iteration(P, x, precond, slot, s);
        }
    }
    if (precond != MBMD_PRECOND_NONE) flush_step(P, x, s);
    if (trace_host) {
        if (n_iter - base == P.trace_cap) {
            MBMD_HIP(hipMemcpyAsync(trace_host + base, P.trace, sizeof(double) * P.trace_cap,
                                    hipMemcpyDeviceToHost, s));
            MBMD_HIP(hipStreamSynchronize(s));
            base = n_iter;
        }
        objective_at(P, x, P.trace + (n_iter - base), s);
        MBMD_HIP(hipMemcpyAsync(trace_host + base, P.trace, sizeof(double) * (n_iter - base + 1),
                                hipMemcpyDeviceToHost, s));
        read_flags(P, s);
    }
}

// Sets the batched-launch setting for the launches of one class (see ZBatch)
// and clears it on leaving, also on an error.
struct ZScope {
    ZScope(const long long* zd, int nz, const void* x0) {
        ZBatch& z = zbatch();
        z.zd = zd;
        z.nz = nz;
        z.x0 = x0;
    }
    ~ZScope() { zbatch() = ZBatch{}; }
    ZScope(const ZScope&) = delete;
    ZScope& operator=(const ZScope&) = delete;
};

// Byte offset of a device buffer in the problem's block; -1 for none, and a
// value no other problem shares when the buffer lies outside the block (blur
// buffers grown after creation in a library block sized without their room).
long long block_offset(const Problem& P, const void* p) {
    if (!p) return -1;
    const uintptr_t b = reinterpret_cast<uintptr_t>(P.arena.base), a = reinterpret_cast<uintptr_t>(p);
    if (a >= b && a < b + P.arena.size) return (long long)(a - b);
    return -2 - (long long)a;
}

// Problems whose iterations can share launches: every host-side launch
// parameter equal (geometry, sizes, penalty kind and delta, blur taps) and
// every device buffer at the same offset of the problem's block, so that one
// byte offset per member moves all of the first member's pointers onto it.
std::string batch_class_key(const Problem& P) {
    const mbmd_geometry& g = P.g;
    std::vector<double> f = {(double)g.kind, (double)g.nx, (double)g.ny, g.dx, g.dy, (double)g.n_views, g.theta0,
                             g.dtheta, (double)g.n_bins, g.du, g.u_offset, g.dso, g.dsd, (double)P.K, (double)P.E,
                             (double)P.C, (double)P.pen_kind, (double)P.has_penalty, (double)(float)P.delta,
                             (double)P.ws_flags, (double)P.fuse_rows, (double)P.blur.h, (double)P.blur.B};
    for (int c = 0; c < kMaxChan; ++c)
        for (int t = 0; t < 2 * P.blur.h + 1; ++t) f.push_back((double)P.blur.taps[c][t]);
    const void* bufs[] = {P.geom_mem, P.Q,      P.S,      P.rowS,  P.Qsum,   P.beta_d, P.y,     P.w,
                          P.gammaA,   P.l,      P.q,      P.u,     P.v,      P.r,      P.sino_tmp, P.g_img,
                          P.d_img,    P.p_img,  P.t_img,  P.t2_img, P.dL_const, P.M0,  P.Linv,  P.Kinv,
                          P.Dinv,     P.W,      P.wb,     P.J,     P.btmp0,  P.btmp1,  P.spec,  P.tw_x,
                          P.tw_y,     P.coef,   P.coarse, P.partials, P.scal, P.flags};
    std::string key(reinterpret_cast<const char*>(f.data()), sizeof(double) * f.size());
    for (const void* b : bufs) {
        const long long o = block_offset(P, b);
        key.append(reinterpret_cast<const char*>(&o), sizeof(o));
    }
    return key;
}

// Preconditioners whose apply kernels have the batched form (all of them).
bool shares_launches(int precond) {
    return precond >= MBMD_PRECOND_NONE && precond < kPreconds;
}

}  // namespace
}  // namespace mbmd

using namespace mbmd;

extern "C" {

int mbmd_version(void) { return 1; }

const char* mbmd_last_error(void) { return g_last_error.c_str(); }

const char* mbmd_status_string(int status) {
    switch (status) {
        case MBMD_OK: return "ok";
        case MBMD_ERR_ARG: return "invalid argument";
        case MBMD_ERR_SHAPE: return "unsupported shape";
        case MBMD_ERR_HIP: return "HIP runtime error";
        case MBMD_ERR_NOT_BUILT: return "preconditioner not built";
        case MBMD_ERR_NUMERIC: return "non-finite objective or step";
        case MBMD_ERR_UNSUPPORTED: return "unsupported option";
        default: return "unknown status";
    }
}

int mbmd_cache_clear(void) {
    return guarded([&] { clear_geometry_cache(); });
}

int mbmd_project(const mbmd_geometry* geom, const float* x_dev, float* sino_dev, int n_mat, void* stream) {
    return guarded([&] {
        MBMD_REQUIRE(geom && x_dev && sino_dev, MBMD_ERR_ARG, "NULL argument");
        validate_geometry(*geom);
        MBMD_REQUIRE(n_mat >= 1 && n_mat <= kMaxMat, MBMD_ERR_SHAPE, "n_mat must be in 1..4");
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (geom->kind == MBMD_GEOM_IDENTITY) {
            MBMD_HIP(hipMemcpyAsync(sino_dev, x_dev, sizeof(float) * (size_t)n_mat * geom->nx * geom->ny,
                                    hipMemcpyDeviceToDevice, s));
            return;
        }
        launch_project(cached_geometry(*geom, kMaxMat, kMaxBackCh, s), x_dev, sino_dev, n_mat, s);
    });
}

int mbmd_backproject(const mbmd_geometry* geom, const float* sino_dev, float* x_dev, int n_ch, void* stream) {
    return guarded([&] {
        MBMD_REQUIRE(geom && x_dev && sino_dev, MBMD_ERR_ARG, "NULL argument");
        validate_geometry(*geom);
        MBMD_REQUIRE(n_ch >= 1 && n_ch <= kMaxBackCh, MBMD_ERR_SHAPE, "n_ch must be in 1..10");
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (geom->kind == MBMD_GEOM_IDENTITY) {
            MBMD_HIP(hipMemcpyAsync(x_dev, sino_dev, sizeof(float) * (size_t)n_ch * geom->nx * geom->ny,
                                    hipMemcpyDeviceToDevice, s));
            return;
        }
        launch_backproject(cached_geometry(*geom, kMaxMat, kMaxBackCh, s), sino_dev, x_dev, n_ch, s);
    });
}

int mbmd_projector_nnz(const mbmd_geometry* geom, long long* nnz_host, void* stream) {
    return guarded([&] {
        MBMD_REQUIRE(geom && nnz_host, MBMD_ERR_ARG, "NULL argument");
        validate_geometry(*geom);
        if (geom->kind == MBMD_GEOM_IDENTITY) {
            *nnz_host = (long long)geom->nx * geom->ny;
            return;
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        *nnz_host = count_nonzeros(cached_geometry(*geom, kMaxMat, kMaxBackCh, s), s);
    });
}

int mbmd_workspace_bytes(const mbmd_geometry* geom, const mbmd_spectral* sp, int flags, size_t* bytes) {
    return guarded([&] {
        MBMD_REQUIRE(geom && sp && bytes, MBMD_ERR_ARG, "NULL argument");
        Problem P;
        size_problem(P, *geom, *sp, flags);
        *bytes = problem_bytes(P);
    });
}

int mbmd_problem_create(const mbmd_geometry* geom, const mbmd_spectral* sp, const mbmd_penalty* pen,
                        const float* y_dev, const float* w_dev, void* workspace_dev, size_t workspace_bytes,
                        int flags, void* stream, mbmd_problem** out) {
    return guarded([&] {
        MBMD_REQUIRE(geom && sp && pen && y_dev && out, MBMD_ERR_ARG, "NULL argument");
        *out = nullptr;
        MBMD_REQUIRE(sp->Q_host && sp->S_host, MBMD_ERR_ARG, "NULL spectral table");
        MBMD_REQUIRE(pen->kind == MBMD_PENALTY_QUADRATIC || pen->kind == MBMD_PENALTY_HUBER, MBMD_ERR_ARG,
                     "unknown penalty kind");
        std::unique_ptr<mbmd_problem> P(new mbmd_problem());
        hipStream_t s = static_cast<hipStream_t>(stream);
        size_problem(*P, *geom, *sp, flags);
        const char* fr = std::getenv("MBMD_FUSE_ROWS");
        P->fuse_rows = !(fr && fr[0] == '0');
        P->pen_kind = pen->kind;
        P->delta = pen->delta;
        for (int i = 0; i < P->K * P->K; ++i) P->beta[i] = pen->beta_host ? pen->beta_host[i] : 0.0;
        for (int i = 0; i < P->K; ++i)
            for (int j = 0; j < P->K; ++j)
                MBMD_REQUIRE(P->beta[i * P->K + j] == P->beta[j * P->K + i], MBMD_ERR_ARG, "beta must be symmetric");
        for (int i = 0; i < P->K * P->K; ++i) P->has_penalty |= P->beta[i] != 0.0;
        if (pen->kind == MBMD_PENALTY_HUBER)
            MBMD_REQUIRE(P->K == 1 && pen->delta > 0.0, MBMD_ERR_ARG, "Huber needs one material and delta > 0");
        GeomHost gh;
        if (!P->identity) build_geometry_host(*geom, gh);      // FP64 on the host, before any device work
        const size_t need = problem_bytes(*P);
        if (workspace_dev) {
            MBMD_REQUIRE(workspace_bytes >= need, MBMD_ERR_ARG,
                         "workspace smaller than mbmd_workspace_bytes reports");
            P->arena.adopt(workspace_dev, workspace_bytes);
        } else {
            P->arena.reserve(need);
        }
        carve(*P);
        if (!P->identity) {
            P->geom = new GeomTables();
            place_geometry(*geom, gh, *P->geom, P->geom_mem, P->K, problem_back_ch(*P), s);
        }
        // spectral model
        const int K = P->K, E = P->E, C = P->C;
        std::vector<float> Qf(E * K), Sf(C * E), rowS(C, 0.0f), Qsum(E, 0.0f), bf(K * K);
        for (int e = 0; e < E; ++e)
            for (int k = 0; k < K; ++k) {
                Qf[e * K + k] = (float)sp->Q_host[e * K + k];
                Qsum[e] += (float)sp->Q_host[e * K + k];
            }
        for (int c = 0; c < C; ++c) {
            double rs = 0.0;
            for (int e = 0; e < E; ++e) {
                Sf[c * E + e] = (float)sp->S_host[c * E + e];
                rs += sp->S_host[c * E + e];
            }
            rowS[c] = (float)rs;
        }
        for (int i = 0; i < K * K; ++i) bf[i] = (float)P->beta[i];
        MBMD_HIP(hipMemcpyAsync(P->Q, Qf.data(), sizeof(float) * Qf.size(), hipMemcpyHostToDevice, s));
        MBMD_HIP(hipMemcpyAsync(P->S, Sf.data(), sizeof(float) * Sf.size(), hipMemcpyHostToDevice, s));
        MBMD_HIP(hipMemcpyAsync(P->rowS, rowS.data(), sizeof(float) * C, hipMemcpyHostToDevice, s));
        MBMD_HIP(hipMemcpyAsync(P->Qsum, Qsum.data(), sizeof(float) * E, hipMemcpyHostToDevice, s));
        MBMD_HIP(hipMemcpyAsync(P->beta_d, bf.data(), sizeof(float) * K * K, hipMemcpyHostToDevice, s));
        MBMD_HIP(hipMemcpyAsync(P->y, y_dev, sizeof(float) * (size_t)C * P->ni, hipMemcpyDeviceToDevice, s));
        if (w_dev)
            MBMD_HIP(hipMemcpyAsync(P->w, w_dev, sizeof(float) * (size_t)C * P->ni, hipMemcpyDeviceToDevice, s));
        else
            launch_inv_var(C * P->ni, P->y, P->w, s);
        launch_fill(4, reinterpret_cast<float*>(P->flags), 0.0f, s);
        // no step pending: alpha = 0 (p and q finite)
        launch_fill_double(kScalars, P->scal, 0.0, s);
        launch_fill(P->K * P->nj, P->p_img, 0.0f, s);
        launch_fill(P->K * P->ni, P->q, 0.0f, s);
        if (P->identity) {
            launch_fill(P->ni, P->gammaA, 1.0f, s);
        } else {
            launch_fill(P->nj, P->t_img, 1.0f, s);
            launch_project(*P->geom, P->t_img, P->gammaA, 1, s);
        }
        if (P->tw_x) {
            fill_twiddles(P->tw_x, P->nx, s);
            fill_twiddles(P->tw_y, P->ny, s);
        }
        MBMD_HIP(hipStreamSynchronize(s));        // the host tables and spectra go out of scope
        P->last_stream = s;
        *out = P.release();
    });
}

void mbmd_problem_destroy(mbmd_problem* prob) {
    if (!prob) return;
    (void)hipStreamSynchronize(prob->last_stream);
    prob->arena.release();
    prob->blur_arena.release();
    delete prob->geom;                 // its memory was part of the arena
    delete prob;
}

int mbmd_problem_check(mbmd_problem* prob, int* flags_host, void* stream) {
    return guarded([&] {
        MBMD_REQUIRE(prob != nullptr, MBMD_ERR_ARG, "NULL problem");
        hipStream_t s = static_cast<hipStream_t>(stream);
        prob->last_stream = s;
        read_flags(*prob, s, flags_host);
    });
}

int mbmd_problem_set_blur(mbmd_problem* prob, const float* taps_host, int half_width, void* stream) {
    return guarded([&] {
        MBMD_REQUIRE(prob != nullptr, MBMD_ERR_ARG, "NULL problem");
        Problem& P = *prob;
        static_assert(MBMD_MAX_BLUR_HALF == kMaxBlurHalf, "blur limit of the header and the kernels");
        MBMD_REQUIRE(half_width >= 0 && half_width <= kMaxBlurHalf, MBMD_ERR_ARG, "blur half width out of range");
        MBMD_REQUIRE(!P.identity || half_width == 0, MBMD_ERR_UNSUPPORTED, "no blur on the identity geometry");
        BlurArgs b;
        if (half_width > 0) {
            MBMD_REQUIRE(taps_host != nullptr, MBMD_ERR_ARG, "NULL blur taps");
            const int nt = 2 * half_width + 1;
            for (int c = 0; c < P.C; ++c)
                for (int t = 0; t < nt; ++t) {
                    const float v = taps_host[c * nt + t];
                    MBMD_REQUIRE(std::isfinite(v) && v >= 0.0f, MBMD_ERR_ARG, "blur taps must be finite and >= 0");
                    b.taps[c][t] = v;
                }
            b.h = half_width;
            b.B = P.B;
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        P.last_stream = s;
        if (b.h > 0 && P.wb == nullptr) {
            // sized without room for a blur: library memory may grow, a caller's workspace may not
            MBMD_REQUIRE(P.arena.owned, MBMD_ERR_UNSUPPORTED,
                         "the problem's workspace was sized without MBMD_WORKSPACE_BLUR");
            Arena& A = P.blur_arena;
            carve_blur(P, A);                               // sizing pass
            A.reserve(A.used);
            carve_blur(P, A);
        }
        if (b.h > 0) {                                      // wb = B^T (w B 1)
            launch_fill(P.C * P.ni, P.btmp0, 1.0f, s);
            launch_blur(b, P.ni, P.C, P.btmp0, P.w, P.btmp1, false, s);
            launch_blur(b, P.ni, P.C, P.btmp1, nullptr, P.wb, true, s);
        }
        P.blur = b;
        ++P.launch_version;                                 // a captured batch iteration is stale
        P.dL_valid = 0;
        P.m0_state = 0;
        for (int k = 0; k < kPreconds; ++k) P.built[k] = 0;
    });
}

int mbmd_precond_build_ex(mbmd_problem* prob, int kind, int flags, const float* x_ref_dev, void* stream) {
    return guarded([&] {
        MBMD_REQUIRE(prob, MBMD_ERR_ARG, "NULL problem");
        MBMD_REQUIRE(kind >= 0 && kind < kPreconds, MBMD_ERR_ARG, "unknown preconditioner");
        MBMD_REQUIRE((flags & ~MBMD_PRECOND_UNMODIFIED) == 0, MBMD_ERR_ARG, "unknown preconditioner build flag");
        hipStream_t s = static_cast<hipStream_t>(stream);
        prob->last_stream = s;
        if (kind == MBMD_PRECOND_NONE) return;
        if (prob->identity)
            MBMD_REQUIRE(kind == MBMD_PRECOND_BLOCKDIAG, MBMD_ERR_UNSUPPORTED,
                         "identity geometry supports the block-diagonal preconditioner only");
        if (kind == MBMD_PRECOND_FOURIER)
            MBMD_REQUIRE(prob->spec != nullptr, MBMD_ERR_SHAPE, "the Fourier preconditioner needs power-of-two sizes");
        if (kind == MBMD_PRECOND_HAAR || kind == MBMD_PRECOND_DAUB4)
            MBMD_REQUIRE(prob->coef != nullptr, MBMD_ERR_SHAPE, "the wavelet preconditioners need a square power-of-two image");
        if (flags == 0 && !x_ref_dev) {
            ensure_fisher_m0(*prob, s);
        } else {
            // reference line integrals into q, which holds nothing between runs
            // (every run ends with its pending step applied)
            const float* lref = nullptr;
            if (x_ref_dev) {
                project(*prob, x_ref_dev, prob->q, prob->K, s);
                lref = prob->q;
            }
            build_fisher_m0(*prob, 2, lref, !(flags & MBMD_PRECOND_UNMODIFIED), s);
        }
        if (kind == MBMD_PRECOND_FOURIER) build_fourier(*prob, s);
        if (kind == MBMD_PRECOND_HAAR) build_haar(*prob, s);
        if (kind == MBMD_PRECOND_DAUB4) build_daub4(*prob, s);
        prob->built[kind] = 1;
    });
}

int mbmd_precond_build(mbmd_problem* prob, int kind, void* stream) {
    return mbmd_precond_build_ex(prob, kind, 0, nullptr, stream);
}

int mbmd_precond_apply(mbmd_problem* prob, int kind, const float* g_dev, float* out_dev, void* stream) {
    return guarded([&] {
        MBMD_REQUIRE(prob && g_dev && out_dev && g_dev != out_dev, MBMD_ERR_ARG, "bad argument");
        MBMD_REQUIRE(kind >= 0 && kind < kPreconds, MBMD_ERR_ARG, "unknown preconditioner");
        if (kind != MBMD_PRECOND_NONE) MBMD_REQUIRE(prob->built[kind], MBMD_ERR_NOT_BUILT, "preconditioner not built");
        hipStream_t s = static_cast<hipStream_t>(stream);
        prob->last_stream = s;
        apply_direction(*prob, kind, g_dev, out_dev, 1.0f, nullptr, s);
    });
}

int mbmd_gradient(mbmd_problem* prob, const float* x_dev, float* grad_dev, float* curv_dev, double* objective_host,
                  void* stream) {
    return guarded([&] {
        MBMD_REQUIRE(prob && x_dev && grad_dev, MBMD_ERR_ARG, "NULL argument");
        Problem& P = *prob;
        hipStream_t s = static_cast<hipStream_t>(stream);
        P.last_stream = s;
        int counts[kRegions] = {0};
        project(P, x_dev, P.l, P.K, s);
        counts[R_PHI_L] = launch_ray_grad(ray_args(P), P.l, P.u, curv_dev ? P.v : nullptr, nullptr,
                                          region(P, R_PHI_L), s);
        backproject(P, P.u, P.g_img, curv_dev ? 2 * P.K : P.K, s);
        counts[R_PHI_R] = launch_penalty_grad(pen_args(P), x_dev, P.g_img, curv_dev ? P.d_img : nullptr, grad_dev,
                                              curv_dev, region(P, R_PHI_R), s);
        if (objective_host) {
            launch_reduce_final(P.partials, counts, P.scal, nullptr, 0, P.flags, s);
            MBMD_HIP(hipMemcpyAsync(objective_host, P.scal + S_PHI, sizeof(double), hipMemcpyDeviceToHost, s));
            read_flags(P, s);
        }
    });
}

int mbmd_sps_step(mbmd_problem* prob, float* x_dev, int precond, int n_iter, double* trace_host, void* stream) {
    return guarded([&] {
        MBMD_REQUIRE(prob && x_dev && n_iter >= 0, MBMD_ERR_ARG, "bad argument");
        sps_run(*prob, x_dev, precond, n_iter, trace_host, static_cast<hipStream_t>(stream));
    });
}

int mbmd_forward(mbmd_problem* prob, const float* x_dev, float* ybar_dev, float* l_dev, void* stream) {
    return guarded([&] {
        MBMD_REQUIRE(prob && x_dev && ybar_dev, MBMD_ERR_ARG, "NULL argument");
        Problem& P = *prob;
        hipStream_t s = static_cast<hipStream_t>(stream);
        P.last_stream = s;
        float* l = l_dev ? l_dev : P.l;
        project(P, x_dev, l, P.K, s);
        launch_forward_model(ray_args(P), l, ybar_dev, s);
    });
}

int mbmd_forward_vjp(mbmd_problem* prob, const float* l_dev, const float* gbar_dev, float* dx_dev, void* stream) {
    return guarded([&] {
        MBMD_REQUIRE(prob && l_dev && gbar_dev && dx_dev, MBMD_ERR_ARG, "NULL argument");
        Problem& P = *prob;
        hipStream_t s = static_cast<hipStream_t>(stream);
        P.last_stream = s;
        launch_forward_vjp(ray_args(P), l_dev, gbar_dev, P.u, s);
        backproject(P, P.u, dx_dev, P.K, s);
    });
}

int mbmd_batch_workspace_bytes(mbmd_problem* const* probs, int n, size_t* bytes) {
    return guarded([&] {
        MBMD_REQUIRE(probs && n > 0 && bytes, MBMD_ERR_ARG, "bad argument");
        *bytes = ((size_t)16 * n + 255) & ~size_t(255);
    });
}

int mbmd_batch_create(mbmd_problem* const* probs, int n, void* workspace_dev, size_t workspace_bytes, int flags,
                      mbmd_batch** out) {
    return guarded([&] {
        MBMD_REQUIRE(probs && n > 0 && out, MBMD_ERR_ARG, "bad argument");
        MBMD_REQUIRE((flags & ~MBMD_BATCH_SEPARATE_LAUNCHES) == 0, MBMD_ERR_ARG, "unknown batch flag");
        *out = nullptr;
        std::unique_ptr<mbmd_batch> b(new mbmd_batch());
        for (int i = 0; i < n; ++i) {
            MBMD_REQUIRE(probs[i] != nullptr, MBMD_ERR_ARG, "NULL problem in batch");
            MBMD_REQUIRE(!probs[i]->identity, MBMD_ERR_UNSUPPORTED, "batches hold projector geometries");
            for (int k = 0; k < i; ++k) MBMD_REQUIRE(probs[k] != probs[i], MBMD_ERR_ARG, "a problem twice in a batch");
            b->probs.push_back(probs[i]);
        }
        b->shared = !(flags & MBMD_BATCH_SEPARATE_LAUNCHES);
        const size_t need = (size_t)16 * n;
        if (workspace_dev) {
            MBMD_REQUIRE(workspace_bytes >= need, MBMD_ERR_ARG, "batch workspace smaller than mbmd_batch_workspace_bytes");
            MBMD_REQUIRE((reinterpret_cast<uintptr_t>(workspace_dev) & 255) == 0, MBMD_ERR_ARG,
                         "workspace must be 256-byte aligned");
            b->zdev = static_cast<long long*>(workspace_dev);
        } else {
            MBMD_HIP(hipMalloc(reinterpret_cast<void**>(&b->zdev), need));
            b->owns_z = true;
        }
        b->zhost.assign((size_t)2 * n, 0);
        b->n_lanes = std::min(n, kBatchStreams);
        for (int i = 0; i < b->n_lanes; ++i) {
            MBMD_HIP(hipStreamCreateWithFlags(&b->branch[i], hipStreamNonBlocking));
            MBMD_HIP(hipEventCreateWithFlags(&b->join[i], hipEventDisableTiming));
        }
        MBMD_HIP(hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
        *out = b.release();
    });
}

void mbmd_batch_destroy(mbmd_batch* b) {
    if (!b) return;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (int i = 0; i < 2; ++i) {
        if (b->exec[i]) (void)hipGraphExecDestroy(b->exec[i]);
        if (b->graph[i]) (void)hipGraphDestroy(b->graph[i]);
    }
    if (b->capture) (void)hipStreamDestroy(b->capture);
    for (int i = 0; i < b->n_lanes; ++i) {
        if (b->branch[i]) {
            (void)hipStreamSynchronize(b->branch[i]);
            (void)hipStreamDestroy(b->branch[i]);
        }
        if (b->join[i]) (void)hipEventDestroy(b->join[i]);
    }
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->owns_z && b->zdev) {
        (void)hipDeviceSynchronize();
        (void)hipFree(b->zdev);
    }
    delete b;
}

int mbmd_batch_sps_step(mbmd_batch* b, float* const* x_dev, int precond, int n_iter, int use_graph, void* stream) {
    return guarded([&] {
        MBMD_REQUIRE(b && x_dev && n_iter >= 0, MBMD_ERR_ARG, "bad argument");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const size_t n = b->probs.size();
        for (size_t i = 0; i < n; ++i) {
            MBMD_REQUIRE(x_dev[i] != nullptr, MBMD_ERR_ARG, "NULL image in batch");
            check_precond_ready(*b->probs[i], precond);
            b->probs[i]->last_stream = s;
            begin_run(*b->probs[i], s);
            if (precond == MBMD_PRECOND_NONE) ensure_dL_const(*b->probs[i], s);
        }
        // Units: classes of problems that share launches (for preconditioners whose
        // kernels have the batched form), else one unit per problem.
        bool same_units = b->zprecond == precond && b->zx.size() == n && b->zversions.size() == n &&
                          std::equal(b->zx.begin(), b->zx.end(), x_dev);
        for (size_t i = 0; same_units && i < n; ++i) same_units = b->zversions[i] == b->probs[i]->launch_version;
        if (!same_units) {
            b->units.clear();
            b->unit_first.clear();
            std::vector<std::string> keys;         // per unit: its class key, empty for a lone problem
            for (size_t i = 0; i < n; ++i) {
                const bool can = b->shared && shares_launches(precond);
                const std::string key = can ? batch_class_key(*b->probs[i]) : std::string();
                size_t u = can ? (size_t)(std::find(keys.begin(), keys.end(), key) - keys.begin()) : keys.size();
                if (u == keys.size()) {
                    keys.push_back(key);
                    b->units.push_back({});
                }
                b->units[u].push_back((int)i);
            }
            // offsets of every class member from its first member: block and image
            int row = 0;
            for (const auto& u : b->units) {
                b->unit_first.push_back(row);
                const Problem& P0 = *b->probs[u[0]];
                for (int m : u) {
                    const Problem& P = *b->probs[m];
                    b->zhost[2 * row] = (long long)(reinterpret_cast<uintptr_t>(P.arena.base) -
                                                    reinterpret_cast<uintptr_t>(P0.arena.base));
                    b->zhost[2 * row + 1] = (long long)(reinterpret_cast<uintptr_t>(x_dev[m]) -
                                                        reinterpret_cast<uintptr_t>(x_dev[u[0]]));
                    ++row;
                }
            }
            MBMD_HIP(hipMemcpyAsync(b->zdev, b->zhost.data(), sizeof(long long) * b->zhost.size(),
                                    hipMemcpyHostToDevice, s));
            MBMD_HIP(hipStreamSynchronize(s));
            b->lane.resize(b->units.size());
            for (size_t u = 0; u < b->units.size(); ++u) b->lane[u] = (int)(u % b->n_lanes);
            b->zprecond = precond;
            b->zx.assign(x_dev, x_dev + n);
            b->zversions.resize(n);
            for (size_t i = 0; i < n; ++i) b->zversions[i] = b->probs[i]->launch_version;
        }
        const size_t nu = b->units.size();
        // one iteration of unit u on its branch stream: a class as one launch per kernel
        auto unit_iter = [&](size_t u, bool refresh) {
            const std::vector<int>& mem = b->units[u];
            Problem& P = *b->probs[mem[0]];
            float* x = x_dev[mem[0]];
            hipStream_t bs = b->branch[b->lane[u]];
            std::unique_ptr<ZScope> zs;
            if (mem.size() > 1) zs.reset(new ZScope(b->zdev + 2 * b->unit_first[u], (int)mem.size(), x));
            if (precond == MBMD_PRECOND_NONE) {
                plain_iteration(P, x, nullptr, bs);
            } else {
                if (refresh) {
                    flush_step(P, x, bs);
                    project(P, x, P.l, P.K, bs);
                }
                precond_iteration(P, x, precond, nullptr, bs);
            }
        };
        // the pending step of each problem, after its last iteration
        auto finish = [&](size_t k, hipStream_t st) {
            if (precond != MBMD_PRECOND_NONE) flush_step(*b->probs[k], x_dev[k], st);
        };
        auto fork = [&](hipStream_t from) {
            MBMD_HIP(hipEventRecord(b->fork, from));
            for (int i = 0; i < b->n_lanes; ++i) MBMD_HIP(hipStreamWaitEvent(b->branch[i], b->fork, 0));
        };
        auto join = [&](hipStream_t into) {
            for (int i = 0; i < b->n_lanes; ++i) {
                MBMD_HIP(hipEventRecord(b->join[i], b->branch[i]));
                MBMD_HIP(hipStreamWaitEvent(into, b->join[i], 0));
            }
        };
        if (!use_graph) {
            // the units are independent: each branch runs all its iterations, then joins
            fork(s);
            for (int it = 0; it < n_iter; ++it)
                for (size_t u = 0; u < nu; ++u) unit_iter(u, it % kRefreshEvery == 0);
            join(s);
            for (size_t k = 0; k < n; ++k) finish(k, s);
            return;
        }
        // Capture on a library-owned stream (the legacy default stream cannot be
        // captured); the branches join the capture through the fork event, and the
        // instantiated graphs are then launched on the caller's stream.
        bool same = b->captured && b->precond == precond && b->xs.size() == n;
        for (size_t i = 0; same && i < n; ++i)
            same = b->xs[i] == x_dev[i] && b->versions[i] == b->probs[i]->launch_version;
        if (!same) {
            for (int i = 0; i < 2; ++i) {
                if (b->exec[i]) (void)hipGraphExecDestroy(b->exec[i]);
                if (b->graph[i]) (void)hipGraphDestroy(b->graph[i]);
                b->exec[i] = nullptr;
                b->graph[i] = nullptr;
            }
            b->captured = false;
            if (!b->capture) MBMD_HIP(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
            MBMD_HIP(hipStreamSynchronize(s));   // set-up launches above must not be captured out of order
            hipStream_t cs = b->capture;
            for (int i = 0; i < 2; ++i) {
                MBMD_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
                try {
                    fork(cs);
                    for (size_t u = 0; u < nu; ++u) unit_iter(u, i == 1);
                    join(cs);
                } catch (...) {
                    hipGraph_t g = nullptr;
                    (void)hipStreamEndCapture(cs, &g);
                    if (g) (void)hipGraphDestroy(g);
                    (void)hipGetLastError();
                    throw;
                }
                MBMD_HIP(hipStreamEndCapture(cs, &b->graph[i]));
                MBMD_HIP(hipGraphInstantiate(&b->exec[i], b->graph[i], nullptr, nullptr, 0));
            }
            b->captured = true;
            b->precond = precond;
            b->xs.assign(x_dev, x_dev + n);
            b->versions.resize(n);
            for (size_t i = 0; i < n; ++i) b->versions[i] = b->probs[i]->launch_version;
        }
        b->stream = s;
        for (int it = 0; it < n_iter; ++it) {
            const bool refresh = precond != MBMD_PRECOND_NONE && it % kRefreshEvery == 0;
            MBMD_HIP(hipGraphLaunch(b->exec[refresh ? 1 : 0], s));
        }
        for (size_t k = 0; k < n; ++k) finish(k, s);
    });
}

}  // extern "C"
