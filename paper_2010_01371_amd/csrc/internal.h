// Internal declarations of the MI355X (gfx950) library behind include/mbmd.h.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>
#include <type_traits>

#include "../../include/mbmd.h"

namespace mbmd {

constexpr int kMaxMat = 4;
constexpr int kMaxChan = 8;
constexpr int kMaxEnergy = 256;
constexpr int kMaxPacked = kMaxMat * (kMaxMat + 1) / 2;   // symmetric N_k x N_k, packed
constexpr int kPreconds = 5;                               // mbmd_precond values 0..4
constexpr int kMaxBlurHalf = 4;                            // projection-domain blur: at most 9 taps
constexpr int kBlurTaps = 2 * kMaxBlurHalf + 1;

// Projection-domain blur, per channel along the bins of each view: row b of
// channel c is (B_c z)_b = sum_{|d|<=h} taps[c][d + h] z_{b+d}, bins beyond
// the detector dropped.  h = 0: no blur.
struct BlurArgs {
    int h = 0;
    int B = 0;                         // bins per view
    float taps[kMaxChan][kBlurTaps] = {};
};
constexpr int kMaxBackCh = 10;                              // channels of one backprojection
constexpr int kBackMaxU = 4;                                // views in flight per back projection group
constexpr int kMaxGpus = 64;                                // devices with cached per-device launch data
constexpr int kRefreshEvery = 25;                           // recompute l = A x this often
constexpr int kMaxPartials = 16384;                         // per reduction region

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);
struct Error {
    int status;
    std::string msg;
};
#define MBMD_HIP(call)                                                                  \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            throw ::mbmd::Error{MBMD_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)}; \
    } while (0)
#define MBMD_REQUIRE(cond, status, msg)                                                 \
    do {                                                                                \
        if (!(cond)) throw ::mbmd::Error{(status), (msg)};                              \
    } while (0)
#define MBMD_LAUNCHED() MBMD_HIP(hipGetLastError())

// Index of packed symmetric entry (k, l) of an n x n matrix, row-major upper.
__host__ __device__ inline int packed_index(int k, int l, int n) {
    if (k > l) { int t = k; k = l; l = t; }
    return k * n - k * (k - 1) / 2 + (l - k);
}

// ---------------------------------------------------------------- optional kernel timing
// Brackets one launch with hipEvents on its stream when profiling is enabled.
class KernelTimer {
  public:
    KernelTimer(const char* name, hipStream_t s);
    ~KernelTimer() {
        try {
            stop();
        } catch (...) {
        }
    }
    void stop();

  private:
    const char* name_;
    hipStream_t s_;
    hipEvent_t a_{}, b_{};
    bool active_ = false;
};

// ---------------------------------------------------------------- batched launches
// A batch runs slices whose launch parameters are identical (a class) as one
// launch per kernel, blockIdx.z selecting the slice.  Every slice's state lies
// at the same offsets of its own block as slice 0's in its block, so slice z's
// pointers are slice 0's plus a byte offset: zd[2 z] for the block, zd[2 z + 1]
// for the caller's image x.  The launchers read the current setting, which only
// the batch sets (thread-local, around one class's launches); kernels given a
// non-null zd shift their pointers by it.  While it is set, KernelTimer refuses
// every kernel without that form (MBMD_ERR_UNSUPPORTED, before the launch).
struct ZBatch {
    const long long* zd = nullptr;   // device [nz][2]
    int nz = 1;
    const void* x0 = nullptr;        // slice 0's image, for launchers whose input may be x
};
ZBatch& zbatch();
inline dim3 zgrid(dim3 g) {
    g.z = (unsigned)zbatch().nz;
    return g;
}
inline const long long* zarg() { return zbatch().zd; }
enum { Z_BLOCK = 0, Z_IMAGE = 1 };
__device__ __forceinline__ long long zoff(const long long* zd, int which) {
    return zd ? zd[2 * (int)blockIdx.z + which] : 0;
}
// Byte arithmetic on the pointer itself (not through an integer), so that the
// compiler still sees a global-memory pointer based on the kernel argument:
// it keeps global (not flat) accesses and, for zadd, its no-alias reasoning,
// which lets read-only tables stay in scalar loads.  zadd is for pointers that
// are never null (d is 0 outside a batch); zshift keeps a null pointer null.
template <class T>
__device__ __forceinline__ T* zadd(T* p, long long d) {
    using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
    return reinterpret_cast<T*>(reinterpret_cast<B*>(p) + d);
}
template <class T>
__device__ __forceinline__ T* zshift(T* p, long long d) {
    return p ? zadd(p, d) : p;
}

// ---------------------------------------------------------------- device memory arena
// Parts are 256-byte aligned offsets from base.  A null base is a sizing pass:
// take() only counts.  The memory is the library's (reserve, freed by release)
// or the caller's (adopt: release forgets it).
struct Arena {
    char* base = nullptr;
    size_t size = 0, used = 0;
    bool owned = false;
    void reserve(size_t bytes);
    void adopt(void* mem, size_t bytes);
    template <class T> T* take(size_t n) {
        size_t off = (used + 255) & ~size_t(255);
        used = off + n * sizeof(T);
        if (base == nullptr) return nullptr;     // sizing pass
        if (used > size) throw Error{MBMD_ERR_ARG, "workspace too small"};
        return reinterpret_cast<T*>(base + off);
    }
    void release();
};

// ---------------------------------------------------------------- geometry tables
// Per-view data of the distance-driven projector.  A view sweeps either the
// image rows (frame 0: line index q = iy, along index p = ix) or the columns
// (frame 1: q = ix, p = iy).  Along-line positions K are in pixel units with
// the origin at the image centre, so pixel p spans [p - Np/2, p + 1 - Np/2].
struct ViewParams {
    // fractional bin index of the point (K, q): beta = num / den with
    // num = n0 + nK K + nq qq, den = d0 + dK K + dq qq, qq = q - (Nq-1)/2
    float n0, nK, nq, d0, dK, dq;
    float orient;      // +1 when bin boundaries run along +K on every sweep line, else -1
    int view_frame;    // original view index | frame << 16
};
__host__ __device__ inline int vp_view(const ViewParams& p) { return p.view_frame & 0xffff; }
__host__ __device__ inline int vp_frame(const ViewParams& p) { return p.view_frame >> 16; }

// One detector cell b of the back projector's cumulative integral: C[b+1] in
// FP64, the width C[b+1] - C[b] of the bin and the width of the next bin in
// FP32 (16 bytes, one vector load, which serves both pixel edges of a lane).
struct alignas(16) DetEntry {
    double c;
    float d;
    float dn;
};

// Per-view tables are in slot order (views of frame 0, then of frame 1).
struct GeomTables {
    mbmd_geometry g{};
    int V = 0, B = 0, nx = 0, ny = 0;
    int n_frame_views[2] = {0, 0};
    ViewParams* view = nullptr;      // [slot]
    // [slot][B+1]: boundary b' crosses sweep line q (0..Nq-1) at along-line
    // position X0 + X1 q, in pixels from the line's first pixel edge; stored in
    // increasing X (boundary B - b' at entry b' for views with orient < 0)
    float2* bound = nullptr;
    // [frame 0 items][frame 1 items]: forward items of each frame in order of
    // decreasing work (active lines), so the heaviest blocks are dispatched first
    int* fwd_order = nullptr;
    float* path = nullptr;           // [slot][B]: path length per sweep line of the bin-centre ray
    int* frame_views = nullptr;      // [slot] -> view index
    // scratch: line prefix sums F[k] = sum_{p<k} img[p] for k < Np and the line total
    // at k = Np .. Np+3; frame 0 lines [n_mat][ny][prefix_row(nx)], then frame 1
    // lines [n_mat][nx][prefix_row(ny)]
    float* prefix = nullptr;
    int prefix_mat = 0;
    // [max(nx,ny)][slot][2]: per sweep line q of the slot's frame, the fractional
    // bin index counted from the detector centre, beta - back_shift(B) =
    // (n + m K) / (1 + c K), as {n, m, c, a} and {g, 0, 0, 0}: with
    // f = b - back_shift(B) for any bin b, (a - g f) scales (n + m K) - f (1 + c K)
    // to the fraction (K - K_b) / (K_b+1 - K_b) of bin b.  beta increases with K:
    // for views with orient < 0 it counts bins from the last one
    float4* back_line = nullptr;
    int back_line_q = 0;             // max(nx, ny)
    // scratch: detector rows of n_ch channels, [n_ch][V][det_row(B)] for one or
    // two, else packed (det_triples, det_single_base, det_scales)
    DetEntry* det_prefix = nullptr;
    // scratch: [back_ch][nx][ny] column-sweep part of a back projection
    float* back_part = nullptr;
    // tile shape picked for the back projector per channel count (-1: not yet tuned)
    mutable int back_variant[kMaxBackCh + 1] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
    // Testing hook: MBMD_BACK_VARIANT=v in the environment when the tables are
    // placed forces back projector candidate v (-1: the tuned choice).
    int forced_back = -1;
    int back_ch = 0;
    void* mem = nullptr;
    int device = -1;
};

// Row stride (floats) of the line prefix table for lines of Np pixels: Np + 4
// entries (a 16-byte read at any k <= Np stays in the row) rounded up to a
// multiple of 4, so that rows start 16-byte aligned.
__host__ __device__ inline int prefix_row(int Np) { return (Np + 4 + 3) & ~3; }
// Detector rows of the back projector: entries 0 .. B-1 are the bins (from the
// last bin for views with orient < 0), B and B+1 repeat the total with zero
// widths, so that the bin index clamped to the symmetric range
// [-back_shift(B), back_shift(B)] around the detector centre (shifted by
// back_shift(B)) always lands inside the row.
__host__ __device__ inline int det_row(int B) { return B + 2; }
// From kPackFrom channels on, whole groups of three channels ("triples") share
// two rows of 16-byte entries, planes A and B ([det_triples(n_ch)][2][V]
// [det_row(B)]), so that two gathers at the same entry offset serve three
// channels: channel k of a triple holds q = hi 2^16 + lo, a 48-bit integer
// with C[b+1] = c0 + q 2^-s for the row's own offset c0 (not stored: it drops
// out of every pixel) and exponent s, as hi (int32, word k of A), lo (16 bits:
// word 3 of A, low / high half for k = 0 / 1, word 3 of B for k = 2), and its
// width w[b] (FP32, word k of B).  The remaining channels keep rows of their
// own (DetEntry, [n_ch - 3 T][V][det_row(B)]) after the triples, and the
// triples' scales 2^-s (FP64, [V][3 T]) follow those.
constexpr int kPackFrom = 3;
__host__ __device__ inline int det_triples(int n_ch) { return n_ch >= kPackFrom ? n_ch / 3 : 0; }
// Byte offset of the rows of the channels outside the triples.
__host__ __device__ inline size_t det_single_base(int n_ch, int V, int B) {
    return (size_t)2 * det_triples(n_ch) * V * det_row(B) * sizeof(DetEntry);
}
// Byte offset of the triples' scale table (the end of the rows).
__host__ __device__ inline size_t det_scales(int n_ch, int V, int B) {
    return det_single_base(n_ch, V, B) + (size_t)(n_ch - 3 * det_triples(n_ch)) * V * det_row(B) * sizeof(DetEntry);
}

// Forward projection tiling: wavefronts of two bin boundaries per lane (127 bins),
// blocks of kFwdWaves such wavefronts along the detector ("chunks"), and each
// block's active lines split into two halves.  Items of a frame are
// (slot in frame, chunk, half), numbered ((slot chunks) + chunk) 2 + half.  One
// wavefront per block lets the dispatcher balance the CUs wavefront by wavefront
// (the work per wavefront ranges from no lines to every line).
constexpr int kFwdBinsPerWave = 127;
constexpr int kFwdWaves = 1;
__host__ __device__ inline int fwd_chunks(int B) { return (B + kFwdWaves * kFwdBinsPerWave - 1) / (kFwdWaves * kFwdBinsPerWave); }

// Lines q in [0, Nq) are active unless the first and the last boundary of a
// wavefront (positions X = x0 + x1 q, affine in q) both lie at least a margin
// beyond the same end of the line; the inactive lines form at most two
// intervals, and [q_lo, q_hi] is the hull of what remains (empty: q_lo > q_hi).
// FP64 with a margin of 1/64 pixel, far above the FP32 error of the positions
// the line loop evaluates, so no line with a nonzero contribution is dropped.
__host__ __device__ inline void active_lines(float2 bf, float2 bl, int Np, int Nq, int& q_lo, int& q_hi) {
    const double m = 1.0 / 64.0, last = (double)(Nq - 1);
    // {q in [0, last] : a + b q <= c} as [lo, hi]
    auto half = [&](double a, double b, double c, double& lo, double& hi) {
        lo = 0.0;
        hi = last;
        if (b == 0.0) {
            if (a > c) lo = 1.0, hi = 0.0;
        } else if (b > 0.0) {
            hi = fmin(last, floor((c - a) / b));
        } else {
            lo = fmax(0.0, ceil((c - a) / b));
        }
    };
    double lo1a, hi1a, lo1b, hi1b, lo2a, hi2a, lo2b, hi2b;
    half(bf.x, bf.y, -m, lo1a, hi1a);                              // first boundary left of the line
    half(bl.x, bl.y, -m, lo1b, hi1b);                              // last boundary left of the line
    half(-(double)bf.x, -(double)bf.y, -((double)Np + m), lo2a, hi2a);   // first right of it
    half(-(double)bl.x, -(double)bl.y, -((double)Np + m), lo2b, hi2b);   // last right of it
    const double i1lo = fmax(lo1a, lo1b), i1hi = fmin(hi1a, hi1b);
    const double i2lo = fmax(lo2a, lo2b), i2hi = fmin(hi2a, hi2b);
    double a = 0.0, b = last;
    for (int r = 0; r < 2; ++r) {                                  // strip inactive runs at both ends
        if (i1lo <= i1hi && i1lo <= a && a <= i1hi) a = i1hi + 1.0;
        if (i2lo <= i2hi && i2lo <= a && a <= i2hi) a = i2hi + 1.0;
        if (i1lo <= i1hi && i1lo <= b && b <= i1hi) b = i1lo - 1.0;
        if (i2lo <= i2hi && i2lo <= b && b <= i2hi) b = i2lo - 1.0;
    }
    q_lo = (int)a;
    q_hi = (int)b;
}


__host__ __device__ inline int back_shift(int B) { return (B + 1) / 2; }
inline size_t prefix_elems(int nx, int ny) { return (size_t)ny * prefix_row(nx) + (size_t)nx * prefix_row(ny); }

// Host copy of a geometry's tables, built in FP64 and stored in FP32.
struct GeomHost {
    std::vector<ViewParams> vp;
    std::vector<float2> bound;
    std::vector<float> path;
    std::vector<int> fv;
    std::vector<float4> line;
    std::vector<int> order;
    int n_frame_views[2] = {0, 0};
};
void build_geometry_host(const mbmd_geometry& g, GeomHost& h);
// Device bytes of the tables and scratch of a geometry (256-byte aligned parts);
// back_ch = 0 leaves out everything the back projection needs.
size_t geometry_bytes(const mbmd_geometry& g, int prefix_mat, int back_ch);
// Points t into base (geometry_bytes(g, ...) bytes, 256-byte aligned, not owned
// by t) and enqueues the uploads of h on s; h must outlive them.
void place_geometry(const mbmd_geometry& g, const GeomHost& h, GeomTables& t, char* base, int prefix_mat,
                    int back_ch, hipStream_t s);
// Builds the tables into memory of its own (t.mem, freed by free_geometry).
void build_geometry(const mbmd_geometry& g, GeomTables& t, int prefix_mat, int back_ch);
void free_geometry(GeomTables& t);
void validate_geometry(const mbmd_geometry& g);
// Tables and scratch of the standalone projector calls, per geometry, device and stream.
GeomTables& cached_geometry(const mbmd_geometry& g, int prefix_mat, int back_ch, hipStream_t s);
void clear_geometry_cache();

// ---------------------------------------------------------------- projector launches
void launch_project(const GeomTables& t, const float* x, float* sino, int n_mat, hipStream_t s);
void launch_backproject(const GeomTables& t, const float* sino, float* x, int n_ch, hipStream_t s);
// A^T sino without the final sum: x receives the row-sweep part, the return value is
// the column-sweep part in image layout (nullptr if none), valid until the next
// back projection with the same geometry.
const float* launch_backproject_parts(const GeomTables& t, const float* sino, float* x, int n_ch, hipStream_t s);
long long count_nonzeros(const GeomTables& t, hipStream_t s);

// Pixels that a back projection adds into, cleared before it: the last w0
// columns of x (row sweeps) and the last h1 rows of part (column sweeps), nch
// channels each -- the tail pixels, or every pixel when the main wavefronts'
// views are split over two wavefronts; zero sizes when there is none.
struct BackClear {
    float* x;
    float* part;
    int nx, ny, w0, h1, nch;
};
// What a producer of a back projection's input needs to write the detector
// rows itself (instead of the detector-prefix launch): the rows, the per-view
// records and path lengths they are built from, and the pixels to clear for the
// tile shape in use.  ok is false until that shape is chosen for n_ch channels
// (the first back projection of a geometry and channel count tunes it), and for
// packed rows (kPackFrom channels or more), which only the detector prefix writes.
struct BackRows {
    bool ok;
    DetEntry* rows;               // [n_ch][V][det_row(B)]
    const ViewParams* view;       // [slot]
    const float* path;            // [slot][B]
    int V, B;
    BackClear clr;
};
BackRows back_rows(const GeomTables& t, float* x, int n_ch);
// The back projection kernel alone in the chosen shape, with the detector rows
// already written (by a launch given back_rows(t, x, n_ch)); returns the
// column-sweep part as launch_backproject_parts does.
const float* launch_back_kernel(const GeomTables& t, float* x, int n_ch, hipStream_t s);

// ---------------------------------------------------------------- problem
struct Problem {
    mbmd_geometry g{};
    GeomTables* geom = nullptr;      // owned (projector geometries only); memory in the arena
    char* geom_mem = nullptr;        // the geometry's part of the arena
    size_t geom_bytes = 0;
    int ws_flags = 0;                // mbmd_workspace_flags the arena was sized with
    int identity = 0;
    int K = 1, E = 1, C = 1, npk = 1;
    int nx = 0, ny = 0, V = 0, B = 0;
    int nj = 0, ni = 0;              // pixels, rays
    int pen_kind = 0;
    double beta[kMaxMat * kMaxMat] = {0};
    double delta = 0.0;
    int has_penalty = 0;
    std::vector<double> Qh, Sh;

    Arena arena;
    // spectral model (device)
    float *Q = nullptr, *S = nullptr, *rowS = nullptr, *Qsum = nullptr, *beta_d = nullptr;
    // data
    float *y = nullptr, *w = nullptr, *gammaA = nullptr;
    // sinogram state
    float *l = nullptr, *q = nullptr, *u = nullptr, *v = nullptr, *r = nullptr, *sino_tmp = nullptr;
    // image state
    float *g_img = nullptr, *d_img = nullptr, *p_img = nullptr, *t_img = nullptr, *t2_img = nullptr;
    float *dL_const = nullptr;       // single-energy data curvature A^T(gamma c), built once
    int dL_valid = 0;
    // preconditioners
    float* M0 = nullptr;             // [npk][nj]
    float* Linv = nullptr;           // [ny][nx][npk]  (L^-1 blocks)
    float* Kinv = nullptr;           // [ny][nx][npk]  (K^-1 blocks)
    float* Dinv = nullptr;           // [npk][nj] Daubechies-4 coefficient blocks (inverse)
    float* W = nullptr;              // [npk][ni] Fisher weights (build)
    // projection-domain blur (mbmd_problem_set_blur); buffers in blur_arena
    BlurArgs blur;
    int launch_version = 0;          // bumped when the iteration's launch sequence or arguments change
    Arena blur_arena;
    float* wb = nullptr;             // [C][ni] B^T W B 1 (the eta factor)
    float* J = nullptr;              // [C][K][ni] Jacobian of the unblurred means (build)
    float* btmp0 = nullptr;          // [C][ni] scratch
    float* btmp1 = nullptr;          // [C][ni] scratch
    float2* spec = nullptr;          // [K][ny][nx] complex scratch
    float2* tw_x = nullptr;          // twiddles for nx
    float2* tw_y = nullptr;          // twiddles for ny
    float* coef = nullptr;           // [K][ny][nx] Haar coefficients
    float* coarse = nullptr;         // [K][ny/T][nx/T]
    int built[kPreconds] = {};
    // Fisher weights W and M0 in use: 0 none, 1 from the data (modified),
    // 2 from a reference image and / or M0 = I (mbmd_precond_build_ex)
    int m0_state = 0;
    int n_floored[kPreconds] = {};
    // reductions
    double* partials = nullptr;      // [kRegions][kMaxPartials]
    double* scal = nullptr;          // device scalars (alpha, phi, flags...)
    double* trace = nullptr;         // device objective trace (grows)
    int trace_cap = 0;
    double* trace_mem_owner = nullptr;
    int* flags = nullptr;
    int l_valid_for_x = 0;
    // Testing hook: MBMD_FUSE_ROWS=0 in the environment at creation keeps the
    // gradient launch and the detector prefix apart (the same iterates).
    bool fuse_rows = true;
    hipStream_t last_stream = nullptr;
};

// Reduction regions and scalar slots.
enum { R_PHI_L = 0, R_PHI_R, R_GP, R_CQ2, R_PRP, R_AUX, kRegions };
// S_PHI_PREV: the objective of the previous evaluation of a run (NaN at its
// start), against which the next one is checked for an increase.
enum { S_ALPHA = 0, S_PHI, S_GP, S_DEN, S_LMAX, S_PHI_PREV, kScalars = 16 };
// Bits of the problem's numeric flags (flags[0] on the device): the mbmd_numeric_flags.
constexpr int kFlagErrors = MBMD_FLAG_NONFINITE | MBMD_FLAG_NO_CURVATURE | MBMD_FLAG_ASCENT;
// Reduction modes of launch_reduce_final: form the step size; check the
// objective against S_PHI_PREV (raising MBMD_FLAG_INCREASE) and replace it.
enum { RED_STEP = 1, RED_MONOTONE = 2 };
// Relative rise of the objective between consecutive evaluations that raises
// MBMD_FLAG_INCREASE (well above the FP32 evaluation noise of about 1e-6).
constexpr double kIncreaseTol = 1e-5;

// ---------------------------------------------------------------- ray (per detector element) passes
struct RayArgs {
    int ni, K, E, C;
    const float *Q, *S, *rowS, *Qsum;    // device spectral model
    const float *y, *w, *gammaA;         // [C][ni], [C][ni], [ni] (NULL gammaA = 1)
    const float* wb;                     // [C][ni] eta factor B^T W B 1 (= w without a blur)
    BlurArgs blur;
    float *tmp0, *tmp1;                  // [C][ni] scratch of the blurred passes
};
struct PenaltyArgs {
    int K, nx, ny, kind;
    const float* beta;     // device [K][K]
    float delta;
};
// The previous preconditioned step, applied at the start of the next ray
// gradient launch: l += alpha q (in place, before l is used) and, in extra
// blocks of the same launch, x += alpha p (n_img floats); alpha is read on the
// device, and a zero alpha (with finite p and q) makes it a no-op.
struct StepUpdate {
    const double* alpha;
    const float* q;
    float* l;
    float* x;
    const float* p;
    int n_img;
};
int launch_ray_grad(const RayArgs& a, const float* l, float* u, float* v, float* r,
                    double* phi_partials, hipStream_t s, const StepUpdate* up = nullptr);
// The ray gradient u (a.K channels) written straight into the back projector's
// detector rows (br = back_rows(...) with br.ok): one workgroup per view slot,
// each computing its rays as launch_ray_grad does and building the rows of u
// times the path length, bit for bit as the detector-prefix launch would from
// the stored u; also clears br.clr.  Residuals r, objective partials (one per
// view slot; returns their count) and the step update as launch_ray_grad.
// Returns -1, launching nothing, when the rows of one slot do not fit in LDS.
int launch_ray_grad_rows(const RayArgs& a, const float* l, float* r, double* phi_partials, hipStream_t s,
                         const StepUpdate& up, const BackRows& br);
int launch_ray_curv(const RayArgs& a, const float* l, const float* r, const float* q,
                    double* partials, hipStream_t s);
// Curvature along the direction in one launch: the rays' c q^2 into region CQ2
// and, with pen, the penalty's p^T R''(x) p into region PRP of partials (the
// base of all regions); sets counts[R_CQ2] and counts[R_PRP].
void launch_curvature(const RayArgs& a, const float* l, const float* r, const float* q, const PenaltyArgs* pen,
                      const float* x, const float* p, double* partials, int* counts, hipStream_t s);
void launch_forward_model(const RayArgs& a, const float* l, float* ybar, hipStream_t s);
void launch_forward_vjp(const RayArgs& a, const float* l, const float* gbar, float* sk, hipStream_t s);
// Fisher weights [npk][ni]; lref [K][ni]: reference line integrals (D the
// transmission there), or NULL for the data-based D.
void launch_fisher(const RayArgs& a, float* W, hipStream_t s, const float* lref = nullptr, float* J = nullptr);
// Per channel c and ray i: out = wt * (B z) (transpose: B^T z; wt NULL: 1).
void launch_blur(const BlurArgs& b, int ni, int C, const float* in, const float* wt, float* out, bool transpose,
                 hipStream_t s);
// Per ray, with J [C][K][ni]: out_c = sum_k J_ck in_k ([K][ni] -> [C][ni]), or
// transposed out_k = sum_c J_ck in_c.
void launch_jmix(int ni, int K, int C, const float* J, const float* in, float* out, bool transpose, hipStream_t s);
void launch_fisher_mix(int ni, int K, const float* W, const float* in, float* out, hipStream_t s);
int launch_identity_iterate(const RayArgs& a, float* x, const float* M0, int precond, int n_iter,
                            double* partials_per_iter, int stride, hipStream_t s);

// ---------------------------------------------------------------- image passes
int launch_penalty_grad(const PenaltyArgs& a, const float* x, const float* gL, const float* dL,
                        float* g, float* d, double* phi_partials, hipStream_t s, const float* gL2 = nullptr);
int launch_penalty_quadform(const PenaltyArgs& a, const float* x, const float* p, double* partials,
                            hipStream_t s);
void launch_penalty_hess_add(const PenaltyArgs& a, const float* v, float* out, hipStream_t s);
void launch_plain_update(int n, float* x, const float* g, const float* d, hipStream_t s);
void launch_inv_var(int n, const float* y, float* w, hipStream_t s);
void launch_scale_by_vec(int n, int nch, const float* in, const float* vec, float* out, hipStream_t s);
void launch_fill_double(int n, double* x, double value, hipStream_t s);
void launch_axpy_alpha(int n, float* x, const float* p, const double* alpha, hipStream_t s);
// x1 += alpha p1 (n1 floats) and x2 += alpha p2 (n2 floats) in one launch.
void launch_axpy2_alpha(int n1, float* x1, const float* p1, int n2, float* x2, const float* p2,
                        const double* alpha, hipStream_t s);
void launch_fill(int n, float* x, float value, hipStream_t s);
void launch_scale_copy(int n, const float* in, float* out, float scale, hipStream_t s);
int launch_dot(int n, const float* a, const float* b, double* partials, hipStream_t s);
void launch_block_apply(int nj, int K, const float* M, const float* in, float* out, float scale,
                        hipStream_t s);
// packed [npk][nj] += the symmetric share of material column k_col, col [K][nj]
// (entry (k2, k_col) of every pixel's block at channel k2).
void launch_block_add_column(int nj, int K, int k_col, const float* col, float* packed, hipStream_t s);
void launch_block_invsqrt(int n, int K, const float* in_packed, float* out_packed, double power,
                          double floor_rel, const double* floor_abs_scaled, double eps,
                          int* n_floored, hipStream_t s);
void launch_block_lmax(int n, int K, const float* in_packed, double* lmax, hipStream_t s);
void launch_reduce_final(double* partials, const int* counts, double* scal, double* trace_slot,
                         int mode, int* flags, hipStream_t s);

// ---------------------------------------------------------------- transforms
void fill_twiddles(float2* tw, int n, hipStream_t s);
// Forward 2D FFT of K real images (optionally pre-multiplied by packed blocks
// M and circularly shifted by (-sy, -sx)); complex output [K][ny][nx].
void launch_fft2_forward(int K, int nx, int ny, const float* in, const float* M, int sy, int sx,
                         float2* spec, const float2* twx, const float2* twy, hipStream_t s);
// out = -scale * M * Re(IFFT2(Filt * FFT2(M * in)))  and partial sums of g.out.
int launch_fourier_apply(int K, int nx, int ny, const float* in, const float* M, const float* Filt,
                         float2* spec, const float2* twx, const float2* twy, float* out,
                         float out_sign, const float* g, double* partials, hipStream_t s);
void launch_spectrum_real_to_blocks(int K, int nj, int k_col, const float2* spec, float* blocks,
                                    hipStream_t s);

int haar_tile(int n);
void launch_haar_forward(int K, int n, const float* in, const float* M, float* coef, float* coarse,
                         hipStream_t s);
void launch_haar_inverse(int K, int n, const float* coef, float* coarse, const float* M, float* out,
                         float out_sign, hipStream_t s);
int launch_haar_apply(int K, int n, const float* in, const float* M, const float* Kinv, float* coef,
                      float* coarse, float* out, float out_sign, const float* g, double* partials,
                      hipStream_t s);
void launch_coef_blocks(int K, int n, int k_col, const float* coef, float* blocks, hipStream_t s);
// Orthonormal Daubechies-4 transform of [K][n][n] images (square power of two):
// coef = U (M in) (M NULL: identity); the inverse out = out_sign M (U^T coef)
// overwrites coef.  scratch: [K][n][n] overwritten (the inverse may pass out).
// The apply is out = out_sign M U^T Dinv U M in, with the partials of g . out
// (returns their count) when partials is not NULL.
void launch_d4_forward(int K, int n, const float* in, const float* M, float* coef, float* scratch, hipStream_t s);
void launch_d4_inverse(int K, int n, float* coef, const float* M, float* out, float out_sign, float* scratch,
                       hipStream_t s);
int launch_d4_apply(int K, int n, const float* in, const float* M, const float* Dinv, float* coef, float* out,
                    float out_sign, const float* g, double* partials, hipStream_t s);

}  // namespace mbmd
