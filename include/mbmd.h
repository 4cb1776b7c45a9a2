/*
 * mbmd.h -- preconditioned separable-paraboloidal-surrogate (SPS) iteration
 * for penalized weighted least-squares CT reconstruction and model-based
 * material decomposition, on AMD Instinct MI355X (gfx950).
 *
 * Method: Tivnan, Wang & Stayman, "A Preconditioned Algorithm for
 * Model-Based Iterative CT Reconstruction and Material Decomposition from
 * Spectral CT Data" (arXiv 2010.01371).  Section names below refer to it.
 *
 * Estimation problem (Methods, "Generalized Models for Data Acquisition and
 * Estimation", eq:meanModel and eq:mapEstimator):
 *     ybar(x) = B S exp(-(Q (x) A) x),
 *     Phi(x)  = 1/2 (y - ybar)^T diag(w) (y - ybar) + R(x),
 * with x the stack of N_k material images, A the 2D projector, Q [N_E x N_k]
 * the attenuation of each material per energy, S [N_c x N_E] the channel
 * sensitivities (gain and I0 folded in), B an optional projection-domain blur
 * along the detector (identity unless mbmd_problem_set_blur sets one), and
 * w = 1/variance per ray and channel.
 * Standard CT is N_k = N_E = N_c = 1 with S = I0 and Q = 1 ("Standard CT
 * Reconstruction"); projection-domain decomposition is the identity geometry
 * (A = I, "Projection-Domain Decomposition"); one-step MBMD is the general
 * case ("One-Step Reconstruction and Material Decomposition").
 *
 * Conventions for every call:
 *   - Arrays named *_dev are device pointers (HIP device memory, float32,
 *     C-contiguous); the caller owns them.  Arrays named *_host are host
 *     pointers.  Descriptor structs are host memory and are copied by the
 *     call that receives them.
 *   - Images are [n_mat][ny][nx] (x fastest).  Sinograms are
 *     [n][n_views][n_bins] (bins fastest).
 *   - `stream` is a hipStream_t (NULL = the default stream).  All work is
 *     enqueued on it asynchronously unless a *_host output is requested,
 *     in which case the call synchronizes that stream before returning.
 *     Three set-up steps also wait: problem creation (for its table
 *     uploads), the first back projection of a geometry and channel count
 *     in the process outside graph capture (it times the candidate tile
 *     shapes, which give identical results, on its own inputs), and a batch
 *     call whose grouping of problems changed (for its offsets table).
 *   - Return value: MBMD_OK (0) or a negative mbmd_status.  No exception
 *     crosses this interface.  mbmd_last_error() returns a thread-local
 *     message for the last failure.  Numeric failures of kernels already
 *     enqueued (mbmd_numeric_flags) surface at the next synchronizing call
 *     on the problem: mbmd_sps_step with a trace, mbmd_gradient with an
 *     objective, or mbmd_problem_check.
 *   - Device memory: a problem's whole device state (geometry tables,
 *     problem state, preconditioner tables, scratch) lives in one block of
 *     mbmd_workspace_bytes bytes, either a workspace the caller passes to
 *     mbmd_problem_create (e.g. a torch uint8 tensor; the library then
 *     allocates nothing for the problem) or, for a NULL workspace, one
 *     allocation made by mbmd_problem_create.  Nothing is allocated inside
 *     the iterations, applies, builds or batches.  The standalone projector
 *     calls (mbmd_project, mbmd_backproject, mbmd_projector_nnz) keep
 *     library-allocated tables per geometry, device and stream (at most 16,
 *     least recently used freed first; mbmd_cache_clear frees them).
 */
#ifndef MBMD_H
#define MBMD_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MBMD_OK = 0,
    MBMD_ERR_ARG = -1,          /* invalid argument (NULL, non-positive size, bad enum) */
    MBMD_ERR_SHAPE = -2,        /* sizes the library does not support (see each call) */
    MBMD_ERR_HIP = -3,          /* a HIP runtime call failed */
    MBMD_ERR_NOT_BUILT = -4,    /* preconditioner requested before mbmd_precond_build */
    MBMD_ERR_NUMERIC = -5,      /* non-finite objective or step size detected */
    MBMD_ERR_UNSUPPORTED = -6   /* option combination not implemented */
} mbmd_status;

typedef enum {
    MBMD_GEOM_PARALLEL = 0,     /* parallel beam */
    MBMD_GEOM_FAN_FLAT = 1,     /* fan beam, flat detector */
    MBMD_GEOM_IDENTITY = 2      /* A = I: the unknown is a sinogram of line integrals */
} mbmd_geom_kind;

typedef enum {
    MBMD_PRECOND_NONE = 0,      /* plain SPS */
    MBMD_PRECOND_FOURIER = 1,   /* (cross-material) modified Fourier: M = M0 U^H L^-1/2 U */
    MBMD_PRECOND_HAAR = 2,      /* (cross-material) Haar wavelet:     M = M0 U^T K^-1/2 U */
    MBMD_PRECOND_BLOCKDIAG = 3, /* per-pixel N_k x N_k block diagonal: M = M0 */
    MBMD_PRECOND_DAUB4 = 4      /* (cross-material) wavelet with the Daubechies-4 transform:
                                   M = M0 U^T K^-1/2 U, U the periodised orthonormal DWT */
} mbmd_precond;

/* Flags of mbmd_precond_build_ex. */
typedef enum {
    MBMD_PRECOND_UNMODIFIED = 1 /* M0 = I: the unmodified preconditioners (the Fourier one of eq:fourierEigenbasis) */
} mbmd_precond_flags;

/* Flags of mbmd_workspace_bytes / mbmd_problem_create. */
typedef enum {
    MBMD_WORKSPACE_BLUR = 1     /* room for a projection-domain blur (mbmd_problem_set_blur) */
} mbmd_workspace_flags;

/* Numeric flags raised on the device by the iterations and read (and
 * cleared) by the synchronizing calls.  The first three are failures
 * (MBMD_ERR_NUMERIC); the last is a warning. */
typedef enum {
    MBMD_FLAG_NONFINITE = 1,    /* objective, g^T p, step denominator or step size not finite */
    MBMD_FLAG_NO_CURVATURE = 2, /* preconditioned step: the 1D majoriser's curvature
                                   sum_iE c q^2 + p^T R'' p is not positive for g^T p != 0
                                   (the step is skipped) */
    MBMD_FLAG_ASCENT = 4,       /* preconditioned step: g^T p > 0, i.e. M M^T is not positive
                                   semi-definite (the step alpha < 0 is still the majoriser's
                                   minimiser) */
    MBMD_FLAG_INCREASE = 8      /* the objective rose between consecutive evaluations of one run
                                   by more than 1e-5 relative (SPS decreases it monotonically when
                                   every line integral stays >= 0, which is not enforced) */
} mbmd_numeric_flags;

typedef enum {
    MBMD_PENALTY_QUADRATIC = 0, /* R = 1/2 x^T (beta (x) Gamma) x */
    MBMD_PENALTY_HUBER = 1      /* R = beta sum_pairs psi_delta(x_j - x_j'), one material */
} mbmd_penalty_kind;

/*
 * 2D geometry.  The projector is distance-driven; the paper only calls A
 * "the forward projector" (standard-CT and one-step MBMD sections), so the
 * model is fixed here:
 *   pixel centre   ((ix-(nx-1)/2) dx, (iy-(ny-1)/2) dy)      [mm]
 *   view angle     theta_v = theta0 + v dtheta                 [rad]
 *   detector axis  e = (cos theta, sin theta); central ray d = (-sin, cos)
 *   bin centre     u_b = (b-(n_bins-1)/2) du + u_offset        [mm]
 *   parallel ray   { u e + s d };  flat-fan ray from -dso d through
 *                  (dsd - dso) d + u e
 * Per view the sweep lines are the rows when |cos theta| >= |sin theta|
 * (decided in FP64 on the host), else the columns; on each line the weight
 * of a pixel is the overlap of the pixel with the bin footprint (cut by the
 * bin's two boundary rays), divided by the footprint width, times the line
 * spacing over |cos| of the bin-centre ray's angle to the line normal.
 * For MBMD_GEOM_IDENTITY, nx must equal n_bins and ny n_views, and the
 * other fields are ignored.
 */
typedef struct {
    int kind;                   /* mbmd_geom_kind */
    int nx, ny;                 /* image size (pixels) */
    double dx, dy;              /* pixel size (mm) */
    int n_views;
    double theta0, dtheta;      /* first view angle and increment (rad) */
    int n_bins;
    double du, u_offset;        /* bin pitch and detector offset (mm) */
    double dso, dsd;            /* source-isocentre and source-detector (mm), fan only */
} mbmd_geometry;

/* Spectral model (one-step MBMD section): Q and S are host FP64 arrays,
 * copied at problem creation.  Limits: n_mat <= 4, n_chan <= 8,
 * n_energy <= 256. */
typedef struct {
    int n_mat, n_energy, n_chan;
    const double* Q_host;       /* [n_energy][n_mat] attenuation per unit of x */
    const double* S_host;       /* [n_chan][n_energy] sensitivity incl. gain and I0 */
} mbmd_spectral;

/* Roughness penalty (eq:quadraticSmoothess, quadReg_summation): 4-neighbour
 * graph Laplacian Gamma with out-of-image neighbours dropped.  beta is a
 * host [n_mat][n_mat] symmetric positive semi-definite matrix.  Huber needs
 * n_mat == 1 and delta > 0. */
typedef struct {
    int kind;                   /* mbmd_penalty_kind */
    const double* beta_host;    /* [n_mat][n_mat] */
    double delta;               /* Huber threshold (units of x) */
} mbmd_penalty;

typedef struct mbmd_problem mbmd_problem;
typedef struct mbmd_batch mbmd_batch;

/* ---------------------------------------------------------------- projector */

/*
 * sino_dev[m] = A x_dev[m] for m < n_mat  (forward projection, the A of
 * eq:meanModel in the standard-CT and one-step MBMD sections).
 * x_dev: [n_mat][ny][nx]; sino_dev: [n_mat][n_views][n_bins]; 1 <= n_mat <= 4.
 * Geometry tables are built on the first call with a given geometry on a
 * given device and stream and cached there (see the conventions above):
 * calls on different streams have separate scratch and may overlap.
 * Errors: MBMD_ERR_ARG (NULL pointer, bad sizes), MBMD_ERR_SHAPE (fan source
 * inside the image circle or between the sweep lines of a view, a bin
 * boundary parallel to the sweep lines, n_mat out of range), MBMD_ERR_HIP.
 */
int mbmd_project(const mbmd_geometry* geom, const float* x_dev, float* sino_dev,
                 int n_mat, void* stream);

/*
 * x_dev[m] = A^T sino_dev[m] for m < n_ch (matched back projection with the
 * same weights; pixel-driven, deterministic, FP64 sums over views).
 * sino_dev: [n_ch][n_views][n_bins]; x_dev: [n_ch][ny][nx] (overwritten);
 * 1 <= n_ch <= 10.  Each view's cumulative detector integral is FP64; from
 * three channels on, groups of three hold it as 48-bit fixed point relative
 * to its own range (within 2^-47 of that range, far below the FP32 widths'
 * rounding), so that one pair of loads serves three channels.  A channel's
 * result does not depend on the other channels' data.  Same caching and errors
 * as mbmd_project.
 */
int mbmd_backproject(const mbmd_geometry* geom, const float* sino_dev, float* x_dev,
                     int n_ch, void* stream);

/* Device bytes of the allocation-free projector's array (per device). */
#define MBMD_NOALLOC_SCRATCH_BYTES (32u << 20)

/*
 * mbmd_project for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.  Same
 * arguments, result and errors as mbmd_project (bit for bit the same kernels),
 * but the projector's tables and line-prefix scratch live in a static device
 * array of MBMD_NOALLOC_SCRATCH_BYTES per device, held until the process ends;
 * the call allocates no device memory.  The array keeps the tables of the last
 * geometry used on the device: a call with another geometry builds that
 * geometry's tables on the host, waits for the device and uploads them
 * (so it is not capturable); later calls with the same geometry only enqueue
 * two kernels on `stream`.  Every call on a device shares its array: calls
 * that overlap on one device race.
 * Errors: those of mbmd_project, and MBMD_ERR_SHAPE when the geometry's tables
 * and scratch (for up to 4 materials) exceed the array.
 */
int mbmd_project_noalloc(const mbmd_geometry* geom, const float* x_dev, float* sino_dev,
                         int n_mat, void* stream);

/*
 * Number of nonzeros of A (pairs of a ray and a pixel with a positive
 * footprint overlap), counted on the device from the projector's own tables;
 * the unit of work of one projection.  Synchronizes `stream`.
 */
int mbmd_projector_nnz(const mbmd_geometry* geom, long long* nnz_host, void* stream);

/* ---------------------------------------------------------------- problems */

/*
 * Device bytes a problem with this geometry and spectral model needs
 * (flags: 0 or MBMD_WORKSPACE_BLUR); the descriptors' table pointers are not
 * read.  Errors: MBMD_ERR_ARG (NULL, unknown flag), MBMD_ERR_SHAPE.
 */
int mbmd_workspace_bytes(const mbmd_geometry* geom, const mbmd_spectral* spectral, int flags,
                         size_t* bytes_host);

/*
 * Create a problem (the estimation problem of eq:mapEstimator with the mean
 * model of eq:meanModel): copies the descriptors, y_dev and w_dev
 * ([n_chan][n_views][n_bins]; w = inverse variance, or NULL for
 * w = 1/max(y, 1)), builds the projector tables in FP64 on the host, and
 * computes A 1 (the gamma of the SPS section).
 *   - workspace_dev: NULL, or caller-owned device memory of workspace_bytes
 *     >= mbmd_workspace_bytes(geom, spectral, flags), 256-byte aligned, that
 *     holds the problem's whole device state until mbmd_problem_destroy (the
 *     library then allocates no device memory for the problem).  NULL: the
 *     library allocates that block itself and frees it at destroy.
 *   - flags: 0 or MBMD_WORKSPACE_BLUR (the blur's buffers are part of the
 *     block; without it a blur needs library memory, so mbmd_problem_set_blur
 *     fails on a caller workspace).
 * Synchronizes `stream` before returning.  Errors: MBMD_ERR_ARG (NULL,
 * workspace too small or misaligned, unknown flag), MBMD_ERR_SHAPE (limits
 * above; identity geometry with nx != n_bins or ny != n_views), MBMD_ERR_HIP.
 */
int mbmd_problem_create(const mbmd_geometry* geom, const mbmd_spectral* spectral,
                        const mbmd_penalty* penalty, const float* y_dev, const float* w_dev,
                        void* workspace_dev, size_t workspace_bytes, int flags, void* stream,
                        mbmd_problem** out);

/* Free a problem (synchronizes its last stream; a caller workspace is then
 * the caller's again). NULL is ignored. */
void mbmd_problem_destroy(mbmd_problem* prob);

/*
 * Synchronizes `stream`, writes the numeric flags raised since they were
 * last read into *flags_host (may be NULL) and clears them.  Returns
 * MBMD_ERR_NUMERIC when a failure bit (MBMD_FLAG_NONFINITE,
 * MBMD_FLAG_NO_CURVATURE, MBMD_FLAG_ASCENT) was among them, MBMD_OK
 * otherwise (MBMD_FLAG_INCREASE alone is a warning).
 */
int mbmd_problem_check(mbmd_problem* prob, int* flags_host, void* stream);

/*
 * Build preconditioner `kind` ("Preconditioned Optimization" and the
 * Fourier, modified Fourier, wavelet and cross-material sections):
 *   - Fisher weights with a data-based D (one energy: D = y / I0; several:
 *     a water-only per-ray Gauss-Newton estimate, the first material playing
 *     water);
 *   - M0_j = Htilde_j^-1/2 from the material columns (F + R) 1_k
 *     (eigenvalues floored at 1e-6 of each block's largest; a pixel no ray
 *     sees gets M0_j = 0);
 *   - FOURIER: impulse response of M0 H M0 at (ny/2, nx/2) per material, DFT
 *     with the phase removed, real part, symmetrised per-frequency blocks,
 *     eigenvalues floored at 1e-2 of the largest over all frequencies;
 *   - HAAR: response to U^T 1 per material, Haar-transformed; same floor;
 *   - DAUB4: the same with the periodised orthonormal Daubechies-4 transform
 *     (the other unitary wavelet the wavelet section names);
 *   - BLOCKDIAG: M0 only.
 * The composition is M = M0 U^H L^-1/2 U (the paper's symmetric sandwich
 * M0^T U^T L^-1/2 U M0 does not whiten M0^T H M0).  Huber problems build
 * with the quadratic Hessian beta Gamma.  FOURIER, HAAR and DAUB4 need nx
 * and ny powers of two (HAAR, DAUB4: nx == ny) and a projector geometry.
 * Errors: MBMD_ERR_ARG, MBMD_ERR_SHAPE, MBMD_ERR_UNSUPPORTED, MBMD_ERR_HIP.
 */
int mbmd_precond_build(mbmd_problem* prob, int kind, void* stream);

/*
 * mbmd_precond_build with options ("Preconditioned Optimization": D
 * approximates the transmission at the solution, and the modified
 * preconditioners differ from the plain ones by M0):
 *   - flags: 0, or MBMD_PRECOND_UNMODIFIED for M0 = I (FOURIER then is
 *     U^H L^-1/2 U with L from the bare Hessian's impulse response; HAAR
 *     likewise; BLOCKDIAG is then no preconditioning);
 *   - x_ref_dev: NULL for the data-based D above, or a device image
 *     [n_mat][ny][nx] (FP32, caller-owned, read only during the call) whose
 *     transmission D = exp(-AA x_ref) replaces it -- the Fisher information
 *     at an iterate, for rebuilding the preconditioner during the iterations.
 * The Fisher weights and M0 are shared by the problem's preconditioners, so
 * any call with options (and the next plain mbmd_precond_build after one)
 * voids the others: apply or iterate with them only after building them
 * again (MBMD_ERR_NOT_BUILT otherwise).  Uses the problem's scratch between
 * runs; asynchronous on `stream` like the other calls.
 * Errors: as mbmd_precond_build, and MBMD_ERR_ARG for an unknown flag.
 */
int mbmd_precond_build_ex(mbmd_problem* prob, int kind, int flags, const float* x_ref_dev, void* stream);

/* Largest half width of a projection-domain blur (9 taps). */
#define MBMD_MAX_BLUR_HALF 4

/*
 * Projection-domain blur (the operator B of the standard-CT,
 * projection-domain and one-step MBMD models: the mean becomes
 * ybar = B S exp(-AA x), e.g. focal spot and detector blur).  Per channel c,
 * along the bins of each view: (B_c z)_b = sum_{|d|<=h} taps[c][d + h]
 * z_{b+d}, bins beyond the detector dropped.
 *   - taps_host: host array [n_chan][2 h + 1] (copied; non-negative and
 *     finite, so that the decoupled SPS surrogate still majorises);
 *   - half_width h: 1..MBMD_MAX_BLUR_HALF, or 0 to remove the blur (taps may
 *     then be NULL).
 * Every later call uses it: the objective, gradient, SPS iterations
 * (eta = BB^T W BB 1 and rho = BB^T W (ybar - y) - eta t of the SPS
 * section, so the one-energy curvature is recomputed every iteration), the
 * forward model and its VJP, and the preconditioner builds (Fisher
 * information A^T J^T B^T W B J A; the data-based D ignores the blur).  It
 * voids every preconditioner built before it.  Its buffers, (3 + n_mat)
 * n_chan n_rays floats, are part of the problem's block when it was sized
 * with MBMD_WORKSPACE_BLUR; otherwise the first call with h > 0 allocates
 * them (library-owned block only), freed by mbmd_problem_destroy.
 * Asynchronous on `stream`.
 * Errors: MBMD_ERR_ARG (NULL problem, h out of range, NULL, negative or
 * non-finite taps), MBMD_ERR_UNSUPPORTED (identity geometry, whose rays the
 * blur would couple; a caller workspace sized without MBMD_WORKSPACE_BLUR),
 * MBMD_ERR_HIP.
 */
int mbmd_problem_set_blur(mbmd_problem* prob, const float* taps_host, int half_width, void* stream);

/*
 * out_dev = M M^T g_dev for a built preconditioner (the direction operator
 * of the preconditioned SPS step, without its minus sign); for
 * MBMD_PRECOND_NONE out = g.  Both [n_mat][ny][nx], distinct buffers.
 * Errors: MBMD_ERR_NOT_BUILT, MBMD_ERR_ARG, MBMD_ERR_HIP.
 */
int mbmd_precond_apply(mbmd_problem* prob, int kind, const float* g_dev, float* out_dev,
                       void* stream);

/*
 * Gradient and SPS curvature of Phi at x_dev (SPS section):
 *   grad = (Q (x) A)^T(-eta t^2 - rho t) + dR/dx
 *        = A^T [sum_E Q_Ek (-t_E sum_c S_cE w_c (ybar_c - y_c))] + dR/dx,
 *   curv = A^T [sum_E Q_Ek gamma_E c_E] + d_R   (the separable surrogate
 *          Hessian diagonal, c_E = max(2 eta_E + rho_E, 0)),
 * with rho read as S^T W (ybar - y) - eta t (the printed x^(n) stands for
 * t^(n)).  grad_dev, curv_dev: [n_mat][ny][nx]; curv_dev and
 * objective_host (Phi(x), FP64) may be NULL.  With objective_host the call
 * synchronizes and returns MBMD_ERR_NUMERIC when Phi is not finite or an
 * earlier call raised a numeric failure flag.
 */
int mbmd_gradient(mbmd_problem* prob, const float* x_dev, float* grad_dev, float* curv_dev,
                  double* objective_host, void* stream);

/*
 * Run n_iter SPS iterations in place on x_dev ([n_mat][ny][nx]).
 *   NONE: x <- x - (g + dR)/(d + d_R) (the SPS update);
 *   others: p = -M M^T grad Phi(x), q = (Q (x) A) p,
 *           alpha = -g^T p / (sum_iE c_iE q_iE^2 + p^T R'' p),  x <- x + alpha p
 *   (unit curvature in x' = M^-1 x, then the exact minimiser of the 1D
 *   majoriser built from the same maximum curvatures; for the identity
 *   geometry without penalty alpha is per ray).  Line integrals A x are
 *   carried across iterations and recomputed every 25.  Reductions are FP64
 *   and alpha stays on the device.
 * objective_trace_host: NULL, or n_iter+1 doubles receiving Phi before each
 * iteration and after the last (synchronizes, and returns MBMD_ERR_NUMERIC
 * when a numeric failure flag was raised).  Without a trace the call only
 * enqueues; its flags are read by the next synchronizing call.
 */
int mbmd_sps_step(mbmd_problem* prob, float* x_dev, int precond, int n_iter,
                  double* objective_trace_host, void* stream);

/*
 * Polyenergetic forward model: ybar_dev [n_chan][V][B] = S exp(-(Q (x) A) x);
 * l_dev (NULL allowed) receives A x [n_mat][V][B] for mbmd_forward_vjp.
 */
int mbmd_forward(mbmd_problem* prob, const float* x_dev, float* ybar_dev, float* l_dev,
                 void* stream);

/*
 * Backward of mbmd_forward: dx_dev [n_mat][ny][nx] =
 *   A^T [ sum_E Q_Ek (-t_E) sum_c S_cE gbar_c ],  t_E = exp(-sum_k Q_Ek l_k),
 * recomputing the energy sums from l_dev = A x (no ray x energy tensor is
 * stored).  gbar_dev: [n_chan][V][B].
 */
int mbmd_forward_vjp(mbmd_problem* prob, const float* l_dev, const float* gbar_dev,
                     float* dx_dev, void* stream);

/* ---------------------------------------------------------------- batches */

/* Flags of mbmd_batch_create. */
typedef enum {
    MBMD_BATCH_SEPARATE_LAUNCHES = 1  /* every problem its own launches (no shared launches) */
} mbmd_batch_flags;

/* Device bytes of a batch of n problems (its table of per-slice offsets). */
int mbmd_batch_workspace_bytes(mbmd_problem* const* probs, int n, size_t* bytes_host);

/*
 * Group problems (uneven sizes allowed, all on the current device) for a
 * batched iteration (the serving form of the one-step MBMD iteration: many
 * slices per call).  The problems are borrowed and must outlive the batch.
 * Problems whose launch parameters are all equal -- same geometry, sizes,
 * penalty kind, blur taps and block layout (same workspace flags, every
 * buffer inside the block) -- form a class: every kernel of an iteration runs
 * once per class, each workgroup working on one member (the per-member byte
 * offsets of the problem blocks and images live in the batch's workspace).  A
 * problem whose blur buffers were grown outside its block (a library block
 * created without MBMD_WORKSPACE_BLUR) gets launches of its own.  Classes and
 * lone problems are dealt round-robin onto up to 4 library-owned streams
 * (default priority) forked from the caller's stream and joined back into it.
 *   - workspace_dev: NULL (the library allocates) or caller-owned device memory
 *     of mbmd_batch_workspace_bytes, 256-byte aligned, kept until destroy;
 *   - flags: 0 or MBMD_BATCH_SEPARATE_LAUNCHES.
 * Errors: MBMD_ERR_ARG (NULL, a problem twice, workspace too small, unknown
 * flag), MBMD_ERR_UNSUPPORTED (identity geometry), MBMD_ERR_HIP.
 */
int mbmd_batch_create(mbmd_problem* const* probs, int n, void* workspace_dev, size_t workspace_bytes,
                      int flags, mbmd_batch** out);
void mbmd_batch_destroy(mbmd_batch* batch);

/*
 * n_iter iterations of every problem of the batch (x_dev[i] belongs to
 * problem i; distinct images; a preconditioner kind every problem has
 * built).  Each problem's iterates are bit for bit those of mbmd_sps_step
 * on that problem alone with the same n_iter (every call starts from x).
 * use_graph != 0 captures one iteration over all problems in a hipGraph on
 * the first call (classes and lone problems as parallel branches) and
 * replays it on `stream`; other x pointers, another preconditioner kind or
 * a member problem's blur set since the capture (mbmd_problem_set_blur) make
 * the call capture again.  Preconditioner tables rebuilt in place need no
 * new capture: a replay reads them as they are.  use_graph == 0 enqueues
 * every iteration of each class or lone problem on its stream.  Either way
 * the work is ordered after what `stream` held before the call and before
 * what it receives after it.  No objective trace; each problem's numeric
 * flags are read by mbmd_problem_check.
 * Errors: MBMD_ERR_ARG (NULL, unknown preconditioner), MBMD_ERR_NOT_BUILT,
 * MBMD_ERR_UNSUPPORTED, MBMD_ERR_HIP.
 */
int mbmd_batch_sps_step(mbmd_batch* batch, float* const* x_dev, int precond, int n_iter,
                        int use_graph, void* stream);

/* ---------------------------------------------------------------- timing */

/*
 * Per-kernel timing for callers that measure the library (benchmarks,
 * roofline reports).  While enabled, every kernel launch of the library is
 * bracketed by two hipEvents recorded on the stream it is launched on
 * (launches enqueued during graph capture are not instrumented).
 * mbmd_profile_query waits for the recorded events and returns, for the
 * kernel named `kernel` (e.g. "k_dd_back"), the number of instrumented
 * launches and their summed duration in ms since the last reset.
 * mbmd_profile_kernels writes the comma-separated names seen so far into
 * `names` (capacity bytes, NUL-terminated).  mbmd_profile_select restricts
 * the instrumentation to a comma-separated list of kernel names (NULL or ""
 * = every kernel), so that a timed region carries only the events it needs.
 * Errors: MBMD_ERR_ARG, MBMD_ERR_HIP.
 */
int mbmd_profile_enable(int on);
int mbmd_profile_select(const char* names);
int mbmd_profile_reset(void);
int mbmd_profile_query(const char* kernel, long long* launches, double* total_ms);
int mbmd_profile_kernels(char* names, size_t capacity);

/* ---------------------------------------------------------------- misc */

const char* mbmd_status_string(int status);
const char* mbmd_last_error(void);
int mbmd_version(void);
/* Frees the cached tables of the standalone projector calls on every device
 * (waits for the devices).  Safe to call at any time; the next call rebuilds. */
int mbmd_cache_clear(void);

#ifdef __cplusplus
}
#endif

#endif /* MBMD_H */
