/*
 * FP64 reference distance-driven projector (test infrastructure only).
 *
 * The paper leaves the system matrix A unspecified (it is "the forward
 * projector" of the standard-CT and one-step MBMD models, Methods,
 * "Standard CT Reconstruction" and "One-Step Reconstruction and Material
 * Decomposition").  This file fixes one: the 2D distance-driven model.
 *
 *   view angle      theta_v = theta0 + v dtheta
 *   detector axis   e = (cos theta, sin theta)
 *   central ray     d = (-sin theta, cos theta)
 *   bin centre      u_b = (b - (B-1)/2) du + u_offset, boundaries u_b -+ du/2
 *   parallel ray    { u e + s d }
 *   flat-fan ray    from S = -dso d through P(u) = (dsd - dso) d + u e
 *
 * Per view the sweep lines are the image rows when |cos theta| >= |sin theta|
 * and the columns otherwise.  For a row sweep, the two boundary rays of bin b
 * cut the line y = y_iy at x_a and x_b; with [lo, hi] = sorted(x_a, x_b) the
 * weight of pixel (ix, iy) is
 *     |[lo, hi] n [x_ix - dx/2, x_ix + dx/2]| / (hi - lo) * dy / |cos phi_b|
 * where phi_b is the angle between the bin-centre ray and the y axis.  The
 * column sweep is the same with x and y exchanged.  The identity geometry
 * is A = I.
 *
 * Everything is FP64 and written for clarity: one function lists the
 * (pixel, weight) pairs of one ray, and both the projector and its exact
 * transpose are built on it.  No code here is shared with the GPU library.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OG_PARALLEL = 0, OG_FAN = 1, OG_IDENTITY = 2 };

typedef struct {
    int kind, nx, ny, n_views, n_bins;
    double dx, dy, theta0, dtheta, du, u_offset, dso, dsd;
} ogeom;

/* Boundary-ray point/direction for detector coordinate u of view (c, s). */
static void ray_of(const ogeom* g, double c, double s, double u, double p[2], double r[2]) {
    const double ex = c, ey = s, dx = -s, dy = c;
    if (g->kind == OG_PARALLEL) {
        p[0] = u * ex; p[1] = u * ey;
        r[0] = dx; r[1] = dy;
    } else {
        const double sx = -g->dso * dx, sy = -g->dso * dy;
        const double qx = (g->dsd - g->dso) * dx + u * ex;
        const double qy = (g->dsd - g->dso) * dy + u * ey;
        p[0] = sx; p[1] = sy;
        r[0] = qx - sx; r[1] = qy - sy;
    }
}

/* 1 when view v sweeps image rows, 0 when it sweeps columns. */
int oracle_sweeps_rows(const ogeom* g, int v) {
    const double th = g->theta0 + v * g->dtheta;
    return fabs(cos(th)) >= fabs(sin(th));
}

/*
 * List the nonzeros of row (v, b) of A.  Writes at most `cap` pairs and
 * returns their number, or -1 when `cap` is too small or the ray runs
 * parallel to the sweep lines.
 */
int oracle_ray_weights(const ogeom* g, int v, int b, int* idx, double* wt, int cap) {
    if (g->kind == OG_IDENTITY) {
        if (cap < 1) return -1;
        idx[0] = v * g->n_bins + b;
        wt[0] = 1.0;
        return 1;
    }
    const double th = g->theta0 + v * g->dtheta;
    const double c = cos(th), s = sin(th);
    const int rows = fabs(c) >= fabs(s);
    const double uc = (b - (g->n_bins - 1) / 2.0) * g->du + g->u_offset;
    double pl[2], rl[2], ph[2], rh[2], pc[2], rc[2];
    ray_of(g, c, s, uc - 0.5 * g->du, pl, rl);
    ray_of(g, c, s, uc + 0.5 * g->du, ph, rh);
    ray_of(g, c, s, uc, pc, rc);
    /* a = sweep-normal axis (y for rows), t = along-line axis (x for rows) */
    const int ia = rows ? 1 : 0, it = rows ? 0 : 1;
    const int n_lines = rows ? g->ny : g->nx;
    const int n_along = rows ? g->nx : g->ny;
    const double d_line = rows ? g->dy : g->dx;
    const double d_along = rows ? g->dx : g->dy;
    const double rnorm = hypot(rc[0], rc[1]);
    if (fabs(rl[ia]) < 1e-12 * rnorm || fabs(rh[ia]) < 1e-12 * rnorm || fabs(rc[ia]) < 1e-12 * rnorm)
        return -1;
    const double path = d_line * rnorm / fabs(rc[ia]);   /* d_line / |cos phi_b| */
    int n = 0;
    for (int q = 0; q < n_lines; ++q) {
        const double a = (q - (n_lines - 1) / 2.0) * d_line;
        const double ta = pl[it] + (a - pl[ia]) * rl[it] / rl[ia];
        const double tb = ph[it] + (a - ph[ia]) * rh[it] / rh[ia];
        const double lo = ta < tb ? ta : tb;
        const double hi = ta < tb ? tb : ta;
        const double width = hi - lo;
        int k0 = (int)floor(lo / d_along + n_along / 2.0);
        int k1 = (int)floor(hi / d_along + n_along / 2.0);
        if (k0 < 0) k0 = 0;
        if (k1 > n_along - 1) k1 = n_along - 1;
        for (int k = k0; k <= k1; ++k) {
            const double e0 = (k - n_along / 2.0) * d_along;
            const double e1 = e0 + d_along;
            const double ov = (hi < e1 ? hi : e1) - (lo > e0 ? lo : e0);
            if (ov <= 0.0) continue;
            if (n >= cap) return -1;
            idx[n] = rows ? q * g->nx + k : k * g->nx + q;
            wt[n] = ov / width * path;
            ++n;
        }
    }
    return n;
}

static int ray_capacity(const ogeom* g) {
    return (g->nx + 2) * (g->ny + 2);
}

/* Threads for one projector call: about one per 2e5 ray-pixel steps, so that
 * small geometries run on one thread (waking a team costs more than their
 * work), capped by oracle_set_threads. */
static int threads_for(const ogeom* g) {
    int nt = 1;
#ifdef _OPENMP
    const double work = (double)g->n_views * g->n_bins * (g->nx > g->ny ? g->nx : g->ny);
    nt = (int)(work / 2e5) + 1;
    if (nt > omp_get_max_threads()) nt = omp_get_max_threads();
#endif
    return nt;
}

/* sino[m][v][b] = sum_j A[(v,b), j] x[m][j] for n_mat images. Returns 0 or -1. */
int oracle_project(const ogeom* g, const double* x, double* sino, int n_mat) {
    const int V = g->n_views, B = g->n_bins, nj = g->nx * g->ny;
    int err = 0;
#pragma omp parallel num_threads(threads_for(g))
    {
        const int cap = ray_capacity(g);
        int* idx = (int*)malloc(sizeof(int) * cap);
        double* wt = (double*)malloc(sizeof(double) * cap);
#pragma omp for schedule(static)
        for (int v = 0; v < V; ++v) {
            for (int b = 0; b < B; ++b) {
                const int n = oracle_ray_weights(g, v, b, idx, wt, cap);
                if (n < 0) { err = -1; continue; }
                for (int m = 0; m < n_mat; ++m) {
                    double acc = 0.0;
                    for (int t = 0; t < n; ++t) acc += wt[t] * x[(size_t)m * nj + idx[t]];
                    sino[((size_t)m * V + v) * B + b] = acc;
                }
            }
        }
        free(idx);
        free(wt);
    }
    return err;
}

/* x[m][j] = sum_i A[i, j] sino[m][i] (exact transpose of oracle_project). */
int oracle_backproject(const ogeom* g, const double* sino, double* x, int n_mat) {
    const int V = g->n_views, B = g->n_bins, nj = g->nx * g->ny;
    const int nthreads = threads_for(g);
    double* part = (double*)calloc((size_t)nthreads * n_mat * nj, sizeof(double));
    if (!part) return -1;
    int err = 0;
#pragma omp parallel num_threads(nthreads)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* mine = part + (size_t)tid * n_mat * nj;
        const int cap = ray_capacity(g);
        int* idx = (int*)malloc(sizeof(int) * cap);
        double* wt = (double*)malloc(sizeof(double) * cap);
#pragma omp for schedule(static)
        for (int v = 0; v < V; ++v) {
            for (int b = 0; b < B; ++b) {
                const int n = oracle_ray_weights(g, v, b, idx, wt, cap);
                if (n < 0) { err = -1; continue; }
                for (int m = 0; m < n_mat; ++m) {
                    const double s = sino[((size_t)m * V + v) * B + b];
                    for (int t = 0; t < n; ++t) mine[(size_t)m * nj + idx[t]] += wt[t] * s;
                }
            }
        }
        free(idx);
        free(wt);
    }
    memset(x, 0, sizeof(double) * (size_t)n_mat * nj);
    for (int t = 0; t < nthreads; ++t)
        for (size_t j = 0; j < (size_t)n_mat * nj; ++j) x[j] += part[(size_t)t * n_mat * nj + j];
    free(part);
    return err;
}

/* Number of threads the projector loops may use (1 without OpenMP). */
int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
