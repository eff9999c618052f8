/*
 * gd_oracle.c -- plain, slow FP64 CPU reference for the deconvolution solve.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or
 * calls this file; it exists so the GPU library can be checked against an
 * implementation simple enough to verify by eye against the paper.  It shares
 * no code, header or constant table with the GPU library.
 *
 * What it computes (San & Vedula, "Generalized deconvolution procedure for
 * structural modeling of turbulence"):
 *   - the approximate-deconvolution problem G u = ubar, Eq. (tau3) of Sec. 3;
 *   - G: by default the separable periodic 3-point trapezoidal filter,
 *     weights (1/4, 1/2, 1/4) per axis, written as the direct 9-point (2D) or
 *     27-point (3D) sum.  The paper leaves G free (Sec. 4 opening) and uses a
 *     spectral differential filter (Sec. 4, Eq. df); or_solve_with takes any
 *     filter as a callback, and the Python side passes that one, applied
 *     through the FFT as the paper does.
 *   - Van Cittert / Richardson iteration, Algorithm 1 (Eqs. adm2, res, ric);
 *   - steepest descent, Algorithm 2 (Eqs. sd, sd-a);
 *   - conjugate gradient, Algorithm 3 (Eqs. cg1 - cg-b);
 *   - BiCGSTAB, Algorithm 4;
 *   - the inner product (a, b) = integral of a*b dx, Eq. (inner), discretised
 *     as h^d * sum_i a_i b_i;
 *   - relative residuals normalised by the initial residual (Sec. 4.1 text
 *     on the residual history, Table 1 caption).
 *
 * Readings where the paper is silent (kept identical on the GPU side):
 *   - N counts loop passes of the algorithms, so Van Cittert from u0 = ubar
 *     after N passes equals sum_{n=0..N} (I-G)^n ubar.
 *   - Stopping: after each completed pass, stop when ||r_n|| <= tol * r_ref
 *     (tol > 0) or when n reaches N.  r_ref = ||ubar - G ubar|| by default,
 *     or ||ubar||.
 *   - Guards: r_ref == 0 -> ZERO_REF (u = u0, 0 passes); ||r0|| == 0 ->
 *     CONVERGED after 0 passes; a zero denominator in alpha -> BREAKDOWN_RHO;
 *     BiCGSTAB: ||s|| <= tol*r_ref (or s == 0) -> take the half step
 *     u += alpha p, r = s and stop CONVERGED; (t,t) == 0 otherwise ->
 *     BREAKDOWN_OMEGA; any non-finite scalar -> NONFINITE.
 *
 * Summation: dot products use Neumaier-compensated summation by default
 * (sum_mode 0).  sum_mode 1 is plain forward summation and sum_mode 2 is
 * pairwise summation; they exist only to measure the oracle's own rounding
 * sensitivity.  sum_mode 3 is the timed mode's: a fixed number of chunks,
 * each Neumaier-summed, then the chunk sums Neumaier-summed in chunk order.
 *
 * Threads (or_set_threads): only for timing on the host's cores.  The filter
 * and vector loops split over points, which changes no result; with more than
 * one thread the dot products must use sum_mode 3, whose chunks do not depend
 * on the thread count, so any thread count gives bitwise the same result.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int or_nthreads = 1;

/* Threads the loops may use (1 = serial); returns the count in effect. */
int or_set_threads(int n)
{
#ifdef _OPENMP
    or_nthreads = n < 1 ? 1 : n;
#else
    (void)n;
    or_nthreads = 1;
#endif
    return or_nthreads;
}

/* Logical processors the host offers (1 without OpenMP). */
int or_host_procs(void)
{
#ifdef _OPENMP
    return omp_get_num_procs();
#else
    return 1;
#endif
}

#define OR_PAR _Pragma("omp parallel for num_threads(or_nthreads) schedule(static) if (or_nthreads > 1)")

/* status values, documented in the library header with the same numbers */
enum {
    OR_CONVERGED = 0,
    OR_MAXITER = 1,
    OR_BREAKDOWN_RHO = 2,
    OR_BREAKDOWN_OMEGA = 3,
    OR_NONFINITE = 4,
    OR_ZERO_REF = 5
};
enum { OR_VC = 0, OR_CG = 1, OR_BICGSTAB = 2, OR_SD = 3 };
enum { OR_INIT_UBAR = 0, OR_INIT_ZERO = 1, OR_INIT_GIVEN = 2 };
enum { OR_REF_R0UBAR = 0, OR_REF_UBAR = 1 };

typedef struct {
    int32_t iters;
    int32_t status;
    double r_ref;
    double r0;
    double r_final;
    double r_true;
} or_info;

static int64_t wrap(int64_t i, int64_t n)
{
    int64_t m = i % n;
    return m < 0 ? m + n : m;
}

/* y = G x on an nx*ny(*nz) periodic grid, x fastest. ndim 2 ignores nz. */
void or_filter(int ndim, int64_t nx, int64_t ny, int64_t nz, const double *x, double *y)
{
    const double w[3] = {0.25, 0.5, 0.25};
    if (ndim == 2) {
        OR_PAR
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                double s = 0.0;
                for (int b = -1; b <= 1; ++b)
                    for (int a = -1; a <= 1; ++a)
                        s += w[b + 1] * w[a + 1] * x[wrap(j + b, ny) * nx + wrap(i + a, nx)];
                y[j * nx + i] = s;
            }
        return;
    }
    OR_PAR
    for (int64_t k = 0; k < nz; ++k)
        for (int64_t j = 0; j < ny; ++j)
            for (int64_t i = 0; i < nx; ++i) {
                double s = 0.0;
                for (int c = -1; c <= 1; ++c)
                    for (int b = -1; b <= 1; ++b)
                        for (int a = -1; a <= 1; ++a)
                            s += w[c + 1] * w[b + 1] * w[a + 1] *
                                 x[(wrap(k + c, nz) * ny + wrap(j + b, ny)) * nx + wrap(i + a, nx)];
                y[(k * ny + j) * nx + i] = s;
            }
}

static double sum_pairwise(const double *a, const double *b, int64_t n)
{
    if (n <= 8) {
        double s = 0.0;
        for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
        return s;
    }
    int64_t h = n / 2;
    return sum_pairwise(a, b, h) + sum_pairwise(a + h, b + h, n - h);
}

/* Neumaier-compensated sum of a_i b_i over [lo, hi) */
static double sum_neumaier(const double *a, const double *b, int64_t lo, int64_t hi)
{
    double s = 0.0, c = 0.0;
    for (int64_t i = lo; i < hi; ++i) {
        double v = a[i] * b[i];
        double t = s + v;
        if (fabs(s) >= fabs(v)) c += (s - t) + v;
        else c += (v - t) + s;
        s = t;
    }
    return s + c;
}

#define OR_CHUNKS 256

/* (a, b) = hw * sum_i a_i b_i, hw = h_x h_y (h_z) */
double or_dot(const double *a, const double *b, int64_t n, double hw, int sum_mode)
{
    double s = 0.0;
    if (sum_mode == 3) {
        double part[OR_CHUNKS];
        OR_PAR
        for (int k = 0; k < OR_CHUNKS; ++k) part[k] = sum_neumaier(a, b, n * k / OR_CHUNKS, n * (k + 1) / OR_CHUNKS);
        double c = 0.0;
        for (int k = 0; k < OR_CHUNKS; ++k) {
            double t = s + part[k];
            if (fabs(s) >= fabs(part[k])) c += (s - t) + part[k];
            else c += (part[k] - t) + s;
            s = t;
        }
        s += c;
    } else if (sum_mode == 1) {
        for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    } else if (sum_mode == 2) {
        s = sum_pairwise(a, b, n);
    } else {
        s = sum_neumaier(a, b, 0, n);
    }
    return hw * s;
}

/* A filter given by the caller: y = G x over one field of n points. */
typedef void (*or_apply_fn)(const double *x, double *y);

typedef struct {
    int ndim;
    int64_t nx, ny, nz, n;
    double hw;
    int sum_mode;
    or_apply_fn apply;  /* NULL: the trapezoidal stencil */
} grid_t;

static void G(const grid_t *g, const double *x, double *y)
{
    if (g->apply) g->apply(x, y);
    else or_filter(g->ndim, g->nx, g->ny, g->nz, x, y);
}
static double dot(const grid_t *g, const double *a, const double *b) { return or_dot(a, b, g->n, g->hw, g->sum_mode); }

/* ||ubar - G x|| */
static double resnorm(const grid_t *g, const double *ubar, const double *x, double *tmp)
{
    G(g, x, tmp);
    OR_PAR
    for (int64_t i = 0; i < g->n; ++i) tmp[i] = ubar[i] - tmp[i];
    return sqrt(dot(g, tmp, tmp));
}

/* Decide whether to stop after `n` completed passes with residual norm rn. */
static int stop_check(double rn, double tol, double r_ref, int n, int max_iter, int *status)
{
    if (!isfinite(rn)) { *status = OR_NONFINITE; return 1; }
    if (rn == 0.0 || (tol > 0.0 && rn <= tol * r_ref)) { *status = OR_CONVERGED; return 1; }
    if (n >= max_iter) { *status = OR_MAXITER; return 1; }
    return 0;
}

/*
 * Solve G u = ubar with one of the four methods.
 *   u:    on entry the initial guess when init == OR_INIT_GIVEN; on exit the
 *         result.  Length n.
 *   hist: NULL or max_iter+1 doubles; hist[k] = ||r_k|| for k <= iters.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int or_solve_with(int solver, int ndim, int64_t nx, int64_t ny, int64_t nz, double hw,
                  const double *ubar, double *u, int max_iter, double tol, int init,
                  int norm_ref, int sum_mode, double *hist, or_info *info, or_apply_fn apply)
{
    if ((ndim != 2 && ndim != 3) || nx < 1 || ny < 1 || (ndim == 3 && nz < 1) || max_iter < 0)
        return -1;
    if (or_nthreads > 1 && sum_mode != 3) return -1; /* only the chunked sums are thread-count independent */
    grid_t g = {ndim, nx, ny, ndim == 3 ? nz : 1, 0, hw, sum_mode, apply};
    g.n = g.nx * g.ny * g.nz;
    const int64_t n = g.n;
    double *r = calloc(n, sizeof(double)), *d = calloc(n, sizeof(double));
    double *p = calloc(n, sizeof(double)), *q = calloc(n, sizeof(double));
    double *f0 = calloc(n, sizeof(double)), *s = calloc(n, sizeof(double));
    double *t = calloc(n, sizeof(double));
    if (!r || !d || !p || !q || !f0 || !s || !t) {
        free(r); free(d); free(p); free(q); free(f0); free(s); free(t);
        return -1;
    }

    /* reference norm */
    double r_ref = norm_ref == OR_REF_UBAR ? sqrt(dot(&g, ubar, ubar)) : resnorm(&g, ubar, ubar, d);

    /* initial guess (Algorithms 1-4 use u0 = ubar) and initial residual */
    if (init == OR_INIT_UBAR) memcpy(u, ubar, n * sizeof(double));
    else if (init == OR_INIT_ZERO) memset(u, 0, n * sizeof(double));
    G(&g, u, d);
    OR_PAR
    for (int64_t i = 0; i < n; ++i) r[i] = ubar[i] - d[i];
    double rr = dot(&g, r, r);
    double r0 = sqrt(rr);
    if (hist) hist[0] = r0;

    int status = OR_MAXITER, iters = 0, stop = 0;
    if (!isfinite(r_ref)) { status = OR_NONFINITE; stop = 1; }
    else if (r_ref == 0.0) { status = OR_ZERO_REF; stop = 1; }
    else stop = stop_check(r0, tol, r_ref, 0, max_iter, &status);

    if (!stop && solver == OR_VC) {
        /* Algorithm 1 */
        while (iters < max_iter) {
            OR_PAR
            for (int64_t i = 0; i < n; ++i) u[i] += r[i];   /* u_{n+1} = u_n + r_n */
            G(&g, r, d);                                     /* d_n = G r_n */
            OR_PAR
            for (int64_t i = 0; i < n; ++i) r[i] -= d[i];    /* r_{n+1} = r_n - d_n */
            ++iters;
            rr = dot(&g, r, r);
            if (hist) hist[iters] = sqrt(rr);
            if (stop_check(sqrt(rr), tol, r_ref, iters, max_iter, &status)) break;
        }
    } else if (!stop && solver == OR_SD) {
        /* Algorithm 2 */
        while (iters < max_iter) {
            G(&g, r, d);                                     /* d_n = G r_n */
            double rd = dot(&g, r, d);
            if (!isfinite(rd)) { status = OR_NONFINITE; break; }
            if (rd == 0.0) { status = OR_BREAKDOWN_RHO; break; }
            double alpha = rr / rd;                          /* Eq. (sd-a) */
            OR_PAR
            for (int64_t i = 0; i < n; ++i) {
                u[i] += alpha * r[i];
                r[i] -= alpha * d[i];
            }
            ++iters;
            rr = dot(&g, r, r);
            if (hist) hist[iters] = sqrt(rr);
            if (stop_check(sqrt(rr), tol, r_ref, iters, max_iter, &status)) break;
        }
    } else if (!stop && solver == OR_CG) {
        /* Algorithm 3 */
        memcpy(p, r, n * sizeof(double));                   /* p_0 = r_0 */
        double rho = rr;                                     /* rho_0 = (r_0, r_0) */
        while (iters < max_iter) {
            G(&g, p, d);                                     /* d_n = G p_n */
            double pd = dot(&g, p, d);
            if (!isfinite(pd)) { status = OR_NONFINITE; break; }
            if (pd == 0.0) { status = OR_BREAKDOWN_RHO; break; }
            double alpha = rho / pd;
            OR_PAR
            for (int64_t i = 0; i < n; ++i) {
                u[i] += alpha * p[i];
                r[i] -= alpha * d[i];
            }
            ++iters;
            double rho_new = dot(&g, r, r);
            if (hist) hist[iters] = sqrt(rho_new);
            if (stop_check(sqrt(rho_new), tol, r_ref, iters, max_iter, &status)) break;
            double beta = rho_new / rho;
            OR_PAR
            for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
            rho = rho_new;
        }
    } else if (!stop && solver == OR_BICGSTAB) {
        /* Algorithm 4 */
        memcpy(f0, r, n * sizeof(double));                  /* frozen shadow residual */
        /* p_0 = q_0 = 0 (calloc) */
        double alpha = 1.0, omega = 1.0, rho = 1.0;
        double thr = tol > 0.0 ? tol * r_ref : 0.0;
        while (iters < max_iter) {
            double rho_new = dot(&g, f0, r);
            if (!isfinite(rho_new)) { status = OR_NONFINITE; break; }
            if (rho_new == 0.0) { status = OR_BREAKDOWN_RHO; break; }
            double beta = (alpha / omega) * (rho_new / rho);
            OR_PAR
            for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * (p[i] - omega * q[i]);
            G(&g, p, q);
            double fq = dot(&g, f0, q);
            if (!isfinite(fq)) { status = OR_NONFINITE; break; }
            if (fq == 0.0) { status = OR_BREAKDOWN_RHO; break; }
            alpha = rho_new / fq;
            OR_PAR
            for (int64_t i = 0; i < n; ++i) s[i] = r[i] - alpha * q[i];
            G(&g, s, t);
            double ss = dot(&g, s, s), st = dot(&g, s, t), tt = dot(&g, t, t);
            if (!isfinite(ss) || !isfinite(st) || !isfinite(tt)) { status = OR_NONFINITE; break; }
            int half = (ss == 0.0) || (sqrt(ss) <= thr);
            if (!half && tt == 0.0) { status = OR_BREAKDOWN_OMEGA; break; }
            omega = half ? 0.0 : st / tt;
            OR_PAR
            for (int64_t i = 0; i < n; ++i) {
                u[i] += alpha * p[i] + omega * s[i];
                r[i] = s[i] - omega * t[i];
            }
            rho = rho_new;
            ++iters;
            rr = dot(&g, r, r);
            if (hist) hist[iters] = sqrt(rr);
            if (half) { status = isfinite(rr) ? OR_CONVERGED : OR_NONFINITE; break; }
            if (stop_check(sqrt(rr), tol, r_ref, iters, max_iter, &status)) break;
        }
    }

    /* recursive residual at exit and the true residual ||ubar - G u|| */
    double r_final = sqrt(dot(&g, r, r));
    double r_true = resnorm(&g, ubar, u, d);
    if (info) {
        info->iters = iters;
        info->status = status;
        info->r_ref = r_ref;
        info->r0 = r0;
        info->r_final = r_final;
        info->r_true = r_true;
    }
    free(r); free(d); free(p); free(q); free(f0); free(s); free(t);
    return 0;
}

/* Algorithms 1-4 with the trapezoidal stencil as G. */
int or_solve(int solver, int ndim, int64_t nx, int64_t ny, int64_t nz, double hw,
             const double *ubar, double *u, int max_iter, double tol, int init,
             int norm_ref, int sum_mode, double *hist, or_info *info)
{
    return or_solve_with(solver, ndim, nx, ny, nz, hw, ubar, u, max_iter, tol, init, norm_ref, sum_mode, hist,
                         info, NULL);
}
