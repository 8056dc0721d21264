/*
 * CPU FP64 oracle for restarted GMRES(m) on the discrete Poisson problem.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the HIP library.
 *
 * Plain, single-threaded, slow and meant to be checked against the paper by
 * eye:
 *   - operator: the zero-Dirichlet discrete Laplacian of Section 1.4
 *     (A u = f, A the discrete Laplacian with its boundary conditions), taken
 *     here with the sign that makes it positive definite, A = -lap_h, on the
 *     unit square / cube with h = 1/(N+1) per axis (5-point in 2D, 7-point in
 *     3D);
 *   - solver: GMRES(k) of Saad & Schultz as used in Section 1.3 -- minimise the
 *     residual over the Krylov space K_k(A, r0) built from r0 = b - A x0, then
 *     restart from the last iterate;
 *   - orthogonalisation: classical Gram-Schmidt applied twice (CGS2), or
 *     modified Gram-Schmidt as a cross-check;
 *   - least squares: Givens rotations on the Hessenberg matrix, then back
 *     substitution.
 * Readings where the paper is silent (tolerance relative to |b|, stop on the
 * Givens estimate and accept on the true residual, breakdown threshold,
 * iteration = one Arnoldi step) are stated at the point of use.
 *
 * Threads (for timing the oracle on every core of a host): the operator and
 * the vector updates split their loops over OpenMP threads; every dot
 * product is the sequential sum of fixed 4096-element chunks, each summed
 * in order, so the result does not depend on the thread count (bitwise).
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t status;             /* 0 converged (or fixed count done), 1 not converged, <0 error */
    int64_t iters;              /* Arnoldi steps (products A v) */
    int32_t cycles;             /* restart cycles started */
    double relres_init;         /* |b - A x0| / |b| */
    double relres_first_cycle;  /* true relative residual after the first cycle (E_k) */
    double relres_est;          /* last Givens estimate / |b| */
    double relres_true;         /* final true relative residual */
} or_stats;

/* Threads used by the loops below (1 by default). */
void or_set_threads(int32_t n)
{
    omp_set_num_threads(n > 0 ? n : 1);
}

/* (A u)_p = sum over axes of (2 u_p - u_{p-e} - u_{p+e}) / h_axis^2, u = 0
 * outside the interior.  Layout: index = (z*ny + y)*nx + x. */
void or_apply(int32_t dim, int64_t nx, int64_t ny, int64_t nz,
              const double *u, double *out)
{
    double hx = 1.0 / (double)(nx + 1), hy = 1.0 / (double)(ny + 1);
    double hz = 1.0 / (double)(nz + 1);
    double cx = 1.0 / (hx * hx), cy = 1.0 / (hy * hy), cz = 1.0 / (hz * hz);
    if (dim == 2) nz = 1;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int64_t z = 0; z < nz; ++z)
        for (int64_t y = 0; y < ny; ++y)
            for (int64_t x = 0; x < nx; ++x) {
                int64_t p = (z * ny + y) * nx + x;
                double c = u[p];
                double w = x > 0 ? u[p - 1] : 0.0;
                double e = x < nx - 1 ? u[p + 1] : 0.0;
                double s = y > 0 ? u[p - nx] : 0.0;
                double nn = y < ny - 1 ? u[p + nx] : 0.0;
                double acc = (2.0 * c - w - e) * cx + (2.0 * c - s - nn) * cy;
                if (dim == 3) {
                    double d = z > 0 ? u[p - nx * ny] : 0.0;
                    double t = z < nz - 1 ? u[p + nx * ny] : 0.0;
                    acc += (2.0 * c - d - t) * cz;
                }
                out[p] = acc;
            }
}

/* sum_i a_i b_i: the chunks of 4096 elements are summed in order, then the
 * chunk sums in order (the same result for any thread count). */
#define OR_CHUNK 4096
static double dot(int64_t n, const double *a, const double *b)
{
    int64_t nc = (n + OR_CHUNK - 1) / OR_CHUNK;
    double part_small[64];
    double *part = nc <= 64 ? part_small : (double *)malloc(sizeof(double) * (size_t)nc);
    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nc; ++c) {
        int64_t i1 = (c + 1) * OR_CHUNK < n ? (c + 1) * OR_CHUNK : n;
        double s = 0.0;
        for (int64_t i = c * OR_CHUNK; i < i1; ++i) s += a[i] * b[i];
        part[c] = s;
    }
    double s = 0.0;
    for (int64_t c = 0; c < nc; ++c) s += part[c];
    if (part != part_small) free(part);
    return s;
}

/* |b - A x| with Neumaier-compensated summation of the squares, and |b|. */
void or_residual_norm(int32_t dim, int64_t nx, int64_t ny, int64_t nz,
                      const double *b, const double *x, double *rnorm, double *bnorm)
{
    int64_t n = nx * ny * (dim == 3 ? nz : 1);
    double *ax = (double *)malloc(sizeof(double) * (size_t)n);
    or_apply(dim, nx, ny, nz, x, ax);
    double s = 0.0, comp = 0.0, sb = 0.0, compb = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double r = b[i] - ax[i];
        double v = r * r, t = s + v;
        comp += fabs(s) >= fabs(v) ? (s - t) + v : (v - t) + s;
        s = t;
        double vb = b[i] * b[i], tb = sb + vb;
        compb += fabs(sb) >= fabs(vb) ? (sb - tb) + vb : (vb - tb) + sb;
        sb = tb;
    }
    *rnorm = sqrt(s + comp);
    *bnorm = sqrt(sb + compb);
    free(ax);
}

/* One Arnoldi step: w holds A v_j on entry and the new unnormalised direction on
 * exit; hcol[0..j] receives the projection coefficients.  ortho 0 = CGS2
 * (project on V_j twice, H = sum of both coefficient vectors), 1 = MGS. */
static void orthogonalise(int ortho, int64_t n, int j, const double *V, double *w,
                          double *hcol, double *tmp)
{
    if (ortho == 1) {
        for (int i = 0; i <= j; ++i) {
            const double *vi = V + (size_t)i * (size_t)n;
            double h = dot(n, vi, w);
            #pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < n; ++p) w[p] -= h * vi[p];
            hcol[i] = h;
        }
        return;
    }
    for (int i = 0; i <= j; ++i) hcol[i] = 0.0;
    for (int pass = 0; pass < 2; ++pass) {
        for (int i = 0; i <= j; ++i) tmp[i] = dot(n, V + (size_t)i * (size_t)n, w);
        for (int i = 0; i <= j; ++i) {
            const double *vi = V + (size_t)i * (size_t)n;
            #pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < n; ++p) w[p] -= tmp[i] * vi[p];
            hcol[i] += tmp[i];
        }
    }
}

/*
 * Restarted GMRES(m).
 *   b, x: length n; x holds x0 on entry and the final iterate on exit.
 *   rtol: stop when the true |b - A x| <= rtol |b| (tolerance relative to |b|,
 *         so every initial guess aims at the same accuracy).
 *   max_iters: cap on Arnoldi steps -> status 1 (not converged), last iterate kept.
 *   fixed_iters > 0: ignore the tolerance and run exactly this many Arnoldi
 *         steps (restarting every m), for trajectory comparisons.
 *   ortho: 0 CGS2, 1 MGS.
 *   hist: optional, length >= max(max_iters, fixed_iters) + 1; receives the
 *         Givens residual estimate |g_{j+1}| / |b| after every step (hist[0] =
 *         relres_init).
 * A cycle ends early when the Givens estimate |g_{j+1}| reaches rtol |b|, on
 * breakdown, or at the step cap; the iterate is accepted only on the true
 * residual b - A x recomputed after the cycle, otherwise GMRES restarts.
 */
int32_t or_gmres(int32_t dim, int64_t nx, int64_t ny, int64_t nz,
                 const double *b, double *x, int32_t m, double rtol,
                 int64_t max_iters, int64_t fixed_iters, int32_t ortho,
                 or_stats *st, double *hist)
{
    if (dim != 2 && dim != 3) return -1;
    if (nx < 1 || ny < 1 || (dim == 3 && nz < 1) || m < 1) return -1;
    int64_t n = nx * ny * (dim == 3 ? nz : 1);
    memset(st, 0, sizeof(*st));

    double bnorm = sqrt(dot(n, b, b));
    if (bnorm == 0.0) {                       /* A x = 0 has the solution x = 0 */
        for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
        if (hist) hist[0] = 0.0;
        return 0;
    }

    size_t nn = (size_t)n;
    double *V = (double *)malloc(sizeof(double) * nn * (size_t)(m + 1));
    double *w = (double *)malloc(sizeof(double) * nn);
    double *r = (double *)malloc(sizeof(double) * nn);
    double *R = (double *)calloc((size_t)(m + 1) * (size_t)m, sizeof(double));
    double *cs = (double *)malloc(sizeof(double) * (size_t)m);
    double *sn = (double *)malloc(sizeof(double) * (size_t)m);
    double *g = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    double *y = (double *)malloc(sizeof(double) * (size_t)m);
    double *hc = (double *)malloc(sizeof(double) * (size_t)(m + 1));
    double *scratch = (double *)malloc(sizeof(double) * (size_t)(m + 1));

    or_apply(dim, nx, ny, nz, x, r);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double beta = sqrt(dot(n, r, r));
    st->relres_init = beta / bnorm;
    st->relres_first_cycle = st->relres_init;
    st->relres_est = st->relres_init;
    st->relres_true = st->relres_init;
    if (hist) hist[0] = st->relres_init;

    int fixed = fixed_iters > 0;
    int64_t limit = fixed ? fixed_iters : max_iters;
    int converged = !fixed && beta <= rtol * bnorm;
    int64_t iters = 0;

    while (!converged && iters < limit && beta > 0.0) {
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) V[i] = r[i] / beta;
        for (int i = 0; i <= m; ++i) g[i] = 0.0;
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            or_apply(dim, nx, ny, nz, V + (size_t)j * nn, w);
            double wnorm = sqrt(dot(n, w, w));
            orthogonalise(ortho, n, j, V, w, hc, scratch);   /* hc[0..j] = H[0..j][j] */
            double hnext = sqrt(dot(n, w, w));                /* H[j+1][j] */
            hc[j + 1] = hnext;
            /* Breakdown: the new direction is rounding noise relative to A v_j,
             * so K_{j+1} is (numerically) invariant and the LS solution exact. */
            int breakdown = hnext <= 1e-14 * wnorm;

            /* apply G_0..G_{j-1} to the new column, then form G_j */
            for (int i = 0; i < j; ++i) {
                double a = hc[i], c = hc[i + 1];
                hc[i] = cs[i] * a + sn[i] * c;
                hc[i + 1] = -sn[i] * a + cs[i] * c;
            }
            double rho = hypot(hc[j], hc[j + 1]);
            if (rho == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
            else { cs[j] = hc[j] / rho; sn[j] = hc[j + 1] / rho; }
            hc[j] = rho;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            for (int i = 0; i <= j; ++i) R[(size_t)i * m + j] = hc[i];

            ++iters;
            k = j + 1;
            st->relres_est = fabs(g[j + 1]) / bnorm;
            if (hist) hist[iters] = st->relres_est;
            if (iters >= limit || breakdown) break;
            if (!fixed && fabs(g[j + 1]) <= rtol * bnorm) break;
            #pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < n; ++p) V[(size_t)(j + 1) * nn + p] = w[p] / hnext;
        }

        /* y = R^{-1} g by back substitution (R = the rotated H, k x k) */
        for (int i = k - 1; i >= 0; --i) {
            double s = g[i];
            for (int l = i + 1; l < k; ++l) s -= R[(size_t)i * m + l] * y[l];
            y[i] = s / R[(size_t)i * m + i];
        }
        for (int l = 0; l < k; ++l) {
            const double *vl = V + (size_t)l * nn;
            #pragma omp parallel for schedule(static)
            for (int64_t p = 0; p < n; ++p) x[p] += y[l] * vl[p];
        }
        or_apply(dim, nx, ny, nz, x, r);
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) r[i] = b[i] - r[i];
        beta = sqrt(dot(n, r, r));
        st->cycles += 1;
        st->relres_true = beta / bnorm;
        if (st->cycles == 1) st->relres_first_cycle = st->relres_true;
        if (!fixed && beta <= rtol * bnorm) converged = 1;
    }
    st->iters = iters;
    st->status = (fixed || converged) ? 0 : 1;

    free(V); free(w); free(r); free(R); free(cs); free(sn); free(g); free(y);
    free(hc); free(scratch);
    return st->status;
}

/*
 * One Arnoldi cycle of exactly k <= m steps from v0 = r0/|r0| with no early
 * exit, for checking the Arnoldi relations A V_k = V_{k+1} Hbar_k and
 * V^T V = I.  V_out: (k+1) x n; H_out: (k+1) x k row-major (unrotated).
 * Returns the number of steps taken (< k on breakdown).
 */
int32_t or_arnoldi(int32_t dim, int64_t nx, int64_t ny, int64_t nz,
                   const double *r0, int32_t k, int32_t ortho,
                   double *V_out, double *H_out)
{
    int64_t n = nx * ny * (dim == 3 ? nz : 1);
    size_t nn = (size_t)n;
    double *w = (double *)malloc(sizeof(double) * nn);
    double *tmp = (double *)malloc(sizeof(double) * (size_t)(2 * (k + 1)));
    double beta = sqrt(dot(n, r0, r0));
    memset(H_out, 0, sizeof(double) * (size_t)(k + 1) * (size_t)k);
    for (int64_t p = 0; p < n; ++p) V_out[p] = r0[p] / beta;
    int steps = 0;
    for (int j = 0; j < k; ++j) {
        or_apply(dim, nx, ny, nz, V_out + (size_t)j * nn, w);
        double wnorm = sqrt(dot(n, w, w));
        orthogonalise(ortho, n, j, V_out, w, tmp, tmp + (k + 1));
        for (int i = 0; i <= j; ++i) H_out[(size_t)i * k + j] = tmp[i];
        double hnext = sqrt(dot(n, w, w));
        H_out[(size_t)(j + 1) * k + j] = hnext;
        steps = j + 1;
        if (hnext <= 1e-14 * wnorm) break;
        for (int64_t p = 0; p < n; ++p) V_out[(size_t)(j + 1) * nn + p] = w[p] / hnext;
    }
    free(w); free(tmp);
    return steps;
}
