/*
 * Test infrastructure: runs every entry point of the C oracle on small 2D and
 * 3D problems, edge cases included (a zero right-hand side, a restart length
 * of 1, an iteration cap that is reached, both orthogonalisations, the
 * residual history), so that a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer checks the oracle's memory accesses and
 * arithmetic.  Exit status 0 when every result meets its expected property.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

typedef struct {
    int32_t status;
    int64_t iters;
    int32_t cycles;
    double relres_init, relres_first_cycle, relres_est, relres_true;
} or_stats;

void or_set_threads(int32_t n);
void or_apply(int32_t dim, int64_t nx, int64_t ny, int64_t nz, const double *u, double *out);
void or_residual_norm(int32_t dim, int64_t nx, int64_t ny, int64_t nz, const double *b,
                      const double *x, double *rnorm, double *bnorm);
int32_t or_gmres(int32_t dim, int64_t nx, int64_t ny, int64_t nz, const double *b, double *x,
                 int32_t m, double rtol, int64_t max_iters, int64_t fixed_iters, int32_t ortho,
                 or_stats *st, double *hist);
int32_t or_arnoldi(int32_t dim, int64_t nx, int64_t ny, int64_t nz, const double *r0, int32_t k,
                   int32_t ortho, double *V_out, double *H_out);

static int fails = 0;
#define CHECK(c, what) do { if (!(c)) { printf("FAIL %s\n", what); ++fails; } } while (0)

static void fill(double *b, int64_t n, unsigned seed) {
    for (int64_t i = 0; i < n; ++i) {
        seed = seed * 1103515245u + 12345u;
        b[i] = (double)(seed >> 8) / 16777216.0 - 0.5;
    }
}

static void solve_case(int32_t dim, int64_t nx, int64_t ny, int64_t nz, int32_t m, int32_t ortho) {
    const int64_t n = nx * ny * (dim == 3 ? nz : 1);
    double *b = malloc(sizeof(double) * n), *x = calloc(n, sizeof(double));
    double *hist = malloc(sizeof(double) * 4001);
    or_stats st;
    fill(b, n, (unsigned)(nx * 131 + ny * 7 + nz + m + ortho));
    int32_t rc = or_gmres(dim, nx, ny, nz, b, x, m, 1e-10, 4000, 0, ortho, &st, hist);
    double rn, bn;
    or_residual_norm(dim, nx, ny, nz, b, x, &rn, &bn);
    CHECK(rc == 0 && st.status == 0, "gmres converged");
    CHECK(rn <= 1e-10 * bn * 1.0001, "true residual within the tolerance");
    CHECK(hist[0] == 1.0 && hist[st.iters] <= 1e-10 * 1.0001, "residual history");
    /* a cap that is reached: not converged, no write past the history */
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    rc = or_gmres(dim, nx, ny, nz, b, x, m, 1e-14, 3, 0, ortho, &st, hist);
    CHECK(st.iters <= 3 && (st.status == 1 || st.relres_true <= 1e-14), "capped run");
    /* fixed step count (trajectory mode) */
    for (int64_t i = 0; i < n; ++i) x[i] = 0.0;
    rc = or_gmres(dim, nx, ny, nz, b, x, m, 1e-10, 0, 2 * m + 1, ortho, &st, hist);
    CHECK(rc == 0 && st.iters <= 2 * m + 1, "fixed steps");
    /* Arnoldi relations: V^T V = I to rounding */
    const int32_t k = m < (int32_t)n ? m : (int32_t)n - 1;
    double *V = malloc(sizeof(double) * (size_t)(k + 1) * n);
    double *H = malloc(sizeof(double) * (size_t)(k + 1) * k);
    int32_t steps = or_arnoldi(dim, nx, ny, nz, b, k, ortho, V, H);
    double worst = 0.0;
    for (int32_t i = 0; i <= steps; ++i)
        for (int32_t j = 0; j <= steps; ++j) {
            double s = 0.0;
            for (int64_t p = 0; p < n; ++p) s += V[(size_t)i * n + p] * V[(size_t)j * n + p];
            worst = fmax(worst, fabs(s - (i == j)));
        }
    CHECK(worst < 1e-11, "orthonormal Krylov basis");
    free(V); free(H); free(b); free(x); free(hist);
}

int main(void) {
    or_set_threads(1);
    for (int32_t ortho = 0; ortho < 2; ++ortho) {
        solve_case(2, 9, 7, 1, 5, ortho);
        solve_case(2, 13, 1, 1, 1, ortho);
        solve_case(3, 5, 4, 3, 8, ortho);
    }
    /* a zero right-hand side: x = 0 at once */
    double b0[12] = {0}, x0[12];
    for (int i = 0; i < 12; ++i) x0[i] = 1.0;
    or_stats st;
    int32_t rc = or_gmres(2, 4, 3, 1, b0, x0, 4, 1e-8, 100, 0, 0, &st, NULL);
    int zero = 1;
    for (int i = 0; i < 12; ++i) zero &= x0[i] == 0.0;
    CHECK(rc == 0 && zero, "zero right-hand side");
    /* invalid arguments are refused */
    CHECK(or_gmres(4, 4, 3, 1, b0, x0, 4, 1e-8, 100, 0, 0, &st, NULL) < 0, "dimension 4 refused");
    CHECK(or_gmres(2, 0, 3, 1, b0, x0, 4, 1e-8, 100, 0, 0, &st, NULL) < 0, "empty grid refused");
    printf(fails ? "oracle sanitizer run: %d failures\n" : "oracle sanitizer run: ok\n", fails);
    return fails != 0;
}
