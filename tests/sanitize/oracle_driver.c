/*
 * Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the oracle's C
 * part (test infrastructure).  Exercises every exported routine on small 1-D, 2-D and 3-D
 * grids, including ragged sizes, a zero column, a warm start, both PCG forms and the
 * error returns (non-SPD operator, iteration limit, non-finite data), and checks a few
 * properties of the results: symmetry of H_sigma (x.Hy = y.Hx), the quadratic form
 * against orc_apply, and the true residual of the solves.  Exit status 0 when all hold.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

void orc_apply(int dim, const int *n, const double *h, double kappa, double sigma,
               const double *V, const double *X, double *Y, int ncols);
void orc_quad(int dim, const int *n, const double *h, double kappa, double sigma,
              const double *V, const double *X, double *out, int ncols);
int orc_pcg(int dim, const int *n, const double *h, double kappa, double sigma,
            const double *V, const double *B, double *X, int ncols, double tol, int maxit,
            int use_x0, int *iters, int *col_status);
int orc_pcg_variant(int dim, const int *n, const double *h, double kappa, double sigma,
                    const double *V, const double *B, double *X, int ncols, double tol,
                    int maxit, int use_x0, int *iters, int *col_status, int variant);
int orc_threads(void);
void orc_set_threads(int n);

static unsigned long long rs = 88172645463325252ull;
static double urand(void) { /* xorshift64, uniform in [-1, 1) */
    rs ^= rs << 13;
    rs ^= rs >> 7;
    rs ^= rs << 17;
    return (double)(rs >> 11) / 4503599627370496.0 - 1.0;
}

static int fails = 0;
#define CHECK(c, ...)                        \
    do {                                     \
        if (!(c)) {                          \
            fprintf(stderr, __VA_ARGS__);    \
            fputc('\n', stderr);             \
            ++fails;                         \
        }                                    \
    } while (0)

static double dotp(const double *a, const double *b, long n) {
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

static void one_grid(int dim, const int *n, int ncols) {
    long ng = 1;
    for (int k = 0; k < dim; ++k) ng *= n[k];
    double h[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < dim; ++k) h[k] = 1.0 / (n[k] + 1) * (1.0 + 0.1 * k);
    const double kappa = 0.5, sigma = 0.25;
    double *V = malloc(sizeof(double) * ng);
    double *X = malloc(sizeof(double) * ng * ncols);
    double *Y = malloc(sizeof(double) * ng * ncols);
    double *Z = malloc(sizeof(double) * ng * ncols);
    double *q = malloc(sizeof(double) * ncols);
    int *its = malloc(sizeof(int) * ncols), *cst = malloc(sizeof(int) * ncols);
    for (long i = 0; i < ng; ++i) V[i] = 3.0 * (urand() + 1.0);
    for (long i = 0; i < ng * ncols; ++i) X[i] = urand();
    for (long i = 0; i < ng; ++i) X[(long)(ncols - 1) * ng + i] = 0.0; /* a zero column */

    orc_apply(dim, n, h, kappa, sigma, V, X, Y, ncols);
    orc_quad(dim, n, h, kappa, sigma, V, X, q, ncols);
    for (int c = 0; c < ncols; ++c) {
        const double ref = dotp(X + (long)c * ng, Y + (long)c * ng, ng);
        CHECK(fabs(q[c] - ref) <= 1e-12 * (fabs(ref) + 1.0), "quad %d: %g vs %g", c, q[c], ref);
    }
    if (ncols >= 2) { /* x.Hy = y.Hx */
        const double a = dotp(X, Y + ng, ng), b = dotp(X + ng, Y, ng);
        CHECK(fabs(a - b) <= 1e-11 * (fabs(a) + 1.0), "symmetry %g vs %g", a, b);
    }
    for (int variant = 0; variant < 2; ++variant)
        for (int warm = 0; warm < 2; ++warm) {
            for (long i = 0; i < ng * ncols; ++i) Z[i] = warm ? 0.5 * X[i] : 0.0;
            const int st = orc_pcg_variant(dim, n, h, kappa, sigma, V, Y, Z, ncols, 1e-11,
                                           5000, warm, its, cst, variant);
            CHECK(st == 0, "pcg status %d (variant %d, warm %d)", st, variant, warm);
            for (int c = 0; c < ncols; ++c) {
                double e = 0.0, s = 0.0;
                for (long i = 0; i < ng; ++i) {
                    e = fmax(e, fabs(Z[(long)c * ng + i] - X[(long)c * ng + i]));
                    s = fmax(s, fabs(X[(long)c * ng + i]));
                }
                CHECK(e <= 1e-7 * (s + 1e-300) || (s == 0.0 && e == 0.0),
                      "solve column %d: error %g (variant %d)", c, e, variant);
                CHECK(cst[c] == 0 && its[c] >= 0, "column status %d", cst[c]);
            }
        }
    /* iteration limit */
    int st = orc_pcg(dim, n, h, kappa, sigma, V, Y, Z, ncols, 1e-14, 1, 0, its, cst);
    CHECK(ng <= 2 || st == 2, "expected NOCONV, got %d", st);
    /* indefinite operator: sigma far below -max diag */
    st = orc_pcg(dim, n, h, kappa, -1e9, V, Y, Z, ncols, 1e-10, 50, 0, its, cst);
    CHECK(st == 1 || st == 3, "expected NOT_SPD, got %d", st);
    /* non-finite right-hand side */
    Y[0] = NAN;
    st = orc_pcg(dim, n, h, kappa, sigma, V, Y, Z, ncols, 1e-10, 50, 0, its, cst);
    CHECK(st == 3, "expected NONFINITE, got %d", st);
    free(V), free(X), free(Y), free(Z), free(q), free(its), free(cst);
}

int main(void) {
    orc_set_threads(3);
    CHECK(orc_threads() == 3, "threads %d", orc_threads());
    const int g1[3] = {17, 1, 1}, g2[3] = {9, 7, 1}, g3[3] = {6, 5, 4}, g4[3] = {1, 1, 1},
              g5[3] = {13, 1, 3};
    one_grid(1, g1, 3);
    one_grid(2, g2, 4);
    one_grid(3, g3, 5);
    one_grid(3, g4, 2);
    one_grid(3, g5, 2);
    if (fails) {
        fprintf(stderr, "%d check(s) failed\n", fails);
        return 1;
    }
    printf("oracle sanitizer driver: all checks passed\n");
    return 0;
}
