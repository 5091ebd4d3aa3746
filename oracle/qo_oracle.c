/*
 * qo_oracle.c -- reference (test-infrastructure) implementation of the grid
 * operations of the quasi-orthogonal inverse-operator method, in plain C, FP64.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct CPU
 * checker the HIP library is compared against.  Nothing in the product path
 * links, loads or calls it; only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark do.  It shares no code, header or
 * constant with the HIP library.
 *
 * What it implements (paper: Wang & Zhou, "A quasi-orthogonal method based on
 * the inverse operator for Schroedinger eigenvalue problems"):
 *
 *  - orc_apply: the discrete Schroedinger operator H_sigma = -kappa*Lap_h + V + sigma
 *    on a uniform interior grid with homogeneous Dirichlet data.  The paper's
 *    bilinear form a(u,v) (Sec. 2.1) is discretised with the textbook second
 *    difference in each axis; kappa = 1/2 gives the operator -1/2 Lap + V of the
 *    examples in Sec. 5, kappa = 1 the form of Sec. 2.1.  sigma is the shift
 *    allowed by the Garding remark at the end of Sec. 2.2.
 *
 *  - orc_pcg: the inverse operator G = H_sigma^{-1} of Sec. 3.1 applied to each
 *    column independently.  The paper defines G but does not say how it is
 *    applied; here it is Jacobi-preconditioned conjugate gradients, stopped per
 *    column at the first iteration whose recursively updated residual satisfies
 *    ||r|| <= tol*||b||.  Two textbook forms of the same iteration:
 *      variant 0: Hestenes-Stiefel (two inner products per iteration, each
 *                 needing the previous one);
 *      variant 1: Chronopoulos-Gear (both inner products of an iteration taken
 *                 together from u = D r and w = H u; the step length follows from
 *                 alpha = gamma / (delta - beta gamma / alpha_prev)).
 *    In exact arithmetic they produce the same iterates.
 *
 * Layout: a block of ncols grid functions is column-major, Ng rows, each
 * column a grid with x fastest: index i + n0*(j + n1*k).
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

/* status codes of orc_pcg */
#define ORC_OK 0
#define ORC_NOT_SPD 1
#define ORC_NOCONV 2
#define ORC_NONFINITE 3

static long grid_size(int dim, const int *n) {
    long ng = 1;
    for (int k = 0; k < dim; ++k) ng *= n[k];
    return ng;
}

/* y = H_sigma x for one grid function.  Second difference per axis:
 * (x[i-e] - 2 x[i] + x[i+e]) / h^2 with x = 0 outside the grid.          */
static void apply_one(int dim, const int *n, const double *h, double kappa,
                      double sigma, const double *V, const double *x, double *y) {
    const int n0 = n[0];
    const int n1 = dim >= 2 ? n[1] : 1;
    const int n2 = dim >= 3 ? n[2] : 1;
    const long s1 = n0, s2 = (long)n0 * n1;
    for (int k = 0; k < n2; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n0; ++i) {
                const long c = i + s1 * j + s2 * k;
                const double xc = x[c];
                double lap = 0.0;
                /* axis 0 */
                {
                    double xm = i > 0 ? x[c - 1] : 0.0;
                    double xp = i < n0 - 1 ? x[c + 1] : 0.0;
                    lap += (xm - 2.0 * xc + xp) / (h[0] * h[0]);
                }
                if (dim >= 2) {
                    double xm = j > 0 ? x[c - s1] : 0.0;
                    double xp = j < n1 - 1 ? x[c + s1] : 0.0;
                    lap += (xm - 2.0 * xc + xp) / (h[1] * h[1]);
                }
                if (dim >= 3) {
                    double xm = k > 0 ? x[c - s2] : 0.0;
                    double xp = k < n2 - 1 ? x[c + s2] : 0.0;
                    lap += (xm - 2.0 * xc + xp) / (h[2] * h[2]);
                }
                y[c] = -kappa * lap + (V[c] + sigma) * xc;
            }
}

/* Y = H_sigma X, ncols columns. */
void orc_apply(int dim, const int *n, const double *h, double kappa, double sigma,
               const double *V, const double *X, double *Y, int ncols) {
    const long ng = grid_size(dim, n);
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < ncols; ++c)
        apply_one(dim, n, h, kappa, sigma, V, X + (long)c * ng, Y + (long)c * ng);
}

/* out[c] = x_c . (H_sigma x_c): the quadratic form of each column (unweighted). */
void orc_quad(int dim, const int *n, const double *h, double kappa, double sigma,
              const double *V, const double *X, double *out, int ncols) {
    const long ng = grid_size(dim, n);
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = 0; c < ncols; ++c) {
        double *y = (double *)malloc(sizeof(double) * ng);
        const double *x = X + (long)c * ng;
        apply_one(dim, n, h, kappa, sigma, V, x, y);
        double s = 0.0;
        for (long i = 0; i < ng; ++i) s += x[i] * y[i];
        out[c] = s;
        free(y);
    }
}

int orc_pcg_variant(int dim, const int *n, const double *h, double kappa, double sigma,
                    const double *V, const double *B, double *X, int ncols, double tol,
                    int maxit, int use_x0, int *iters, int *col_status, int variant);

static double dot(const double *a, const double *b, long n) {
    double s = 0.0;
    for (long i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/*
 * Solve H_sigma x_c = b_c for every column by Jacobi-PCG.
 *   X     in: initial guesses when use_x0 != 0 (else ignored, x0 = 0); out: solutions
 *   iters out: iterations used per column
 *   col_status out (may be NULL): per-column status
 * Returns the worst status over the columns (NONFINITE > NOT_SPD > NOCONV > OK).
 */
static int cg_one_reduction(int dim, const int *n, const double *h, double kappa,
                            double sigma, const double *V, const double *Dinv,
                            const double *b, double *x, long ng, double tol, int maxit,
                            int use_x0, int *iters, double *r, double *u, double *w,
                            double *p, double *s);

int orc_pcg(int dim, const int *n, const double *h, double kappa, double sigma,
            const double *V, const double *B, double *X, int ncols, double tol,
            int maxit, int use_x0, int *iters, int *col_status) {
    return orc_pcg_variant(dim, n, h, kappa, sigma, V, B, X, ncols, tol, maxit, use_x0,
                           iters, col_status, 0);
}

int orc_pcg_variant(int dim, const int *n, const double *h, double kappa, double sigma,
                    const double *V, const double *B, double *X, int ncols, double tol,
                    int maxit, int use_x0, int *iters, int *col_status, int variant) {
    const long ng = grid_size(dim, n);
    /* Jacobi preconditioner: inverse of the diagonal of H_sigma. */
    double diag0 = 0.0;
    for (int k = 0; k < dim; ++k) diag0 += 2.0 * kappa / (h[k] * h[k]);
    double *Dinv = (double *)malloc(sizeof(double) * ng);
    for (long i = 0; i < ng; ++i) Dinv[i] = 1.0 / (diag0 + V[i] + sigma);

    int worst = ORC_OK;
#pragma omp parallel
    {
        double *r = (double *)malloc(sizeof(double) * ng);
        double *z = (double *)malloc(sizeof(double) * ng);
        double *p = (double *)malloc(sizeof(double) * ng);
        double *q = (double *)malloc(sizeof(double) * ng);
        double *w = (double *)malloc(sizeof(double) * ng);
#pragma omp for schedule(dynamic, 1)
        for (int c = 0; c < ncols; ++c) {
            const double *b = B + (long)c * ng;
            double *x = X + (long)c * ng;
            int st = ORC_OK, it = 0;
            if (variant == 1) {
                st = cg_one_reduction(dim, n, h, kappa, sigma, V, Dinv, b, x, ng, tol, maxit,
                                      use_x0, &it, r, z, w, p, q);
                goto done;
            }
            if (use_x0) {
                apply_one(dim, n, h, kappa, sigma, V, x, q);
                for (long i = 0; i < ng; ++i) r[i] = b[i] - q[i];
            } else {
                for (long i = 0; i < ng; ++i) { x[i] = 0.0; r[i] = b[i]; }
            }
            const double bnorm = sqrt(dot(b, b, ng));
            for (long i = 0; i < ng; ++i) { z[i] = Dinv[i] * r[i]; p[i] = z[i]; }
            double rho = dot(r, z, ng);
            if (!isfinite(rho) || !isfinite(bnorm)) st = ORC_NONFINITE;
            else if (!(sqrt(dot(r, r, ng)) <= tol * bnorm)) {
                for (;;) {
                    if (it >= maxit) { st = ORC_NOCONV; break; }
                    apply_one(dim, n, h, kappa, sigma, V, p, q);
                    const double gamma = dot(p, q, ng);
                    if (!isfinite(gamma)) { st = ORC_NONFINITE; break; }
                    if (!(gamma > 0.0)) { st = ORC_NOT_SPD; break; }
                    const double alpha = rho / gamma;
                    for (long i = 0; i < ng; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
                    ++it;
                    const double rn = sqrt(dot(r, r, ng));
                    if (!isfinite(rn)) { st = ORC_NONFINITE; break; }
                    if (rn <= tol * bnorm) break;
                    for (long i = 0; i < ng; ++i) z[i] = Dinv[i] * r[i];
                    const double rho_new = dot(r, z, ng);
                    const double beta = rho_new / rho;
                    rho = rho_new;
                    for (long i = 0; i < ng; ++i) p[i] = z[i] + beta * p[i];
                }
            }
        done:
            iters[c] = it;
            if (col_status) col_status[c] = st;
#pragma omp critical
            {
                /* rank: NONFINITE(3) > NOT_SPD(1) > NOCONV(2) > OK(0) */
                static const int rank[4] = {0, 2, 1, 3};
                if (rank[st] > rank[worst]) worst = st;
            }
        }
        free(r); free(z); free(p); free(q); free(w);
    }
    free(Dinv);
    return worst;
}

/* Chronopoulos-Gear form of Jacobi-PCG for one column (variant 1).
 *   r = b - H x0; u = D r; w = H u; gamma = r.u; delta = w.u
 *   beta = 0, alpha = gamma / delta; p = 0
 *   repeat: p = u + beta p; s = H p; x += alpha p; r -= alpha s
 *           u = D r; w = H u; gamma' = r.u; delta = w.u; stop test on ||r||
 *           beta = gamma'/gamma; alpha = gamma' / (delta - beta gamma' / alpha)
 * (u, w, p, s are work arrays of length ng.) */
static int cg_one_reduction(int dim, const int *n, const double *h, double kappa,
                            double sigma, const double *V, const double *Dinv,
                            const double *b, double *x, long ng, double tol, int maxit,
                            int use_x0, int *iters, double *r, double *u, double *w,
                            double *p, double *s) {
    int it = 0;
    if (use_x0) {
        apply_one(dim, n, h, kappa, sigma, V, x, s);
        for (long i = 0; i < ng; ++i) r[i] = b[i] - s[i];
    } else {
        for (long i = 0; i < ng; ++i) { x[i] = 0.0; r[i] = b[i]; }
    }
    const double bnorm = sqrt(dot(b, b, ng));
    for (long i = 0; i < ng; ++i) u[i] = Dinv[i] * r[i];
    apply_one(dim, n, h, kappa, sigma, V, u, w);
    double gamma = dot(r, u, ng);
    double delta = dot(w, u, ng);
    double rn = sqrt(dot(r, r, ng));
    *iters = 0;
    if (!isfinite(gamma) || !isfinite(delta) || !isfinite(rn) || !isfinite(bnorm))
        return ORC_NONFINITE;
    if (rn <= tol * bnorm) return ORC_OK;
    double beta = 0.0, den = delta, alpha = 0.0;
    for (long i = 0; i < ng; ++i) p[i] = 0.0;
    for (;;) {
        if (it >= maxit) { *iters = it; return ORC_NOCONV; }
        if (!isfinite(den)) { *iters = it; return ORC_NONFINITE; }
        if (!(den > 0.0)) { *iters = it; return ORC_NOT_SPD; }
        alpha = gamma / den;
        for (long i = 0; i < ng; ++i) p[i] = u[i] + beta * p[i];
        apply_one(dim, n, h, kappa, sigma, V, p, s);
        for (long i = 0; i < ng; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * s[i]; }
        ++it;
        for (long i = 0; i < ng; ++i) u[i] = Dinv[i] * r[i];
        apply_one(dim, n, h, kappa, sigma, V, u, w);
        const double gnew = dot(r, u, ng);
        delta = dot(w, u, ng);
        rn = sqrt(dot(r, r, ng));
        if (!isfinite(rn) || !isfinite(gnew)) { *iters = it; return ORC_NONFINITE; }
        if (rn <= tol * bnorm) break;
        beta = gnew / gamma;
        den = delta - beta * gnew / alpha;
        gamma = gnew;
    }
    *iters = it;
    return ORC_OK;
}

/* Threads of the OpenMP loops above (for the record of a timing), and a way to change
 * them (1: the single-thread rate).  Not part of the method. */
int orc_threads(void) { return omp_get_max_threads(); }
void orc_set_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
}
