/*
 * Driver for the AddressSanitizer / UndefinedBehaviorSanitizer build of the HIP
 * library's host code (CPU only: built without device code, run where no GPU is
 * visible).  Checks the error conventions of the C ABI: every call validates its
 * arguments before any device work and returns a status instead of aborting; null
 * handles give QO_ERR_ARG; qo_create rejects each invalid configuration field with
 * QO_ERR_ARG and, when no device can be used, returns QO_ERR_DEVICE (or QO_ERR_ALLOC)
 * with *out == NULL and nothing leaked; status strings exist for every code.
 * Exit status 0 when every check holds.
 */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "qo.h"

static int fails = 0;
#define CHECK(c, ...)                     \
    do {                                  \
        if (!(c)) {                       \
            fprintf(stderr, __VA_ARGS__); \
            fputc('\n', stderr);          \
            ++fails;                      \
        }                                 \
    } while (0)

static qo_config base(void) {
    qo_config c;
    memset(&c, 0, sizeof c);
    c.dim = 3;
    c.n[0] = 16, c.n[1] = 12, c.n[2] = 10;
    c.L[0] = c.L[1] = c.L[2] = 1.0;
    c.kinetic = 0.5;
    c.N = 4;
    c.sigma = 0.0;
    c.pcg_tol = 1e-10;
    c.pcg_maxit = 100;
    c.pcg_check = 1;
    c.precision = QO_FP64;
    c.refine_inner_tol = 1e-5;
    c.warm_start = 1;
    c.pcg_variant = 0;
    c.precond = 1;
    return c;
}

static void expect_arg(qo_config c, const char *what) {
    qo_handle h = (qo_handle)0x1;
    qo_status s = qo_create(&c, NULL, &h);
    CHECK(s == QO_ERR_ARG, "qo_create(%s): status %d, expected QO_ERR_ARG", what, (int)s);
    CHECK(h == NULL, "qo_create(%s): handle not cleared", what);
}

int main(void) {
    /* status strings */
    for (int s = 0; s <= 7; ++s) {
        const char *m = qo_status_string((qo_status)s);
        CHECK(m && strlen(m) > 0, "no string for status %d", s);
    }
    CHECK(qo_status_string((qo_status)99) != NULL, "no string for an unknown status");
    CHECK(qo_last_error(NULL) != NULL, "qo_last_error(NULL) is NULL");

    /* qo_create: each invalid field */
    qo_config c;
    CHECK(qo_create(NULL, NULL, NULL) == QO_ERR_ARG, "null out");
    qo_handle h = (qo_handle)0x1;
    CHECK(qo_create(NULL, NULL, &h) == QO_ERR_ARG && h == NULL, "null config");
    c = base(); c.dim = 1; expect_arg(c, "dim 1");
    c = base(); c.dim = 4; expect_arg(c, "dim 4");
    c = base(); c.n[1] = 0; expect_arg(c, "n[1] = 0");
    c = base(); c.L[2] = -1.0; expect_arg(c, "L[2] < 0");
    c = base(); c.L[0] = NAN; expect_arg(c, "L[0] NaN");
    c = base(); c.n[0] = 1025; c.precond = 0; expect_arg(c, "n[0] > 1024");
    c = base(); c.pcg_variant = 3; expect_arg(c, "pcg_variant 3");
    c = base(); c.pcg_variant = 2; expect_arg(c, "block CG with fast-Poisson");
    c = base(); c.pcg_variant = 2; c.precond = 0; c.precision = QO_MIXED;
    expect_arg(c, "block CG mixed");
    c = base(); c.precond = 2; expect_arg(c, "precond 2");
    c = base(); c.n[0] = 257; expect_arg(c, "fast-Poisson axis of more than 256 points");
    c = base(); c.N = 0; expect_arg(c, "N = 0");
    c = base(); c.N = 16 * 12 * 10; expect_arg(c, "N = Ng");
    c = base(); c.kinetic = 0.0; expect_arg(c, "kinetic 0");
    c = base(); c.sigma = INFINITY; expect_arg(c, "sigma inf");
    c = base(); c.pcg_tol = 0.0; expect_arg(c, "pcg_tol 0");
    c = base(); c.pcg_maxit = 0; expect_arg(c, "pcg_maxit 0");
    c = base(); c.pcg_check = 0; expect_arg(c, "pcg_check 0");
    c = base(); c.precision = 2; expect_arg(c, "precision 2");
    c = base(); c.precision = QO_MIXED; c.refine_inner_tol = 1.0;
    expect_arg(c, "inner tol 1");

    /* a valid configuration without a usable device */
    c = base();
    h = (qo_handle)0x1;
    qo_status s = qo_create(&c, NULL, &h);
    CHECK(s == QO_ERR_DEVICE || s == QO_ERR_ALLOC, "valid config without a GPU: status %d", (int)s);
    CHECK(h == NULL, "valid config without a GPU: handle not cleared");

    /* null handles */
    double x[4] = {0, 0, 0, 0};
    qo_step_stats st;
    qo_checkpoint ck;
    memset(&ck, 0, sizeof ck);
    CHECK(qo_set_potential(NULL, x, 0) == QO_ERR_ARG, "set_potential(NULL)");
    CHECK(qo_set_state(NULL, x, 4, 0) == QO_ERR_ARG, "set_state(NULL)");
    CHECK(qo_get_state(NULL, x, 4, 0) == QO_ERR_ARG, "get_state(NULL)");
    CHECK(qo_get_checkpoint(NULL, x, x, 4, x, 0, &ck) == QO_ERR_ARG, "get_checkpoint(NULL)");
    CHECK(qo_set_checkpoint(NULL, x, x, 4, x, 0, &ck) == QO_ERR_ARG, "set_checkpoint(NULL)");
    CHECK(qo_step(NULL, 1.0, 1, &st) == QO_ERR_ARG, "step(NULL)");
    CHECK(qo_energy(NULL, x, x) == QO_ERR_ARG, "energy(NULL)");
    CHECK(qo_gram(NULL, x, x) == QO_ERR_ARG, "gram(NULL)");
    CHECK(qo_eigenpairs(NULL, 0, x, NULL, 4, 0) == QO_ERR_ARG, "eigenpairs(NULL)");
    CHECK(qo_run(NULL, 1.0, 0.0, 1, 1e-5, NULL, NULL, NULL, NULL) == QO_ERR_ARG, "run(NULL)");
    CHECK(qo_eigsum_gradient(NULL, x, 0) == QO_ERR_ARG, "eigsum_gradient(NULL)");
    CHECK(qo_apply(NULL, x, x, 4, 1) == QO_ERR_ARG, "apply(NULL)");
    CHECK(qo_solve(NULL, x, x, 4, 1, 0, NULL) == QO_ERR_ARG, "solve(NULL)");
    CHECK(qo_precond(NULL, x, x, 4, 1, NULL) == QO_ERR_ARG, "precond(NULL)");
    CHECK(qo_get_block(NULL, 0, x, 4, 0) == QO_ERR_ARG, "get_block(NULL)");
    CHECK(qo_get_matrix(NULL, 0, x) == QO_ERR_ARG, "get_matrix(NULL)");
    CHECK(qo_energy_mode(NULL, 0, 0) == QO_ERR_ARG, "energy_mode(NULL)");
    CHECK(qo_tape_forward(NULL, 1.0, 1, 0, x) == QO_ERR_ARG, "tape_forward(NULL)");
    CHECK(qo_profile(NULL, 1) == QO_ERR_ARG, "profile(NULL)");
    CHECK(qo_destroy(NULL) == QO_ERR_ARG || qo_destroy(NULL) == QO_OK, "destroy(NULL)");

    /* the allocation-free Gram: argument errors before any device work */
    CHECK(qo_gram_pair_noalloc(NULL, x, 4, 4, 1, 1.0, x, NULL) == QO_ERR_ARG, "noalloc X null");
    CHECK(qo_gram_pair_noalloc(x, x, 2, 4, 1, 1.0, x, NULL) == QO_ERR_ARG, "noalloc ld < ng");
    CHECK(qo_gram_pair_noalloc(x, x, 4, 4, 0, 1.0, x, NULL) == QO_ERR_ARG, "noalloc ncols 0");
    CHECK(qo_gram_pair_noalloc(x, x, 4, 4, QO_NOALLOC_MAX_COLS + 1, 1.0, x, NULL) == QO_ERR_ARG,
          "noalloc ncols too large");
    CHECK(qo_gram_pair_noalloc(x, x, 4, 4, 1, -1.0, x, NULL) == QO_ERR_ARG, "noalloc w < 0");
    CHECK(strlen(qo_last_error(NULL)) > 0, "noalloc error message empty");

    /* batches */
    qo_batch b = (qo_batch)0x1;
    CHECK(qo_batch_create(NULL, 1, NULL, &b) == QO_ERR_ARG, "batch null configs");
    c = base();
    b = (qo_batch)0x1;
    CHECK(qo_batch_create(&c, 0, NULL, &b) == QO_ERR_ARG, "batch count 0");
    c.N = 0;
    b = (qo_batch)0x1;
    CHECK(qo_batch_create(&c, 1, NULL, &b) == QO_ERR_ARG, "batch bad config");
    CHECK(qo_batch_step(NULL, NULL, 1, 0, NULL) == QO_ERR_ARG, "batch_step(NULL)");
    CHECK(qo_batch_last_error(NULL) != NULL, "batch_last_error(NULL)");

    if (fails) {
        fprintf(stderr, "%d check(s) failed\n", fails);
        return 1;
    }
    printf("ABI sanitizer driver: all checks passed\n");
    return 0;
}
