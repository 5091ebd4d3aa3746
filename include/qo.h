/*
 * qo.h -- C ABI of libqo_hip.so, the MI355X (gfx950) implementation of one
 * evolution step of the quasi-orthogonal inverse-operator method for the N
 * lowest eigenpairs of the discrete Schroedinger operator H = -kappa Lap_h + V.
 *
 * Paper: S. Wang and A. Zhou, "A quasi-orthogonal method based on the inverse
 * operator for Schroedinger eigenvalue problems".
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Grid: dim = 2 or 3, n[k] interior points per axis of the box
 *    [0,L_0] x [0,L_1] (x [0,L_2]), spacing h_k = L_k / (n_k + 1), homogeneous
 *    Dirichlet data.  Ng = n_0 n_1 (n_2).  A grid function is Ng values with x
 *    fastest: index i + n_0 (j + n_1 k).
 *  - Block: N grid functions stored column-major, column j at offset j*ld
 *    (ld >= Ng), every column a contiguous grid function.  This is the
 *    coefficient-matrix orientation of the paper's Sec. 5 (C in R^{Ng x N}).
 *  - Inner product (Sec. 2.1): <X,Y> = ((x_i, y_j))_ij with the grid L2 inner
 *    product (u,v) = h^d sum_i u_i v_i, h^d = prod_k h_k.
 *  - Operator: H_sigma = -kappa Lap_h + V + sigma (5-point stencil in 2-D,
 *    7-point in 3-D); the shift sigma is the one allowed by the Garding remark
 *    at the end of Sec. 2.2 and must make H_sigma positive definite.  The
 *    inverse operator of Sec. 3.1 is G = H_sigma^{-1}.
 *  - Pointers flagged on_device are HIP device pointers (e.g. a torch tensor's
 *    data_ptr()); others are host pointers.  The caller owns every pointer it
 *    passes; the library owns the workspace it allocates in qo_create and frees
 *    it in qo_destroy.  All device work is ordered on the stream given to
 *    qo_create; host outputs are complete when a call returns.
 *  - Every function returns a qo_status and never aborts.  Arguments are
 *    validated before any device work.  qo_last_error(h) gives a message for
 *    the last failing call on h.  A handle is not thread-safe; distinct handles
 *    are independent.
 */
#ifndef QO_H
#define QO_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct qo_ctx *qo_handle;

typedef enum {
    QO_OK = 0,
    QO_ERR_ARG = 1,        /* invalid argument, null pointer, unsupported size */
    QO_ERR_ALLOC = 2,      /* device or host allocation failed */
    QO_ERR_DEVICE = 3,     /* a HIP runtime call failed */
    QO_ERR_STATE = 4,      /* call out of order (no potential / no state yet) */
    QO_ERR_NOT_SPD = 5,    /* <U,U> not positive definite, or p.H_sigma p <= 0 in PCG */
    QO_ERR_PCG_NOCONV = 6, /* PCG (or refinement) hit its iteration limit */
    QO_ERR_NONFINITE = 7   /* NaN or Inf met in the data */
} qo_status;

typedef enum { QO_FP64 = 0, QO_MIXED = 1 } qo_precision;
typedef enum { QO_EIG_RITZ = 0, QO_EIG_PAPER = 1 } qo_eig_mode;

typedef struct {
    int dim;                 /* 2 or 3 */
    int n[3];                /* interior points per axis (n[2] ignored when dim == 2) */
    double L[3];             /* box side lengths */
    double kinetic;          /* kappa: 0.5 for H = -1/2 Lap + V (Sec. 5), 1.0 for a(u,v) of Sec. 2.1 */
    int N;                   /* number of eigenpairs, 1 <= N < Ng */
    double sigma;            /* shift of H */
    double pcg_tol;          /* per-column stop: ||r|| <= pcg_tol ||b|| (recursive residual) */
    int pcg_maxit;           /* PCG iterations per solve (per refinement round in QO_MIXED) */
    int pcg_check;           /* host polls convergence every pcg_check iterations (>= 1) */
    int precision;           /* qo_precision */
    double refine_inner_tol; /* QO_MIXED: relative tolerance of each FP32 inner PCG solve */
    int warm_start;          /* 1: G U_n starts from the previous G U_hat and G U_hat from
                                P (X + C Y); 0: both start from zero */
    int pcg_variant;         /* 0: Hestenes-Stiefel form, two sweeps per iteration;
                                1: Chronopoulos-Gear form, one sweep per iteration
                                   (3-D, or 2-D with n_0 <= 256); same iterates in exact
                                   arithmetic;
                                2: block CG (O'Leary): one search block for all
                                   columns, N x N step matrices, converged columns
                                   deflated, the column solver finishing if the block
                                   loses rank; QO_FP64 with precond 0 only */
    int precond;             /* PCG preconditioner (the solver of G is left open by Sec. 4.1;
                                the concluding section asks for a better one than the diagonal):
                                0: Jacobi, M = diag(H_sigma);
                                1: fast-Poisson, M = kappa (-Lap_h) + vbar with
                                   vbar = max(0, mean(V + sigma)), inverted exactly by type-I
                                   discrete sine transforms (FP16 matrix cores, FP32
                                   accumulation); iteration count independent of h.  Needs
                                   pcg_variant 0 and every axis of at most 256 points
                                   (qo_create returns QO_ERR_ARG otherwise) */
} qo_config;

typedef struct {
    double energy;         /* E(U_{n+1}) = 1/2 tr <U, H U> (Sec. 2.2), unshifted */
    double energy_shifted; /* E_sigma(U_{n+1}) = 1/2 tr <U, H_sigma U>: the dissipated quantity */
    double orth_err_fro;   /* ||<U_hat,U_hat> - I||_F, i.e. ||O_n||_F (Sec. 4.1) */
    double grad_norm;      /* ||G U_n - U_n <G U_n, U_n>|| (Sec. 3.1, Alg. 1 stop test) */
    int pcg_iters[2];      /* max over columns of PCG iterations for G U_n and G U_hat
                              (QO_MIXED: summed over refinement rounds) */
    int refine_rounds[2];  /* QO_MIXED: refinement rounds per solve; 1 in QO_FP64 */
    int energy_rose;       /* 1 if E_sigma(U_{n+1}) > E_sigma(U_n) (tau too large); 0 at
                              the first step after qo_set_state / qo_set_potential, whose
                              starting energy is not evaluated */
    int step_index;        /* n + 1 after the step */
    double orth_err_next;  /* ||O_{n+1}||_F from the Gram recurrence of Sec. 4.1,
                              O_{n+1} = O_n - tau (A_n O_n + O_n A_n) + tau^2 O_n B_n O_n */
    double t_phase_ms[8];  /* solve1, gram1, small, update, solve2, gram2, correct, energy */
} qo_step_stats;

/* Block and matrix selectors of the diagnostic getters. */
typedef enum { QO_BLOCK_U = 0, QO_BLOCK_UHAT = 1, QO_BLOCK_P = 2, QO_BLOCK_Q = 3 } qo_block;
typedef enum {
    QO_MAT_S = 0, /* <U_n,U_n>                          */
    QO_MAT_M = 1, /* <U_n, G U_n>                       */
    QO_MAT_R = 2, /* <G U_n, G U_n>                     */
    QO_MAT_X = 3, /* U_hat = U_n X + (G U_n) Y          */
    QO_MAT_Y = 4,
    QO_MAT_O = 5, /* <U_hat,U_hat> - I   (O_n, Sec. 4.1) */
    QO_MAT_A = 6, /* <U_hat, G U_hat>    (A_n, Sec. 4.1) */
    QO_MAT_B = 7  /* <G U_hat, G U_hat>  (B_n, Sec. 4.1) */
} qo_matrix;

/* Create a solver for the grid and options in cfg.  hip_stream is a
 * hipStream_t (NULL: the default stream).  Allocates the device workspace, in
 * blocks of ld x N values with ld = Ng rounded up to a multiple of 64:
 *   QO_FP64: 9 FP64 blocks (U, U_hat, the G U / G U_hat pair, r, two search
 *            directions, two scratch blocks); 10 with pcg_variant 1;
 *   QO_MIXED adds 5 FP32 blocks (6 with pcg_variant 1) and a BF16 copy of two
 *            blocks for the Gram (the bytes of one FP32 block);
 *   precond 1 adds two FP16 blocks and one block of the PCG's precision (z);
 * plus O(Ng + N^2) per-point and N x N arrays.  At Ng = 96^3, N = 256 the mixed
 * fast-Poisson workspace is about 25 GB.  qo_tape_forward adds K + 1 FP64 blocks when
 * it is called (fewer under qo_tape_budget).  Sizes: 1 <= N < Ng, n_0 <= 1024 (n_0 <= 256 with
 * pcg_variant 1).  On error *out is NULL. */
qo_status qo_create(const qo_config *cfg, void *hip_stream, qo_handle *out);

/* Potential V: Ng values, x fastest (the V of H = -kappa Lap + V, Sec. 2.1). */
qo_status qo_set_potential(qo_handle h, const double *V, int on_device);

/* Current iterate U_n (Ng x N, column-major, leading dimension ld >= Ng).
 * Resets the step counter and drops the warm-start vectors. */
qo_status qo_set_state(qo_handle h, const double *U, long ld, int on_device);
qo_status qo_get_state(qo_handle h, double *U, long ld, int on_device);

/* Checkpoint of the iteration of Sec. 4.1 at step n, for a resume that continues
 * bit for bit (qo_set_state restarts cold instead).  Besides U_n it holds what the
 * next step reads from earlier steps: the warm start of the solve G U_n (the block
 * G U_hat_{n-1} of the previous step; warm starts are not part of the paper's scheme),
 * E_sigma(U_n) for the energy_rose flag, and, in energy mode 1, the carried matrix
 * K = <U_n, H_sigma U_n>. */
typedef struct {
    long step_index;       /* n */
    int has_warm;          /* 1: warm holds the warm-start block (warm starts on, n > 0) */
    int has_energy;        /* 1: energy_shifted is E_sigma(U_n) from the last step */
    double energy_shifted;
    int has_K;             /* 1: K holds the carried N x N matrix (energy mode 1) */
} qo_checkpoint;

/* Writes U_n into U and, when info->has_warm comes back 1 and warm is not NULL, the
 * warm-start block into warm (both Ng x N, leading dimension ld >= Ng, device pointers
 * when on_device), and the carried K into K (N x N column-major host array; may be
 * NULL).  info (not NULL) receives the scalars.  QO_ERR_STATE without a state. */
qo_status qo_get_checkpoint(qo_handle h, double *U, double *warm, long ld, double *K,
                            int on_device, qo_checkpoint *info);

/* Restores a checkpoint taken by qo_get_checkpoint on a handle of the same
 * configuration and potential (set the potential first).  warm must be given when
 * info->has_warm, K when info->has_K (it is then used only in energy mode 1).
 * QO_ERR_ARG for missing blocks or a negative step index, QO_ERR_NONFINITE for
 * non-finite values (the handle then has no state). */
qo_status qo_set_checkpoint(qo_handle h, const double *U, const double *warm, long ld,
                            const double *K, int on_device, const qo_checkpoint *info);

/* nsteps evolution steps of the two-stage scheme of Sec. 4.1 (Alg. 1 with a
 * fixed step tau): P = G U_n; U_hat = Cayley transform of U_n by the skew
 * operator A V = P<U_n,V> - U_n<P,V> (solved exactly through an N x N
 * system); Q = G U_hat; U_{n+1} = U_hat - tau Q (<U_hat,U_hat> - I).
 * Transactional: on error U_n and the step counter are unchanged.  last (may
 * be NULL) receives the statistics of the last step taken. */
qo_status qo_step(qo_handle h, double tau, int nsteps, qo_step_stats *last);

/* E(U_n) and E_sigma(U_n) of the current iterate (Sec. 2.2). Host outputs. */
qo_status qo_energy(qo_handle h, double *E, double *E_shifted);

/* S = <U_n,U_n> and K = <U_n, H_sigma U_n> (N x N column-major host arrays;
 * K may be NULL). */
qo_status qo_gram(qo_handle h, double *S, double *K);

/* Eigenvalue read-out of Sec. 5.  QO_EIG_RITZ: Rayleigh-Ritz on span U_n,
 * K c = theta S c, lambda = theta - sigma; evecs (may be NULL) receives U_n c
 * (Ng x N, leading dimension ld, S-orthonormal).  QO_EIG_PAPER: lambda =
 * eigenvalues of <G U_n, U_n>^{-1} minus sigma (needs one extra solve; evecs
 * must be NULL).  evals: N host doubles, ascending. */
qo_status qo_eigenpairs(qo_handle h, int mode, double *evals, double *evecs, long ld,
                        int on_device);

/* Algorithm 1 of Sec. 5: take steps while ||grad_G E_G(U_n)|| > grad_tol, at most
 * max_steps.  The gradient of U_n is evaluated inside the step (after G U_n), so the
 * loop stops before updating a U_n that already passes the test.  tau_max > 0
 * selects the adaptive time step (tau is kept <= tau_max) of the algorithm's "select tau_n <= delta_T": a
 * step that fails (singular Gram matrix, PCG limit, non-finite data), raises E_sigma
 * or lets ||<U,U> - I|| grow is undone and retried with tau/2 (E_sigma alone can fall
 * by shrinking U out of the quasi-Stiefel set when tau is too large); an accepted step
 * grows tau by 1.25 up to tau_max; tau_max <= 0 keeps tau fixed.  out_steps (may be
 * NULL): accepted steps; out_tau (may be NULL): the step size at exit; last (may be
 * NULL): statistics of the last accepted step; *converged (may be NULL): 1 when the
 * gradient test passed. */
qo_status qo_run(qo_handle h, double tau, double tau_max, int max_steps, double grad_tol,
                 int *out_steps, double *out_tau, int *converged, qo_step_stats *last);

/* Gradient of the sum of the N Ritz values of span U_n with respect to the potential:
 * g_j = d(theta_1 + ... + theta_N)/dV_j = h^d (U S^{-1} U^T)_jj, S = <U,U> (U held fixed;
 * at convergence this is the Hellmann-Feynman gradient of lambda_1 + ... + lambda_N, the
 * eigenvalues of Sec. 2.2).  g: Ng values (device pointer when on_device). */
qo_status qo_eigsum_gradient(qo_handle h, double *g, int on_device);

qo_status qo_destroy(qo_handle h);
const char *qo_status_string(qo_status s);
/* Message of the last failing call on h; with h == NULL, of the calling thread's last
 * failing handle-free call (qo_gram_pair_noalloc). */
const char *qo_last_error(qo_handle h);

/* ---- kernel-level entry points (device pointers, ncols <= N, ld >= Ng) ---- */

/* Y = H_sigma X (the stencil of the operator, Sec. 2.1 discretised). */
qo_status qo_apply(qo_handle h, const double *X, double *Y, long ld, int ncols);

/* X = G B = H_sigma^{-1} B per column (Sec. 3.1), PCG (preconditioner per
 * cfg.precond) in FP64, or in QO_MIXED FP32 PCG with FP64 residual replacement.  use_x0: X holds the
 * starting guess.  iters (host, ncols ints, may be NULL): iterations per
 * column (QO_MIXED: summed over rounds). */
qo_status qo_solve(qo_handle h, const double *B, double *X, long ld, int ncols, int use_x0,
                   int *iters);

/* Z = M^{-1} R per column with the fast-Poisson preconditioner of the PCG
 * (precond = 1; needs the potential, which fixes vbar): the same FP16
 * transform passes the solve runs, so Z equals the exact M^{-1} R up to FP16
 * rounding (about 1e-3 relative).  rz (host, ncols doubles, may be NULL):
 * the per-column sums r_i z_i.  A zero column gives a zero column. */
qo_status qo_precond(qo_handle h, const double *R, double *Z, long ld, int ncols, double *rz);

/* G = <Z,Z> for Z = [X | Y] (2 ncols columns): the 2ncols x 2ncols Gram matrix
 * of Sec. 2.1, column-major host output.  BF16 tiles with FP32 accumulation
 * in QO_MIXED, FP64 otherwise. */
qo_status qo_gram_pair(qo_handle h, const double *X, const double *Y, long ld, int ncols,
                       double *G);

/* Allocation-free variant of qo_gram_pair (FP64 path), for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Needs no handle and calls no allocating routine.  G = w [X | Y]^T [X | Y]
 * (the 2 ncols x 2 ncols Gram matrix of Sec. 2.1 with the grid weight w = h^d), written
 * column-major to the device array G; X, Y are device blocks of ncols columns of ng
 * values with leading dimension ld >= ng; all three are owned by the caller.  The work is
 * enqueued on hip_stream (a hipStream_t, NULL: the default stream) of the current device
 * and the call returns without waiting for it.  The split-K partial sums live in a
 * 32 MiB device array of the library (one per device, kept until the process ends,
 * located at the first call on the device); 1 <= ncols <= QO_NOALLOC_MAX_COLS so that at
 * least one row chunk of partials fits.  Every call on a device uses that device's one
 * array: calls that overlap on one device (other streams or threads) race and must be
 * serialised by the caller.  Errors: QO_ERR_ARG (null pointer, ng < 1, ld < ng, ncols out
 * of range, w not positive and finite), QO_ERR_DEVICE (no current device, launch
 * failure); nothing is enqueued then, and qo_last_error(NULL) gives the message. */
#define QO_NOALLOC_MAX_COLS 1024
qo_status qo_gram_pair_noalloc(const double *X, const double *Y, long ld, long ng, int ncols,
                               double w, double *G, void *hip_stream);

/* Diagnostics of the last step: a block (Ng x N into out with leading
 * dimension ld) or an N x N matrix (column-major host array). */
qo_status qo_get_block(qo_handle h, int which, double *out, long ld, int on_device);
qo_status qo_get_matrix(qo_handle h, int which, double *out);

/* ---- grouped batches of independent problems ----
 * count instances, each with its own qo_config (grid, N, sigma, tolerance, potential and
 * state), stepped together with the scheme of Sec. 4.1.  Instances whose grids agree (dim,
 * n, L, kinetic, precond) form a group: the grid-sized kernels (stencil, PCG sweeps,
 * preconditioner passes, energy) run once over all columns of a group, the Grams, block
 * updates and N x N algebra once per group with one tile set or workgroup per instance.
 * Restrictions: pcg_variant 0, N <= 1024; instances of one group share precision (and
 * refine_inner_tol).  The PCG runs a fixed
 * number of iterations per solve: pcg_maxit (the largest value in the group) until
 * iteration counts have been observed, then the largest count of a previous step plus
 * a margin of 50% + 4, at most pcg_maxit (kept while it stays within max(2, 25%) above
 * the observed counts and max(4, 25%) above that target); columns freeze on convergence,
 * and a column still above its tolerance after them makes the step fail with
 * QO_ERR_PCG_NOCONV.
 * With precision QO_MIXED a solve is a fixed number of restarted refinement rounds
 * (six until counts have been observed, then the most any column used plus one, at
 * most 30): FP64 residual, FP32 PCG with a fixed iteration count per round (pcg_maxit
 * at first, then the round's largest observed count plus max(2, 25%)) on the columns
 * still above tolerance (inner tolerance as the single-instance mixed path), FP64
 * update; the FP64 residual after the last round decides convergence.  Grams, N x N
 * algebra and energy stay FP64 (BF16 Grams are single-instance only); pcg_iters then
 * counts FP32 iterations summed over the rounds and refine_rounds the rounds used.
 * The solve of G U_n always starts from the previous G U_hat (zero after
 * qo_batch_set_state).  qo_batch_set_state and qo_batch_set_potential return the
 * instance's group to the counts of a fresh batch (pcg_maxit; six rounds in mixed
 * precision) and drop its captured graphs, since a cold start or a new operator needs
 * more iterations than the warm-started steps before it; a step that fails with
 * QO_ERR_PCG_NOCONV does the same for every group.  With use_graph != 0 each step is replayed from a HIP graph
 * captured at its first use (one per parity of the P / Q buffers); the stream given to
 * qo_batch_create must then not be the null stream (NULL creates a private stream).  At
 * creation the band height of the stencil kernels is chosen per group by timing the
 * candidates on the device (qo_batch_tile reports it).  A failed step leaves the states
 * undefined (no undo).  Instances are numbered 0 .. count-1 in the order of cfgs. */
typedef struct qo_batch_ctx *qo_batch;
qo_status qo_batch_create(const qo_config *cfgs, int count, void *hip_stream, qo_batch *out);
qo_status qo_batch_set_potential(qo_batch b, int i, const double *V, int on_device);
qo_status qo_batch_set_state(qo_batch b, int i, const double *U, long ld, int on_device);
qo_status qo_batch_get_state(qo_batch b, int i, double *U, long ld, int on_device);
/* nsteps steps of every instance.  taus: count step sizes (NULL: the previous ones).
 * stats (may be NULL): count entries, the last step's statistics per instance. */
qo_status qo_batch_step(qo_batch b, const double *taus, int nsteps, int use_graph,
                        qo_step_stats *stats);
qo_status qo_batch_tile(qo_batch b, int i, int *ty);
qo_status qo_batch_destroy(qo_batch b);
const char *qo_batch_last_error(qo_batch b);

/* ---- kernel timing (for roofline measurement) ----
 * When enabled, every launch of the kernels below is bracketed by HIP events
 * on the handle's stream; durations are harvested at the library's own
 * synchronisation points.  work[k] counts column-iterations for the PCG sweeps
 * (bytes moved = bytes per point-column x Ng x work) and launches otherwise.  A second
 * sweep that starts a solve from x = 0 without reading x moves 4 of the 5 arrays of a
 * regular one and counts 0.8 of a column-iteration.  QO_KERNEL_RESID covers the FP64
 * residual passes of QO_MIXED, the ones that also apply the previous round's correction
 * x + d included. */
typedef enum {
    QO_KERNEL_SWEEP1_F64 = 0, QO_KERNEL_SWEEP2_F64 = 1, QO_KERNEL_SWEEP1_F32 = 2,
    QO_KERNEL_SWEEP2_F32 = 3, QO_KERNEL_GRAM = 4, QO_KERNEL_UPDATE = 5, QO_KERNEL_RESID = 6,
    QO_KERNEL_CG_F64 = 7, QO_KERNEL_CG_F32 = 8, QO_KERNEL_DST_FWD = 9, QO_KERNEL_DST_PENCIL = 10,
    QO_KERNEL_DST_INV = 11, QO_KERNEL_COUNT = 12
} qo_kernel_id;
typedef struct {
    long launches[QO_KERNEL_COUNT];
    double ms[QO_KERNEL_COUNT];
    double work[QO_KERNEL_COUNT];
} qo_profile_data;

/* How qo_step computes the energy it reports.  mode 0 (default): the stencil quadratic
 * form of U_{n+1} (one pass over the block).  mode 1: K = <U, H_sigma U> is carried from
 * step to step by exact identities of the two stages (Sec. 4.1; the second-stage energy
 * identity of Sec. 4.2 is its trace): with the solves H_sigma P = U, H_sigma Q = U_hat,
 *   K_hat   = X^T K X + X^T S Y + Y^T S X + Y^T M^T Y,
 *   K_{n+1} = K_hat - tau (S_hat O + O S_hat) + tau^2 O A^T O,
 * E_sigma = 1/2 tr K_{n+1}, tr <U,U> = tr O_{n+1} + N, all N x N work.  K is computed
 * with the stencil at the first step after the mode is set or the state or potential
 * changes, and again every `anchor` steps (anchor 0: never again).  The propagated value
 * inherits the solves' tolerance each step.  mode 1 needs precision QO_FP64 (the BF16
 * Grams of QO_MIXED would enter the identities); QO_ERR_ARG otherwise or for a bad mode
 * or a negative anchor. */
qo_status qo_energy_mode(qo_handle h, int mode, int anchor);

/* ---- reverse mode through K steps -------------------------------------------------
 *
 * qo_tape_forward takes K steps of Sec. 4.1 (Algorithm 1 of Sec. 5 with a fixed tau) from
 * the current state and records a checkpoint of every step's starting block U_0 .. U_K
 * (K + 1 blocks of ld x N doubles held by the handle until it is destroyed; they grow
 * with the largest K taped).  The linear solves start from zero while taping, so a step
 * can be recomputed bit for bit from its checkpoint; the handle's warm_start setting is
 * restored afterwards.  *L receives the loss of U_K:
 *   loss 0: E(U_K) = h^d/2 sum_c u_c^T H u_c, the energy of Sec. 2.2;
 *   loss 1: theta_1 + ... + theta_N, the sum of the Ritz values of span U_K (the
 *           eigenvalue read-out of Sec. 5), = tr(S^{-1} K_sigma) - N sigma.
 * FP64 only (QO_ERR_ARG for precision QO_MIXED); QO_ERR_STATE without potential or
 * state; solver errors as qo_step.  On error the tape is invalid and the state is the
 * last completed step's.
 *
 * qo_tape_backward returns seed * dL/dV (gV, Ng values) and seed * dL/dU_0 (gU0, N
 * columns of Ng values with leading dimension ld >= Ng, the layout of qo_set_state);
 * either may be NULL.  Device pointers when on_device, else host.  It goes back through
 * the steps, recomputing each from its checkpoint, with the adjoints of the corrector,
 * of the solves Q = G U_hat and P = G U (each an extra solve with the same symmetric
 * H_sigma; dG/dV = -G diag(dV) G), of the predictor's N x N algebra and of the Gram
 * matrices.  The result is the derivative of the computed K-step map (the solves taken
 * as exact); it uses 2K solves of N columns more than the forward.  The state is U_K
 * again afterwards.  QO_ERR_STATE before a successful qo_tape_forward. */
qo_status qo_tape_forward(qo_handle h, double tau, int K, int loss, double *L);

/* Memory bound of the tape: at most `blocks` FP64 blocks of ld x N for the states
 * (0, the default: every one of U_0 .. U_K).  With a bound, qo_tape_forward keeps every
 * s-th state and U_K, with the smallest stride s for which those checkpoints and the s - 1
 * states of one segment fit (s ~ sqrt(K): about 2 sqrt(K) blocks); qo_tape_backward
 * recomputes each segment's states from its checkpoint once, just before the adjoint goes
 * through it (about K extra steps), and returns the same gradients bit for bit.
 * QO_ERR_ARG for blocks < 0 or 1 <= blocks < 3; qo_tape_forward returns QO_ERR_ARG when
 * no stride fits K in the bound. */
qo_status qo_tape_budget(qo_handle h, int blocks);
qo_status qo_tape_backward(qo_handle h, double seed, double *gV, double *gU0, long ld,
                           int on_device);

/* enable != 0 turns timing on and clears the counters; 0 turns it off. */
qo_status qo_profile(qo_handle h, int enable);
qo_status qo_profile_get(qo_handle h, qo_profile_data *out);

#ifdef __cplusplus
}
#endif
#endif /* QO_H */
