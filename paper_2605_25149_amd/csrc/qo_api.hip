// C ABI of libqo_hip (declared in include/qo.h) and the step engine: the
// sequence of kernels of one evolution step of the two-stage scheme of
// Sec. 4.1, the batched PCG driver for the inverse operator of Sec. 3.1, and
// the eigenvalue read-out of Sec. 5.
//
// Step n (all device work on the handle's stream):
//   solve    P = G U_n                      (Jacobi-PCG; QO_MIXED: FP32 PCG in FP64 refinement)
//   gram1    [U P]^T [U P] h^d  -> S = <U,U>, M = <U,P>, R = <P,P>
//   small    N x N predictor system in the basis {U, W}, W = P - U C, C = S^{-1} M:
//              R_W = R - M^T C,  D = C S - M^T,  alpha = tau/2
//              (I + alpha^2 R_W S - alpha D) b = D - alpha R_W S
//              a = S (I + alpha b),  X = I + tau (b - C a),  Y = tau a
//            (the exact solution of the implicit first stage; its matrix is
//             close to I, unlike the 2N x 2N system in the basis {U, P})
//   update   U_hat = U X + P Y;  warm start x0 = P (X + C Y) for the next solve
//   solve    Q = G U_hat
//   gram2    [U_hat Q]^T [U_hat Q] h^d -> O = <U_hat,U_hat> - I, A_n, B_n
//   correct  U_{n+1} = U_hat - tau Q O
//   energy   E_sigma = 1/2 h^d sum_j u_j . H_sigma u_j  (stencil pass)
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/qo.h"
#include "qo_internal.h"

using namespace qo;

namespace {

struct Buf {
    void *p = nullptr;
};

}  // namespace

struct qo_ctx {
    qo_config cfg{};
    hipStream_t st = nullptr;
    int device = 0;
    Grid g{};    // tiling of the two-sweep kernels and the stencil family
    Grid gcg{};  // tiling of the one-sweep PCG kernels
    long qsmax = 0;  // partial-sum stride: N * max(tiles)
    long ng = 0, ld = 0;
    int N = 0;
    double w = 1.0;
    bool mixed = false;

    // per-point arrays
    double *vs = nullptr, *dinv = nullptr;
    float *vs32 = nullptr, *dinv32 = nullptr;
    // blocks (ld x N)
    double *U = nullptr, *Uh = nullptr, *PQ[2] = {nullptr, nullptr}, *r = nullptr,
           *r2 = nullptr, *pa = nullptr, *pb = nullptr, *W = nullptr, *W2 = nullptr;
    float *r32 = nullptr, *d32 = nullptr, *rr32 = nullptr, *rr32b = nullptr, *pa32 = nullptr,
          *pb32 = nullptr;
    // reductions and small matrices
    double *part = nullptr;
    double *gpart = nullptr;
    // BF16 copies of the Gram operands (mixed precision): U (written by the corrector, or
    // packed when it has changed otherwise), U_hat (written by its update) and the solution
    // block of the current Gram (packed)
    __bf16 *zbU = nullptr, *zbUh = nullptr, *zbPQ = nullptr;
    __bf16 *split3 = nullptr;  // BF16 parts of the block update's small operands (mixed)
    bool zbU_ok = false;  // zbU holds U rounded to BF16
    int gnsplit = 1;
    double *G1 = nullptr, *G2 = nullptr;
    double *mpool = nullptr;
    double *colsums = nullptr;
    double *dscal = nullptr;
    double *sortwork = nullptr;
    double *gjw = nullptr;  // blocked Gauss-Jordan workspace
    int *gjpiv = nullptr;
    PcgState ps{};
    int *mask = nullptr, *nact = nullptr, *dstatus = nullptr;
    double *coltol = nullptr;
    // reliable-update state of the mixed-precision solve
    double *zerotol = nullptr, *rref = nullptr, *bb64 = nullptr;
    int *need = nullptr, *nneed = nullptr;
    double rel_delta = 0.1;
    bool rel = true;
    // fast-Poisson preconditioner (precond == 1)
    bool dst = false;
    DstPlan dp{};
    _Float16 *dS = nullptr, *t1 = nullptr, *t2 = nullptr;
    float *dmu = nullptr, *pcs = nullptr;
    float *z32 = nullptr;  // preconditioned residual z = M^{-1} r (FP32 in either precision)
    float *pbeta = nullptr;  // beta of the FP32 PCG, formed before the inverse plane pass
    double *rzc = nullptr;   // and r.z per column
    double *wzp = nullptr;   // partial sums of (V + sigma - vbar) z^2: per column, slab, wave
    double *rzp = nullptr, *dsum = nullptr;
    double mu0 = 0.0;  // mu_x[0] + mu_y[0] (+ mu_z[0]): smallest eigenvalue of -Lap_h
    // block CG (pcg_variant 2): Z and ping-pong partners of X, R, P; small matrices;
    // per-column norms and active flags
    double *bcgb[4] = {nullptr, nullptr, nullptr, nullptr};
    double *bcgm = nullptr, *bcgv = nullptr;
    int *bcga = nullptr;
    // energy by the Gram identities (qo_energy_mode): K = <U, H_sigma U> carried from step
    // to step, recomputed with the stencil every eanchor steps
    int emode = 0, eanchor = 0;
    bool have_K = false;
    double *Kprop = nullptr, *epool = nullptr;
    // reverse mode through taped steps (qo_tape_forward / qo_tape_backward)
    std::vector<double *> tape;  // checkpoints U_0, U_s, U_2s, ... and U_K (s = tape_s)
    std::vector<double *> tseg;  // the s - 1 recomputed states of one segment (s > 1)
    int tape_budget = 0;         // at most this many state blocks (0: no bound)
    int tape_s = 1;              // checkpoint stride of the last tape
    int tape_K = 0, tape_loss = 0;
    double tape_tau = 0.0;
    bool have_tape = false;
    double *ab[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    double *gVd = nullptr, *adpool = nullptr, *admat = nullptr;
    // pinned host: PCG activity flags (two slots, by iteration parity), the refinement
    // round's flags, the predictor's status, and one iteration-count slot per round
    int *h_poll = nullptr;
    double *h_scal = nullptr;
    // events marking those read-backs (poll: by parity; round; predictor status)
    hipEvent_t pev[2] = {nullptr, nullptr}, rev = nullptr, sev = nullptr;

    std::vector<void *> allocs;
    bool have_V = false, have_U = false, have_warm = false;
    int cur = 0;
    const double *lastP = nullptr, *lastQ = nullptr;
    long nstep = 0;
    bool have_Es = false;
    double last_Es = 0.0;
    std::string err;
    hipEvent_t ev[9] = {};
    bool ev_ok = false;
    std::vector<int> h_its;
    // kernel timing
    struct Pend {
        int kid;
        hipEvent_t a, b;
    };
    bool prof = false;
    std::vector<hipEvent_t> evpool;
    std::vector<Pend> pend;
    qo_profile_data pdata{};
};

namespace {
int env_int(const char *name, int dflt) {
    const char *v = getenv(name);
    if (!v || !*v) return dflt;
    return atoi(v);
}
}  // namespace

// Tiling of the stencil family (g) and of the one-sweep PCG kernels (q) for a grid of
// dim / n[] interior points with N columns: band height, z-chunks, points per thread.
// Host code, also called by the CPU checks of the kernels' index arithmetic.
void qo::plan_grid(int dim, const int n[3], const double L[3], double kinetic, int N, Grid &g,
                   Grid &q) {
    g.cinst = nullptr;
    g.dim = dim;
    g.nx = n[0];
    g.ny = n[1];
    g.nz = dim == 3 ? n[2] : 1;
    g.ng = (long)g.nx * g.ny * g.nz;
    double h[3];
    for (int k = 0; k < 3; ++k) h[k] = (k < dim) ? L[k] / (n[k] + 1) : 1.0;
    g.ihx2 = 1.0 / (h[0] * h[0]);
    g.ihy2 = 1.0 / (h[1] * h[1]);
    g.ihz2 = dim == 3 ? 1.0 / (h[2] * h[2]) : 0.0;
    g.kappa = kinetic;
    g.c0 = 2.0 * kinetic * (g.ihx2 + g.ihy2 + g.ihz2);

    // band height: ~1536 points per plane in 2-D; 3-D bands are kept near 768
    // points (measured faster for the FP32 sweeps at 96^3 because of occupancy)
    int TY = (dim == 3 ? 768 : 1536) / g.nx;
    if (TY < 1) TY = 1;
    TY = env_int("QO_TY", TY);
    if (TY > g.ny) TY = g.ny;
    if (TY < 1) TY = 1;
    while (pick_ppt(TY * g.nx) < 0 && TY > 1) --TY;
    g.TY = TY;
    g.ppt = pick_ppt(TY * g.nx);
    // The engine for fewer than 4 points per thread stages one halo column per thread
    // between planes, so a 3-D grid (several planes per tile) wider than a workgroup takes
    // the engine for 4 or more, which loops over the halo columns.
    if (dim == 3 && g.nx > kThreads && g.ppt < 4) g.ppt = 4;
    g.nbands = (g.ny + TY - 1) / TY;
    if (dim == 2) {
        g.ZC = 1;
        g.nzc = 1;
    } else {
        long want = (2048 + (long)N * g.nbands - 1) / ((long)N * g.nbands);
        int maxc = g.nz / 16;
        if (maxc < 1) maxc = 1;
        if (want > maxc) want = maxc;
        if (want < 1) want = 1;
        int ZC = (g.nz + (int)want - 1) / (int)want;
        ZC = env_int("QO_ZC", ZC);
        if (ZC < 1) ZC = 1;
        if (ZC > g.nz) ZC = g.nz;
        g.ZC = ZC;
        g.nzc = (g.nz + ZC - 1) / ZC;
    }
    // one-sweep PCG: rows [-2, TY+1] per plane in at most 5 (8 for wide rows) points per
    // thread, and 3 + 3 LDS planes of (TY+4) and (TY+2) rows within 64 KiB in FP64
    q = g;
    {
        const int target = g.nx <= 128 ? 5 : 8;
        int ty = kThreads * target / g.nx - 4;
        const int ty_lds = ((65536 / (24 * g.nx)) - 6) / 2;
        if (ty > ty_lds) ty = ty_lds;
        ty = env_int("QO_CG_TY", ty);
        if (ty > g.ny) ty = g.ny;
        if (ty < 1) ty = 1;
        q.TY = ty;
        const int raw = ((ty + 4) * g.nx + kThreads - 1) / kThreads;
        const int opts[6] = {2, 3, 4, 5, 6, 8};
        q.ppt = -1;
        for (int o : opts)
            if (o >= raw) { q.ppt = o; break; }
        q.nbands = (g.ny + ty - 1) / ty;
        if (dim == 2) {
            q.ZC = 1;
            q.nzc = 1;
        } else {
            long want = (2048 + (long)N * q.nbands - 1) / ((long)N * q.nbands);
            int maxc = g.nz / 16;
            if (maxc < 1) maxc = 1;
            if (want > maxc) want = maxc;
            if (want < 1) want = 1;
            int ZC = (g.nz + (int)want - 1) / (int)want;
            ZC = env_int("QO_CG_ZC", ZC);
            if (ZC < 1) ZC = 1;
            if (ZC > g.nz) ZC = g.nz;
            q.ZC = ZC;
            q.nzc = (g.nz + ZC - 1) / ZC;
        }
    }
}

namespace {

qo_status fail(qo_ctx *c, qo_status s, const char *fmt, ...) {
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return s;
}

#define HIPC(ctx, call)                                                                    \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(ctx, QO_ERR_DEVICE, "%s failed: %s (%s:%d)", #call,                \
                        hipGetErrorString(e_), __FILE__, __LINE__);                        \
    } while (0)

#define QOC(call)                       \
    do {                                \
        qo_status s_ = (call);          \
        if (s_ != QO_OK) return s_;     \
    } while (0)

template <typename T>
qo_status dalloc(qo_ctx *c, T **p, size_t n) {
    void *q = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&q, n * sizeof(T));
    if (e != hipSuccess)
        return fail(c, QO_ERR_ALLOC, "hipMalloc(%zu bytes) failed: %s", n * sizeof(T),
                    hipGetErrorString(e));
    c->allocs.push_back(q);
    e = hipMemsetAsync(q, 0, n * sizeof(T), c->st);
    if (e != hipSuccess) return fail(c, QO_ERR_DEVICE, "hipMemsetAsync failed");
    *p = static_cast<T *>(q);
    return QO_OK;
}


void setup_grid(qo_ctx *c) {
    const qo_config &cf = c->cfg;
    plan_grid(cf.dim, cf.n, cf.L, cf.kinetic, c->N, c->g, c->gcg);
    double h[3];
    for (int k = 0; k < 3; ++k) h[k] = (k < cf.dim) ? cf.L[k] / (cf.n[k] + 1) : 1.0;
    c->w = h[0] * h[1] * (cf.dim == 3 ? h[2] : 1.0);
    const Grid &g = c->g, &q = c->gcg;
    c->qsmax = (long)c->N * (g.tiles() > q.tiles() ? g.tiles() : q.tiles());
}

// ----------------------------------------------------------------- solves

// ---- kernel timing
hipEvent_t prof_event(qo_ctx *c) {
    if (!c->evpool.empty()) {
        hipEvent_t e = c->evpool.back();
        c->evpool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

hipEvent_t prof_begin(qo_ctx *c) {
    if (!c->prof) return nullptr;
    hipEvent_t a = prof_event(c);
    if (a) (void)hipEventRecord(a, c->st);
    return a;
}

void prof_end(qo_ctx *c, int kid, hipEvent_t a) {
    if (!c->prof || !a) return;
    hipEvent_t b = prof_event(c);
    if (!b) {
        c->evpool.push_back(a);
        return;
    }
    (void)hipEventRecord(b, c->st);
    c->pend.push_back({kid, a, b});
}

// Durations of the launches that have completed (in stream order: the first one still
// running ends the harvest; it and the later ones are kept for the next harvest).
void prof_harvest(qo_ctx *c) {
    size_t i = 0;
    for (; i < c->pend.size(); ++i) {
        auto &p = c->pend[i];
        if (hipEventQuery(p.b) != hipSuccess) break;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            c->pdata.ms[p.kid] += ms;
            c->pdata.launches[p.kid] += 1;
            if (p.kid >= QO_KERNEL_GRAM && p.kid <= QO_KERNEL_RESID) c->pdata.work[p.kid] += 1.0;
        }
        c->evpool.push_back(p.a);
        c->evpool.push_back(p.b);
    }
    c->pend.erase(c->pend.begin(), c->pend.begin() + (long)i);
}

// Layout of the pinned read-back area (ints).
constexpr int kMaxRounds = 30;  // refinement rounds per mixed-precision solve, at most
long poll_ints(int N) { return 2L * (N + 8) + 16 + (long)(kMaxRounds + 2) * N; }
int *poll_slot(qo_ctx *c, int parity) { return c->h_poll + (long)parity * (c->N + 8); }
int *round_slot(qo_ctx *c) { return c->h_poll + 2L * (c->N + 8); }
int *stat_slot(qo_ctx *c) { return round_slot(c) + 8; }
int *its_slot(qo_ctx *c, int round) { return round_slot(c) + 16 + (long)round * c->N; }

// Kernel-time work counters of one PCG solve from its per-column iteration counts.
// pform: the FP32 form whose inverse pass reads P_old except at k = 0 (0.6 of its bytes)
// and which runs no first sweep.
void pcg_account(qo_ctx *c, bool f64, const int *its, int ncols, bool zero_start_dst, bool dst,
                 bool pform = false) {
    if (!c->prof) return;
    double colits = 0.0;
    int started = 0;  // columns whose first second sweep ran (x = 0 then: 4 of 5 arrays)
    for (int j = 0; j < ncols; ++j) {
        colits += its[j];
        started += its[j] > 0 ? 1 : 0;
    }
    const int k1 = f64 ? QO_KERNEL_SWEEP1_F64 : QO_KERNEL_SWEEP1_F32;
    const int k2 = f64 ? QO_KERNEL_SWEEP2_F64 : QO_KERNEL_SWEEP2_F32;
    if (!pform) c->pdata.work[k1] += colits;  // the FP32 form has no first sweep
    c->pdata.work[k2] += colits - (zero_start_dst ? 0.2 * started : 0.0);
    if (dst)
        for (int kid : {(int)QO_KERNEL_DST_FWD, (int)QO_KERNEL_DST_PENCIL, (int)QO_KERNEL_DST_INV})
            c->pdata.work[kid] += colits;
    if (pform) c->pdata.work[QO_KERNEL_DST_INV] -= 0.4 * started;
}

qo_status check_poll_err(qo_ctx *c, int code, int col, const char *what) {
    if (code == 5)
        return fail(c, QO_ERR_NOT_SPD,
                    "%s: p.H_sigma p <= 0 in column %d (H_sigma not positive definite; "
                    "increase sigma)",
                    what, col);
    if (code == 7) return fail(c, QO_ERR_NONFINITE, "%s: non-finite value in column %d", what, col);
    return fail(c, QO_ERR_DEVICE, "%s: device error code %d", what, code);
}

// z = M^{-1} r (fast-Poisson preconditioner) for the columns that PCG iteration
// k updates; partial sums of r.z (from the spectral coefficients) into c->rzp.
template <typename T>
qo_status precondition(qo_ctx *c, const T *R, float *Z, int ncols, int k, double tol,
                       const int *mask, const PcgState &s) {
    hipStream_t st = c->st;
    const long qs = (long)ncols * c->g.tiles();
    HIPC(c, launch_pc_prep(k, ncols, mask, s, qs, c->g.tiles(), tol, c->ng, c->pcs, st));
    hipEvent_t e0 = prof_begin(c);
    HIPC(c, launch_dst_fwd<T>(c->dp, R, c->ld, ncols, c->t1, c->pcs, st));
    prof_end(c, QO_KERNEL_DST_FWD, e0);
    hipEvent_t e1 = prof_begin(c);
    HIPC(c, launch_dst_pencil(c->dp, c->t1, c->t2, c->ld, ncols, c->pcs, c->rzp, st));
    prof_end(c, QO_KERNEL_DST_PENCIL, e1);
    hipEvent_t e2 = prof_begin(c);
    HIPC(c, launch_dst_inv(c->dp, c->t2, Z, c->ld, ncols, c->pcs, st));
    prof_end(c, QO_KERNEL_DST_INV, e2);
    return QO_OK;
}

// The flags of a refinement round (active columns, error code and column), copied back
// asynchronously; ev completes when they have arrived.
struct RoundPoll {
    hipEvent_t ev;
    const int *h;
};

// The FP32 form: the same passes, with beta of the PCG step taken from the pencil's r.z
// partials before the inverse plane pass, which then writes the search direction
// P = z + beta P_old (P = z at k = 0) instead of z, and the partial sums of w z^2 that give
// gamma = P.H P without a pass over the grid (launch_pcg_gamma).
qo_status precondition_p(qo_ctx *c, const float *R, const float *Pold, float *Pnew, int ncols,
                         int k, double tol, const int *mask, const PcgState &s) {
    hipStream_t st = c->st;
    const long qs = (long)ncols * c->g.tiles();
    HIPC(c, launch_pc_prep(k, ncols, mask, s, qs, c->g.tiles(), tol, c->ng, c->pcs, st));
    hipEvent_t e0 = prof_begin(c);
    HIPC(c, launch_dst_fwd<float>(c->dp, R, c->ld, ncols, c->t1, c->pcs, st));
    prof_end(c, QO_KERNEL_DST_FWD, e0);
    hipEvent_t e1 = prof_begin(c);
    HIPC(c, launch_dst_pencil(c->dp, c->t1, c->t2, c->ld, ncols, c->pcs, c->rzp, st));
    prof_end(c, QO_KERNEL_DST_PENCIL, e1);
    HIPC(c, launch_rho_beta(k, ncols, c->pcs, c->rzp, c->dp.rzparts, s, c->pbeta, c->rzc, st));
    hipEvent_t e2 = prof_begin(c);
    HIPC(c, launch_dst_inv_p(c->dp, c->t2, k == 0 ? nullptr : Pold, c->pbeta, Pnew, c->ld, ncols,
                             c->pcs, c->vs32, c->wzp, st));
    prof_end(c, QO_KERNEL_DST_INV, e2);
    return QO_OK;
}

// PCG on all columns of B (ld c->ld) into X, precision T: Jacobi, or the
// fast-Poisson preconditioner when c->dst.
//
// The host learns that every column has converged from the activity flags of the first
// sweep, copied back asynchronously every pcg_check iterations.  Those of iteration k are
// read only after iteration k + 1 has been enqueued, so the device never waits for the
// host: if iteration k was the last, the kernels of iteration k + 1 find every column
// inactive and return at once (converged columns are frozen on the device; iteration
// counts and results are those of a synchronous poll).  At pcg_maxit the flags are read
// synchronously.
//
// skip_init: R already holds the residual, X is zero and the partial sums of ||r||^2 and
// of the norm the stop test is relative to sit in s.part (+qs, +2qs); B is not read.
// Only with the fast-Poisson preconditioner (the Jacobi form also needs r.D r).
// outer (may be NULL): the flags of the refinement round that asked for this solve, not
// yet read; they are read once the first iteration is enqueued, and when no column is
// active *outer_done is set and nothing else is done (the enqueued kernels do nothing).
// its_async (may be NULL): the per-column iteration counts are copied there (pinned host
// memory) without waiting, its_out is not written and the caller accounts for the
// work once the copy has completed; otherwise the counts are waited for.
template <typename T>
qo_status pcg(qo_ctx *c, const T *vs, const T *dinv, const T *B, T *X, T *R, T *P0, T *P1,
              int ncols, int use_x0, double tol, const int *mask, const double *coltol,
              int *its_out, const char *what, bool skip_init = false,
              const RoundPoll *outer = nullptr, bool *outer_done = nullptr,
              int *its_async = nullptr) {
    const Grid &g = c->g;
    hipStream_t st = c->st;
    PcgState s = c->ps;
    s.coltol = coltol;
    HIPC(c, hipMemsetAsync(s.its, 0, sizeof(int) * ncols, st));
    int init_err[2] = {0, INT_MAX};
    HIPC(c, hipMemcpyAsync(s.err, init_err, sizeof init_err, hipMemcpyHostToDevice, st));
    if (!(skip_init && c->dst))
        HIPC(c, launch_pcg_init<T>(g, vs, dinv, B, X, R, c->ld, ncols, use_x0, s.part, st));
    T *pbuf[2] = {P0, P1};
    const int check = c->cfg.pcg_check;
    const int maxit = c->cfg.pcg_maxit;
    const bool f64 = sizeof(T) == 8;
    const int k1 = f64 ? QO_KERNEL_SWEEP1_F64 : QO_KERNEL_SWEEP1_F32;
    const int k2 = f64 ? QO_KERNEL_SWEEP2_F64 : QO_KERNEL_SWEEP2_F32;
    float *Z = c->dst ? c->z32 : nullptr;
    const bool pform = !f64 && Z != nullptr;  // FP32 fast-Poisson: P formed by the inverse pass
    // activity flags and error code of iteration k into the slot of its parity
    auto post_poll = [&](int k) -> qo_status {
        int *h = poll_slot(c, k & 1);
        HIPC(c, hipMemcpyAsync(h, s.active + (k & 1) * ncols, sizeof(int) * ncols,
                               hipMemcpyDeviceToHost, st));
        HIPC(c, hipMemcpyAsync(h + ncols, s.err, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPC(c, hipEventRecord(c->pev[k & 1], st));
        return QO_OK;
    };
    // wait for the flags of iteration k; *nact: columns still active
    auto read_poll = [&](int k, int *nact) -> qo_status {
        HIPC(c, hipEventSynchronize(c->pev[k & 1]));
        prof_harvest(c);
        const int *h = poll_slot(c, k & 1);
        if (h[ncols]) return check_poll_err(c, h[ncols], h[ncols + 1], what);
        int n = 0;
        for (int j = 0; j < ncols; ++j) n += h[j] ? 1 : 0;
        *nact = n;
        return QO_OK;
    };
    int pend = -1;  // the iteration whose flags are in flight
    for (int k = 0;; ++k) {
        if (pform)
            QOC(precondition_p(c, reinterpret_cast<const float *>(R),
                               reinterpret_cast<const float *>(pbuf[(k + 1) & 1]),
                               reinterpret_cast<float *>(pbuf[k & 1]), ncols, k, tol, mask, s));
        else if (Z)
            QOC(precondition<T>(c, R, Z, ncols, k, tol, mask, s));
        if (pform) {
            HIPC(c, launch_pcg_gamma(g, k, ncols, tol, mask, s, c->rzc, c->wzp,
                                     c->dp.nslab * (c->dp.RP / 16), st));
        } else {
            hipEvent_t ea = prof_begin(c);
            HIPC(c, launch_pcg_sweep1<T>(g, vs, dinv, R, pbuf[(k + 1) & 1], pbuf[k & 1], c->ld,
                                         ncols, k, tol, mask, s, st, Z, c->rzp, c->dp.rzparts));
            prof_end(c, k1, ea);
        }
        if (outer && k == 0) {
            HIPC(c, hipEventSynchronize(outer->ev));
            prof_harvest(c);
            if (outer->h[1]) return check_poll_err(c, outer->h[1], outer->h[2], what);
            if (outer->h[0] == 0) {
                *outer_done = true;
                return QO_OK;
            }
        }
        if (k >= maxit) {
            int nact = 0;
            QOC(post_poll(k));
            QOC(read_poll(k, &nact));
            if (nact == 0) break;
            return fail(c, QO_ERR_PCG_NOCONV, "%s: %d of %d columns not converged after %d "
                        "PCG iterations (tol %.3g)", what, nact, ncols, maxit, tol);
        }
        const bool poll_now = k % check == 0;
        if (poll_now) QOC(post_poll(k));
        if (pend >= 0) {
            int nact = 0;
            QOC(read_poll(pend, &nact));
            if (nact == 0) break;
        }
        pend = poll_now ? k : -1;
        hipEvent_t eb = prof_begin(c);
        HIPC(c, launch_pcg_sweep2<T>(g, vs, dinv, pbuf[k & 1], X, R, c->ld, ncols, k, s, st,
                                     Z == nullptr, k == 0 && skip_init && Z != nullptr));
        prof_end(c, k2, eb);
    }
    if (its_async) {
        HIPC(c, hipMemcpyAsync(its_async, s.its, sizeof(int) * ncols, hipMemcpyDeviceToHost, st));
        return QO_OK;
    }
    int *h = poll_slot(c, 0);
    HIPC(c, hipMemcpyAsync(h, s.its, sizeof(int) * ncols, hipMemcpyDeviceToHost, st));
    HIPC(c, hipStreamSynchronize(st));
    prof_harvest(c);
    for (int j = 0; j < ncols; ++j) its_out[j] = h[j];
    pcg_account(c, f64, its_out, ncols, skip_init && Z, Z != nullptr, pform);
    return QO_OK;
}

// One-sweep (Chronopoulos-Gear) Jacobi-PCG on all columns of B into X.
template <typename T>
qo_status pcg_cg(qo_ctx *c, const T *vs, const T *dinv, const T *B, T *X, T *R0, T *R1, T *P0,
                 T *P1, int ncols, int use_x0, double tol, const int *mask,
                 const double *coltol, int *its_out, const char *what) {
    const Grid &g = c->gcg;
    hipStream_t st = c->st;
    PcgState s = c->ps;
    s.coltol = coltol;
    HIPC(c, hipMemsetAsync(s.its, 0, sizeof(int) * ncols, st));
    int init_err[2] = {0, INT_MAX};
    HIPC(c, hipMemcpyAsync(s.err, init_err, sizeof init_err, hipMemcpyHostToDevice, st));
    double *pbuf[2] = {c->part, c->part + 4 * c->qsmax};
    T *Rb[2] = {R0, R1};
    T *Pb[2] = {P0, P1};
    HIPC(c, launch_pcg_init<T>(g, vs, dinv, B, X, R0, c->ld, ncols, use_x0, pbuf[0], st));
    HIPC(c, launch_cg_delta0<T>(g, vs, dinv, R0, c->ld, ncols, pbuf[0], st));
    const int check = c->cfg.pcg_check;
    const int maxit = c->cfg.pcg_maxit;
    const int kid = sizeof(T) == 8 ? QO_KERNEL_CG_F64 : QO_KERNEL_CG_F32;
    for (int k = 0;; ++k) {
        hipEvent_t ea = prof_begin(c);
        HIPC(c, launch_cg_step<T>(g, vs, dinv, Rb[k & 1], Rb[(k + 1) & 1], Pb[(k + 1) & 1],
                                  Pb[k & 1], X, c->ld, ncols, k, tol, mask, s, pbuf[k & 1],
                                  pbuf[(k + 1) & 1], st));
        prof_end(c, kid, ea);
        if (k % check == 0 || k >= maxit) {
            HIPC(c, hipMemcpyAsync(c->h_poll, s.active + (k & 1) * ncols, sizeof(int) * ncols,
                                   hipMemcpyDeviceToHost, st));
            HIPC(c, hipMemcpyAsync(c->h_poll + ncols, s.err, 2 * sizeof(int),
                                   hipMemcpyDeviceToHost, st));
            HIPC(c, hipStreamSynchronize(st));
            prof_harvest(c);
            if (c->h_poll[ncols]) return check_poll_err(c, c->h_poll[ncols], c->h_poll[ncols + 1], what);
            int nact = 0;
            for (int j = 0; j < ncols; ++j) nact += c->h_poll[j] ? 1 : 0;
            if (nact == 0) break;
            if (k >= maxit)
                return fail(c, QO_ERR_PCG_NOCONV, "%s: %d of %d columns not converged after %d "
                            "PCG iterations (tol %.3g)", what, nact, ncols, maxit, tol);
        }
    }
    HIPC(c, hipMemcpyAsync(c->h_poll, s.its, sizeof(int) * ncols, hipMemcpyDeviceToHost, st));
    HIPC(c, hipStreamSynchronize(st));
    prof_harvest(c);
    double colits = 0.0;
    for (int j = 0; j < ncols; ++j) {
        its_out[j] = c->h_poll[j];
        colits += c->h_poll[j];
    }
    if (c->prof) c->pdata.work[kid] += colits;
    return QO_OK;
}

// Mixed-precision solve with reliable updates: Jacobi-PCG runs in FP32 on the
// correction d (x_true = x + d) and is never restarted; at poll points every
// column whose FP32 recursive residual fell by `rel_delta` since its last
// replacement (or reached the tolerance) gets x += d, d = 0 and its residual
// replaced by the FP64 residual b - H x (rounded to FP32).  The search direction
// is kept, so the Krylov progress of the FP32 iteration is not lost; the FP64
// residual decides convergence.
qo_status solve_mixed_rel(qo_ctx *c, const double *B, double *X, int ncols, int use_x0, int *its,
                          int *rounds, const char *what) {
    const Grid &g = c->g;
    hipStream_t st = c->st;
    PcgState s = c->ps;
    s.coltol = c->zerotol;  // the FP32 stop test is off; the FP64 residual decides
    const double tol = c->cfg.pcg_tol;
    const int tiles = g.tiles();
    double *outer = c->part + 4 * c->qsmax;
    if (!use_x0) HIPC(c, hipMemsetAsync(X, 0, sizeof(double) * c->ld * ncols, st));
    HIPC(c, hipMemsetAsync(c->d32, 0, sizeof(float) * c->ld * ncols, st));
    HIPC(c, hipMemsetAsync(s.its, 0, sizeof(int) * ncols, st));
    int init_err[2] = {0, INT_MAX};
    HIPC(c, hipMemcpyAsync(s.err, init_err, sizeof init_err, hipMemcpyHostToDevice, st));
    std::vector<int> ones(ncols, 1);
    HIPC(c, hipMemcpyAsync(c->need, ones.data(), sizeof(int) * ncols, hipMemcpyHostToDevice, st));
    hipEvent_t er = prof_begin(c);
    HIPC(c, launch_resid_rel(g, c->vs, c->dinv32, B, X, c->ld, c->r32, ncols, c->need, c->part,
                             outer, st));
    prof_end(c, QO_KERNEL_RESID, er);
    HIPC(c, hipMemsetAsync(c->nact, 0, sizeof(int), st));
    HIPC(c, launch_rel_finalize(outer, tiles, ncols, c->need, c->mask, c->rref, c->bb64, tol, 1,
                                c->nact, s.err, st));
    HIPC(c, hipMemcpyAsync(c->h_poll, c->nact, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPC(c, hipMemcpyAsync(c->h_poll + 1, s.err, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
    HIPC(c, hipStreamSynchronize(st));
    prof_harvest(c);
    if (c->h_poll[1]) return check_poll_err(c, c->h_poll[1], c->h_poll[2], what);
    int nrep = 1;
    const int check = c->cfg.pcg_check;
    const int maxit = c->cfg.pcg_maxit;
    if (c->h_poll[0] > 0) {
        float *pbuf[2] = {c->pa32, c->pb32};
        for (int k = 0;; ++k) {
            if (c->dst) QOC(precondition<float>(c, c->r32, c->z32, ncols, k, tol, c->mask, s));
            hipEvent_t ea = prof_begin(c);
            HIPC(c, launch_pcg_sweep1<float>(g, c->vs32, c->dinv32, c->r32, pbuf[(k + 1) & 1],
                                             pbuf[k & 1], c->ld, ncols, k, tol, c->mask, s, st,
                                             c->dst ? c->z32 : nullptr, c->rzp, c->dp.rzparts));
            prof_end(c, QO_KERNEL_SWEEP1_F32, ea);
            hipEvent_t eb = prof_begin(c);
            HIPC(c, launch_pcg_sweep2<float>(g, c->vs32, c->dinv32, pbuf[k & 1], c->d32, c->r32,
                                             c->ld, ncols, k, s, st, !c->dst));
            prof_end(c, QO_KERNEL_SWEEP2_F32, eb);
            if ((k + 1) % check != 0 && k + 1 < maxit) continue;
            int *act = s.active + (k & 1) * ncols;
            HIPC(c, hipMemsetAsync(c->nneed, 0, sizeof(int), st));
            HIPC(c, launch_rel_check(c->part, tiles, ncols, act, c->rref, c->bb64, c->rel_delta,
                                     tol, c->need, c->nneed, st));
            HIPC(c, launch_refine_axpy(X, c->ld, c->d32, c->ld, c->ng, ncols, c->need, 1, st));
            hipEvent_t ec = prof_begin(c);
            HIPC(c, launch_resid_rel(g, c->vs, c->dinv32, B, X, c->ld, c->r32, ncols, c->need,
                                     c->part, outer, st));
            prof_end(c, QO_KERNEL_RESID, ec);
            HIPC(c, hipMemsetAsync(c->nact, 0, sizeof(int), st));
            HIPC(c, launch_rel_finalize(outer, tiles, ncols, c->need, act, c->rref, c->bb64, tol,
                                        0, c->nact, s.err, st));
            HIPC(c, hipMemcpyAsync(c->h_poll, c->nact, sizeof(int), hipMemcpyDeviceToHost, st));
            HIPC(c, hipMemcpyAsync(c->h_poll + 1, s.err, 2 * sizeof(int), hipMemcpyDeviceToHost,
                                   st));
            HIPC(c, hipMemcpyAsync(c->h_poll + 3, c->nneed, sizeof(int), hipMemcpyDeviceToHost,
                                   st));
            HIPC(c, hipStreamSynchronize(st));
            prof_harvest(c);
            if (c->h_poll[1]) return check_poll_err(c, c->h_poll[1], c->h_poll[2], what);
            if (c->h_poll[3] > 0) ++nrep;
            if (c->h_poll[0] == 0) break;
            if (k + 1 >= maxit)
                return fail(c, QO_ERR_PCG_NOCONV, "%s: %d of %d columns above tol %.3g after %d "
                            "FP32 iterations", what, c->h_poll[0], ncols, tol, maxit);
        }
    }
    HIPC(c, hipMemcpyAsync(c->h_poll, s.its, sizeof(int) * ncols, hipMemcpyDeviceToHost, st));
    HIPC(c, hipStreamSynchronize(st));
    double colits = 0.0;
    for (int j = 0; j < ncols; ++j) {
        // its[j] is the last iteration index in which the column was active
        its[j] = c->h_poll[j] + 1;
        colits += its[j];
    }
    if (c->prof) {
        c->pdata.work[QO_KERNEL_SWEEP1_F32] += colits;
        c->pdata.work[QO_KERNEL_SWEEP2_F32] += colits;
        if (c->dst)
            for (int kid : {(int)QO_KERNEL_DST_FWD, (int)QO_KERNEL_DST_PENCIL, (int)QO_KERNEL_DST_INV})
                c->pdata.work[kid] += colits;
    }
    *rounds = nrep;
    return QO_OK;
}


// ---- block CG (O'Leary), Jacobi preconditioner, FP64 -----------------------------------

qo_status check_status(qo_ctx *c, const char *what);
__global__ void k_block_axpby(double *__restrict__ Y, const double *__restrict__ X, long ld,
                              long ng, double a, double b);

// out[c] = sum_i X[i][c]^2 (one block per column)
__global__ void k_colnorm2(const double *__restrict__ X, long ld, long ng,
                           double *__restrict__ out) {
    __shared__ double red[16];
    const double *x = X + (long)blockIdx.x * ld;
    double s = 0.0;
    for (long i = threadIdx.x; i < ng; i += blockDim.x) s += x[i] * x[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        out[blockIdx.x] = t;
    }
}

// act_new[c] = act_old[c] (1 when null) and ||r_c|| > tol ||b_c||; a column that stops
// records its iteration k; counts into nact; non-finite norms set err = 7.
__global__ void k_bcg_active(const double *__restrict__ rr, const double *__restrict__ bb,
                             double tol, const int *__restrict__ act_old,
                             int *__restrict__ act_new, int *__restrict__ its, int k, int n,
                             int *__restrict__ nact, int *__restrict__ err) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const int was = act_old ? act_old[c] : 1;
        int a = 0;
        if (!isfinite(rr[c]) || !isfinite(bb[c])) {
            atomicMax(err, 7);
        } else {
            a = was && sqrt(rr[c]) > tol * sqrt(bb[c]);
        }
        if (was && !a) its[c] = k;
        act_new[c] = a;
        if (a) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) *nact = cnt;
}

// Z = D^{-1} R on active columns, 0 elsewhere (column in blockIdx.y)
__global__ void k_bcg_jacobi(double *__restrict__ Z, const double *__restrict__ R,
                             const double *__restrict__ dinv, long ld, long ng,
                             const int *__restrict__ act) {
    const int c = blockIdx.y;
    const long o = (long)c * ld;
    const bool a = act[c] != 0;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < ng;
         i += (long)gridDim.x * blockDim.x)
        Z[o + i] = a ? dinv[i] * R[o + i] : 0.0;
}

// dst = src on active rows and columns, the identity on the others (n x n)
__global__ void k_bcg_mask(double *__restrict__ dst, const double *__restrict__ src, int n,
                           const int *__restrict__ act) {
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
        const int i = e % n, j = e / n;
        dst[e] = (act[i] && act[j]) ? src[e] : (i == j ? 1.0 : 0.0);
    }
}

// X = G B for ncols columns by block PCG: one search block for all columns, s x s step
// matrices alpha = (P^T H P)^{-1} (Z^T R) and beta = (Z^T R)_old^{-1} (Z^T R)_new, Jacobi
// preconditioner; a column that meets ||r|| <= tol ||b|| is deflated (identity rows and
// columns in the small matrices, zero search direction).  Converged columns' iteration
// counts into its.  Host polls the active count after every iteration.
qo_status solve_bcg(qo_ctx *c, const double *B, double *X, int n, int use_x0, double tol,
                    int *its_out, const char *what) {
    hipStream_t st = c->st;
    const long ld = c->ld, ng = c->ng;
    const int N = c->N;
    const size_t blk = (size_t)ld * N, nn = (size_t)N * N;
    for (int i = 0; i < 4; ++i)
        if (!c->bcgb[i]) QOC(dalloc(c, &c->bcgb[i], blk));
    if (!c->bcgm) QOC(dalloc(c, &c->bcgm, 8 * nn));
    if (!c->bcgv) QOC(dalloc(c, &c->bcgv, (size_t)2 * N));
    if (!c->bcga) QOC(dalloc(c, &c->bcga, (size_t)3 * N + 4));
    double *Z = c->bcgb[0];
    double *Xc = X, *Xn = c->bcgb[1];
    double *Rc = c->r, *Rn = c->bcgb[2];
    double *Pc = c->pa, *Pn = c->bcgb[3];
    double *Q = c->pb;
    double *Gt = c->bcgm, *Gm = Gt + nn, *rho = Gm + nn, *rhon = rho + nn, *alpha = rhon + nn,
           *aT = alpha + nn, *naT = aT + nn, *rhom = naT + nn;
    double *rr = c->bcgv, *bb = rr + N;
    int *act = c->bcga, *actn = act + N, *its = actn + N, *nact = its + N, *err = nact + 1;
    long vb = (ng + 255) / 256;
    if (vb > 1024) vb = 1024;
    const dim3 vgrid((unsigned)vb, (unsigned)n);
    HIPC(c, hipMemsetAsync(its, 0, sizeof(int) * n, st));
    HIPC(c, hipMemsetAsync(err, 0, sizeof(int), st));
    if (use_x0) {
        HIPC(c, launch_apply(c->g, c->vs, Xc, Rc, ld, n, st));
        hipLaunchKernelGGL(k_block_axpby, vgrid, dim3(256), 0, st, Rc, B, ld, ng, 1.0, -1.0);
        HIPC(c, hipGetLastError());
    } else {
        HIPC(c, hipMemsetAsync(Xc, 0, sizeof(double) * ld * n, st));
        HIPC(c, hipMemcpyAsync(Rc, B, sizeof(double) * ld * n, hipMemcpyDeviceToDevice, st));
    }
    hipLaunchKernelGGL(k_colnorm2, dim3(n), dim3(256), 0, st, B, ld, ng, bb);
    hipLaunchKernelGGL(k_colnorm2, dim3(n), dim3(256), 0, st, Rc, ld, ng, rr);
    hipLaunchKernelGGL(k_bcg_active, dim3(1), dim3(256), 0, st, rr, bb, tol, nullptr, act, its,
                       0, n, nact, err);
    hipLaunchKernelGGL(k_bcg_jacobi, vgrid, dim3(256), 0, st, Z, Rc, c->dinv, ld, ng, act);
    HIPC(c, hipMemcpyAsync(Pc, Z, sizeof(double) * ld * n, hipMemcpyDeviceToDevice, st));
    HIPC(c, launch_gram_cross_f64(Z, Rc, ld, ng, n, 1.0, c->gpart, c->gnsplit, Gt, st));
    hipLaunchKernelGGL(k_bcg_mask, dim3(64), dim3(256), 0, st, rho, Gt, n, act);
    HIPC(c, hipGetLastError());
    const int maxit = c->cfg.pcg_maxit;
    const int stall = 50;
    std::vector<double> h_rr(n), h_bb(n);
    std::vector<int> h_act(n);
    HIPC(c, hipMemcpyAsync(h_bb.data(), bb, sizeof(double) * n, hipMemcpyDeviceToHost, st));
    double best = INFINITY;
    int k = 0, kbest = 0;
    bool breakdown = false;
    // the search block can lose rank while columns are still active: singular P^T H P or
    // (Z^T R)_old, or no halving of the largest relative residual in `stall` iterations;
    // the column solver then finishes from the current X
    auto status_clear = [&]() -> qo_status {
        int hs = 0;
        HIPC(c, hipMemcpyAsync(&hs, c->dstatus, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPC(c, hipStreamSynchronize(st));
        if (hs == 7) return fail(c, QO_ERR_NONFINITE, "%s: non-finite block CG matrices", what);
        breakdown = hs != 0;
        return QO_OK;
    };
    for (;;) {
        int poll[2] = {0, 0};
        HIPC(c, hipMemcpyAsync(poll, nact, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPC(c, hipMemcpyAsync(h_rr.data(), rr, sizeof(double) * n, hipMemcpyDeviceToHost, st));
        HIPC(c, hipMemcpyAsync(h_act.data(), act, sizeof(int) * n, hipMemcpyDeviceToHost, st));
        HIPC(c, hipStreamSynchronize(st));
        if (poll[1]) return fail(c, QO_ERR_NONFINITE, "%s: non-finite residual in block CG", what);
        if (poll[0] == 0) break;
        if (k >= maxit)
            return fail(c, QO_ERR_PCG_NOCONV, "%s: %d of %d columns not converged after %d "
                        "block CG iterations (tol %.3g)", what, poll[0], n, maxit, tol);
        double worst = 0.0;
        for (int j = 0; j < n; ++j)
            if (h_act[j]) worst = std::max(worst, std::sqrt(h_rr[j] / h_bb[j]));
        if (worst < 0.5 * best) {
            best = worst;
            kbest = k;
        }
        if (k - kbest > stall) {
            breakdown = true;
            break;
        }
        ++k;
        // Q = H P; alpha = mask(P^T Q)^{-1} rho
        HIPC(c, launch_apply(c->g, c->vs, Pc, Q, ld, n, st));
        HIPC(c, launch_gram_cross_f64(Pc, Q, ld, ng, n, 1.0, c->gpart, c->gnsplit, Gt, st));
        hipLaunchKernelGGL(k_bcg_mask, dim3(64), dim3(256), 0, st, Gm, Gt, n, act);
        HIPC(c, hipMemcpyAsync(alpha, rho, sizeof(double) * n * n, hipMemcpyDeviceToDevice, st));
        HIPC(c, hipMemsetAsync(c->dstatus, 0, sizeof(int), st));
        HIPC(c, nn_gj_solve(Gm, n, alpha, n, n, n, false, c->dstatus, st, c->gjw, c->gjpiv));
        QOC(status_clear());
        if (breakdown) {
            --k;
            break;
        }
        // X += P alpha, R -= Q alpha (the small operand is passed row-major: alpha^T)
        HIPC(c, nn_axpby(aT, n, 0.0, nullptr, n, 1.0, alpha, n, true, 0.0, n, n, st));
        HIPC(c, nn_axpby(naT, n, 0.0, nullptr, n, -1.0, alpha, n, true, 0.0, n, n, st));
        HIPC(c, launch_tsgemm(Xn, ld, Xc, Pc, aT, nullptr, nullptr, ld, ng, n, st));
        HIPC(c, launch_tsgemm(Rn, ld, Rc, Q, naT, nullptr, nullptr, ld, ng, n, st));
        std::swap(Xc, Xn);
        std::swap(Rc, Rn);
        // deflate the columns that met the tolerance
        hipLaunchKernelGGL(k_colnorm2, dim3(n), dim3(256), 0, st, Rc, ld, ng, rr);
        hipLaunchKernelGGL(k_bcg_active, dim3(1), dim3(256), 0, st, rr, bb, tol, act, actn, its,
                           k, n, nact, err);
        // Z = D^{-1} R; beta = mask(rho)^{-1} mask(Z^T R); P = Z + P beta
        hipLaunchKernelGGL(k_bcg_jacobi, vgrid, dim3(256), 0, st, Z, Rc, c->dinv, ld, ng, actn);
        HIPC(c, launch_gram_cross_f64(Z, Rc, ld, ng, n, 1.0, c->gpart, c->gnsplit, Gt, st));
        hipLaunchKernelGGL(k_bcg_mask, dim3(64), dim3(256), 0, st, rhon, Gt, n, actn);
        hipLaunchKernelGGL(k_bcg_mask, dim3(64), dim3(256), 0, st, rhom, rho, n, actn);
        HIPC(c, hipMemcpyAsync(alpha, rhon, sizeof(double) * n * n, hipMemcpyDeviceToDevice, st));
        HIPC(c, hipMemsetAsync(c->dstatus, 0, sizeof(int), st));
        HIPC(c, nn_gj_solve(rhom, n, alpha, n, n, n, false, c->dstatus, st, c->gjw, c->gjpiv));
        std::swap(act, actn);
        QOC(status_clear());
        if (breakdown) break;
        HIPC(c, nn_axpby(aT, n, 0.0, nullptr, n, 1.0, alpha, n, true, 0.0, n, n, st));
        HIPC(c, launch_tsgemm(Pn, ld, Z, Pc, aT, nullptr, nullptr, ld, ng, n, st));
        std::swap(Pc, Pn);
        std::swap(rho, rhon);
    }
    if (breakdown) {
        // finish with the column solver from the current X (it reuses r, pa, pb)
        std::vector<int> h_its(n), col_its(n);
        HIPC(c, hipMemcpyAsync(h_its.data(), its, sizeof(int) * n, hipMemcpyDeviceToHost, st));
        HIPC(c, hipMemcpyAsync(h_act.data(), act, sizeof(int) * n, hipMemcpyDeviceToHost, st));
        HIPC(c, hipStreamSynchronize(st));
        QOC(pcg<double>(c, c->vs, c->dinv, B, Xc, c->r, c->pa, c->pb, n, 1, tol, nullptr,
                        nullptr, col_its.data(), what));
        if (Xc != X)
            HIPC(c, hipMemcpyAsync(X, Xc, sizeof(double) * ld * n, hipMemcpyDeviceToDevice, st));
        HIPC(c, hipStreamSynchronize(st));
        for (int j = 0; j < n; ++j) its_out[j] = h_act[j] ? k + col_its[j] : h_its[j];
        return QO_OK;
    }
    if (Xc != X) HIPC(c, hipMemcpyAsync(X, Xc, sizeof(double) * ld * n, hipMemcpyDeviceToDevice, st));
    std::vector<int> h_its(n);
    HIPC(c, hipMemcpyAsync(h_its.data(), its, sizeof(int) * n, hipMemcpyDeviceToHost, st));
    HIPC(c, hipStreamSynchronize(st));
    for (int j = 0; j < n; ++j) its_out[j] = h_its[j];
    return QO_OK;
}

// X = G B for ncols columns of internal-layout blocks.  its: per column.
// zb (optional, mixed fast-Poisson solves of all N columns): the row-blocked BF16 copy of
// X that the Gram of the solution block reads; *zb_ok says whether the solve left it
// holding X (its last residual pass formed X), so the Gram need not pack X itself.
qo_status solve_block(qo_ctx *c, const double *B, double *X, int ncols, int use_x0, int *its,
                      int *rounds, const char *what, __bf16 *zb = nullptr,
                      bool *zb_ok = nullptr) {
    if (zb_ok) *zb_ok = false;
    const double tol = c->cfg.pcg_tol;
    const bool one_sweep = c->cfg.pcg_variant == 1;
    if (!c->mixed && c->cfg.pcg_variant == 2) {
        *rounds = 1;
        return solve_bcg(c, B, X, ncols, use_x0, tol, its, what);
    }
    if (!c->mixed) {
        *rounds = 1;
        if (one_sweep)
            return pcg_cg<double>(c, c->vs, c->dinv, B, X, c->r, c->r2, c->pa, c->pb, ncols,
                                  use_x0, tol, nullptr, nullptr, its, what);
        return pcg<double>(c, c->vs, c->dinv, B, X, c->r, c->pa, c->pb, ncols, use_x0, tol,
                           nullptr, nullptr, its, what);
    }
    // Reliable updates keep the FP32 search direction across a residual replacement,
    // which suits slowly converging Jacobi-PCG (the FP32 and FP64 residuals still agree
    // when a replacement is due).  With the fast-Poisson preconditioner a few iterations
    // take the FP32 residual to its rounding floor, the replaced residual is no longer
    // close to the recursive one, and the kept direction stalls the iteration: there the
    // inner FP32 solve is restarted each round instead.
    if (c->rel && !one_sweep && !c->dst)
        return solve_mixed_rel(c, B, X, ncols, use_x0, its, rounds, what);
    // FP64 iterative refinement around FP32 PCG (restarted each round)
    hipStream_t st = c->st;
    const Grid &g = c->g;
    if (!use_x0) HIPC(c, hipMemsetAsync(X, 0, sizeof(double) * c->ld * ncols, st));
    for (int j = 0; j < ncols; ++j) its[j] = 0;
    std::vector<int> inner(ncols);
    const long qs = (long)ncols * g.tiles();
    const int max_rounds = kMaxRounds;
    // With the fast-Poisson solve the update x += d of one round is taken by the residual
    // pass of the next, which writes x + d out of place: the iterate moves between X and
    // the spare FP64 block r (not used by the mixed solve otherwise).  There the round's
    // convergence flags are read only after the next inner solve's first iteration has
    // been enqueued (that iteration does nothing when the round found every column
    // converged), and the inner iteration counts are gathered at the end.
    const bool fused = c->dst && !one_sweep;
    double *xc = X, *xs = c->r;
    bool pending = false;
    int done_rounds = 0;
    for (int round = 0;; ++round) {
        int init_err[2] = {0, INT_MAX};
        HIPC(c, hipMemcpyAsync(c->ps.err, init_err, sizeof init_err, hipMemcpyHostToDevice, st));
        hipEvent_t er = prof_begin(c);
        if (pending) {
            HIPC(c, launch_resid_next(g, c->vs, B, xc, c->d32, xs, c->ld, c->r32, ncols, c->mask,
                                      c->ps.its, c->part, st, ncols == c->N ? zb : nullptr,
                                      c->N));
            std::swap(xc, xs);
            pending = false;
        } else {
            HIPC(c, launch_resid(g, c->vs, B, xc, c->ld, c->r32, c->ld, ncols, nullptr, c->part,
                                 st));
        }
        prof_end(c, QO_KERNEL_RESID, er);
        HIPC(c, launch_colsum(c->part + qs, g.tiles(), ncols, 2, qs, c->colsums, st));
        HIPC(c, launch_refine_mask(c->colsums, ncols, tol, c->cfg.refine_inner_tol, c->mask,
                                   c->coltol, c->nact, c->ps.err, st));
        int *hr = round_slot(c);
        HIPC(c, hipMemcpyAsync(hr, c->nact, sizeof(int), hipMemcpyDeviceToHost, st));
        HIPC(c, hipMemcpyAsync(hr + 1, c->ps.err, 2 * sizeof(int), hipMemcpyDeviceToHost, st));
        HIPC(c, hipEventRecord(c->rev, st));
        bool done = false;
        const bool speculate = fused && round < max_rounds;
        if (!speculate) {
            HIPC(c, hipEventSynchronize(c->rev));
            prof_harvest(c);
            if (hr[1]) return check_poll_err(c, hr[1], hr[2], what);
            done = hr[0] == 0;
            if (!done && round >= max_rounds)
                return fail(c, QO_ERR_PCG_NOCONV,
                            "%s: refinement did not reach tol %.3g in %d rounds", what, tol,
                            max_rounds);
        }
        if (!done) {
            if (one_sweep) {
                QOC(pcg_cg<float>(c, c->vs32, c->dinv32, c->r32, c->d32, c->rr32, c->rr32b,
                                  c->pa32, c->pb32, ncols, 0, c->cfg.refine_inner_tol, c->mask,
                                  c->coltol, inner.data(), what));
            } else if (c->dst) {
                // The FP32 solve works on r32 in place (the next round recomputes it) and
                // skips its init pass: it starts from d = 0 without clearing d (its first
                // update writes d = alpha p instead of adding), and ||r||^2 from the residual
                // pass serves as both the starting residual and the norm the inner stop test
                // is relative to.
                HIPC(c, hipMemcpyAsync(c->part + 2 * qs, c->part + qs, sizeof(double) * qs,
                                       hipMemcpyDeviceToDevice, st));
                const RoundPoll rp{c->rev, hr};
                bool outer_done = false;
                QOC(pcg<float>(c, c->vs32, c->dinv32, c->r32, c->d32, c->r32, c->pa32, c->pb32,
                               ncols, 0, c->cfg.refine_inner_tol, c->mask, c->coltol,
                               inner.data(), what, true, speculate ? &rp : nullptr, &outer_done,
                               its_slot(c, round)));
                done = outer_done;
            } else {
                QOC(pcg<float>(c, c->vs32, c->dinv32, c->r32, c->d32, c->rr32, c->pa32, c->pb32,
                               ncols, 0, c->cfg.refine_inner_tol, c->mask, c->coltol,
                               inner.data(), what));
            }
        }
        if (done) {
            *rounds = round;
            done_rounds = round;
            // round >= 1: the last pass was a fused residual pass, which formed X
            if (zb_ok) *zb_ok = zb && fused && ncols == c->N && round >= 1;
            if (xc != X)
                HIPC(c, hipMemcpyAsync(X, xc, sizeof(double) * c->ld * ncols,
                                       hipMemcpyDeviceToDevice, st));
            break;
        }
        if (!c->dst || one_sweep)
            for (int j = 0; j < ncols; ++j) its[j] += inner[j];
        // With the fast-Poisson solve d was written only in columns that took at least one
        // inner iteration (the others hold an older correction): those alone are updated.
        if (fused)
            pending = true;
        else
            HIPC(c, launch_refine_axpy(xc, c->ld, c->d32, c->ld, c->ng, ncols, c->mask, 0, st));
    }
    if (fused) {
        // every round's counts were copied before the last round's flags, which have been
        // read: the copies are complete
        for (int r = 0; r < done_rounds; ++r) {
            const int *h = its_slot(c, r);
            for (int j = 0; j < ncols; ++j) its[j] += h[j];
            pcg_account(c, false, h, ncols, true, true, true);
        }
    }
    return QO_OK;
}

// Grams of [X | Y]; in a step [U | P] and [U_hat | Q].  Mixed precision takes the BF16
// copies of U and U_hat that their producers wrote (U is packed if it has changed otherwise
// since) and packs the solution block; any other X is packed into the U_hat copy, which
// only the step's own U_hat update fills before its Gram.
qo_status gram(qo_ctx *c, const double *X, const double *Y, long ld, int n, double *G,
               bool y_packed = false) {
    hipEvent_t e = prof_begin(c);
    if (c->mixed) {
        const bool xu = X == c->U && n == c->N, xh = X == c->Uh && n == c->N;
        HIPC(c, launch_gram_bf16(X, Y, ld, c->ng, n, c->w, c->gpart, c->gnsplit, G,
                                 xu ? c->zbU : c->zbUh, c->zbPQ, !xh && !(xu && c->zbU_ok),
                                 !(y_packed && n == c->N), c->st));
        if (xu) c->zbU_ok = true;
    } else
        HIPC(c, launch_gram_f64(X, Y, ld, c->ng, n, c->w, c->gpart, c->gnsplit, G, c->st));
    prof_end(c, QO_KERNEL_GRAM, e);
    return QO_OK;
}

// fp32: the FP32-arithmetic update of the mixed-precision step (see launch_tsgemm); zb
// receives its BF16 copy
qo_status tsgemm(qo_ctx *c, double *Out, const double *C0, const double *A, const double *Xr,
                 const double *Bm, const double *Yr, bool fp32 = false, __bf16 *zb = nullptr,
                 double *Out2 = nullptr, const double *Zr = nullptr) {
    hipEvent_t e = prof_begin(c);
    HIPC(c, launch_tsgemm(Out, c->ld, C0, A, Xr, Bm, Yr, c->ld, c->ng, c->N, c->st, fp32, zb,
                          fp32 ? c->split3 : nullptr, Out2, Zr));
    prof_end(c, QO_KERNEL_UPDATE, e);
    return QO_OK;
}

// Gram in FP64 regardless of precision (outputs and diagnostics)
qo_status gram64(qo_ctx *c, const double *X, const double *Y, long ld, int n, double *G) {
    HIPC(c, launch_gram_f64(X, Y, ld, c->ng, n, c->w, c->gpart, c->gnsplit, G, c->st));
    return QO_OK;
}

// named N x N matrices in the pool
enum {
    MP_SW, MP_C, MP_RW, MP_D, MP_RWS, MP_MAT, MP_RHS, MP_A, MP_X, MP_Y, MP_Z, MP_XR, MP_YR,
    MP_ZR, MP_O, MP_OR, MP_MS, MP_T1, MP_T2, MP_T3, MP_COUNT
};

double *mp(qo_ctx *c, int i) { return c->mpool + (size_t)i * c->N * c->N; }

qo_status energy_of(qo_ctx *c, const double *U, double *Es, double *trS) {
    const Grid &g = c->g;
    const int N = c->N;
    const long qs = (long)N * g.tiles();
    HIPC(c, launch_quad(g, c->vs, U, c->ld, N, c->part, c->st));
    HIPC(c, launch_colsum(c->part, g.tiles(), N, 2, qs, c->colsums, c->st));
    HIPC(c, nn_energy_finish(c->colsums, N, c->w, c->dscal + 4, c->st));
    HIPC(c, hipMemcpyAsync(c->h_scal + 4, c->dscal + 4, 2 * sizeof(double), hipMemcpyDeviceToHost,
                           c->st));
    HIPC(c, hipStreamSynchronize(c->st));
    *Es = c->h_scal[4];
    *trS = c->h_scal[5];
    return QO_OK;
}

qo_status status_error(qo_ctx *c, int hs, const char *what) {
    if (hs == 5) return fail(c, QO_ERR_NOT_SPD, "%s: matrix not positive definite / singular", what);
    if (hs == 7) return fail(c, QO_ERR_NONFINITE, "%s: non-finite matrix entries", what);
    if (hs) return fail(c, QO_ERR_DEVICE, "%s: status %d", what, hs);
    return QO_OK;
}

qo_status check_status(qo_ctx *c, const char *what) {
    int hs = 0;
    HIPC(c, hipMemcpyAsync(&hs, c->dstatus, sizeof(int), hipMemcpyDeviceToHost, c->st));
    HIPC(c, hipStreamSynchronize(c->st));
    if (hs == 5) return fail(c, QO_ERR_NOT_SPD, "%s: matrix not positive definite / singular", what);
    if (hs == 7) return fail(c, QO_ERR_NONFINITE, "%s: non-finite matrix entries", what);
    if (hs) return fail(c, QO_ERR_DEVICE, "%s: status %d", what, hs);
    return QO_OK;
}

void rec(qo_ctx *c, int i) {
    if (c->ev_ok) (void)hipEventRecord(c->ev[i], c->st);
}

// out[0] = 1/2 tr(A) + a tr(B) + b for n x n column-major A, B (one block)
__global__ void k_trace2(const double *__restrict__ A, const double *__restrict__ B, int n,
                         double a, double b, double *__restrict__ out) {
    __shared__ double red[16];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) s += 0.5 * A[(long)i * n + i] + a * B[(long)i * n + i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        out[0] = t + b;
    }
}

// K = <U, H_sigma U> of the current state from the stencil (FP64): apply into the residual
// buffer (free between solves), Gram of [U | H U], block (0,1).
qo_status anchor_K(qo_ctx *c) {
    const int N = c->N, N2 = 2 * N;
    HIPC(c, launch_apply(c->g, c->vs, c->U, c->r, c->ld, N, c->st));
    QOC(gram64(c, c->U, c->r, c->ld, N, c->G2));
    HIPC(c, nn_axpby(c->Kprop, N, 1.0, c->G2 + (size_t)N * N2, N2, 0.0, nullptr, N, false, 0.0,
                     N, N, c->st));
    c->have_K = true;
    return QO_OK;
}

// K_{n+1} from K_n and the step's small matrices.  With H_sigma P = U and H_sigma Q = U_hat
// (the solves), <U, H P> = <P, H U> = S and <P, H P> = M^T, so
//   K_hat = X^T K X + X^T S Y + Y^T S X + Y^T M^T Y      (U_hat = U X + P Y),
// and with <U_hat, H Q> = S_hat, <Q, H Q> = A^T (A = <U_hat, Q>),
//   K_{n+1} = K_hat - tau (S_hat O + O S_hat) + tau^2 O A^T O   (U_{n+1} = U_hat - tau Q O).
// E_sigma(U_{n+1}) = 1/2 tr K_{n+1} and tr S_{n+1} = tr O_{n+1} + N go to dscal[4..5].
qo_status propagate_K(qo_ctx *c, double tau, const double *X, const double *Y,
                      const double *O, const double *On) {
    const int N = c->N, N2 = 2 * N;
    hipStream_t st = c->st;
    const double *S = c->G1, *M = c->G1 + (size_t)N * N2;
    const double *Sh = c->G2, *A = c->G2 + (size_t)N * N2;
    double *T1 = c->epool, *T2 = T1 + (size_t)N * N, *T3 = T2 + (size_t)N * N,
           *Kh = T3 + (size_t)N * N, *Kn = Kh + (size_t)N * N;
    HIPC(c, nn_gemm(T1, N, c->Kprop, N, false, X, N, false, N, N, N, 1.0, 0.0, 0.0, st));
    HIPC(c, nn_gemm(Kh, N, X, N, true, T1, N, false, N, N, N, 1.0, 0.0, 0.0, st));
    HIPC(c, nn_gemm(T2, N, S, N2, false, Y, N, false, N, N, N, 1.0, 0.0, 0.0, st));
    HIPC(c, nn_gemm(T1, N, X, N, true, T2, N, false, N, N, N, 1.0, 0.0, 0.0, st));
    HIPC(c, nn_axpby(T3, N, 1.0, T1, N, 1.0, T1, N, true, 0.0, N, N, st));
    HIPC(c, nn_axpby(Kh, N, 1.0, Kh, N, 1.0, T3, N, false, 0.0, N, N, st));
    HIPC(c, nn_gemm(T2, N, M, N2, true, Y, N, false, N, N, N, 1.0, 0.0, 0.0, st));
    HIPC(c, nn_gemm(Kh, N, Y, N, true, T2, N, false, N, N, N, 1.0, 1.0, 0.0, st));
    HIPC(c, nn_gemm(T1, N, Sh, N2, false, O, N, false, N, N, N, 1.0, 0.0, 0.0, st));
    HIPC(c, nn_axpby(T3, N, 1.0, T1, N, 1.0, T1, N, true, 0.0, N, N, st));
    HIPC(c, nn_axpby(Kn, N, 1.0, Kh, N, -tau, T3, N, false, 0.0, N, N, st));
    HIPC(c, nn_gemm(T1, N, A, N2, true, O, N, false, N, N, N, 1.0, 0.0, 0.0, st));
    HIPC(c, nn_gemm(Kn, N, O, N, false, T1, N, false, N, N, N, tau * tau, 1.0, 0.0, st));
    HIPC(c, hipMemcpyAsync(c->Kprop, Kn, sizeof(double) * N * N, hipMemcpyDeviceToDevice, st));
    hipLaunchKernelGGL(k_trace2, dim3(1), dim3(1024), 0, st, Kn, On, N, 0.0, 0.0, c->dscal + 4);
    HIPC(c, hipGetLastError());
    hipLaunchKernelGGL(k_trace2, dim3(1), dim3(1024), 0, st, On, On, N, 0.5, (double)N,
                       c->dscal + 5);
    HIPC(c, hipGetLastError());
    return QO_OK;
}

// grad_stop > 0: after G U_n and the Gram matrix, stop (return QO_OK with
// *stopped = 1, U_n untouched) when ||grad_G E_G(U_n)|| <= grad_stop.
qo_status one_step(qo_ctx *c, double tau, qo_step_stats *stats, double grad_stop = 0.0,
                   int *stopped = nullptr) {
    const int N = c->N;
    const int N2 = 2 * N;
    hipStream_t st = c->st;
    const long ld = c->ld;
    double *P = c->PQ[c->cur];
    double *Q = c->PQ[c->cur ^ 1];
    const int warm = c->cfg.warm_start ? 1 : 0;
    std::vector<int> itsP(N), itsQ(N);
    int rP = 0, rQ = 0;

    if (c->emode == 1 && (!c->have_K || (c->eanchor > 0 && c->nstep % c->eanchor == 0)))
        QOC(anchor_K(c));
    rec(c, 0);
    bool pP = false, pQ = false;  // the solves left the BF16 Gram copies of P, Q (mixed)
    QOC(solve_block(c, c->U, P, N, warm && c->have_warm, itsP.data(), &rP, "solve G U_n",
                    c->mixed ? c->zbPQ : nullptr, &pP));
    rec(c, 1);
    QOC(gram(c, c->U, P, ld, N, c->G1, pP));
    rec(c, 2);
    double *S = c->G1;
    double *M = c->G1 + (size_t)N * N2;
    double *R = c->G1 + (size_t)N * N2 + N;
    const double alpha = 0.5 * tau;
    HIPC(c, hipMemsetAsync(c->dstatus, 0, sizeof(int), st));
    HIPC(c, nn_grad2(S, M, R, N2, N, mp(c, MP_MS), N, c->dscal + 0, st));
    if (stopped) *stopped = 0;
    if (grad_stop > 0.0) {
        HIPC(c, hipMemcpyAsync(c->h_scal, c->dscal, sizeof(double), hipMemcpyDeviceToHost, st));
        HIPC(c, hipStreamSynchronize(st));
        const double g2 = c->h_scal[0];
        if ((g2 > 0.0 ? sqrt(g2) : 0.0) <= grad_stop) {
            // U_n passes the test: keep it; G U_n is the warm start of a later solve
            if (stopped) *stopped = 1;
            if (stats) {
                memset(stats, 0, sizeof *stats);
                stats->grad_norm = g2 > 0.0 ? sqrt(g2) : 0.0;
                stats->step_index = (int)c->nstep;
            }
            return QO_OK;
        }
    }
    // C = S^{-1} M
    HIPC(c, nn_axpby(mp(c, MP_SW), N, 1.0, S, N2, 0.0, nullptr, N, false, 0.0, N, N, st));
    HIPC(c, nn_axpby(mp(c, MP_C), N, 1.0, M, N2, 0.0, nullptr, N, false, 0.0, N, N, st));
    HIPC(c, nn_gj_solve(mp(c, MP_SW), N, mp(c, MP_C), N, N, N, true, c->dstatus, st, c->gjw, c->gjpiv));
    // R_W = sym(R - M^T C)
    HIPC(c, nn_axpby(mp(c, MP_T1), N, 1.0, R, N2, 0.0, nullptr, N, false, 0.0, N, N, st));
    HIPC(c, nn_gemm(mp(c, MP_T1), N, M, N2, true, mp(c, MP_C), N, false, N, N, N, -1.0, 1.0, 0.0, st));
    HIPC(c, nn_axpby(mp(c, MP_RW), N, 0.5, mp(c, MP_T1), N, 0.5, mp(c, MP_T1), N, true, 0.0, N, N, st));
    // D = C S - M^T
    HIPC(c, nn_gemm(mp(c, MP_D), N, mp(c, MP_C), N, false, S, N2, false, N, N, N, 1.0, 0.0, 0.0, st));
    HIPC(c, nn_axpby(mp(c, MP_D), N, 1.0, mp(c, MP_D), N, -1.0, M, N2, true, 0.0, N, N, st));
    // RWS = R_W S
    HIPC(c, nn_gemm(mp(c, MP_RWS), N, mp(c, MP_RW), N, false, S, N2, false, N, N, N, 1.0, 0.0, 0.0, st));
    // (I + alpha^2 RWS - alpha D) b = D - alpha RWS
    HIPC(c, nn_axpby(mp(c, MP_MAT), N, alpha * alpha, mp(c, MP_RWS), N, -alpha, mp(c, MP_D), N, false, 1.0, N, N, st));
    HIPC(c, nn_axpby(mp(c, MP_RHS), N, 1.0, mp(c, MP_D), N, -alpha, mp(c, MP_RWS), N, false, 0.0, N, N, st));
    HIPC(c, nn_gj_solve(mp(c, MP_MAT), N, mp(c, MP_RHS), N, N, N, false, c->dstatus, st, c->gjw, c->gjpiv));
    double *bm = mp(c, MP_RHS);
    // a = S + alpha S b
    HIPC(c, nn_axpby(mp(c, MP_A), N, 1.0, S, N2, 0.0, nullptr, N, false, 0.0, N, N, st));
    HIPC(c, nn_gemm(mp(c, MP_A), N, S, N2, false, bm, N, false, N, N, N, alpha, 1.0, 0.0, st));
    // X = I + tau b - tau C a ; Y = tau a ; Z = X + C Y
    HIPC(c, nn_axpby(mp(c, MP_X), N, tau, bm, N, 0.0, nullptr, N, false, 1.0, N, N, st));
    HIPC(c, nn_gemm(mp(c, MP_X), N, mp(c, MP_C), N, false, mp(c, MP_A), N, false, N, N, N, -tau, 1.0, 0.0, st));
    HIPC(c, nn_axpby(mp(c, MP_Y), N, tau, mp(c, MP_A), N, 0.0, nullptr, N, false, 0.0, N, N, st));
    HIPC(c, nn_axpby(mp(c, MP_Z), N, 1.0, mp(c, MP_X), N, 0.0, nullptr, N, false, 0.0, N, N, st));
    HIPC(c, nn_gemm(mp(c, MP_Z), N, mp(c, MP_C), N, false, mp(c, MP_Y), N, false, N, N, N, 1.0, 1.0, 0.0, st));
    // row-major copies for the block update
    HIPC(c, nn_axpby(mp(c, MP_XR), N, 0.0, nullptr, N, 1.0, mp(c, MP_X), N, true, 0.0, N, N, st));
    HIPC(c, nn_axpby(mp(c, MP_YR), N, 0.0, nullptr, N, 1.0, mp(c, MP_Y), N, true, 0.0, N, N, st));
    HIPC(c, nn_axpby(mp(c, MP_ZR), N, 0.0, nullptr, N, 1.0, mp(c, MP_Z), N, true, 0.0, N, N, st));
    // The predictor's status is read back without waiting; it is looked at once the second
    // solve is done (before any error of that solve, which a failed N x N solve may cause).
    // U_n is not written before then, so a failure still leaves the step undone.
    HIPC(c, hipMemcpyAsync(stat_slot(c), c->dstatus, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPC(c, hipEventRecord(c->sev, st));
    rec(c, 3);
    // U_hat = U X + P Y and, with warm starts, x0 = P Z in one launch that reads P once
    // (QO_MIXED: FP32-accurate arithmetic; the Grams of that path are BF16)
    QOC(tsgemm(c, c->Uh, nullptr, c->U, mp(c, MP_XR), P, mp(c, MP_YR), c->mixed,
               c->mixed ? c->zbUh : nullptr, warm ? Q : nullptr,
               warm ? mp(c, MP_ZR) : nullptr));
    rec(c, 4);
    const qo_status sQ = solve_block(c, c->Uh, Q, N, warm, itsQ.data(), &rQ, "solve G U_hat",
                                     c->mixed ? c->zbPQ : nullptr, &pQ);
    HIPC(c, hipEventSynchronize(c->sev));
    QOC(status_error(c, stat_slot(c)[0], "predictor N x N solve"));
    if (sQ != QO_OK) return sQ;
    rec(c, 5);
    QOC(gram(c, c->Uh, Q, ld, N, c->G2, pQ));
    rec(c, 6);
    // O = sym(<U_hat,U_hat>) - I ; corrector coefficient -tau O (symmetric => its own transpose)
    HIPC(c, nn_axpby(mp(c, MP_O), N, 0.5, c->G2, N2, 0.5, c->G2, N2, true, -1.0, N, N, st));
    HIPC(c, nn_axpby(mp(c, MP_OR), N, -tau, mp(c, MP_O), N, 0.0, nullptr, N, false, 0.0, N, N, st));
    HIPC(c, nn_fro(mp(c, MP_O), N, N, c->dscal + 1, st));
    // ||O_{n+1}|| by the Gram recurrence with A = sym<U_hat,Q>, B = <Q,Q>
    {
        double *Am = mp(c, MP_T1), *T2 = mp(c, MP_T2), *On = mp(c, MP_T3);
        HIPC(c, nn_axpby(Am, N, 0.5, c->G2 + (size_t)N * N2, N2, 0.5, c->G2 + (size_t)N * N2, N2,
                         true, 0.0, N, N, st));
        HIPC(c, nn_axpby(On, N, 1.0, mp(c, MP_O), N, 0.0, nullptr, N, false, 0.0, N, N, st));
        HIPC(c, nn_gemm(On, N, Am, N, false, mp(c, MP_O), N, false, N, N, N, -tau, 1.0, 0.0, st));
        HIPC(c, nn_gemm(On, N, mp(c, MP_O), N, false, Am, N, false, N, N, N, -tau, 1.0, 0.0, st));
        HIPC(c, nn_gemm(T2, N, c->G2 + (size_t)N * N2 + N, N2, false, mp(c, MP_O), N, false, N, N,
                        N, 1.0, 0.0, 0.0, st));
        HIPC(c, nn_gemm(On, N, mp(c, MP_O), N, false, T2, N, false, N, N, N, tau * tau, 1.0, 0.0,
                        st));
        HIPC(c, nn_fro(On, N, N, c->dscal + 2, st));
    }
    c->zbU_ok = false;
    QOC(tsgemm(c, c->U, c->Uh, nullptr, nullptr, Q, mp(c, MP_OR), c->mixed,
               c->mixed ? c->zbU : nullptr));
    c->zbU_ok = c->mixed;
    rec(c, 7);
    // the state has moved: commit bookkeeping before the (non-failing) diagnostics
    c->lastP = P;
    c->lastQ = Q;
    c->cur ^= 1;
    c->have_warm = warm != 0;
    c->nstep += 1;
    double Es = 0.0, trS = 0.0;
    if (c->emode == 1) {
        QOC(propagate_K(c, tau, mp(c, MP_X), mp(c, MP_Y), mp(c, MP_O), mp(c, MP_T3)));
        HIPC(c, hipMemcpyAsync(c->h_scal + 4, c->dscal + 4, 2 * sizeof(double),
                               hipMemcpyDeviceToHost, st));
        HIPC(c, hipStreamSynchronize(st));
        Es = c->h_scal[4];
        trS = c->h_scal[5];
    } else {
        QOC(energy_of(c, c->U, &Es, &trS));
    }
    rec(c, 8);
    HIPC(c, hipMemcpyAsync(c->h_scal, c->dscal, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPC(c, hipStreamSynchronize(st));
    prof_harvest(c);
    if (stats) {
        memset(stats, 0, sizeof *stats);
        stats->energy_shifted = Es;
        stats->energy = Es - 0.5 * c->cfg.sigma * trS;
        stats->orth_err_fro = c->h_scal[1];
        const double g2 = c->h_scal[0];
        stats->grad_norm = g2 > 0.0 ? sqrt(g2) : 0.0;
        int mp_ = 0, mq = 0;
        for (int j = 0; j < N; ++j) {
            mp_ = itsP[j] > mp_ ? itsP[j] : mp_;
            mq = itsQ[j] > mq ? itsQ[j] : mq;
        }
        stats->pcg_iters[0] = mp_;
        stats->pcg_iters[1] = mq;
        stats->refine_rounds[0] = rP;
        stats->refine_rounds[1] = rQ;
        stats->energy_rose = (c->have_Es && Es > c->last_Es) ? 1 : 0;
        stats->orth_err_next = c->h_scal[2];
        stats->step_index = (int)c->nstep;
        if (c->ev_ok)
            for (int i = 0; i < 8; ++i) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]) == hipSuccess)
                    stats->t_phase_ms[i] = ms;
            }
    }
    c->have_Es = true;
    c->last_Es = Es;
    return QO_OK;
}

qo_status copy_block_in(qo_ctx *c, double *dst, const double *src, long ld, int on_device) {
    HIPC(c, hipMemcpy2DAsync(dst, c->ld * sizeof(double), src, ld * sizeof(double),
                             c->ng * sizeof(double), c->N,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->st));
    HIPC(c, hipStreamSynchronize(c->st));
    return QO_OK;
}

qo_status copy_block_out(qo_ctx *c, double *dst, long ld, const double *src, int on_device,
                         int ncols) {
    HIPC(c, hipMemcpy2DAsync(dst, ld * sizeof(double), src, c->ld * sizeof(double),
                             c->ng * sizeof(double), ncols,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->st));
    HIPC(c, hipStreamSynchronize(c->st));
    return QO_OK;
}

__global__ void k_prep_potential(const double *__restrict__ V, long ng, double sigma, double c0,
                                 double *__restrict__ vs, double *__restrict__ dinv,
                                 float *__restrict__ vs32, float *__restrict__ dinv32,
                                 int *__restrict__ bad) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < ng;
         i += (long)gridDim.x * blockDim.x) {
        const double v = V[i];
        if (!isfinite(v)) atomicMax(bad, 7);
        const double s = v + sigma;
        const double d = 1.0 / (c0 + s);
        vs[i] = s;
        dinv[i] = d;
        if (vs32) {
            vs32[i] = (float)s;
            dinv32[i] = (float)(1.0 / ((double)(float)c0 + (double)(float)s));
        }
        if (!(c0 + s > 0.0)) atomicMax(bad, 5);
    }
}

// g[j] = w * sum_c Y[c][j] U[c][j]   (row-wise dot of two column-major blocks)
__global__ void k_rowdot(const double *__restrict__ Y, const double *__restrict__ U, long ld,
                         long ng, int n, double w, double *__restrict__ g) {
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < ng;
         j += (long)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < n; ++c) s += Y[(long)c * ld + j] * U[(long)c * ld + j];
        g[j] = w * s;
    }
}

// g[j] += a sum_c Y[c][j] X[c][j]
__global__ void k_rowdot_acc(const double *__restrict__ Y, const double *__restrict__ X, long ld,
                             long ng, int n, double a, double *__restrict__ g) {
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < ng;
         j += (long)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int c = 0; c < n; ++c) s += Y[(long)c * ld + j] * X[(long)c * ld + j];
        g[j] += a * s;
    }
}

// Y = a X + b Y over ng rows of ncols columns (column c in blockIdx.y)
__global__ void k_block_axpby(double *__restrict__ Y, const double *__restrict__ X, long ld,
                              long ng, double a, double b) {
    const long o = (long)blockIdx.y * ld;
    for (long j = (long)blockIdx.x * blockDim.x + threadIdx.x; j < ng;
         j += (long)gridDim.x * blockDim.x)
        Y[o + j] = a * X[o + j] + (b == 0.0 ? 0.0 : b * Y[o + j]);
}

// out[0] = tr(A B) for n x n column-major A, B (one block)
__global__ void k_trace_prod(const double *__restrict__ A, int lda, const double *__restrict__ B,
                             int ldb, int n, double *__restrict__ out) {
    __shared__ double red[16];
    double s = 0.0;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const int i = e % n, j = e / n;
        s += A[(long)j * lda + i] * B[(long)i * ldb + j];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
        out[0] = t;
    }
}

__global__ void k_scan_finite(const double *__restrict__ X, long ld, long ng, int ncols,
                              int *__restrict__ bad) {
    const int c = blockIdx.y;
    const double *x = X + (long)c * ld;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < ng;
         i += (long)gridDim.x * blockDim.x)
        if (!isfinite(x[i])) atomicMax(bad, 7);
}

}  // namespace

// =================================================================== ABI

extern "C" {

const char *qo_status_string(qo_status s) {
    // read as int: a C caller may pass any int, and a C++ load of an out-of-range value as
    // the enum type is undefined
    static_assert(sizeof(qo_status) == sizeof(int), "qo_status is passed as an int");
    int v;
    memcpy(&v, &s, sizeof v);
    switch (v) {
        case QO_OK: return "QO_OK";
        case QO_ERR_ARG: return "QO_ERR_ARG";
        case QO_ERR_ALLOC: return "QO_ERR_ALLOC";
        case QO_ERR_DEVICE: return "QO_ERR_DEVICE";
        case QO_ERR_STATE: return "QO_ERR_STATE";
        case QO_ERR_NOT_SPD: return "QO_ERR_NOT_SPD";
        case QO_ERR_PCG_NOCONV: return "QO_ERR_PCG_NOCONV";
        case QO_ERR_NONFINITE: return "QO_ERR_NONFINITE";
    }
    return "QO_ERR_UNKNOWN";
}

const char *qo_last_error(qo_handle h) { return h ? h->err.c_str() : qo::noalloc_last_error(); }

qo_status qo_destroy(qo_handle h) {
    if (!h) return QO_ERR_ARG;
    if (h->st) (void)hipStreamSynchronize(h->st);
    else (void)hipDeviceSynchronize();
    for (void *p : h->allocs) (void)hipFree(p);
    if (h->h_poll) (void)hipHostFree(h->h_poll);
    if (h->h_scal) (void)hipHostFree(h->h_scal);
    if (h->ev_ok)
        for (auto &e : h->ev) (void)hipEventDestroy(e);
    for (hipEvent_t e : {h->pev[0], h->pev[1], h->rev, h->sev})
        if (e) (void)hipEventDestroy(e);
    for (auto &p : h->pend) {
        (void)hipEventDestroy(p.a);
        (void)hipEventDestroy(p.b);
    }
    for (auto e : h->evpool) (void)hipEventDestroy(e);
    delete h;
    return QO_OK;
}

qo_status qo_create(const qo_config *cfg, void *hip_stream, qo_handle *out) {
    if (!out) return QO_ERR_ARG;
    *out = nullptr;
    if (!cfg) return QO_ERR_ARG;
    const qo_config &c = *cfg;
    if (c.dim != 2 && c.dim != 3) return QO_ERR_ARG;
    long ng = 1;
    for (int k = 0; k < c.dim; ++k) {
        if (c.n[k] < 1 || !(c.L[k] > 0.0)) return QO_ERR_ARG;
        ng *= c.n[k];
    }
    if (c.n[0] > 1024) return QO_ERR_ARG;
    if (c.pcg_variant < 0 || c.pcg_variant > 2) return QO_ERR_ARG;
    // block CG: FP64 with the Jacobi preconditioner
    if (c.pcg_variant == 2 && (c.precision != QO_FP64 || c.precond != 0)) return QO_ERR_ARG;
    if (c.pcg_variant == 1 && c.n[0] > 256) return QO_ERR_ARG;
    if (c.precond != 0 && c.precond != 1) return QO_ERR_ARG;
    if (c.precond == 1 && (c.pcg_variant != 0 || dst_plan_check(c.dim, c.n))) return QO_ERR_ARG;
    if (c.N < 1 || c.N >= ng || c.N > 4096) return QO_ERR_ARG;
    if (!(c.kinetic > 0.0) || !std::isfinite(c.sigma)) return QO_ERR_ARG;
    if (!(c.pcg_tol > 0.0) || c.pcg_maxit < 1 || c.pcg_check < 1) return QO_ERR_ARG;
    if (c.precision != QO_FP64 && c.precision != QO_MIXED) return QO_ERR_ARG;
    if (c.precision == QO_MIXED && !(c.refine_inner_tol > 0.0 && c.refine_inner_tol < 1.0))
        return QO_ERR_ARG;

    qo_ctx *h = new (std::nothrow) qo_ctx();
    if (!h) return QO_ERR_ALLOC;
    h->cfg = c;
    h->st = static_cast<hipStream_t>(hip_stream);
    h->N = c.N;
    h->mixed = c.precision == QO_MIXED;
    setup_grid(h);
    h->ng = h->g.ng;
    h->ld = (h->ng + 63) / 64 * 64;
    const int N = h->N;
    const size_t blk = (size_t)h->ld * N;
    qo_status s = QO_OK;
    auto A = [&](auto **p, size_t n) {
        if (s == QO_OK) s = dalloc(h, p, n);
    };
    if (hipGetDevice(&h->device) != hipSuccess) s = QO_ERR_DEVICE;
    A(&h->vs, h->ng);
    A(&h->dinv, h->ng);
    A(&h->U, blk);
    A(&h->Uh, blk);
    A(&h->PQ[0], blk);
    A(&h->PQ[1], blk);
    A(&h->r, blk);
    if (c.pcg_variant == 1) A(&h->r2, blk);
    A(&h->pa, blk);
    A(&h->pb, blk);
    A(&h->W, blk);
    A(&h->W2, blk);
    if (h->mixed) {
        A(&h->vs32, h->ng);
        A(&h->dinv32, h->ng);
        A(&h->r32, blk);
        A(&h->d32, blk);
        A(&h->rr32, blk);
        if (c.pcg_variant == 1) A(&h->rr32b, blk);
        A(&h->pa32, blk);
        A(&h->pb32, blk);
    }
    A(&h->part, (size_t)8 * h->qsmax);
    h->gnsplit = gram_nsplit(h->ng, N);
    A(&h->gpart, gram_part_elems(N, h->gnsplit));
    if (h->mixed) {
        A(&h->zbU, blk);
        A(&h->zbUh, blk);
        A(&h->zbPQ, blk);
        A(&h->split3, tsgemm_split_elems(N));
    }
    A(&h->G1, (size_t)4 * N * N);
    A(&h->G2, (size_t)4 * N * N);
    A(&h->mpool, (size_t)MP_COUNT * N * N);
    A(&h->colsums, (size_t)4 * N);
    A(&h->dscal, 16);
    A(&h->sortwork, (size_t)N + (size_t)N * N);
    A(&h->gjw, nn_gj_work_elems(N));
    A(&h->gjpiv, (size_t)N);
    A(&h->ps.rho, (size_t)2 * N);
    A(&h->ps.alpha, (size_t)2 * N);
    A(&h->ps.active, (size_t)2 * N);
    A(&h->ps.its, (size_t)N);
    A(&h->ps.bb, (size_t)N);
    A(&h->ps.err, 2);
    A(&h->mask, (size_t)N);
    A(&h->coltol, (size_t)N);
    A(&h->zerotol, (size_t)N);
    A(&h->rref, (size_t)N);
    A(&h->bb64, (size_t)N);
    A(&h->need, (size_t)N);
    A(&h->nneed, 1);
    h->rel = env_int("QO_MIXED_RESTART", 0) == 0;
    if (const char *d = getenv("QO_REL_DELTA")) h->rel_delta = atof(d);
    A(&h->nact, 1);
    A(&h->dstatus, 1);
    if (c.precond == 1) {
        h->dst = true;
        DstPlan &dp = h->dp;
        dst_plan_geometry(dp, c.dim, h->g.nx, h->g.ny, h->g.nz);
        const size_t sx = (size_t)dp.NXP * dp.NXP, sy = (size_t)dp.NYP * dp.NYP,
                     ss = (size_t)dp.NSP * dp.NSP;
        A(&h->dS, sx + sy + ss);
        A(&h->dmu, (size_t)dp.nx + dp.ny + dp.ns);
        A(&h->t1, blk);
        A(&h->t2, blk);
        A(&h->pcs, (size_t)N);
        A(&h->rzp, (size_t)N * dp.rzparts);
        A(&h->dsum, 1);
        A(&h->z32, blk);
        A(&h->pbeta, (size_t)N);
        A(&h->rzc, (size_t)N);
        A(&h->wzp, (size_t)N * dp.nslab * (dp.RP / 16));
        if (s == QO_OK) {
            dp.Sx = h->dS;
            dp.Sy = h->dS + sx;
            dp.Ss = h->dS + sx + sy;
            dp.mux = h->dmu;
            dp.muy = h->dmu + dp.nx;
            dp.mus = h->dmu + dp.nx + dp.ny;
            // eigenvalues of the 1-D Dirichlet -d^2/dx^2: (4/h^2) sin^2(pi (j+1) / (2 (n+1)))
            std::vector<float> mu;
            auto push = [&](int n, double L) {
                const double hh = L / (n + 1);
                for (int j = 0; j < n; ++j) {
                    const double sn = std::sin(M_PI * (j + 1) / (2.0 * (n + 1)));
                    mu.push_back((float)(4.0 * sn * sn / (hh * hh)));
                }
            };
            push(dp.nx, c.L[0]);
            push(dp.ny, c.L[1]);
            if (c.dim == 3) push(dp.nz, c.L[2]);
            else push(dp.ny, c.L[1]);
            if (hipMemcpy(h->dmu, mu.data(), sizeof(float) * mu.size(), hipMemcpyHostToDevice) !=
                    hipSuccess ||
                launch_dst_matrix(dp.nx, dp.NXP, h->dS, h->st) != hipSuccess ||
                launch_dst_matrix(dp.ny, dp.NYP, h->dS + sx, h->st) != hipSuccess ||
                launch_dst_matrix(dp.ns, dp.NSP, h->dS + sx + sy, h->st) != hipSuccess)
                s = QO_ERR_DEVICE;
            dp.kap = (float)c.kinetic;
            h->mu0 = (double)mu[0] + (double)mu[dp.nx] * (c.dim == 3 ? 1.0 : 0.0) +
                     (double)mu[dp.nx + dp.ny];
            dp.vbar = 0.f;
            dp.lmin = (float)(c.kinetic * h->mu0);
        }
    }
    h->ps.part = h->part;
    if (s == QO_OK) {
        if (hipHostMalloc((void **)&h->h_poll, sizeof(int) * poll_ints(N)) != hipSuccess ||
            hipHostMalloc((void **)&h->h_scal, sizeof(double) * 16) != hipSuccess)
            s = QO_ERR_ALLOC;
    }
    if (s == QO_OK) {
        for (hipEvent_t *e : {&h->pev[0], &h->pev[1], &h->rev, &h->sev})
            if (hipEventCreateWithFlags(e, hipEventDisableTiming) != hipSuccess) s = QO_ERR_DEVICE;
    }
    if (s == QO_OK) {
        h->ev_ok = true;
        for (auto &e : h->ev)
            if (hipEventCreate(&e) != hipSuccess) h->ev_ok = false;
        if (hipStreamSynchronize(h->st) != hipSuccess) s = QO_ERR_DEVICE;
    }
    if (s != QO_OK) {
        qo_destroy(h);
        return s;
    }
    *out = h;
    return QO_OK;
}

qo_status qo_set_potential(qo_handle h, const double *V, int on_device) {
    if (!h || !V) return h ? fail(h, QO_ERR_ARG, "null potential") : QO_ERR_ARG;
    const double *src = V;
    if (!on_device) {
        HIPC(h, hipMemcpyAsync(h->W, V, sizeof(double) * h->ng, hipMemcpyHostToDevice, h->st));
        src = h->W;
    }
    HIPC(h, hipMemsetAsync(h->dstatus, 0, sizeof(int), h->st));
    long blocks = (h->ng + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_prep_potential, dim3((unsigned)blocks), dim3(256), 0, h->st, src, h->ng,
                       h->cfg.sigma, h->g.c0, h->vs, h->dinv, h->vs32, h->dinv32, h->dstatus);
    HIPC(h, hipGetLastError());
    int bad = 0;
    HIPC(h, hipMemcpyAsync(&bad, h->dstatus, sizeof(int), hipMemcpyDeviceToHost, h->st));
    HIPC(h, hipStreamSynchronize(h->st));
    if (bad == 7) {
        h->have_V = false;
        return fail(h, QO_ERR_NONFINITE, "potential has non-finite values");
    }
    if (bad == 5) {
        h->have_V = false;
        return fail(h, QO_ERR_NOT_SPD, "diagonal of H_sigma not positive: increase sigma");
    }
    if (h->dst) {
        // vbar = max(0, mean(V + sigma)): M = kappa (-Lap_h) + vbar stays SPD
        HIPC(h, launch_sum(h->vs, h->ng, h->dsum, h->st));
        double sum = 0.0;
        HIPC(h, hipMemcpyAsync(&sum, h->dsum, sizeof(double), hipMemcpyDeviceToHost, h->st));
        HIPC(h, hipStreamSynchronize(h->st));
        const double vbar = std::max(0.0, sum / (double)h->ng);
        h->dp.vbar = (float)vbar;
        h->dp.lmin = (float)(h->cfg.kinetic * h->mu0 + vbar);
    }
    h->have_V = true;
    h->have_warm = false;
    h->have_K = false;
    h->have_Es = false;  // energies of the old operator are not comparable
    return QO_OK;
}

qo_status qo_set_state(qo_handle h, const double *U, long ld, int on_device) {
    if (!h) return QO_ERR_ARG;
    if (!U || ld < h->ng) return fail(h, QO_ERR_ARG, "bad state pointer or ld");
    h->zbU_ok = false;
    QOC(copy_block_in(h, h->U, U, ld, on_device));
    HIPC(h, hipMemsetAsync(h->dstatus, 0, sizeof(int), h->st));
    long blocks = (h->ng + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_scan_finite, dim3((unsigned)blocks, h->N), dim3(256), 0, h->st, h->U,
                       h->ld, h->ng, h->N, h->dstatus);
    HIPC(h, hipGetLastError());
    int bad = 0;
    HIPC(h, hipMemcpyAsync(&bad, h->dstatus, sizeof(int), hipMemcpyDeviceToHost, h->st));
    HIPC(h, hipStreamSynchronize(h->st));
    if (bad) {
        h->have_U = false;
        return fail(h, QO_ERR_NONFINITE, "state has non-finite values");
    }
    h->have_U = true;
    h->have_warm = false;
    h->have_Es = false;
    h->have_K = false;
    h->nstep = 0;
    return QO_OK;
}

qo_status qo_get_state(qo_handle h, double *U, long ld, int on_device) {
    if (!h) return QO_ERR_ARG;
    if (!U || ld < h->ng) return fail(h, QO_ERR_ARG, "bad output pointer or ld");
    if (!h->have_U) return fail(h, QO_ERR_STATE, "no state set");
    return copy_block_out(h, U, ld, h->U, on_device, h->N);
}

// The warm start of the next first solve sits in that solve's output block PQ[cur] (the
// previous step's G U_hat); the BF16 copy of U (mixed) is re-derived from U, bit for bit.
qo_status qo_get_checkpoint(qo_handle h, double *U, double *warm, long ld, double *K,
                            int on_device, qo_checkpoint *info) {
    if (!h) return QO_ERR_ARG;
    if (!U || !info || ld < h->ng) return fail(h, QO_ERR_ARG, "bad output pointer or ld");
    if (!h->have_U) return fail(h, QO_ERR_STATE, "no state set");
    QOC(copy_block_out(h, U, ld, h->U, on_device, h->N));
    qo_checkpoint ck{};
    ck.step_index = h->nstep;
    ck.has_warm = h->have_warm ? 1 : 0;
    if (h->have_warm && warm) QOC(copy_block_out(h, warm, ld, h->PQ[h->cur], on_device, h->N));
    ck.has_energy = h->have_Es ? 1 : 0;
    ck.energy_shifted = h->have_Es ? h->last_Es : 0.0;
    ck.has_K = (h->emode == 1 && h->have_K) ? 1 : 0;
    if (ck.has_K && K) {
        HIPC(h, hipMemcpyAsync(K, h->Kprop, sizeof(double) * h->N * h->N, hipMemcpyDeviceToHost,
                               h->st));
        HIPC(h, hipStreamSynchronize(h->st));
    }
    *info = ck;
    return QO_OK;
}

qo_status qo_set_checkpoint(qo_handle h, const double *U, const double *warm, long ld,
                            const double *K, int on_device, const qo_checkpoint *info) {
    if (!h) return QO_ERR_ARG;
    if (!info || info->step_index < 0 || (info->has_warm && !warm) || (info->has_K && !K) ||
        (info->has_energy && !std::isfinite(info->energy_shifted)))
        return fail(h, QO_ERR_ARG, "incomplete checkpoint (warm, K, energy or step index)");
    QOC(qo_set_state(h, U, ld, on_device));  // validates U; resets the carried quantities
    if (info->has_warm) {
        QOC(copy_block_in(h, h->PQ[h->cur], warm, ld, on_device));
        HIPC(h, hipMemsetAsync(h->dstatus, 0, sizeof(int), h->st));
        long blocks = (h->ng + 255) / 256;
        if (blocks > 1024) blocks = 1024;
        hipLaunchKernelGGL(k_scan_finite, dim3((unsigned)blocks, h->N), dim3(256), 0, h->st,
                           h->PQ[h->cur], h->ld, h->ng, h->N, h->dstatus);
        HIPC(h, hipGetLastError());
        int bad = 0;
        HIPC(h, hipMemcpyAsync(&bad, h->dstatus, sizeof(int), hipMemcpyDeviceToHost, h->st));
        HIPC(h, hipStreamSynchronize(h->st));
        if (bad) {
            h->have_U = false;
            return fail(h, QO_ERR_NONFINITE, "warm-start block has non-finite values");
        }
        h->have_warm = true;
    }
    if (info->has_K && h->emode == 1) {
        for (long i = 0; i < (long)h->N * h->N; ++i)
            if (!std::isfinite(K[i])) {
                h->have_U = false;
                return fail(h, QO_ERR_NONFINITE, "carried K has non-finite values");
            }
        HIPC(h, hipMemcpyAsync(h->Kprop, K, sizeof(double) * h->N * h->N,
                               hipMemcpyHostToDevice, h->st));
        HIPC(h, hipStreamSynchronize(h->st));
        h->have_K = true;
    }
    h->have_Es = info->has_energy != 0;
    h->last_Es = info->has_energy ? info->energy_shifted : 0.0;
    h->nstep = info->step_index;
    return QO_OK;
}

qo_status qo_step(qo_handle h, double tau, int nsteps, qo_step_stats *last) {
    if (!h) return QO_ERR_ARG;
    if (!(tau > 0.0) || !std::isfinite(tau) || nsteps < 0)
        return fail(h, QO_ERR_ARG, "tau must be positive and finite, nsteps >= 0");
    if (!h->have_V || !h->have_U) return fail(h, QO_ERR_STATE, "set potential and state first");
    for (int i = 0; i < nsteps; ++i) QOC(one_step(h, tau, last));
    return QO_OK;
}

qo_status qo_run(qo_handle h, double tau, double tau_max, int max_steps, double grad_tol,
                 int *out_steps, double *out_tau, int *converged, qo_step_stats *last) {
    if (!h) return QO_ERR_ARG;
    if (!(tau > 0.0) || !std::isfinite(tau) || max_steps < 0 || !(grad_tol >= 0.0) ||
        !std::isfinite(tau_max))
        return fail(h, QO_ERR_ARG, "bad tau, tau_max, max_steps or grad_tol");
    if (!h->have_V || !h->have_U) return fail(h, QO_ERR_STATE, "set potential and state first");
    const bool adapt = tau_max > 0.0;
    if (adapt && tau > tau_max) tau = tau_max;
    int steps = 0, conv = 0;
    qo_step_stats st{};
    while (steps < max_steps) {
        if (adapt) {  // backup for an undo
            HIPC(h, hipMemcpyAsync(h->W2, h->U, sizeof(double) * h->ld * h->N,
                                   hipMemcpyDeviceToDevice, h->st));
        }
        const int cur0 = h->cur;
        const bool warm0 = h->have_warm, hasE0 = h->have_Es;
        const double E0 = h->last_Es;
        const long n0 = h->nstep;
        int stopped = 0;
        const qo_status ss = one_step(h, tau, &st, grad_tol, &stopped);
        const bool step_failed =
            ss == QO_ERR_NOT_SPD || ss == QO_ERR_PCG_NOCONV || ss == QO_ERR_NONFINITE;
        if (ss != QO_OK && !(adapt && step_failed)) return ss;
        if (ss == QO_OK && stopped) {
            conv = 1;
            break;
        }
        const bool o_grew = st.orth_err_next > st.orth_err_fro * (1.0 + 1e-12) &&
                            st.orth_err_next > 1e-10;
        const bool reject = step_failed || st.energy_rose || o_grew;
        if (adapt && reject) {
            if (!(tau > 1e-12 * tau_max))
                return fail(h, ss != QO_OK ? ss : QO_ERR_NOT_SPD,
                            "adaptive time step fell below 1e-12 tau_max");
            // undo: U_n back, its G U_n (in PQ[cur0]) stays the warm start
            HIPC(h, hipMemcpyAsync(h->U, h->W2, sizeof(double) * h->ld * h->N,
                                   hipMemcpyDeviceToDevice, h->st));
            h->zbU_ok = false;
            HIPC(h, hipStreamSynchronize(h->st));
            h->cur = cur0;
            h->have_warm = ss == QO_OK ? true : warm0;
            h->have_K = false;  // a propagated K belongs to the undone step
            h->have_Es = hasE0;
            h->last_Es = E0;
            h->nstep = n0;
            tau *= 0.5;
            continue;
        }
        ++steps;
        if (last) *last = st;
        if (adapt) tau = fmin(tau_max, 1.25 * tau);
    }
    if (out_steps) *out_steps = steps;
    if (out_tau) *out_tau = tau;
    if (converged) *converged = conv;
    return QO_OK;
}

qo_status qo_energy(qo_handle h, double *E, double *E_shifted) {
    if (!h) return QO_ERR_ARG;
    if (!h->have_V || !h->have_U) return fail(h, QO_ERR_STATE, "set potential and state first");
    double Es = 0.0, trS = 0.0;
    QOC(energy_of(h, h->U, &Es, &trS));
    if (E) *E = Es - 0.5 * h->cfg.sigma * trS;
    if (E_shifted) *E_shifted = Es;
    return QO_OK;
}

qo_status qo_gram(qo_handle h, double *S, double *K) {
    if (!h || !S) return h ? fail(h, QO_ERR_ARG, "null output") : QO_ERR_ARG;
    if (!h->have_V || !h->have_U) return fail(h, QO_ERR_STATE, "set potential and state first");
    const int N = h->N;
    HIPC(h, launch_apply(h->g, h->vs, h->U, h->W, h->ld, N, h->st));
    QOC(gram64(h, h->U, h->W, h->ld, N, h->G2));
    HIPC(h, hipMemcpy2DAsync(S, N * sizeof(double), h->G2, 2 * N * sizeof(double),
                             N * sizeof(double), N, hipMemcpyDeviceToHost, h->st));
    if (K)
        HIPC(h, hipMemcpy2DAsync(K, N * sizeof(double), h->G2 + (size_t)N * 2 * N,
                                 2 * N * sizeof(double), N * sizeof(double), N,
                                 hipMemcpyDeviceToHost, h->st));
    HIPC(h, hipStreamSynchronize(h->st));
    return QO_OK;
}

qo_status qo_eigenpairs(qo_handle h, int mode, double *evals, double *evecs, long ld,
                        int on_device) {
    if (!h || !evals) return h ? fail(h, QO_ERR_ARG, "null output") : QO_ERR_ARG;
    if (mode != QO_EIG_RITZ && mode != QO_EIG_PAPER) return fail(h, QO_ERR_ARG, "bad mode");
    if (mode == QO_EIG_PAPER && evecs) return fail(h, QO_ERR_ARG, "paper mode gives no vectors");
    if (evecs && ld < h->ng) return fail(h, QO_ERR_ARG, "bad ld");
    if (!h->have_V || !h->have_U) return fail(h, QO_ERR_STATE, "set potential and state first");
    const int N = h->N, N2 = 2 * N;
    hipStream_t st = h->st;
    double *ev = h->dscal + 8;  // too small for N; use pool
    ev = mp(h, MP_T3);
    HIPC(h, hipMemsetAsync(h->dstatus, 0, sizeof(int), st));
    if (mode == QO_EIG_RITZ) {
        HIPC(h, launch_apply(h->g, h->vs, h->U, h->W, h->ld, N, st));
        QOC(gram64(h, h->U, h->W, h->ld, N, h->G2));
        double *S = h->G2, *K = h->G2 + (size_t)N * N2;
        // S = V diag(l) V^T ; F = V diag(l)^{-1/2}
        HIPC(h, nn_axpby(mp(h, MP_T1), N, 0.5, S, N2, 0.5, S, N2, true, 0.0, N, N, st));
        HIPC(h, nn_jacobi(mp(h, MP_T1), N, N, ev, mp(h, MP_T2), N, nullptr, st));
        HIPC(h, nn_scale_cols_rsqrt(mp(h, MP_SW), mp(h, MP_T2), N, ev, N, h->dstatus, st));
        // K' = F^T sym(K) F
        HIPC(h, nn_axpby(mp(h, MP_T1), N, 0.5, K, N2, 0.5, K, N2, true, 0.0, N, N, st));
        HIPC(h, nn_gemm(mp(h, MP_T2), N, mp(h, MP_T1), N, false, mp(h, MP_SW), N, false, N, N, N, 1.0, 0.0, 0.0, st));
        HIPC(h, nn_gemm(mp(h, MP_T1), N, mp(h, MP_SW), N, true, mp(h, MP_T2), N, false, N, N, N, 1.0, 0.0, 0.0, st));
        HIPC(h, nn_axpby(mp(h, MP_T2), N, 0.5, mp(h, MP_T1), N, 0.5, mp(h, MP_T1), N, true, 0.0, N, N, st));
        HIPC(h, nn_jacobi(mp(h, MP_T2), N, N, ev, mp(h, MP_Z), N, nullptr, st));
        HIPC(h, nn_sort(ev, mp(h, MP_Z), N, N, false, h->sortwork, st));
        HIPC(h, nn_eval_map(ev, ev, N, false, h->cfg.sigma, st));
        QOC(check_status(h, "Rayleigh-Ritz: <U,U> not positive definite"));
        if (evecs) {
            // c = F Z ; vectors = U c
            HIPC(h, nn_gemm(mp(h, MP_C), N, mp(h, MP_SW), N, false, mp(h, MP_Z), N, false, N, N, N, 1.0, 0.0, 0.0, st));
            HIPC(h, nn_axpby(mp(h, MP_ZR), N, 0.0, nullptr, N, 1.0, mp(h, MP_C), N, true, 0.0, N, N, st));
            if (on_device) {
                HIPC(h, launch_tsgemm(evecs, ld, nullptr, h->U, mp(h, MP_ZR), nullptr, nullptr, h->ld, h->ng, N, st));
            } else {
                HIPC(h, launch_tsgemm(h->W, h->ld, nullptr, h->U, mp(h, MP_ZR), nullptr, nullptr, h->ld, h->ng, N, st));
                QOC(copy_block_out(h, evecs, ld, h->W, 0, N));
            }
        }
    } else {
        // P = G U (side-effect free: scratch start from the warm-start block)
        std::vector<int> its(N);
        int rounds = 0;
        HIPC(h, hipMemcpyAsync(h->W2, h->PQ[h->cur], sizeof(double) * h->ld * N,
                               hipMemcpyDeviceToDevice, st));
        QOC(solve_block(h, h->U, h->W2, N, h->have_warm ? 1 : 0, its.data(), &rounds,
                        "solve G U (paper eigenvalues)"));
        QOC(gram64(h, h->U, h->W2, h->ld, N, h->G2));
        double *M = h->G2 + (size_t)N * N2;
        HIPC(h, nn_axpby(mp(h, MP_T1), N, 0.5, M, N2, 0.5, M, N2, true, 0.0, N, N, st));
        HIPC(h, nn_jacobi(mp(h, MP_T1), N, N, ev, mp(h, MP_T2), N, nullptr, st));
        HIPC(h, nn_eval_map(ev, ev, N, true, h->cfg.sigma, st));
        HIPC(h, nn_sort(ev, nullptr, N, N, false, h->sortwork, st));
    }
    HIPC(h, hipMemcpyAsync(evals, ev, sizeof(double) * N, hipMemcpyDeviceToHost, st));
    HIPC(h, hipStreamSynchronize(st));
    return QO_OK;
}

qo_status qo_eigsum_gradient(qo_handle h, double *g, int on_device) {
    if (!h || !g) return h ? fail(h, QO_ERR_ARG, "null output") : QO_ERR_ARG;
    if (!h->have_U) return fail(h, QO_ERR_STATE, "set the state first");
    const int N = h->N;
    hipStream_t st = h->st;
    // S = <U,U>;  Sinv by Gauss-Jordan (SPD);  Y = U S^{-1};  g = h^d rowdot(Y, U)
    QOC(gram64(h, h->U, h->U, h->ld, N, h->G2));
    HIPC(h, hipMemsetAsync(h->dstatus, 0, sizeof(int), st));
    HIPC(h, nn_axpby(mp(h, MP_T1), N, 1.0, h->G2, 2 * N, 0.0, nullptr, N, false, 0.0, N, N, st));
    HIPC(h, nn_axpby(mp(h, MP_T2), N, 0.0, nullptr, N, 0.0, nullptr, N, false, 1.0, N, N, st));
    HIPC(h, nn_gj_solve(mp(h, MP_T1), N, mp(h, MP_T2), N, N, N, true, h->dstatus, st, h->gjw, h->gjpiv));
    QOC(check_status(h, "eigsum gradient: <U,U> not positive definite"));
    // row-major copy of S^{-1} (symmetric up to rounding; symmetrise)
    HIPC(h, nn_axpby(mp(h, MP_T3), N, 0.5, mp(h, MP_T2), N, 0.5, mp(h, MP_T2), N, true, 0.0, N, N, st));
    HIPC(h, launch_tsgemm(h->W, h->ld, nullptr, h->U, mp(h, MP_T3), nullptr, nullptr, h->ld, h->ng,
                          N, st));
    double *dst = on_device ? g : h->W2;
    long blocks = (h->ng + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_rowdot, dim3((unsigned)blocks), dim3(256), 0, st, h->W, h->U, h->ld,
                       h->ng, N, h->w, dst);
    HIPC(h, hipGetLastError());
    if (!on_device)
        HIPC(h, hipMemcpyAsync(g, h->W2, sizeof(double) * h->ng, hipMemcpyDeviceToHost, st));
    HIPC(h, hipStreamSynchronize(st));
    return QO_OK;
}

qo_status qo_apply(qo_handle h, const double *X, double *Y, long ld, int ncols) {
    if (!h) return QO_ERR_ARG;
    if (!X || !Y || ld < h->ng || ncols < 0 || ncols > h->N)
        return fail(h, QO_ERR_ARG, "bad arguments to qo_apply");
    if (!h->have_V) return fail(h, QO_ERR_STATE, "set the potential first");
    HIPC(h, launch_apply(h->g, h->vs, X, Y, ld, ncols, h->st));
    HIPC(h, hipStreamSynchronize(h->st));
    return QO_OK;
}

qo_status qo_solve(qo_handle h, const double *B, double *X, long ld, int ncols, int use_x0,
                   int *iters) {
    if (!h) return QO_ERR_ARG;
    if (!B || !X || ld < h->ng || ncols < 0 || ncols > h->N)
        return fail(h, QO_ERR_ARG, "bad arguments to qo_solve");
    if (!h->have_V) return fail(h, QO_ERR_STATE, "set the potential first");
    if (ncols == 0) return QO_OK;
    hipStream_t st = h->st;
    const size_t row = h->ng * sizeof(double), lds = ld * sizeof(double),
                 ldi = h->ld * sizeof(double);
    HIPC(h, hipMemcpy2DAsync(h->W, ldi, B, lds, row, ncols, hipMemcpyDeviceToDevice, st));
    if (use_x0) HIPC(h, hipMemcpy2DAsync(h->W2, ldi, X, lds, row, ncols, hipMemcpyDeviceToDevice, st));
    std::vector<int> its(ncols);
    int rounds = 0;
    QOC(solve_block(h, h->W, h->W2, ncols, use_x0 ? 1 : 0, its.data(), &rounds, "qo_solve"));
    HIPC(h, hipMemcpy2DAsync(X, lds, h->W2, ldi, row, ncols, hipMemcpyDeviceToDevice, st));
    HIPC(h, hipStreamSynchronize(st));
    if (iters)
        for (int j = 0; j < ncols; ++j) iters[j] = its[j];
    return QO_OK;
}

qo_status qo_precond(qo_handle h, const double *R, double *Z, long ld, int ncols, double *rz) {
    if (!h) return QO_ERR_ARG;
    if (!R || !Z) return fail(h, QO_ERR_ARG, "null pointer");
    if (!h->dst) return fail(h, QO_ERR_ARG, "qo_precond needs precond = 1");
    if (!h->have_V) return fail(h, QO_ERR_STATE, "no potential set");
    if (ld < h->ng || ncols < 1 || ncols > h->N)
        return fail(h, QO_ERR_ARG, "bad ld/ncols (ld %ld, ncols %d)", ld, ncols);
    hipStream_t st = h->st;
    const size_t row = sizeof(double) * h->ng;
    HIPC(h, hipMemcpy2DAsync(h->W, sizeof(double) * h->ld, R, sizeof(double) * ld, row, ncols,
                             hipMemcpyDeviceToDevice, st));
    HIPC(h, hipMemsetAsync(h->W2, 0, sizeof(double) * h->ld * ncols, st));
    HIPC(h, launch_col_scale(h->W, h->ld, h->ng, ncols, h->pcs, st));
    HIPC(h, launch_dst_fwd<double>(h->dp, h->W, h->ld, ncols, h->t1, h->pcs, st));
    HIPC(h, launch_dst_pencil(h->dp, h->t1, h->t2, h->ld, ncols, h->pcs, h->rzp, st));
    HIPC(h, launch_dst_inv(h->dp, h->t2, h->z32, h->ld, ncols, h->pcs, st));
    HIPC(h, launch_z_expand(h->z32, h->pcs, h->W2, h->ld, h->ng, ncols, st));
    HIPC(h, hipMemcpy2DAsync(Z, sizeof(double) * ld, h->W2, sizeof(double) * h->ld, row, ncols,
                             hipMemcpyDeviceToDevice, st));
    if (rz) {
        const int ns = h->dp.rzparts;
        std::vector<double> part((size_t)ncols * ns);
        std::vector<float> sc(ncols);
        HIPC(h, hipMemcpyAsync(part.data(), h->rzp, sizeof(double) * part.size(),
                               hipMemcpyDeviceToHost, st));
        HIPC(h, hipMemcpyAsync(sc.data(), h->pcs, sizeof(float) * ncols, hipMemcpyDeviceToHost,
                               st));
        HIPC(h, hipStreamSynchronize(st));
        for (int j = 0; j < ncols; ++j) {
            double t = 0.0;
            if (sc[j] != 0.f)
                for (int q = 0; q < ns; ++q) t += part[(size_t)j * ns + q];
            rz[j] = t;
        }
    } else {
        HIPC(h, hipStreamSynchronize(st));
    }
    return QO_OK;
}

qo_status qo_gram_pair(qo_handle h, const double *X, const double *Y, long ld, int ncols,
                       double *G) {
    if (!h) return QO_ERR_ARG;
    if (!X || !Y || !G || ld < h->ng || ncols < 1 || ncols > h->N)
        return fail(h, QO_ERR_ARG, "bad arguments to qo_gram_pair");
    if (h->mixed) {
        // the BF16 path packs from the internal layout (leading dimension h->ld)
        const size_t row = sizeof(double) * h->ng;
        HIPC(h, hipMemcpy2DAsync(h->W, sizeof(double) * h->ld, X, sizeof(double) * ld, row, ncols,
                                 hipMemcpyDeviceToDevice, h->st));
        HIPC(h, hipMemcpy2DAsync(h->W2, sizeof(double) * h->ld, Y, sizeof(double) * ld, row,
                                 ncols, hipMemcpyDeviceToDevice, h->st));
        QOC(gram(h, h->W, h->W2, h->ld, ncols, h->G2));
    } else {
        QOC(gram(h, X, Y, ld, ncols, h->G2));
    }
    HIPC(h, hipMemcpyAsync(G, h->G2, sizeof(double) * 4 * ncols * ncols, hipMemcpyDeviceToHost,
                           h->st));
    HIPC(h, hipStreamSynchronize(h->st));
    return QO_OK;
}

qo_status qo_get_block(qo_handle h, int which, double *out, long ld, int on_device) {
    if (!h) return QO_ERR_ARG;
    if (!out || ld < h->ng) return fail(h, QO_ERR_ARG, "bad output");
    const double *src = nullptr;
    switch (which) {
        case QO_BLOCK_U: src = h->have_U ? h->U : nullptr; break;
        case QO_BLOCK_UHAT: src = h->nstep > 0 ? h->Uh : nullptr; break;
        case QO_BLOCK_P: src = h->lastP; break;
        case QO_BLOCK_Q: src = h->lastQ; break;
        default: return fail(h, QO_ERR_ARG, "bad block selector");
    }
    if (!src) return fail(h, QO_ERR_STATE, "block not available yet");
    return copy_block_out(h, out, ld, src, on_device, h->N);
}

qo_status qo_get_matrix(qo_handle h, int which, double *out) {
    if (!h) return QO_ERR_ARG;
    if (!out) return fail(h, QO_ERR_ARG, "null output");
    if (h->nstep == 0) return fail(h, QO_ERR_STATE, "no step taken yet");
    const int N = h->N;
    const size_t N2 = 2 * (size_t)N;
    const double *src = nullptr;
    size_t lds = N;
    switch (which) {
        case QO_MAT_S: src = h->G1; lds = N2; break;
        case QO_MAT_M: src = h->G1 + N * N2; lds = N2; break;
        case QO_MAT_R: src = h->G1 + N * N2 + N; lds = N2; break;
        case QO_MAT_X: src = mp(h, MP_X); break;
        case QO_MAT_Y: src = mp(h, MP_Y); break;
        case QO_MAT_O: src = mp(h, MP_O); break;
        case QO_MAT_A: src = h->G2 + N * N2; lds = N2; break;
        case QO_MAT_B: src = h->G2 + N * N2 + N; lds = N2; break;
        default: return fail(h, QO_ERR_ARG, "bad matrix selector");
    }
    HIPC(h, hipMemcpy2DAsync(out, N * sizeof(double), src, lds * sizeof(double),
                             N * sizeof(double), N, hipMemcpyDeviceToHost, h->st));
    HIPC(h, hipStreamSynchronize(h->st));
    return QO_OK;
}

qo_status qo_profile(qo_handle h, int enable) {
    if (!h) return QO_ERR_ARG;
    HIPC(h, hipStreamSynchronize(h->st));
    prof_harvest(h);
    h->prof = enable != 0;
    memset(&h->pdata, 0, sizeof h->pdata);
    return QO_OK;
}

qo_status qo_profile_get(qo_handle h, qo_profile_data *out) {
    if (!h || !out) return h ? fail(h, QO_ERR_ARG, "null output") : QO_ERR_ARG;
    HIPC(h, hipStreamSynchronize(h->st));
    prof_harvest(h);
    *out = h->pdata;
    return QO_OK;
}

}  // extern "C"

// ---- reverse mode through K evolution steps ------------------------------------------
//
// qo_tape_forward takes K steps from the current state with cold-started solves (so every
// step can be recomputed exactly from its starting state) and keeps U_0 .. U_K; the loss
// is E(U_K) or the sum of the Ritz values of span U_K.  qo_tape_backward runs the adjoint
// of the steps in reverse order: each step is recomputed from its checkpoint, then the
// adjoints go back through the corrector, the solve Q = G U_hat, the predictor update,
// the N x N algebra, the Grams and the solve P = G U.  The adjoint of a solve is a solve
// with the same (symmetric) G; dG/dV = -G diag(dV) G gives the potential's share.
namespace {

enum { AM_XB, AM_YB, AM_SB, AM_MB, AM_RB, AM_SHB, AM_T, AM_T2, AM_T3, AM_G, AM_COUNT = AM_G + 4 };

double *am(qo_ctx *c, int i) { return c->admat + (size_t)i * c->N * c->N; }

// Checkpoints of a tape of K steps with stride s: U_0, U_s, ..., U_{floor(K/s) s}, and U_K.
int tape_points(int K, int s) { return K / s + 1 + (K % s ? 1 : 0); }
// Slot of checkpoint n (a multiple of s, or K).
int tape_slot(int K, int s, int n) { return n % s ? K / s + 1 : n / s; }

// The smallest stride whose checkpoints and one segment's s - 1 states fit the budget.
int tape_stride(int K, int budget) {
    if (budget <= 0) return 1;
    for (int s = 1; s <= K + 1; ++s)
        if (tape_points(K, s) + (s - 1) <= budget) return s;
    return 0;
}

qo_status tape_alloc(qo_ctx *c, int K, int s) {
    const size_t blk = (size_t)c->ld * c->N;
    qo_status st = QO_OK;
    auto grow = [&](std::vector<double *> &v, int count) {
        while (st == QO_OK && (int)v.size() < count) {
            double *p = nullptr;
            st = dalloc(c, &p, blk);
            if (st == QO_OK) v.push_back(p);
        }
    };
    grow(c->tape, tape_points(K, s));
    grow(c->tseg, s - 1);
    for (int i = 0; i < 6 && st == QO_OK; ++i)
        if (!c->ab[i]) st = dalloc(c, &c->ab[i], blk);
    if (st == QO_OK && !c->gVd) st = dalloc(c, &c->gVd, (size_t)c->ng);
    if (st == QO_OK && !c->adpool) st = dalloc(c, &c->adpool, nn_adjoint_pool_elems(c->N));
    if (st == QO_OK && !c->admat) st = dalloc(c, &c->admat, (size_t)AM_COUNT * c->N * c->N);
    return st;
}

qo_status blk_axpby(qo_ctx *c, double *Y, const double *X, double a, double b) {
    long blocks = (c->ng + 255) / 256;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_block_axpby, dim3((unsigned)blocks, (unsigned)c->N), dim3(256), 0, c->st,
                       Y, X, c->ld, c->ng, a, b);
    HIPC(c, hipGetLastError());
    return QO_OK;
}

qo_status rowdot_acc(qo_ctx *c, const double *Y, const double *X, double a) {
    long blocks = (c->ng + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_rowdot_acc, dim3((unsigned)blocks), dim3(256), 0, c->st, Y, X, c->ld,
                       c->ng, c->N, a, c->gVd);
    HIPC(c, hipGetLastError());
    return QO_OK;
}

// Loss at U (the current state) and, when grad, seed times its gradient: Ubar into ab[0]
// and the explicit potential term into gVd (overwritten).
qo_status loss_and_grad(qo_ctx *c, int kind, double *L, bool grad, double seed = 1.0) {
    hipStream_t st = c->st;
    const int N = c->N, N2 = 2 * N;
    const double w = c->w, sigma = c->cfg.sigma;
    double *U = c->U, *HU = c->ab[4];
    if (grad) HIPC(c, hipMemsetAsync(c->gVd, 0, sizeof(double) * c->ng, st));
    if (kind == 0) {
        double Es = 0.0, trS = 0.0;
        QOC(energy_of(c, U, &Es, &trS));
        *L = Es - 0.5 * sigma * trS;
        if (!grad) return QO_OK;
        HIPC(c, launch_apply(c->g, c->vs, U, HU, c->ld, N, st));
        QOC(blk_axpby(c, c->ab[0], HU, seed * w, 0.0));
        QOC(blk_axpby(c, c->ab[0], U, -seed * w * sigma, 1.0));
        return rowdot_acc(c, U, U, 0.5 * seed * w);
    }
    // sum of the Ritz values: tr(S^{-1} K) - N sigma with S = <U,U>, K = <U, H_sigma U>
    HIPC(c, launch_apply(c->g, c->vs, U, HU, c->ld, N, st));
    QOC(gram64(c, U, HU, c->ld, N, am(c, AM_G)));
    double *S = am(c, AM_G), *Kb = am(c, AM_G) + (size_t)N * N2;
    HIPC(c, hipMemsetAsync(c->dstatus, 0, sizeof(int), st));
    HIPC(c, nn_axpby(am(c, AM_T), N, 1.0, S, N2, 0.0, nullptr, N, false, 0.0, N, N, st));
    HIPC(c, nn_axpby(am(c, AM_T2), N, 0.0, nullptr, N, 0.0, nullptr, N, false, 1.0, N, N, st));
    HIPC(c, nn_gj_solve(am(c, AM_T), N, am(c, AM_T2), N, N, N, true, c->dstatus, st, c->gjw,
                        c->gjpiv));
    QOC(check_status(c, "Ritz-sum loss: <U,U> not positive definite"));
    double *Si = am(c, AM_T3);
    HIPC(c, nn_axpby(Si, N, 0.5, am(c, AM_T2), N, 0.5, am(c, AM_T2), N, true, 0.0, N, N, st));
    hipLaunchKernelGGL(k_trace_prod, dim3(1), dim3(1024), 0, st, Si, N, Kb, N2, N, c->dscal + 8);
    HIPC(c, hipGetLastError());
    HIPC(c, hipMemcpyAsync(c->h_scal + 8, c->dscal + 8, sizeof(double), hipMemcpyDeviceToHost, st));
    HIPC(c, hipStreamSynchronize(st));
    *L = c->h_scal[8] - N * sigma;
    if (!grad) return QO_OK;
    // Ubar = 2w (H_sigma U S^{-1} - U S^{-1} K S^{-1}); gV = w diag(U S^{-1} U^T)
    HIPC(c, nn_gemm(am(c, AM_T), N, Si, N, false, Kb, N2, false, N, N, N, 1.0, 0.0, 0.0, st));
    HIPC(c, nn_gemm(am(c, AM_T2), N, am(c, AM_T), N, false, Si, N, false, N, N, N, 1.0, 0.0, 0.0, st));
    HIPC(c, nn_axpby(am(c, AM_T), N, -seed * w, am(c, AM_T2), N, -seed * w, am(c, AM_T2), N, true,
                     0.0, N, N, st));
    HIPC(c, nn_axpby(am(c, AM_SHB), N, 2.0 * seed * w, Si, N, 0.0, nullptr, N, false, 0.0, N, N, st));
    QOC(tsgemm(c, c->ab[0], nullptr, HU, am(c, AM_SHB), U, am(c, AM_T)));
    QOC(tsgemm(c, c->ab[5], nullptr, U, Si, nullptr, nullptr));
    return rowdot_acc(c, c->ab[5], U, seed * w);
}

}  // namespace

extern "C" {

qo_status qo_tape_forward(qo_handle h, double tau, int K, int loss, double *L) {
    if (!h || !L) return h ? fail(h, QO_ERR_ARG, "null output") : QO_ERR_ARG;
    if (!h->have_V || !h->have_U) return fail(h, QO_ERR_STATE, "set the potential and the state first");
    if (h->mixed) return fail(h, QO_ERR_ARG, "the tape needs precision QO_FP64");
    if (!(tau > 0.0) || K < 0 || K > 100000 || (loss != 0 && loss != 1))
        return fail(h, QO_ERR_ARG, "bad tau, K or loss");
    const int stride = tape_stride(K, h->tape_budget);
    if (stride < 1)
        return fail(h, QO_ERR_ARG, "no checkpoint stride fits %d steps in %d blocks", K,
                    h->tape_budget);
    h->have_tape = false;
    QOC(tape_alloc(h, K, stride));
    const size_t bytes = sizeof(double) * h->ld * h->N;
    const int warm = h->cfg.warm_start;
    h->cfg.warm_start = 0;
    qo_status s = QO_OK;
    if (hipMemcpyAsync(h->tape[0], h->U, bytes, hipMemcpyDeviceToDevice, h->st) != hipSuccess)
        s = fail(h, QO_ERR_DEVICE, "tape copy failed");
    for (int n = 0; n < K && s == QO_OK; ++n) {
        s = one_step(h, tau, nullptr);
        if (s == QO_OK && ((n + 1) % stride == 0 || n + 1 == K) &&
            hipMemcpyAsync(h->tape[tape_slot(K, stride, n + 1)], h->U, bytes,
                           hipMemcpyDeviceToDevice, h->st) != hipSuccess)
            s = fail(h, QO_ERR_DEVICE, "tape copy failed");
    }
    h->cfg.warm_start = warm;
    h->have_warm = false;
    h->have_K = false;
    if (s != QO_OK) return s;
    QOC(loss_and_grad(h, loss, L, false));
    h->tape_K = K;
    h->tape_s = stride;
    h->tape_tau = tau;
    h->tape_loss = loss;
    h->have_tape = true;
    return QO_OK;
}

qo_status qo_tape_budget(qo_handle h, int blocks) {
    if (!h) return QO_ERR_ARG;
    if (blocks < 0 || (blocks > 0 && blocks < 3))
        return fail(h, QO_ERR_ARG, "tape budget must be 0 or at least 3 blocks");
    h->tape_budget = blocks;
    h->have_tape = false;  // a tape taken under another bound is not reused
    return QO_OK;
}

qo_status qo_tape_backward(qo_handle h, double seed, double *gV, double *gU0, long ld,
                           int on_device) {
    if (!h) return QO_ERR_ARG;
    if (!h->have_tape) return fail(h, QO_ERR_STATE, "run qo_tape_forward first");
    if (gU0 && ld < h->ng) return fail(h, QO_ERR_ARG, "ld %ld < Ng %ld", ld, h->ng);
    hipStream_t st = h->st;
    const int N = h->N, N2 = 2 * N, K = h->tape_K;
    const double w = h->w, tau = h->tape_tau;
    const size_t bytes = sizeof(double) * h->ld * N;
    std::vector<int> its(N);
    int rounds = 0;
    const int warm = h->cfg.warm_start;
    h->cfg.warm_start = 0;
    const int sd = h->tape_s;
    double *const UK = h->tape[tape_slot(K, sd, K)];
    auto body = [&]() -> qo_status {
        double L = 0.0;
        HIPC(h, hipMemcpyAsync(h->U, UK, bytes, hipMemcpyDeviceToDevice, st));
        h->zbU_ok = false;
        QOC(loss_and_grad(h, h->tape_loss, &L, true, seed));
        for (int n = K - 1; n >= 0; --n) {
            // U_n: a checkpoint, or a state of the segment [n0, n0 + sd) recomputed from
            // checkpoint U_n0 (all of them when the adjoint enters the segment from above)
            const int n0 = n - n % sd;
            if (n % sd && (n == K - 1 || (n + 1) % sd == 0)) {
                HIPC(h, hipMemcpyAsync(h->U, h->tape[n0 / sd], bytes, hipMemcpyDeviceToDevice,
                                       st));
                for (int m = n0; m < n; ++m) {
                    h->zbU_ok = false;
                    h->have_warm = false;
                    QOC(one_step(h, tau, nullptr));
                    HIPC(h, hipMemcpyAsync(h->tseg[m - n0], h->U, bytes,
                                           hipMemcpyDeviceToDevice, st));
                }
            }
            double *Un = n % sd ? h->tseg[n % sd - 1] : h->tape[n / sd];
            // recompute step n (cold solves: the same arithmetic as the taped forward)
            HIPC(h, hipMemcpyAsync(h->U, Un, bytes, hipMemcpyDeviceToDevice, st));
            h->zbU_ok = false;
            h->have_warm = false;
            QOC(one_step(h, tau, nullptr));
            const double *P = h->lastP, *Q = h->lastQ, *Uh = h->Uh;
            double *Ub = h->ab[0], *Uhb = h->ab[1], *Pb = h->ab[2], *Qb = h->ab[3],
                   *Wt = h->ab[4], *Unb = h->ab[5];
            // corrector U' = U_hat - tau Q O:  Qb = Ub (-tau O), Shb = sym(-tau Q^T Ub)
            QOC(tsgemm(h, Qb, nullptr, Ub, mp(h, MP_OR), nullptr, nullptr));
            QOC(gram64(h, Q, Ub, h->ld, N, am(h, AM_G)));
            const double *Bx = am(h, AM_G) + (size_t)N * N2;
            HIPC(h, nn_axpby(am(h, AM_SHB), N, -0.5 * tau / w, Bx, N2, -0.5 * tau / w, Bx, N2,
                             true, 0.0, N, N, st));
            // O = sym <U_hat,U_hat> - I:  Uhb = Ub + 2 w U_hat Shb
            HIPC(h, nn_axpby(am(h, AM_T), N, 2.0 * w, am(h, AM_SHB), N, 0.0, nullptr, N, false,
                             0.0, N, N, st));
            QOC(tsgemm(h, Uhb, Ub, Uh, am(h, AM_T), nullptr, nullptr));
            // Q = G U_hat:  Uhb += G Qb, gV -= rowdot(G Qb, Q)
            QOC(solve_block(h, Qb, Wt, N, 0, its.data(), &rounds, "adjoint solve G Q_bar"));
            QOC(blk_axpby(h, Uhb, Wt, 1.0, 1.0));
            QOC(rowdot_acc(h, Wt, Q, -1.0));
            // U_hat = U X + P Y:  Xb = U^T Uhb, Yb = P^T Uhb
            QOC(gram64(h, Un, Uhb, h->ld, N, am(h, AM_G)));
            HIPC(h, nn_axpby(am(h, AM_XB), N, 1.0 / w, Bx, N2, 0.0, nullptr, N, false, 0.0, N, N,
                             st));
            QOC(gram64(h, P, Uhb, h->ld, N, am(h, AM_G)));
            HIPC(h, nn_axpby(am(h, AM_YB), N, 1.0 / w, Bx, N2, 0.0, nullptr, N, false, 0.0, N, N,
                             st));
            HIPC(h, hipMemsetAsync(h->dstatus, 0, sizeof(int), st));
            HIPC(h, launch_nn_adjoint(h->G1, N, tau, am(h, AM_XB), am(h, AM_YB), h->adpool,
                                      am(h, AM_SB), h->dstatus, st));
            QOC(check_status(h, "adjoint of the predictor algebra"));
            // Ub <- Uhb X^T + U w(Sb + Sb^T) + P w Mb^T  (Ub itself is no longer needed)
            HIPC(h, nn_axpby(am(h, AM_T), N, w, am(h, AM_SB), N, w, am(h, AM_SB), N, true, 0.0,
                             N, N, st));
            QOC(tsgemm(h, Unb, nullptr, Uhb, mp(h, MP_X), Un, am(h, AM_T)));
            HIPC(h, nn_axpby(am(h, AM_T2), N, w, am(h, AM_MB), N, 0.0, nullptr, N, false, 0.0, N,
                             N, st));
            QOC(tsgemm(h, Ub, Unb, P, am(h, AM_T2), nullptr, nullptr));
            // Pb = Uhb Y^T + U w Mb + P w(Rb + Rb^T), built in Pb then Qb
            HIPC(h, nn_axpby(am(h, AM_T3), N, 0.0, nullptr, N, w, am(h, AM_MB), N, true, 0.0, N,
                             N, st));
            QOC(tsgemm(h, Pb, nullptr, Uhb, mp(h, MP_Y), Un, am(h, AM_T3)));
            HIPC(h, nn_axpby(am(h, AM_T), N, w, am(h, AM_RB), N, w, am(h, AM_RB), N, true, 0.0,
                             N, N, st));
            QOC(tsgemm(h, Qb, Pb, P, am(h, AM_T), nullptr, nullptr));
            // P = G U:  Ub += G Pb, gV -= rowdot(G Pb, P)
            QOC(solve_block(h, Qb, Wt, N, 0, its.data(), &rounds, "adjoint solve G P_bar"));
            QOC(blk_axpby(h, Ub, Wt, 1.0, 1.0));
            QOC(rowdot_acc(h, Wt, P, -1.0));
        }
        // outputs, state back at U_K
        if (gU0)
            HIPC(h, hipMemcpy2DAsync(gU0, sizeof(double) * ld, h->ab[0], sizeof(double) * h->ld,
                                     sizeof(double) * h->ng, N,
                                     on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                     st));
        if (gV)
            HIPC(h, hipMemcpyAsync(gV, h->gVd, sizeof(double) * h->ng,
                                   on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                                   st));
        HIPC(h, hipMemcpyAsync(h->U, UK, bytes, hipMemcpyDeviceToDevice, st));
        h->zbU_ok = false;
        HIPC(h, hipStreamSynchronize(st));
        return QO_OK;
    };
    const qo_status s = body();
    h->cfg.warm_start = warm;
    h->have_warm = false;
    h->have_K = false;
    return s;
}

}  // extern "C"

extern "C" qo_status qo_energy_mode(qo_handle h, int mode, int anchor) {
    if (!h) return QO_ERR_ARG;
    if (mode != 0 && mode != 1) return fail(h, QO_ERR_ARG, "energy mode must be 0 or 1");
    if (anchor < 0) return fail(h, QO_ERR_ARG, "anchor must be >= 0");
    if (mode == 1 && h->mixed)
        return fail(h, QO_ERR_ARG, "the propagated energy needs precision QO_FP64 (BF16 Grams)");
    if (mode == 1) {
        const size_t nn = (size_t)h->N * h->N;
        if (!h->Kprop) QOC(dalloc(h, &h->Kprop, nn));
        if (!h->epool) QOC(dalloc(h, &h->epool, 5 * nn));
    }
    h->emode = mode;
    h->eanchor = anchor;
    h->have_K = false;
    return QO_OK;
}
