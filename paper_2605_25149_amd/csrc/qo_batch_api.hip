// Grouped batches of independent problems (many potentials, uneven grids and N) stepped
// together with the scheme of Sec. 4.1.
//
// Instances whose grids agree form a group.  A group concatenates the columns of its
// instances into one block, so every grid-sized kernel (stencil, PCG sweeps,
// preconditioner passes, energy) runs once over all columns of the group; the per-point
// potential and the preconditioner constants are looked up per column.  The Grams, the
// block updates and the N x N algebra run once per group with one tile set or one
// workgroup per instance.  The PCG runs a fixed number of iterations per solve with
// converged columns frozen on the device, so a step needs no host synchronisation and is
// captured once per parity of the P/Q ping-pong into a HIP graph that later steps
// replay.  Band heights are chosen per group by timing the stencil on the device.
//
// In mixed precision a solve is a fixed number of restarted refinement rounds: the FP64
// residual, a per-column mask and inner tolerance, a fixed-count FP32 PCG on the
// residual (frozen columns skip their work) and the FP64 update; a final FP64 residual
// decides convergence.  The Grams, the N x N algebra and the energy stay in FP64.
#include "qo.h"
#include "qo_internal.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

using namespace qo;

struct qo_batch_ctx {
    hipStream_t st = nullptr;
    bool own_stream = false;
    int count = 0;
    std::vector<qo_config> cfg;
    struct Inst {
        int group = 0, local = 0, col0 = 0, N = 0;
        double tau = 0.0;
        bool have_V = false, have_U = false, have_Es = false;
        double last_Es = 0.0;
        long nstep = 0;
    };
    std::vector<Inst> inst;
    struct Group {
        qo_config cf{};
        Grid g{};
        DstPlan dp{};
        bool dst = false;
        long ng = 0, ld = 0, qs = 0;
        int C = 0, kmax = 0, ninst = 0, max_n = 0, max_gram_grid = 0, ty = 0;
        int kuse = 0;  // iterations per solve in use: kmax until counts are observed
        // mixed precision: FP32 PCG inside restarted FP64 refinement rounds
        bool mixed = false;
        double inner_tol = 1e-5;
        int ruse = 0;  // refinement rounds per solve in use
        std::vector<int> kr;  // FP32 iterations of each round in use
        float *vs32 = nullptr, *dinv32 = nullptr, *r32 = nullptr, *d32 = nullptr,
              *rr32 = nullptr, *pa32 = nullptr, *pb32 = nullptr;
        double *colsums = nullptr, *cin = nullptr;
        int *mask = nullptr, *nact = nullptr, *its32 = nullptr;
        // per solve: per column the FP32 iterations summed over the rounds and the rounds
        // taken part in; per round the largest count and the columns taking part
        int *itot[2] = {nullptr, nullptr}, *irounds[2] = {nullptr, nullptr},
            *rstat[2] = {nullptr, nullptr};
        double w = 1.0;
        std::vector<int> members;
        double *U = nullptr, *Uh = nullptr, *PQ[2] = {nullptr, nullptr}, *r = nullptr,
               *pa = nullptr, *pb = nullptr;
        _Float16 *t1 = nullptr, *t2 = nullptr, *dS = nullptr;
        float *z = nullptr;  // preconditioned residual (FP32 in either precision)
        float *dmu = nullptr, *pcs = nullptr, *cvbar = nullptr, *clmin = nullptr;
        double *vs = nullptr, *dinv = nullptr, *coltol = nullptr, *part = nullptr, *rzp = nullptr;
        double *G1 = nullptr, *G2 = nullptr, *pool = nullptr, *gpart = nullptr, *scal = nullptr,
               *energy = nullptr, *dsum = nullptr;
        int *cinst = nullptr, *coff = nullptr, *nstatus = nullptr, *its[2] = {nullptr, nullptr};
        PcgState ps{};
        GramJob *gjob[2][2] = {};
        TsJob *tjob[2][3] = {};
        NnJob *njob = nullptr;
        std::vector<NnJob> h_njob;
        hipStream_t st = nullptr;  // stream of the group's step work
    };
    std::vector<Group> groups;
    std::vector<void *> allocs;
    std::string err;
    int *err_dev = nullptr;  // sticky PCG error flag pair of the batch (code, first column)
    int cur = 0;             // parity of the P/Q ping-pong (common to all groups)
    hipGraphExec_t gexec[2] = {nullptr, nullptr};
    std::vector<hipStream_t> side;  // streams of groups 1.. (default priority)
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
    bool gvalid[2] = {false, false};
};

namespace {

constexpr int kMaxRounds = 30;  // refinement rounds per mixed-precision solve, at most

qo_status bfail(qo_batch_ctx *b, qo_status s, const char *fmt, ...) {
    if (b) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        b->err = buf;
    }
    return s;
}

#define BHIP(b, call)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return bfail(b, QO_ERR_DEVICE, "%s failed: %s (%s:%d)", #call,                 \
                         hipGetErrorString(e_), __FILE__, __LINE__);                       \
    } while (0)

#define BQO(call)                       \
    do {                                \
        qo_status s_ = (call);          \
        if (s_ != QO_OK) return s_;     \
    } while (0)

template <typename T>
qo_status balloc(qo_batch_ctx *b, T **p, size_t n) {
    void *q = nullptr;
    if (n == 0) n = 1;
    if (hipMalloc(&q, n * sizeof(T)) != hipSuccess)
        return bfail(b, QO_ERR_ALLOC, "hipMalloc(%zu bytes) failed", n * sizeof(T));
    b->allocs.push_back(q);
    if (hipMemsetAsync(q, 0, n * sizeof(T), b->st) != hipSuccess)
        return bfail(b, QO_ERR_DEVICE, "hipMemsetAsync failed");
    *p = static_cast<T *>(q);
    return QO_OK;
}

bool same_grid(const qo_config &a, const qo_config &c) {
    if (a.dim != c.dim || a.kinetic != c.kinetic || a.precond != c.precond) return false;
    if (a.precision != c.precision ||
        (a.precision == QO_MIXED && a.refine_inner_tol != c.refine_inner_tol))
        return false;
    for (int k = 0; k < a.dim; ++k)
        if (a.n[k] != c.n[k] || a.L[k] != c.L[k]) return false;
    return true;
}

// Grid of a group with band height TY (the other tiling rules of the single-instance path).
Grid group_grid(const qo_config &cf, int ncols, int TY, double *w) {
    Grid g{};
    g.dim = cf.dim;
    g.nx = cf.n[0];
    g.ny = cf.n[1];
    g.nz = cf.dim == 3 ? cf.n[2] : 1;
    g.ng = (long)g.nx * g.ny * g.nz;
    double h[3];
    for (int k = 0; k < 3; ++k) h[k] = (k < cf.dim) ? cf.L[k] / (cf.n[k] + 1) : 1.0;
    g.ihx2 = 1.0 / (h[0] * h[0]);
    g.ihy2 = 1.0 / (h[1] * h[1]);
    g.ihz2 = cf.dim == 3 ? 1.0 / (h[2] * h[2]) : 0.0;
    g.kappa = cf.kinetic;
    g.c0 = 2.0 * cf.kinetic * (g.ihx2 + g.ihy2 + g.ihz2);
    *w = h[0] * h[1] * (cf.dim == 3 ? h[2] : 1.0);
    if (TY > g.ny) TY = g.ny;
    if (TY < 1) TY = 1;
    while (pick_ppt(TY * g.nx) < 0 && TY > 1) --TY;
    g.TY = TY;
    g.ppt = pick_ppt(TY * g.nx);
    // as in the single-instance plan: several planes per tile and rows wider than a
    // workgroup need the engine for 4 or more points per thread (it loops over halo columns)
    if (cf.dim == 3 && g.nx > kThreads && g.ppt < 4) g.ppt = 4;
    g.nbands = (g.ny + TY - 1) / TY;
    if (cf.dim == 2) {
        g.ZC = 1;
        g.nzc = 1;
    } else {
        long want = (2048 + (long)ncols * g.nbands - 1) / ((long)ncols * g.nbands);
        int maxc = g.nz / 16;
        if (maxc < 1) maxc = 1;
        if (want > maxc) want = maxc;
        if (want < 1) want = 1;
        g.ZC = (g.nz + (int)want - 1) / (int)want;
        g.nzc = (g.nz + g.ZC - 1) / g.ZC;
    }
    return g;
}

// Band heights worth timing: 256 to 2048 points per plane (one to eight per thread).
std::vector<int> ty_candidates(const qo_config &cf) {
    std::vector<int> out;
    const int nx = cf.n[0], ny = cf.n[1];
    for (int ty = 1; ty <= ny; ++ty) {
        const int pts = ty * nx;
        if (pts < 256 && ty < ny) continue;
        if (pts > 2048 || pick_ppt(pts) < 0) break;
        const int ppt = pick_ppt(pts);
        // keep the tallest band of each points-per-thread class (fewest halo rows)
        if (pick_ppt((ty + 1) * nx) == ppt && ty + 1 <= ny && (ty + 1) * nx <= 2048) continue;
        out.push_back(ty);
    }
    if (out.empty()) out.push_back(std::max(1, std::min(ny, 1536 / nx)));
    return out;
}

void dst_tables_host(const qo_config &cf, const DstPlan &dp, std::vector<float> &mu,
                     double *mu0) {
    auto push = [&](int n, double L) {
        const double hh = L / (n + 1);
        for (int j = 0; j < n; ++j) {
            const double sn = std::sin(M_PI * (j + 1) / (2.0 * (n + 1)));
            mu.push_back((float)(4.0 * sn * sn / (hh * hh)));
        }
    };
    push(dp.nx, cf.L[0]);
    push(dp.ny, cf.L[1]);
    if (cf.dim == 3) push(dp.nz, cf.L[2]);
    else push(dp.ny, cf.L[1]);
    *mu0 = (double)mu[0] + (cf.dim == 3 ? (double)mu[dp.nx] : 0.0) + (double)mu[dp.nx + dp.ny];
}

qo_status group_pcg(qo_batch_ctx *b, qo_batch_ctx::Group &G, const double *B, double *X,
                    int which) {
    hipStream_t st = G.st;
    PcgState s = G.ps;
    s.its = G.its[which];
    s.coltol = G.coltol;
    s.err = b->err_dev;
    const Grid &g = G.g;
    const int tiles = g.tiles();
    BHIP(b, launch_fill_int(s.its, G.C, 0, st));
    BHIP(b, launch_pcg_init<double>(g, G.vs, G.dinv, B, X, G.r, G.ld, G.C, 1, s.part, st));
    double *pbuf[2] = {G.pa, G.pb};
    const int K = G.kuse;
    for (int k = 0; k <= K; ++k) {
        if (G.dst) {
            BHIP(b, launch_pc_prep(k, G.C, nullptr, s, G.qs, tiles, 0.0, G.ng, G.pcs, st));
            BHIP(b, launch_dst_fwd<double>(G.dp, G.r, G.ld, G.C, G.t1, G.pcs, st));
            BHIP(b, launch_dst_pencil(G.dp, G.t1, G.t2, G.ld, G.C, G.pcs, G.rzp, st));
            BHIP(b, launch_dst_inv(G.dp, G.t2, G.z, G.ld, G.C, G.pcs, st));
        }
        BHIP(b, launch_pcg_sweep1<double>(g, G.vs, G.dinv, G.r, pbuf[(k + 1) & 1], pbuf[k & 1],
                                          G.ld, G.C, k, 0.0, nullptr, s, st,
                                          G.dst ? G.z : nullptr, G.rzp, G.dp.rzparts));
        if (k == K) break;
        BHIP(b, launch_pcg_sweep2<double>(g, G.vs, G.dinv, pbuf[k & 1], X, G.r, G.ld, G.C, k, s,
                                          st, !G.dst));
    }
    // a column still active after the final test did not converge
    BHIP(b, launch_noconv_check(s.active + (K & 1) * G.C, G.C, b->err_dev, st));
    return QO_OK;
}

// Mixed-precision solve X = G B (X holds the starting guess): ruse restarted rounds of
// FP64 residual -> FP32 PCG with kuse iterations on the columns still above their
// tolerance -> X += d, then the final FP64 residual test.  which selects the solve's
// bookkeeping arrays (per column the FP32 iterations summed over the rounds and the
// rounds in which it took part; per round the largest count and the columns taking part).
qo_status group_solve_mixed(qo_batch_ctx *b, qo_batch_ctx::Group &G, const double *B,
                            double *X, int which) {
    hipStream_t st = G.st;
    const Grid &g = G.g;
    const int tiles = g.tiles();
    PcgState s = G.ps;
    s.its = G.its32;
    s.coltol = G.cin;
    s.err = b->err_dev;
    BHIP(b, launch_fill_int(G.itot[which], G.C, 0, st));
    BHIP(b, launch_fill_int(G.irounds[which], G.C, 0, st));
    BHIP(b, launch_fill_int(G.rstat[which], 2 * kMaxRounds, 0, st));
    float *pbuf[2] = {G.pa32, G.pb32};
    for (int round = 0; round <= G.ruse; ++round) {
        BHIP(b, launch_resid(g, G.vs, B, X, G.ld, G.r32, G.ld, G.C, nullptr, G.part, st));
        BHIP(b, launch_colsum(G.part + G.qs, tiles, G.C, 2, G.qs, G.colsums, st));
        BHIP(b, launch_refine_mask(G.colsums, G.C, 0.0, G.inner_tol, G.mask, G.cin, G.nact,
                                   b->err_dev, st, G.coltol));
        if (round == G.ruse) break;
        const int K = G.kr[round];
        BHIP(b, launch_fill_int(G.its32, G.C, 0, st));
        BHIP(b, launch_pcg_init<float>(g, G.vs32, G.dinv32, G.r32, G.d32, G.rr32, G.ld, G.C, 0,
                                       s.part, st));
        for (int k = 0; k <= K; ++k) {
            if (G.dst) {
                BHIP(b, launch_pc_prep(k, G.C, G.mask, s, G.qs, tiles, 0.0, G.ng, G.pcs, st));
                BHIP(b, launch_dst_fwd<float>(G.dp, G.rr32, G.ld, G.C, G.t1, G.pcs, st));
                BHIP(b, launch_dst_pencil(G.dp, G.t1, G.t2, G.ld, G.C, G.pcs, G.rzp, st));
                BHIP(b, launch_dst_inv(G.dp, G.t2, G.z, G.ld, G.C, G.pcs, st));
            }
            BHIP(b, launch_pcg_sweep1<float>(g, G.vs32, G.dinv32, G.rr32, pbuf[(k + 1) & 1],
                                             pbuf[k & 1], G.ld, G.C, k, 0.0, G.mask, s, st,
                                             G.dst ? G.z : nullptr, G.rzp, G.dp.rzparts));
            if (k == K) break;
            BHIP(b, launch_pcg_sweep2<float>(g, G.vs32, G.dinv32, pbuf[k & 1], G.d32, G.rr32,
                                             G.ld, G.C, k, s, st, !G.dst));
        }
        BHIP(b, launch_its_accum(G.its32, G.mask, G.C, G.itot[which], G.irounds[which],
                                 G.rstat[which] + 2 * round, st));
        BHIP(b, launch_refine_axpy(X, G.ld, G.d32, G.ld, G.ng, G.C, G.mask, 0, st));
    }
    // a column still above its tolerance after the last round did not converge
    BHIP(b, launch_noconv_check(G.mask, G.C, b->err_dev, st));
    return QO_OK;
}

// One group's share of a step, on the group's stream.
qo_status group_step_enqueue(qo_batch_ctx *b, qo_batch_ctx::Group &G, int par) {
    hipStream_t st = G.st;
    double *P = G.PQ[par], *Q = G.PQ[par ^ 1];
    if (G.mixed) BQO(group_solve_mixed(b, G, G.U, P, 0));
    else BQO(group_pcg(b, G, G.U, P, 0));
    BHIP(b, launch_gram_f64_batch(G.gjob[par][0], G.ninst, G.max_gram_grid, G.ld, G.ng, G.w, st));
    BHIP(b, launch_nn_predict(G.njob, G.ninst, G.max_n, st));
    BHIP(b, launch_tsgemm_batch(G.tjob[par][0], G.ninst, G.max_n, G.ld, G.ng, st));
    BHIP(b, launch_tsgemm_batch(G.tjob[par][1], G.ninst, G.max_n, G.ld, G.ng, st));
    if (G.mixed) BQO(group_solve_mixed(b, G, G.Uh, Q, 1));
    else BQO(group_pcg(b, G, G.Uh, Q, 1));
    BHIP(b, launch_gram_f64_batch(G.gjob[par][1], G.ninst, G.max_gram_grid, G.ld, G.ng, G.w, st));
    BHIP(b, launch_nn_correct(G.njob, G.ninst, st));
    BHIP(b, launch_tsgemm_batch(G.tjob[par][2], G.ninst, G.max_n, G.ld, G.ng, st));
    BHIP(b, launch_quad(G.g, G.vs, G.U, G.ld, G.C, G.part, st));
    BHIP(b, launch_instance_energy(G.part, G.qs, G.g.tiles(), G.coff, G.ninst, G.w, G.energy, st));
    return QO_OK;
}

// One step of every group without host synchronisation.  Groups are independent: the
// first runs on the batch stream, every other one on a stream of its own that forks from
// the batch stream and joins it again at the end, so the small groups' launches overlap
// the large ones (captured graphs keep this as parallel branches).  The joins are made
// even when a group's enqueue fails, so no stream is left forked (or in a capture).
qo_status batch_step_enqueue(qo_batch_ctx *b, int par) {
    const size_t ng = b->groups.size();
    if (ng > 1) {
        BHIP(b, hipEventRecord(b->ev_fork, b->st));
        for (size_t k = 1; k < ng; ++k) BHIP(b, hipStreamWaitEvent(b->groups[k].st, b->ev_fork, 0));
    }
    qo_status first = QO_OK;
    for (auto &G : b->groups) {
        const qo_status s = group_step_enqueue(b, G, par);
        if (s != QO_OK && first == QO_OK) first = s;
        if (first != QO_OK) break;
    }
    for (size_t k = 1; k < ng; ++k) {
        const hipError_t e1 = hipEventRecord(b->ev_join[k], b->groups[k].st);
        const hipError_t e2 = hipStreamWaitEvent(b->st, b->ev_join[k], 0);
        if ((e1 != hipSuccess || e2 != hipSuccess) && first == QO_OK)
            first = bfail(b, QO_ERR_DEVICE, "stream join failed");
    }
    return first;
}

qo_status build_group(qo_batch_ctx *b, qo_batch_ctx::Group &G) {
    const qo_config &cf = G.cf;
    G.ninst = (int)G.members.size();
    std::vector<int> cinst, coff(G.ninst + 1, 0);
    std::vector<double> coltol;
    int kmax = 0;
    for (int li = 0; li < G.ninst; ++li) {
        auto &I = b->inst[G.members[li]];
        const qo_config &c = b->cfg[G.members[li]];
        I.local = li;
        I.col0 = G.C;
        I.N = c.N;
        coff[li] = G.C;
        for (int j = 0; j < c.N; ++j) {
            cinst.push_back(li);
            coltol.push_back(c.pcg_tol);
        }
        G.C += c.N;
        G.max_n = std::max(G.max_n, c.N);
        kmax = std::max(kmax, c.pcg_maxit);
    }
    coff[G.ninst] = G.C;
    G.kmax = kmax;
    G.kuse = kmax;
    G.mixed = cf.precision == QO_MIXED;
    G.inner_tol = cf.refine_inner_tol;
    G.ruse = 6;
    G.kr.assign(kMaxRounds, kmax);
    G.ng = (long)cf.n[0] * cf.n[1] * (cf.dim == 3 ? cf.n[2] : 1);
    G.ld = (G.ng + 63) / 64 * 64;
    const size_t blk = (size_t)G.ld * G.C;
    // tiling: the finest candidate band bounds the partial-sum storage
    const std::vector<int> cands = ty_candidates(cf);
    long max_tiles = 0;
    for (int ty : cands) {
        double w;
        max_tiles = std::max(max_tiles, (long)group_grid(cf, G.C, ty, &w).tiles());
    }
    G.g = group_grid(cf, G.C, cands.back(), &G.w);
    G.ty = G.g.TY;
    auto A = [&](auto **p, size_t n) { return balloc(b, p, n); };
    BQO(A(&G.U, blk));
    BQO(A(&G.Uh, blk));
    BQO(A(&G.PQ[0], blk));
    BQO(A(&G.PQ[1], blk));
    BQO(A(&G.r, blk));
    BQO(A(&G.pa, blk));
    BQO(A(&G.pb, blk));
    BQO(A(&G.vs, (size_t)G.ninst * G.ng));
    BQO(A(&G.dinv, (size_t)G.ninst * G.ng));
    BQO(A(&G.cinst, (size_t)G.C));
    BQO(A(&G.coff, (size_t)G.ninst + 1));
    BQO(A(&G.coltol, (size_t)G.C));
    BQO(A(&G.part, (size_t)8 * G.C * max_tiles));
    BQO(A(&G.ps.rho, (size_t)2 * G.C));
    BQO(A(&G.ps.alpha, (size_t)2 * G.C));
    BQO(A(&G.ps.active, (size_t)2 * G.C));
    BQO(A(&G.its[0], (size_t)G.C));
    BQO(A(&G.its[1], (size_t)G.C));
    BQO(A(&G.ps.bb, (size_t)G.C));
    BQO(A(&G.dsum, 1));
    BQO(A(&G.energy, (size_t)2 * G.ninst));
    BQO(A(&G.scal, (size_t)3 * G.ninst));
    BQO(A(&G.nstatus, (size_t)G.ninst));
    G.ps.part = G.part;
    if (G.mixed) {
        BQO(A(&G.vs32, (size_t)G.ninst * G.ng));
        BQO(A(&G.dinv32, (size_t)G.ninst * G.ng));
        BQO(A(&G.r32, blk));
        BQO(A(&G.d32, blk));
        BQO(A(&G.rr32, blk));
        BQO(A(&G.pa32, blk));
        BQO(A(&G.pb32, blk));
        BQO(A(&G.colsums, (size_t)2 * G.C));
        BQO(A(&G.cin, (size_t)G.C));
        BQO(A(&G.mask, (size_t)G.C));
        BQO(A(&G.nact, 1));
        BQO(A(&G.its32, (size_t)G.C));
        for (int k = 0; k < 2; ++k) {
            BQO(A(&G.itot[k], (size_t)G.C));
            BQO(A(&G.irounds[k], (size_t)G.C));
            BQO(A(&G.rstat[k], (size_t)2 * kMaxRounds));
        }
    }
    BHIP(b, hipMemcpyAsync(G.cinst, cinst.data(), sizeof(int) * G.C, hipMemcpyHostToDevice, b->st));
    BHIP(b, hipMemcpyAsync(G.coff, coff.data(), sizeof(int) * (G.ninst + 1), hipMemcpyHostToDevice,
                           b->st));
    BHIP(b, hipMemcpyAsync(G.coltol, coltol.data(), sizeof(double) * G.C, hipMemcpyHostToDevice,
                           b->st));
    // fast-Poisson preconditioner tables
    if (cf.precond == 1) {
        G.dst = true;
        DstPlan &dp = G.dp;
        dst_plan_geometry(dp, cf.dim, G.g.nx, G.g.ny, G.g.nz);
        const size_t sx = (size_t)dp.NXP * dp.NXP, sy = (size_t)dp.NYP * dp.NYP,
                     ss = (size_t)dp.NSP * dp.NSP;
        BQO(A(&G.dS, sx + sy + ss));
        BQO(A(&G.dmu, (size_t)dp.nx + dp.ny + dp.ns));
        BQO(A(&G.t1, blk));
        BQO(A(&G.t2, blk));
        BQO(A(&G.z, blk));
        BQO(A(&G.pcs, (size_t)G.C));
        BQO(A(&G.cvbar, (size_t)G.C));
        BQO(A(&G.clmin, (size_t)G.C));
        BQO(A(&G.rzp, (size_t)G.C * dp.rzparts));
        dp.Sx = G.dS;
        dp.Sy = G.dS + sx;
        dp.Ss = G.dS + sx + sy;
        dp.mux = G.dmu;
        dp.muy = G.dmu + dp.nx;
        dp.mus = G.dmu + dp.nx + dp.ny;
        dp.kap = (float)cf.kinetic;
        dp.cvbar = G.cvbar;
        dp.clmin = G.clmin;
        std::vector<float> mu;
        double mu0;
        dst_tables_host(cf, dp, mu, &mu0);
        BHIP(b, hipMemcpyAsync(G.dmu, mu.data(), sizeof(float) * mu.size(), hipMemcpyHostToDevice,
                               b->st));
        BHIP(b, hipStreamSynchronize(b->st));
        BHIP(b, launch_dst_matrix(dp.nx, dp.NXP, G.dS, b->st));
        BHIP(b, launch_dst_matrix(dp.ny, dp.NYP, G.dS + sx, b->st));
        BHIP(b, launch_dst_matrix(dp.ns, dp.NSP, G.dS + sx + sy, b->st));
        // until a potential is set: vbar = 0
        std::vector<float> vb(G.C, 0.f), lm(G.C, (float)(cf.kinetic * mu0));
        BHIP(b, hipMemcpyAsync(G.cvbar, vb.data(), sizeof(float) * G.C, hipMemcpyHostToDevice,
                               b->st));
        BHIP(b, hipMemcpyAsync(G.clmin, lm.data(), sizeof(float) * G.C, hipMemcpyHostToDevice,
                               b->st));
        BHIP(b, hipStreamSynchronize(b->st));
    }
    // per-instance N x N workspaces, Gram partials and job tables
    size_t pool_tot = 0, g_tot = 0, gp_tot = 0;
    std::vector<int> nsplit(G.ninst);
    for (int li = 0; li < G.ninst; ++li) {
        const int n = b->cfg[G.members[li]].N;
        // K-chunks per Gram: about 8192 wavefronts over the whole group (the
        // single-instance rule targets 4096 for one Gram), at least 256 rows each, and the
        // instance's partials capped like the single-instance ones
        {
            const int np = gram_pairs(n);
            long ns = 8192 / ((long)np * G.ninst);
            ns = std::min(ns, (G.ng + 255) / 256);
            ns = std::min(ns, (long)gram_nsplit(G.ng, n));
            nsplit[li] = (int)std::max(1L, ns);
        }
        pool_tot += nn_pool_elems(n);
        g_tot += (size_t)4 * n * n;
        gp_tot += gram_part_elems(n, nsplit[li]);
        G.max_gram_grid = std::max(G.max_gram_grid, gram_pairs(n) * nsplit[li]);
    }
    BQO(A(&G.pool, pool_tot));
    BQO(A(&G.G1, g_tot));
    BQO(A(&G.G2, g_tot));
    BQO(A(&G.gpart, gp_tot));
    std::vector<GramJob> gj[2][2];
    std::vector<TsJob> tj[2][3];
    G.h_njob.resize(G.ninst);
    size_t po = 0, go = 0, gpo = 0;
    for (int li = 0; li < G.ninst; ++li) {
        const int n = b->cfg[G.members[li]].N;
        const long off = (long)coff[li] * G.ld;
        double *pool = G.pool + po, *G1 = G.G1 + go, *G2 = G.G2 + go, *gp = G.gpart + gpo;
        NnJob &J = G.h_njob[li];
        J.G1 = G1;
        J.G2 = G2;
        J.pool = pool;
        J.scal = G.scal + 3 * li;
        J.status = G.nstatus + li;
        J.n = n;
        J.tau = 0.0;
        const double *XR = pool + (size_t)nn_slot_xr() * n * n;
        const double *YR = pool + (size_t)nn_slot_yr() * n * n;
        const double *ZR = pool + (size_t)nn_slot_zr() * n * n;
        const double *OR = pool + (size_t)nn_slot_or() * n * n;
        for (int par = 0; par < 2; ++par) {
            double *P = G.PQ[par] + off, *Q = G.PQ[par ^ 1] + off;
            const long kc = gram_kchunk(G.ng, nsplit[li]);
            gj[par][0].push_back(GramJob{G.U + off, P, gp, G1, n, nsplit[li], kc});
            gj[par][1].push_back(GramJob{G.Uh + off, Q, gp, G2, n, nsplit[li], kc});
            tj[par][0].push_back(TsJob{G.Uh + off, nullptr, G.U + off, XR, P, YR, n});
            tj[par][1].push_back(TsJob{Q, nullptr, P, ZR, nullptr, nullptr, n});
            tj[par][2].push_back(TsJob{G.U + off, G.Uh + off, nullptr, nullptr, Q, OR, n});
        }
        po += nn_pool_elems(n);
        go += (size_t)4 * n * n;
        gpo += gram_part_elems(n, nsplit[li]);
    }
    for (int par = 0; par < 2; ++par) {
        for (int k = 0; k < 2; ++k) {
            BQO(A(&G.gjob[par][k], (size_t)G.ninst));
            BHIP(b, hipMemcpyAsync(G.gjob[par][k], gj[par][k].data(), sizeof(GramJob) * G.ninst,
                                   hipMemcpyHostToDevice, b->st));
        }
        for (int k = 0; k < 3; ++k) {
            BQO(A(&G.tjob[par][k], (size_t)G.ninst));
            BHIP(b, hipMemcpyAsync(G.tjob[par][k], tj[par][k].data(), sizeof(TsJob) * G.ninst,
                                   hipMemcpyHostToDevice, b->st));
        }
    }
    BQO(A(&G.njob, (size_t)G.ninst));
    BHIP(b, hipMemcpyAsync(G.njob, G.h_njob.data(), sizeof(NnJob) * G.ninst, hipMemcpyHostToDevice,
                           b->st));
    BHIP(b, hipStreamSynchronize(b->st));
    G.g.cinst = G.cinst;
    G.qs = (long)G.C * G.g.tiles();
    return QO_OK;
}

// Time the stencil engine over the group's columns for every candidate band height and
// keep the fastest (median of 3 launches after one warm-up launch).
qo_status autotune_group(qo_batch_ctx *b, qo_batch_ctx::Group &G) {
    const std::vector<int> cands = ty_candidates(G.cf);
    if (cands.size() <= 1) return QO_OK;
    hipEvent_t e0, e1;
    BHIP(b, hipEventCreate(&e0));
    BHIP(b, hipEventCreate(&e1));
    float best = 1e30f;
    int best_ty = G.g.TY;
    for (int ty : cands) {
        double w;
        Grid g = group_grid(G.cf, G.C, ty, &w);
        g.cinst = G.cinst;
        float t[3];
        hipError_t e = launch_apply(g, G.vs, G.U, G.Uh, G.ld, G.C, b->st);
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
            e = hipEventRecord(e0, b->st);
            if (e == hipSuccess) e = launch_apply(g, G.vs, G.U, G.Uh, G.ld, G.C, b->st);
            if (e == hipSuccess) e = hipEventRecord(e1, b->st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            if (e == hipSuccess) e = hipEventElapsedTime(&t[rep], e0, e1);
        }
        if (e != hipSuccess) {
            (void)hipEventDestroy(e0);
            (void)hipEventDestroy(e1);
            return bfail(b, QO_ERR_DEVICE, "band-height tuning failed: %s", hipGetErrorString(e));
        }
        std::sort(t, t + 3);
        if (t[1] < best) {
            best = t[1];
            best_ty = ty;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    G.g = group_grid(G.cf, G.C, best_ty, &G.w);
    G.g.cinst = G.cinst;
    G.ty = G.g.TY;
    G.qs = (long)G.C * G.g.tiles();
    return QO_OK;
}

}  // namespace

extern "C" {

const char *qo_batch_last_error(qo_batch b) { return b ? b->err.c_str() : "null batch"; }

qo_status qo_batch_destroy(qo_batch b) {
    if (!b) return QO_ERR_ARG;
    if (b->st) (void)hipStreamSynchronize(b->st);
    for (int p = 0; p < 2; ++p)
        if (b->gexec[p]) (void)hipGraphExecDestroy(b->gexec[p]);
    for (hipStream_t s : b->side) (void)hipStreamSynchronize(s);
    for (void *p : b->allocs) (void)hipFree(p);
    for (hipEvent_t e : b->ev_join)
        if (e) (void)hipEventDestroy(e);
    if (b->ev_fork) (void)hipEventDestroy(b->ev_fork);
    for (hipStream_t s : b->side) (void)hipStreamDestroy(s);
    if (b->own_stream && b->st) (void)hipStreamDestroy(b->st);
    delete b;
    return QO_OK;
}

qo_status qo_batch_create(const qo_config *cfgs, int count, void *hip_stream, qo_batch *out) {
    if (!out) return QO_ERR_ARG;
    *out = nullptr;
    if (!cfgs || count < 1) return QO_ERR_ARG;
    for (int i = 0; i < count; ++i) {
        const qo_config &c = cfgs[i];
        if (c.dim != 2 && c.dim != 3) return QO_ERR_ARG;
        long ng = 1;
        for (int k = 0; k < c.dim; ++k) {
            if (c.n[k] < 1 || !(c.L[k] > 0.0)) return QO_ERR_ARG;
            ng *= c.n[k];
        }
        if (c.n[0] > 1024 || c.N < 1 || c.N >= ng || c.N > 1024) return QO_ERR_ARG;
        if (!(c.kinetic > 0.0) || !std::isfinite(c.sigma)) return QO_ERR_ARG;
        if (!(c.pcg_tol > 0.0) || c.pcg_maxit < 1 || c.pcg_maxit > 100000) return QO_ERR_ARG;
        if ((c.precision != QO_FP64 && c.precision != QO_MIXED) || c.pcg_variant != 0)
            return QO_ERR_ARG;
        if (c.precision == QO_MIXED &&
            !(c.refine_inner_tol > 0.0 && c.refine_inner_tol < 1.0))
            return QO_ERR_ARG;
        if (c.precond != 0 && c.precond != 1) return QO_ERR_ARG;
        if (c.precond == 1 && dst_plan_check(c.dim, c.n)) return QO_ERR_ARG;
    }
    qo_batch_ctx *b = new (std::nothrow) qo_batch_ctx();
    if (!b) return QO_ERR_ALLOC;
    b->count = count;
    b->cfg.assign(cfgs, cfgs + count);
    b->inst.resize(count);
    if (hip_stream) {
        b->st = static_cast<hipStream_t>(hip_stream);
    } else {
        // graph capture needs a stream other than the null stream
        if (hipStreamCreate(&b->st) != hipSuccess) {
            delete b;
            return QO_ERR_DEVICE;
        }
        b->own_stream = true;
    }
    for (int i = 0; i < count; ++i) {
        int gi = -1;
        for (size_t k = 0; k < b->groups.size(); ++k)
            if (same_grid(b->groups[k].cf, cfgs[i])) gi = (int)k;
        if (gi < 0) {
            b->groups.emplace_back();
            b->groups.back().cf = cfgs[i];
            gi = (int)b->groups.size() - 1;
        }
        b->groups[gi].members.push_back(i);
        b->inst[i].group = gi;
    }
    qo_status s = balloc(b, &b->err_dev, 2);
    b->ev_join.assign(b->groups.size(), nullptr);
    if (s == QO_OK && b->groups.size() > 1 &&
        hipEventCreateWithFlags(&b->ev_fork, hipEventDisableTiming) != hipSuccess)
        s = QO_ERR_DEVICE;
    for (size_t k = 0; k < b->groups.size() && s == QO_OK; ++k) {
        if (k == 0) {
            b->groups[k].st = b->st;
            continue;
        }
        hipStream_t hs = nullptr;
        if (hipStreamCreate(&hs) != hipSuccess) {
            s = QO_ERR_DEVICE;
            break;
        }
        b->side.push_back(hs);
        b->groups[k].st = hs;
        if (hipEventCreateWithFlags(&b->ev_join[k], hipEventDisableTiming) != hipSuccess)
            s = QO_ERR_DEVICE;
    }
    for (auto &G : b->groups)
        if (s == QO_OK) s = build_group(b, G);
    for (auto &G : b->groups)
        if (s == QO_OK) s = autotune_group(b, G);
    if (s == QO_OK && hipStreamSynchronize(b->st) != hipSuccess) s = QO_ERR_DEVICE;
    if (s != QO_OK) {
        qo_batch_destroy(b);
        return s;
    }
    *out = b;
    return QO_OK;
}

// Back to the counts of a fresh batch for group G: pcg_maxit iterations per solve (six
// rounds of pcg_maxit FP32 iterations in mixed precision) until counts are observed
// again, and the captured graphs re-recorded.  Taken when a new state or potential makes
// the counts of earlier warm-started steps meaningless, and after a solve ran out of
// iterations.
static void reset_counts(qo_batch b, int group) {
    auto &G = b->groups[group];
    G.kuse = G.kmax;
    G.ruse = 6;
    G.kr.assign(kMaxRounds, G.kmax);
    b->gvalid[0] = b->gvalid[1] = false;
}

qo_status qo_batch_set_potential(qo_batch b, int i, const double *V, int on_device) {
    if (!b) return QO_ERR_ARG;
    if (i < 0 || i >= b->count || !V) return bfail(b, QO_ERR_ARG, "bad instance or null potential");
    auto &I = b->inst[i];
    auto &G = b->groups[I.group];
    const qo_config &c = b->cfg[i];
    hipStream_t st = b->st;
    const double *src = V;
    if (!on_device) {
        BHIP(b, hipMemcpyAsync(G.r, V, sizeof(double) * G.ng, hipMemcpyHostToDevice, st));
        src = G.r;
    }
    double *vs = G.vs + (size_t)I.local * G.ng, *dinv = G.dinv + (size_t)I.local * G.ng;
    BHIP(b, hipMemsetAsync(G.nstatus + I.local, 0, sizeof(int), st));
    float *vs32 = G.mixed ? G.vs32 + (size_t)I.local * G.ng : nullptr;
    float *dinv32 = G.mixed ? G.dinv32 + (size_t)I.local * G.ng : nullptr;
    BHIP(b, launch_batch_potential(src, G.ng, c.sigma, G.g.c0, vs, dinv, vs32, dinv32,
                                   G.nstatus + I.local, st));
    int bad = 0;
    BHIP(b, hipMemcpyAsync(&bad, G.nstatus + I.local, sizeof(int), hipMemcpyDeviceToHost, st));
    if (G.dst) BHIP(b, launch_sum(vs, G.ng, G.dsum, st));
    double sum = 0.0;
    if (G.dst) BHIP(b, hipMemcpyAsync(&sum, G.dsum, sizeof(double), hipMemcpyDeviceToHost, st));
    BHIP(b, hipStreamSynchronize(st));
    BHIP(b, hipMemsetAsync(G.nstatus + I.local, 0, sizeof(int), st));
    if (bad == 7) return bfail(b, QO_ERR_NONFINITE, "instance %d: non-finite potential", i);
    if (bad == 5) return bfail(b, QO_ERR_NOT_SPD, "instance %d: diagonal of H_sigma not positive", i);
    if (G.dst) {
        std::vector<float> mu;
        double mu0;
        dst_tables_host(G.cf, G.dp, mu, &mu0);
        const double vbar = std::max(0.0, sum / (double)G.ng);
        std::vector<float> vb(I.N, (float)vbar), lm(I.N, (float)(G.cf.kinetic * mu0 + vbar));
        BHIP(b, hipMemcpyAsync(G.cvbar + I.col0, vb.data(), sizeof(float) * I.N,
                               hipMemcpyHostToDevice, st));
        BHIP(b, hipMemcpyAsync(G.clmin + I.col0, lm.data(), sizeof(float) * I.N,
                               hipMemcpyHostToDevice, st));
        BHIP(b, hipStreamSynchronize(st));
    }
    I.have_V = true;
    reset_counts(b, I.group);
    return QO_OK;
}

qo_status qo_batch_set_state(qo_batch b, int i, const double *U, long ld, int on_device) {
    if (!b) return QO_ERR_ARG;
    if (i < 0 || i >= b->count || !U) return bfail(b, QO_ERR_ARG, "bad instance or null state");
    auto &I = b->inst[i];
    auto &G = b->groups[I.group];
    if (ld < G.ng) return bfail(b, QO_ERR_ARG, "ld %ld < Ng %ld", ld, G.ng);
    const size_t row = sizeof(double) * G.ng;
    BHIP(b, hipMemcpy2DAsync(G.U + (size_t)I.col0 * G.ld, sizeof(double) * G.ld, U,
                             sizeof(double) * ld, row, I.N,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, b->st));
    // drop the instance's warm start: its next solve of G U starts from zero
    BHIP(b, hipMemset2DAsync(G.PQ[b->cur] + (size_t)I.col0 * G.ld, sizeof(double) * G.ld, 0, row,
                             I.N, b->st));
    BHIP(b, hipStreamSynchronize(b->st));
    I.have_U = true;
    I.have_Es = false;
    I.nstep = 0;
    reset_counts(b, I.group);
    return QO_OK;
}

qo_status qo_batch_get_state(qo_batch b, int i, double *U, long ld, int on_device) {
    if (!b) return QO_ERR_ARG;
    if (i < 0 || i >= b->count || !U) return bfail(b, QO_ERR_ARG, "bad instance or null output");
    auto &I = b->inst[i];
    auto &G = b->groups[I.group];
    if (ld < G.ng) return bfail(b, QO_ERR_ARG, "ld %ld < Ng %ld", ld, G.ng);
    BHIP(b, hipMemcpy2DAsync(U, sizeof(double) * ld, G.U + (size_t)I.col0 * G.ld,
                             sizeof(double) * G.ld, sizeof(double) * G.ng, I.N,
                             on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, b->st));
    BHIP(b, hipStreamSynchronize(b->st));
    return QO_OK;
}

qo_status qo_batch_tile(qo_batch b, int i, int *ty) {
    if (!b) return QO_ERR_ARG;
    if (i < 0 || i >= b->count || !ty) return bfail(b, QO_ERR_ARG, "bad instance or null output");
    *ty = b->groups[b->inst[i].group].ty;
    return QO_OK;
}

qo_status qo_batch_step(qo_batch b, const double *taus, int nsteps, int use_graph,
                        qo_step_stats *stats) {
    if (!b) return QO_ERR_ARG;
    if (nsteps < 1) return bfail(b, QO_ERR_ARG, "nsteps < 1");
    for (int i = 0; i < b->count; ++i) {
        if (!b->inst[i].have_V || !b->inst[i].have_U)
            return bfail(b, QO_ERR_STATE, "instance %d: set the potential and the state first", i);
        if (taus && !(taus[i] > 0.0 && std::isfinite(taus[i])))
            return bfail(b, QO_ERR_ARG, "instance %d: tau must be positive", i);
        if (!taus && !(b->inst[i].tau > 0.0))
            return bfail(b, QO_ERR_ARG, "no time steps given");
    }
    hipStream_t st = b->st;
    // time steps live in the device job tables (read by the N x N kernels), so a new tau
    // does not invalidate captured graphs
    if (taus) {
        for (auto &G : b->groups) {
            bool changed = false;
            for (int li = 0; li < G.ninst; ++li) {
                const double t = taus[G.members[li]];
                if (G.h_njob[li].tau != t) changed = true;
                G.h_njob[li].tau = t;
                b->inst[G.members[li]].tau = t;
            }
            if (changed)
                BHIP(b, hipMemcpyAsync(G.njob, G.h_njob.data(), sizeof(NnJob) * G.ninst,
                                       hipMemcpyHostToDevice, st));
        }
    }
    const int init_err[2] = {0, INT_MAX};
    BHIP(b, hipMemcpyAsync(b->err_dev, init_err, sizeof init_err, hipMemcpyHostToDevice, st));
    for (auto &G : b->groups) BHIP(b, hipMemsetAsync(G.nstatus, 0, sizeof(int) * G.ninst, st));
    BHIP(b, hipStreamSynchronize(st));
    for (int step = 0; step < nsteps; ++step) {
        const int par = b->cur;
        if (use_graph) {
            if (!b->gvalid[par]) {
                hipGraph_t graph = nullptr;
                BHIP(b, hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
                qo_status s = batch_step_enqueue(b, par);
                hipError_t ec = hipStreamEndCapture(st, &graph);
                if (s != QO_OK) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return s;
                }
                if (ec != hipSuccess)
                    return bfail(b, QO_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(ec));
                if (b->gexec[par]) {
                    (void)hipGraphExecDestroy(b->gexec[par]);
                    b->gexec[par] = nullptr;
                }
                hipError_t ei = hipGraphInstantiate(&b->gexec[par], graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (ei != hipSuccess)
                    return bfail(b, QO_ERR_DEVICE, "graph instantiation failed: %s",
                                 hipGetErrorString(ei));
                b->gvalid[par] = true;
            }
            BHIP(b, hipGraphLaunch(b->gexec[par], st));
        } else {
            BQO(batch_step_enqueue(b, par));
        }
        b->cur ^= 1;
        for (auto &I : b->inst) I.nstep += 1;
        const bool last = step == nsteps - 1;
        if (!stats && !last) continue;
        // statistics and error checks of this step
        int herr[2];
        BHIP(b, hipMemcpyAsync(herr, b->err_dev, sizeof herr, hipMemcpyDeviceToHost, st));
        std::vector<std::vector<double>> hen(b->groups.size()), hsc(b->groups.size());
        // per column and solve: iterations (FP32 ones summed over the rounds in mixed
        // precision), and in mixed precision the per-round maximum and the rounds used
        std::vector<std::vector<int>> hst(b->groups.size()), hit0(b->groups.size()),
            hit1(b->groups.size()), hrs0(b->groups.size()), hrs1(b->groups.size()),
            hro0(b->groups.size()), hro1(b->groups.size());
        for (size_t k = 0; k < b->groups.size(); ++k) {
            auto &G = b->groups[k];
            hen[k].resize(2 * G.ninst);
            hsc[k].resize(3 * G.ninst);
            hst[k].resize(G.ninst);
            hit0[k].resize(G.C);
            hit1[k].resize(G.C);
            BHIP(b, hipMemcpyAsync(hen[k].data(), G.energy, sizeof(double) * 2 * G.ninst,
                                   hipMemcpyDeviceToHost, st));
            BHIP(b, hipMemcpyAsync(hsc[k].data(), G.scal, sizeof(double) * 3 * G.ninst,
                                   hipMemcpyDeviceToHost, st));
            BHIP(b, hipMemcpyAsync(hst[k].data(), G.nstatus, sizeof(int) * G.ninst,
                                   hipMemcpyDeviceToHost, st));
            BHIP(b, hipMemcpyAsync(hit0[k].data(), G.mixed ? G.itot[0] : G.its[0],
                                   sizeof(int) * G.C, hipMemcpyDeviceToHost, st));
            BHIP(b, hipMemcpyAsync(hit1[k].data(), G.mixed ? G.itot[1] : G.its[1],
                                   sizeof(int) * G.C, hipMemcpyDeviceToHost, st));
            if (G.mixed) {
                for (auto *v : {&hro0[k], &hro1[k]}) v->resize(G.C);
                for (auto *v : {&hrs0[k], &hrs1[k]}) v->resize(2 * kMaxRounds);
                BHIP(b, hipMemcpyAsync(hrs0[k].data(), G.rstat[0], sizeof(int) * 2 * kMaxRounds,
                                       hipMemcpyDeviceToHost, st));
                BHIP(b, hipMemcpyAsync(hrs1[k].data(), G.rstat[1], sizeof(int) * 2 * kMaxRounds,
                                       hipMemcpyDeviceToHost, st));
                BHIP(b, hipMemcpyAsync(hro0[k].data(), G.irounds[0], sizeof(int) * G.C,
                                       hipMemcpyDeviceToHost, st));
                BHIP(b, hipMemcpyAsync(hro1[k].data(), G.irounds[1], sizeof(int) * G.C,
                                       hipMemcpyDeviceToHost, st));
            }
        }
        BHIP(b, hipStreamSynchronize(st));
        // PCG failures first: an unconverged solve can also spoil the N x N algebra
        if (herr[0]) {
            const qo_status s = herr[0] == 6 ? QO_ERR_PCG_NOCONV
                                : herr[0] == 5 ? QO_ERR_NOT_SPD : QO_ERR_NONFINITE;
            // the fixed counts were too small for this step: the next steps start again
            // from pcg_maxit
            if (s == QO_ERR_PCG_NOCONV)
                for (int k = 0; k < (int)b->groups.size(); ++k) reset_counts(b, k);
            return bfail(b, s, "PCG error code %d (first column %d of its group)", herr[0],
                         herr[1]);
        }
        for (size_t k = 0; k < b->groups.size(); ++k) {
            auto &G = b->groups[k];
            for (int li = 0; li < G.ninst; ++li)
                if (hst[k][li]) {
                    const int i = G.members[li];
                    return bfail(b, hst[k][li] == 7 ? QO_ERR_NONFINITE : QO_ERR_NOT_SPD,
                                 "instance %d: N x N predictor solve failed (code %d)", i,
                                 hst[k][li]);
                }
        }
        // fixed iteration count for the next steps: the counts just observed with a margin
        // of 50% + 4 (warm-started counts change slowly), at most pcg_maxit.  The count
        // in use is kept while it still leaves a margin of max(2, 25%) over the observed
        // counts and exceeds the target by no more than max(4, 25%), so that small
        // fluctuations do not invalidate the captured graphs.
        for (size_t k = 0; k < b->groups.size(); ++k) {
            auto &G = b->groups[k];
            if (!G.mixed) {
                int m = 0;
                for (int c = 0; c < G.C; ++c) m = std::max(m, std::max(hit0[k][c], hit1[k][c]));
                const int want = std::min(G.kmax, m + std::max(4, m / 2));
                const bool keep = G.kuse >= std::min(G.kmax, m + std::max(2, m / 4)) &&
                                  G.kuse <= want + std::max(4, want / 4);
                if (!keep && want != G.kuse) {
                    G.kuse = want;
                    b->gvalid[0] = b->gvalid[1] = false;
                }
            } else {
                // rounds: the most any column used plus one; iterations of a used round r:
                // its largest count plus max(2, 25%) (a column cut short continues in the
                // next round, so the margin only saves rounds), kept while within 2 of
                // that; rounds not used get the last used round's count
                bool changed = false;
                int mr = 0;
                for (int r = 0; r < G.ruse; ++r)
                    if (hrs0[k][2 * r + 1] > 0 || hrs1[k][2 * r + 1] > 0) mr = r + 1;
                const int rw = std::min(kMaxRounds, mr + 1);
                if (G.ruse < rw || G.ruse > rw + 1) {
                    G.ruse = rw;
                    changed = true;
                }
                for (int r = 0; r < kMaxRounds; ++r) {
                    int want;
                    if (r < mr) {
                        const int m = std::max(hrs0[k][2 * r], hrs1[k][2 * r]);
                        want = std::min(G.kmax, m + std::max(2, m / 4));
                        if (G.kr[r] >= std::min(G.kmax, m + 1) && G.kr[r] <= want + 2) continue;
                    } else {
                        want = mr > 0 ? G.kr[mr - 1] : G.kmax;
                    }
                    if (G.kr[r] != want) {
                        G.kr[r] = want;
                        if (r < G.ruse) changed = true;
                    }
                }
                if (changed) b->gvalid[0] = b->gvalid[1] = false;
            }
        }
        for (size_t k = 0; k < b->groups.size(); ++k) {
            auto &G = b->groups[k];
            for (int li = 0; li < G.ninst; ++li) {
                auto &I = b->inst[G.members[li]];
                const double Es = hen[k][2 * li], trS = hen[k][2 * li + 1];
                if (stats) {
                    qo_step_stats &o = stats[G.members[li]];
                    memset(&o, 0, sizeof o);
                    o.energy_shifted = Es;
                    o.energy = Es - 0.5 * b->cfg[G.members[li]].sigma * trS;
                    const double g2 = hsc[k][3 * li];
                    o.grad_norm = g2 > 0.0 ? std::sqrt(g2) : 0.0;
                    o.orth_err_fro = hsc[k][3 * li + 1];
                    o.orth_err_next = hsc[k][3 * li + 2];
                    int m0 = 0, m1 = 0;
                    for (int c = I.col0; c < I.col0 + I.N; ++c) {
                        m0 = std::max(m0, hit0[k][c]);
                        m1 = std::max(m1, hit1[k][c]);
                    }
                    o.pcg_iters[0] = m0;
                    o.pcg_iters[1] = m1;
                    o.refine_rounds[0] = o.refine_rounds[1] = 1;
                    if (G.mixed) {
                        int r0 = 0, r1 = 0;
                        for (int c = I.col0; c < I.col0 + I.N; ++c) {
                            r0 = std::max(r0, hro0[k][c]);
                            r1 = std::max(r1, hro1[k][c]);
                        }
                        o.refine_rounds[0] = r0;
                        o.refine_rounds[1] = r1;
                    }
                    o.energy_rose = (I.have_Es && Es > I.last_Es) ? 1 : 0;
                    o.step_index = (int)I.nstep;
                }
                I.have_Es = true;
                I.last_Es = Es;
            }
        }
    }
    return QO_OK;
}

}  // extern "C"
