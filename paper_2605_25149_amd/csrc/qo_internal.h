// Private declarations of libqo_hip: grid descriptor, kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace qo {

// Rows [y0, y0 + ty) and planes [z0, z1) of one tile of a Grid.
struct TileExtent {
    int band, zc, y0, ty, z0, z1;
};

// Geometry of one column grid and of its band/z-chunk tiling.
//   A tile is TY consecutive y-rows (full x extent) of ZC consecutive z-planes;
//   one workgroup of 256 threads streams one tile of one column, marching in z.
struct Grid {
    int dim;
    int nx, ny, nz;      // nz = 1 in 2-D
    long ng;             // nx*ny*nz
    int TY, ZC;          // tile rows, tile planes
    int nbands, nzc;     // tiles per column = nbands*nzc
    int ppt;             // points per thread per plane: ceil(TY*nx/256) rounded up to 1,2,4,6,8
    double ihx2, ihy2, ihz2;  // 1/h_k^2 (ihz2 = 0 in 2-D)
    double kappa;
    double c0;           // 2 kappa (ihx2 + ihy2 + ihz2): stencil diagonal without V
    // Grouped batches concatenate the columns of several instances on one grid:
    // cinst[col] is a column's instance, whose per-point arrays (V + sigma,
    // 1/diag) start at instance * ng.  nullptr for a single instance.
    const int *cinst;
    __host__ __device__ int tiles() const { return nbands * nzc; }
    __host__ __device__ TileExtent extent(int tile) const {
        TileExtent e;
        e.band = tile / nzc;
        e.zc = tile - e.band * nzc;
        e.y0 = e.band * TY;
        e.ty = min(TY, ny - e.y0);
        e.z0 = e.zc * ZC;
        e.z1 = min(nz, e.z0 + ZC);
        return e;
    }
};

constexpr int kThreads = 256;

// Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2):
// dispatch index b runs on XCD b % 8.  Remap so that XCD x works through one
// contiguous range of logical indices in order; neighbouring tiles (which share
// halo rows or operand panels) then meet in the same L2.  A bijection of [0, B).
// The index maps below are host-callable so that a CPU program can check them
// (bijections, coverage, bounds) for every launch shape without a GPU.
__host__ __device__ __forceinline__ int xcd_remap(int b, int B) {
    const int x = b & 7, s = b >> 3;
    const int q = B >> 3, r = B & 7;
    return x * q + (x < r ? x : r) + s;
}

// Stencil-family launches: logical workgroup L of an ncols x tiles grid -> (column,
// tile), column-major: an XCD works through whole columns, so a column's neighbouring
// bands (whose rows are its halo) run side by side and meet in the same L2.  (Grouping a
// few columns tile-major, to share the per-point V + sigma of a tile in L2, measured 2%
// slower for the sweeps.)
__host__ __device__ __forceinline__ void stencil_tile_of(int L, int ncols, int tiles, int &col,
                                                         int &tile) {
    (void)ncols;
    col = L / tiles;
    tile = L - col * tiles;
}

// DST plane passes: logical workgroup L of an ncols x nslab grid -> (column, slab),
// column-major: consecutive workgroups of an XCD stream consecutive slabs of one column.
// (Column-fastest order, which shares the per-point V + sigma of a slab in L2, measured no
// faster for the inverse pass and 7% slower for the forward pass.)
__host__ __device__ __forceinline__ void plane_slab_of(int L, int nslab, int &col, int &slab) {
    col = L / nslab;
    slab = L - col * nslab;
}

// Row-blocked BF16 layout of a Gram operand with n columns: grid row m of column c sits
// at ((m / 32) * n + c) * 32 + m % 32, so a 32-row step of consecutive columns is
// contiguous.  Rows are padded to the block's leading dimension (a multiple of 64).
__host__ __device__ __forceinline__ long bf16_rowblock_index(long m, int c, int n) {
    return ((m >> 5) * n + c) * 32 + (m & 31);
}

// Fast-Poisson pencil pass: offset (in halves) of slowest-axis index s of in-plane
// position m (0 <= m < 64) in an m-major LDS tile with row pitch SP.  The 16-byte blocks
// of row m are permuted by XOR with (m >> 3) & 3, so rows 8 apart start in different
// banks while 8 consecutive s (s a multiple of 8) stay contiguous.
__host__ __device__ __forceinline__ int pen_off(int m, int s, int SP) {
    return m * SP + ((((s >> 3) ^ (m >> 3)) & 3) | ((s >> 3) & ~3)) * 8 + (s & 7);
}

// Floats of the pencil pass's LDS ahead of its per-column constants: the slowest-axis
// eigenvalues (NSP), then those along x and y, each padded to a multiple of 4.
__host__ __device__ constexpr int pen_mu_floats(int NSP, int nx, int ny) {
    return NSP + ((nx + 3) & ~3) + ((ny + 3) & ~3);
}

// Per-column PCG bookkeeping on the device (double-buffered by iteration parity).
struct PcgState {
    double *rho;    // [2][ncap]
    double *alpha;  // [2][ncap] (one-reduction form)
    int *active;    // [2][ncap]
    int *its;       // [ncap]
    double *bb;     // [ncap]
    double *part;   // partial sums [4][ncap * tiles]
    int *err;       // [2]: error code, first failing column
    const double *coltol;  // optional per-column relative tolerance (else the scalar tol)
};

// ---- fast-Poisson (DST-I) preconditioner (qo_dst.hip) ----
// Geometry and tables of M = kappa (-Lap_h) + vbar on the column grid.  The
// slowest axis is z in 3-D and y in 2-D; a "slab" is one z-plane (3-D) or 64
// rows (2-D); a pencil workgroup covers 64 consecutive in-slice positions.
struct DstPlan {
    int dim, nx, ny, nz;
    int ns, nf;          // slowest-axis length; points per slowest-axis slice
    int NXP, NYP, NSP;   // lengths padded to multiples of 32
    int RP, rows;        // padded / real grid rows per slab
    int nslab, npen;     // plane and pencil workgroups per column
    int rzparts;         // partial sums of r.z per column: npen pencil jobs x NSP / 16 waves
    const _Float16 *Sx, *Sy, *Ss;   // DST-I matrices, FP16, row-major, padded with zeros
    const float *mux, *muy, *mus;   // eigenvalues of the 1-D -Lap_h along x, y, slowest axis
    float kap, vbar, lmin;          // lambda = kap (mu_x + mu_y + mu_z) + vbar; lmin its minimum
    const float *cvbar, *clmin;     // per-column vbar, lmin (grouped batches), else nullptr
};

// null if the grid is supported, else the reason
const char *dst_plan_check(int dim, const int n[3]);
void dst_plan_geometry(DstPlan &p, int dim, int nx, int ny, int nz);
hipError_t launch_dst_matrix(int n, int NP, _Float16 *S, hipStream_t st);
hipError_t launch_sum(const double *v, long n, double *out, hipStream_t st);
// pcs[c] = sqrt(Ng / ||r_c||^2) (0 for a zero column)
hipError_t launch_col_scale(const double *R, long ld, long ng, int ncols, float *pcs,
                            hipStream_t st);
// pcs[c] = sqrt(Ng / ||r_c||^2) for the columns the PCG iteration k updates, else 0
hipError_t launch_pc_prep(int k, int ncols, const int *mask, PcgState s, long qs, int tiles,
                          double tol, long ng, float *pcs, hipStream_t st);
// z = M^{-1} r in three passes: forward plane (r -> t1), pencil (t1 -> t2, and the
// partials rzp[c * rzparts + i] of r.z, summed in the spectral domain), inverse plane
// (t2 -> z).
template <typename T>
hipError_t launch_dst_fwd(const DstPlan &p, const T *R, long ld, int ncols, _Float16 *t1,
                          const float *pcs, hipStream_t st);
hipError_t launch_dst_pencil(const DstPlan &p, const _Float16 *t1, _Float16 *t2, long ld,
                             int ncols, const float *pcs, double *rzp, hipStream_t st);
// z is FP32 in either precision (its values carry FP32 precision); launch_z_expand gives
// an FP64 copy.
hipError_t launch_dst_inv(const DstPlan &p, const _Float16 *t2, float *Z, long ld, int ncols,
                          const float *pcs, hipStream_t st);
// FP32 PCG with the fast-Poisson preconditioner, iteration k: rzc[c] = rho_k = r.z from the
// pencil's partials and beta[c] = rho_k / rho_{k-1} (0 at k = 0) for the preconditioned
// columns; then the inverse plane pass forms the search direction P = z + beta P_old
// itself (P = z when Pold is null), and the first sweep takes rho_k from rzc.
hipError_t launch_rho_beta(int k, int ncols, const float *pcs, const double *rzp, int rzt,
                           PcgState s, float *beta, double *rzc, hipStream_t st);
hipError_t launch_dst_inv_p(const DstPlan &p, const _Float16 *t2, const float *Pold,
                            const float *beta, float *P, long ld, int ncols, const float *pcs,
                            const float *vs, double *wzp, hipStream_t st);
// ... and, with the inverse pass's partials wzp of sum (V + sigma - vbar) z^2 (nwz per
// column), the first
// sweep's bookkeeping and gamma = p.Hp from the identities of the iteration, one block per
// column, no pass over the grid (qo_stencil.hip).
hipError_t launch_pcg_gamma(const Grid &g, int k, int ncols, double tol, const int *mask,
                            PcgState s, const double *rzc, const double *wzp, int nwz,
                            hipStream_t st);
// Z (FP64) = Z32 for the columns with pcs[c] != 0, zero elsewhere.
hipError_t launch_z_expand(const float *Z32, const float *pcs, double *Z, long ld, long ng,
                           int ncols, hipStream_t st);

// ---- stencil family (qo_stencil.hip) ----
// All take a column count `ncols`, a column stride `ld` and per-point arrays
// vs = V + sigma and dinv = 1/(c0 + vs) of the matching precision.
hipError_t launch_apply(const Grid &g, const double *vs, const double *X, double *Y, long ld,
                        int ncols, hipStream_t st);
// partial sums per (column, tile): part[0] = x.Hx, part[1] = x.x
hipError_t launch_quad(const Grid &g, const double *vs, const double *X, long ld, int ncols,
                       double *part, hipStream_t st);
// Mixed-precision residual: r = b - H x (FP64), r32 = (float) r; partials rr, bb.
// Columns with mask[c] == 0 are skipped (their partials are set to zero).
hipError_t launch_resid(const Grid &g, const double *vs, const double *B, const double *X,
                        long ld, float *R32, long ld32, int ncols, const int *mask, double *part,
                        hipStream_t st);

template <typename T>
hipError_t launch_pcg_init(const Grid &g, const T *vs, const T *dinv, const T *B, T *X, T *R,
                           long ld, int ncols, int use_x0, double *part, hipStream_t st);
template <typename T>
hipError_t launch_pcg_sweep1(const Grid &g, const T *vs, const T *dinv, const T *R,
                             const T *Pold, T *Pnew, long ld, int ncols, int k, double tol,
                             const int *mask, PcgState s, hipStream_t st,
                             const float *Z = nullptr, const double *rzp = nullptr,
                             int rzt = 0, bool p_given = false);
template <typename T>
// xzero: X is zero on entry (first iteration without an init pass; preconditioned form
// only): X = alpha p is written without reading X.
hipError_t launch_pcg_sweep2(const Grid &g, const T *vs, const T *dinv, const T *Pn, T *X, T *R,
                             long ld, int ncols, int k, PcgState s, hipStream_t st,
                             bool jac = true, bool xzero = false);

// One-reduction (Chronopoulos-Gear) PCG: delta0 = u.Hu with u = D r0 into
// part[3] (after launch_pcg_init on the same grid), then one sweep per iteration.
template <typename T>
hipError_t launch_cg_delta0(const Grid &g, const T *vs, const T *dinv, const T *R, long ld,
                            int ncols, double *part, hipStream_t st);
template <typename T>
hipError_t launch_cg_step(const Grid &g, const T *vs, const T *dinv, const T *Rin, T *Rout,
                          const T *Pold, T *Pnew, T *X, long ld, int ncols, int k, double tol,
                          const int *mask, PcgState s, const double *pin, double *pout,
                          hipStream_t st);
size_t cg_lds_bytes(const Grid &g, size_t elem);

// Sum partials per column: out[c] = sum_t part[q][c*tiles + t] for q < nq; out is [nq][ncols].
hipError_t launch_colsum(const double *part, int tiles, int ncols, int nq, long qstride,
                         double *out, hipStream_t st);

// The refinement update fused into the next residual, out of place: Xn = X + D in the
// columns with mask != 0 and its > 0 (the others: Xn = X), then the launch_resid outputs for
// Xn.  X, D, Xn, R32 share the stride ld; Xn must not overlap X.
// zb (optional): x_new rounded to BF16 into the row-blocked copy of a zn-column block.
hipError_t launch_resid_next(const Grid &g, const double *vs, const double *B, const double *X,
                             const float *D, double *Xn, long ld, float *R32, int ncols,
                             const int *mask, const int *its, double *part, hipStream_t st,
                             __bf16 *zb = nullptr, int zn = 0);
// x += d (FP64 += FP32) for columns with mask != 0 (and d = 0 when zero_d).
hipError_t launch_refine_axpy(double *X, long ld, float *D, long ld32, long ng, int ncols,
                              const int *mask, int zero_d, hipStream_t st);
// Reliable updates of the mixed-precision solve (see qo_stencil.hip).
hipError_t launch_resid_rel(const Grid &g, const double *vs, const float *dinv32, const double *B,
                            const double *X, long ld, float *R32, int ncols, const int *mask,
                            double *part, double *outer, hipStream_t st);
hipError_t launch_rel_check(const double *part, int tiles, int ncols, const int *active,
                            const double *rref, const double *bb64, double delta, double tol,
                            int *need, int *nneed, hipStream_t st);
hipError_t launch_rel_finalize(const double *outer, int tiles, int ncols, const int *need,
                               int *active, double *rref, double *bb64, double tol, int init,
                               int *nactive, int *err, hipStream_t st);
// mask[c] = (sqrt(rr[c]) > tol * sqrt(bb[c])); counts into *nactive (device int);
// coltol[c] (may be null): inner FP32 tolerance for the next round; ctol (may be null):
// per-column outer tolerances in place of tol
hipError_t launch_refine_mask(const double *sums, int ncols, double tol, double tol_in,
                              int *mask, double *coltol, int *nactive, int *err, hipStream_t st,
                              const double *ctol = nullptr);

// ---- Gram (qo_gram.hip) ----
// G (2n x 2n, col-major, ld 2n) = w * [X Y]^T [X Y]; part: workspace of
// gram_part_elems(n, nsplit) doubles.
size_t gram_part_elems(int n, int nsplit);
int gram_nsplit(long ng, int n);
// message of the calling thread's last failing handle-free call (qo_last_error(NULL))
const char *noalloc_last_error();
// G = w X^T Y (n x n, column-major), FP64 MFMA split over nsplit row chunks; part holds
// nsplit n x n partials (gram_part_elems(n, nsplit) suffices)
hipError_t launch_gram_cross_f64(const double *X, const double *Y, long ld, long ng, int n,
                                 double w, double *part, int nsplit, double *G, hipStream_t st);
hipError_t launch_gram_f64(const double *X, const double *Y, long ld, long ng, int n,
                           double w, double *part, int nsplit, double *G, hipStream_t st);
// BF16 tiles from the BF16 copies zx of X and zy of Y (ld x n each, row-blocked: element
// (r, c) at ((r / 32) n + c) 32 + r % 32; 16-byte aligned, ld a multiple of 32; rows
// ng..ld-1 zero): 256-column super-tile pairs accumulate in FP32 per K-chunk.
// pack_x / pack_y: round that block into its copy first (false where its producer has
// already written the copy).
hipError_t launch_gram_bf16(const double *X, const double *Y, long ld, long ng, int n,
                            double w, double *part, int nsplit, double *G, __bf16 *zx,
                            __bf16 *zy, bool pack_x, bool pack_y, hipStream_t st);

// Grouped batches: one Gram per job (instance), FP64 MFMA; part holds nsplit x (2n)^2
// doubles of the job; max_grid >= gram_pairs(n) * nsplit over the jobs.
struct GramJob {
    const double *X, *Y;
    double *part, *G;
    int n, nsplit;
    long kchunk;
};
int gram_pairs(int n);
long gram_kchunk(long ng, int nsplit);
hipError_t launch_gram_f64_batch(const GramJob *jobs, int njobs, int max_grid, long ld, long ng,
                                 double w, hipStream_t st);

// ---- grouped batches: N x N algebra per instance (qo_batch.hip) ----
struct NnJob {
    const double *G1, *G2;  // Grams of [U P] and [U_hat Q], 2n x 2n, leading dimension 2n
    double *pool;           // nn_pool_elems(n) doubles of coefficient matrices
    double *scal;           // [0] squared gradient norm, [1] ||O||_F, [2] ||O_{n+1}||_F
    int *status;            // 0, or the qo_status code of a failed N x N solve
    int n;
    double tau;
};
size_t nn_pool_elems(int n);
int nn_slot_xr();
int nn_slot_yr();
int nn_slot_zr();
int nn_slot_or();
hipError_t launch_nn_predict(const NnJob *jobs, int njobs, int max_n, hipStream_t st);
hipError_t launch_nn_correct(const NnJob *jobs, int njobs, hipStream_t st);
hipError_t launch_instance_energy(const double *part, long qs, int tiles, const int *coff,
                                  int ninst, double w, double *out, hipStream_t st);
// vs = V + sigma, dinv = 1/(c0 + vs); status = 7 (non-finite) or 5 (diagonal <= 0)
hipError_t launch_batch_potential(const double *V, long ng, double sigma, double c0, double *vs,
                                  double *dinv, float *vs32, float *dinv32, int *status,
                                  hipStream_t st);
// per column total += its, rounds += mask (masked-out columns: its 0); rstat[0] = the
// largest count, rstat[1] = the number of masked-in columns (one workgroup)
hipError_t launch_its_accum(const int *its, const int *mask, int n, int *total, int *rounds,
                            int *rstat, hipStream_t st);
// its[c] = 0 for c < n
hipError_t launch_fill_int(int *p, int n, int v, hipStream_t st);
// err: code 6 (PCG limit) for the first column still active
hipError_t launch_noconv_check(const int *active, int n, int *err, hipStream_t st);

// Reverse mode of the predictor algebra: (Xb, Yb) -> out = [Sb | Mb | Rb] (3 n x n blocks,
// column-major); G1 the 2n x 2n Gram of [U P]; pool nn_adjoint_pool_elems(n) doubles.
size_t nn_adjoint_pool_elems(int n);
hipError_t launch_nn_adjoint(const double *G1, int n, double tau, const double *Xb,
                             const double *Yb, double *pool, double *out, int *status,
                             hipStream_t st);

int pick_ppt(int pts);
// Tiling of the stencil family (g) and of the one-sweep PCG kernels (q) for a grid of
// dim / n[] interior points on a box with sides L[] and N columns (qo_api.hip).
void plan_grid(int dim, const int n[3], const double L[3], double kinetic, int N, Grid &g,
               Grid &q);

// ---- tall-skinny update (qo_tsgemm.hip) ----
// Out = C0 + A * Xs + B * Ys  (Ng x n, col-major), small operands given
// transposed: XsT[i*n + k] = Xs[k][i] (i.e. Xs stored row-major).  Any of C0,
// A, B may be null.  Out may alias C0 only.
// Grouped batches: Out = C0 + A Xs + B Ys per job (shared ld, ng; job column count n).
struct TsJob {
    double *Out;
    const double *C0, *A, *Xr, *B, *Yr;
    int n;
};
hipError_t launch_tsgemm_batch(const TsJob *jobs, int njobs, int max_n, long ld, long ng,
                               hipStream_t st);
// fp32: FP32-accurate arithmetic (operands rounded to FP32, FP32 accumulation, C0 added
// in FP64) on BF16 MFMA with each operand split into three BF16 parts, for the
// mixed-precision path; needs `split` (tsgemm_split_elems(n) BF16 of scratch).  There Zb
// (optional) receives Out rounded to BF16 (nearest-even from the stored FP64 value) in the
// row-blocked layout of the BF16 Gram operands (see launch_gram_bf16).  Out2 (with its
// small operand ZsT; both big operands given, no C0) receives the second product B Zs in
// the same launch, so that B is read from HBM once for both (the predictor update U_hat =
// U X + P Y with the warm start P (X + C Y) of the next solve).
size_t tsgemm_split_elems(int n);
hipError_t launch_tsgemm(double *Out, long ldo, const double *C0, const double *A,
                         const double *XsT, const double *B, const double *YsT, long ld,
                         long ng, int n, hipStream_t st, bool fp32 = false,
                         __bf16 *Zb = nullptr, __bf16 *split = nullptr,
                         double *Out2 = nullptr, const double *ZsT = nullptr);

// ---- small dense FP64 (qo_small.hip), all column-major with explicit ld ----
// C = alpha op(A) op(B) + beta C + gamma I
hipError_t nn_gemm(double *C, int ldc, const double *A, int lda, bool ta, const double *B,
                   int ldb, bool tb, int m, int n, int k, double alpha, double beta,
                   double gamma, hipStream_t st);
// C = a A + b op(B) + g I   (C may alias A or B only when op(B) = B)
hipError_t nn_axpby(double *C, int ldc, double a, const double *A, int lda, double b,
                    const double *B, int ldb, bool tb, double g, int m, int n, hipStream_t st);
// B <- A^{-1} B by Gauss-Jordan on [A | B] (A destroyed).  spd: no pivoting and
// fail when a pivot is not > 0; else partial pivoting.  status: device int,
// set to the qo_status code on failure (left untouched on success).
// n <= kGjBlockedMax with work (nn_gj_work_elems(n) doubles) and piv (n ints): blocked
// multi-workgroup form; otherwise one workgroup.
constexpr int kGjBlockedMax = 512;
hipError_t nn_gj_solve(double *A, int lda, double *B, int ldb, int n, int m, bool spd,
                       int *status, hipStream_t st, double *work = nullptr, int *piv = nullptr);
size_t nn_gj_work_elems(int n);
// Symmetric eigen-decomposition by cyclic Jacobi: A (n x n, destroyed) ->
// evals (n), V (n x n, ld n) with A = V diag V^T; unsorted.
hipError_t nn_jacobi(double *A, int lda, int n, double *evals, double *V, int ldv,
                     double *work, hipStream_t st);
// Sort evals ascending (or descending) and permute the columns of V (may be null).
hipError_t nn_sort(double *evals, double *V, int ldv, int n, bool descending, double *work,
                   hipStream_t st);
// out[0] = tr(R) - 2 tr(M M) + tr(M S M^T) (squared gradient norm),
// out[1] = ||A||_F (for A = O)
hipError_t nn_grad2(const double *S, const double *M, const double *R, int ld, int n,
                    double *MS, int ldms, double *out, hipStream_t st);
hipError_t nn_fro(const double *A, int lda, int n, double *out, hipStream_t st);
// F = V diag(1/sqrt(ev)) (columns scaled); fails (status) if ev <= 0
hipError_t nn_scale_cols_rsqrt(double *F, const double *V, int ld, const double *ev, int n,
                               int *status, hipStream_t st);
// out[i] = 1/ev[i] - sigma  or ev[i] - sigma
hipError_t nn_eval_map(double *out, const double *ev, int n, bool invert, double sigma,
                       hipStream_t st);
// energy finish: out[0] = E_sigma = 0.5 w sum_c sums[0][c], out[1] = w sum_c sums[1][c]
hipError_t nn_energy_finish(const double *sums, int ncols, double w, double *out,
                            hipStream_t st);

}  // namespace qo
