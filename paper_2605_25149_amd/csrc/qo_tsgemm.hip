// Tall-skinny block updates of the scheme of Sec. 4.1:
//   predictor   U_hat = U X + P Y          (P = G U_n)
//   warm start  x0    = P (X + C Y)        for the solve G U_hat
//   corrector   U_{n+1} = U_hat + Q (-tau O)   (Q = G U_hat, O = <U_hat,U_hat> - I)
// as one FP64 MFMA kernel Out = C0 + A Xs + B Ys (Ng x n), with an FP32-accurate twin on
// BF16 MFMA (three-part operand split) for the mixed-precision path.
//
// Computed transposed, Out^T = Xs^T A^T + Ys^T B^T, so that the MFMA output
// rows run along the grid: lane l of a 16x16 block owns grid row m0 + l%16 of
// four output columns, and each store instruction writes 16 consecutive grid
// values per column.  The small operand is passed row-major (Xr[k*n + i] =
// Xs[k][i]) so that its loads are contiguous too.  One wavefront computes a
// 64 (grid rows) x 64 (columns) tile.
#include "qo_device.h"

#include <algorithm>

#ifndef QO_TSG_KSC
#define QO_TSG_KSC 2
#endif

namespace qo {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// Global-address-space view: the batch kernel reads its operand pointers from a job
// table, and generic loads through them would make the compiler wait for every load in
// flight (they count on the LDS/scalar counter too) before the MFMAs.
typedef const double __attribute__((address_space(1))) gdouble;
__device__ __forceinline__ gdouble *gptr(const double *p) { return (gdouble *)p; }

// One 64 (grid rows from m0) x 64 (columns from c0) tile of Out, one wavefront.
__device__ __forceinline__ void tsgemm_tile(double *__restrict__ Out, long ldo,
                                            const double *__restrict__ C0,
                                            const double *__restrict__ A,
                                            const double *__restrict__ Xr,
                                            const double *__restrict__ B,
                                            const double *__restrict__ Yr, long ld, long ng,
                                            int n, long m0, int c0, bool b_first = false) {
    const int lane = threadIdx.x;
    const int lr = lane & 15, lg = lane >> 4;

    v4d acc[4][4];  // [column block j][row block i]
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const long m = m0 + 16 * i + lr;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = c0 + 16 * j + lg + 4 * v;
                acc[j][i][v] = (C0 && m < ng && c < n) ? C0[(long)c * ld + m] : 0.0;
            }
        }

    // One pipelined pass per operand pair (A, Xr) and (B, Yr), either of which may be
    // absent, in chunks of 16 k-values (4 MFMA k-steps): the next chunk's loads are issued
    // before the current chunk's 64 MFMAs.  The loads are unconditional, with row and
    // column indices clamped into the operands: a product of a clamped row m >= ng or
    // column c >= n only reaches an output that is never stored.  (Guarded loads become
    // branches, and the compiler then waits for every load in flight before the MFMAs.)
    // The scheduling barriers keep the prefetch ahead of the MFMAs it overlaps.  k beyond
    // n occurs only in a tail chunk when n is not a multiple of 16; its loads are zeroed.
    long moff[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const long m = m0 + 16 * i + lr;
        moff[i] = m < ng ? m : ng - 1;
    }
    int coff[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int c = c0 + 16 * j + lr;
        coff[j] = c < n ? c : n - 1;
    }
    auto pass = [&](const double *Tp, const double *Sp) {
        constexpr int KSC = QO_TSG_KSC, KC = 4 * KSC;  // MFMA k-steps and k-values per chunk
        gdouble *__restrict__ T = gptr(Tp);
        gdouble *__restrict__ S = gptr(Sp);
        auto load_chunk = [&](int kc, double (&sa)[KSC][4], double (&tb)[KSC][4]) {
#pragma unroll
            for (int ks = 0; ks < KSC; ++ks) {
                const long k = kc + 4 * ks + lg;
#pragma unroll
                for (int j = 0; j < 4; ++j) sa[ks][j] = S[k * n + coff[j]];
#pragma unroll
                for (int i = 0; i < 4; ++i) tb[ks][i] = T[k * ld + moff[i]];
            }
        };
        auto mma_chunk = [&](const double (&sa)[KSC][4], const double (&tb)[KSC][4]) {
#pragma unroll
            for (int ks = 0; ks < KSC; ++ks)
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        acc[j][i] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[ks][j], tb[ks][i],
                                                                        acc[j][i], 0, 0, 0);
        };
        const int nfull = n & ~(KC - 1);
        double sa0[KSC][4], tb0[KSC][4], sa1[KSC][4], tb1[KSC][4];
        if (nfull > 0) {
            // past the end the prefetch re-reads the final chunk
            const int last = nfull - KC;
            const int npairs = nfull / (2 * KC);
            load_chunk(0, sa0, tb0);
            for (int p = 0; p < npairs; ++p) {
                const int kc = p * 2 * KC;
                load_chunk(kc + KC, sa1, tb1);
                __builtin_amdgcn_sched_barrier(0);
                mma_chunk(sa0, tb0);
                __builtin_amdgcn_sched_barrier(0);
                load_chunk(min(kc + 2 * KC, last), sa0, tb0);
                __builtin_amdgcn_sched_barrier(0);
                mma_chunk(sa1, tb1);
                __builtin_amdgcn_sched_barrier(0);
            }
            if (nfull & KC) mma_chunk(sa0, tb0);
        }
        if (nfull < n) {
#pragma unroll
            for (int ks = 0; ks < KSC; ++ks) {
                const int k = nfull + 4 * ks + lg;
                const bool kin = k < n;
                const long kk = kin ? k : n - 1;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const double v = S[kk * n + coff[j]];
                    sa0[ks][j] = kin ? v : 0.0;
                }
#pragma unroll
                for (int i = 0; i < 4; ++i) tb0[ks][i] = T[kk * ld + moff[i]];
            }
            mma_chunk(sa0, tb0);
        }
    };
    // b_first: the second operand pair first (the predictor update with its warm start, whose
    // tiles of one row panel then read P at about the same time)
    if (b_first && B) pass(B, Yr);
    if (A) pass(A, Xr);
    if (!b_first && B) pass(B, Yr);
    // FP64 16x16 accumulator layout: value v of lane l is row l/16 + 4v, column l%16,
    // so acc[j][i][v] = Out^T[c0 + 16j + lg + 4v][m0 + 16i + lr]
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const long m = m0 + 16 * i + lr;
            if (m >= ng) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = c0 + 16 * j + lg + 4 * v;
                if (c < n) Out[(long)c * ldo + m] = acc[j][i][v];
            }
        }
}

// ---- FP32-accurate update on BF16 MFMA (mixed-precision path) --------------------------
//
// Every operand value is rounded to FP32 and split exactly into three BF16 parts,
// a = a1 + a2 + a3 (8 significant bits each; an FP32 significand has 24).  Of the nine
// part products, the six with a_i b_j, i + j <= 4, are accumulated (the others are below
// 2^-24 |a b|); BF16 products are exact in the FP32 accumulator, so the result carries
// FP32 input rounding and FP32 accumulation like an FP32 product, at six BF16 MFMAs
// (16 cycles each per 32 k-values) instead of eight FP32 ones (32 cycles per 4).

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef float v2f __attribute__((ext_vector_type(2)));

// f = b1 + b2 + b3 exactly, each part rounded to nearest-even from what is left
__device__ __forceinline__ void split3(float f, __bf16 &b1, __bf16 &b2, __bf16 &b3) {
    __asm__("" : "+v"(f));  // see split3_pair
    b1 = (__bf16)f;
    const float r1 = f - (float)b1;
    b2 = (__bf16)r1;
    b3 = (__bf16)(r1 - (float)b2);
}

// Two FP64 values rounded to FP32 and split, with the packed FP32 -> BF16 conversion (one
// instruction per pair and part).  The empty asm keeps the FP32 rounding a separate step:
// the compiler would otherwise fuse it with the first BF16 rounding into one double ->
// bfloat16 conversion, which needs a dozen instructions per value.
__device__ __forceinline__ void split3_pair(double x0, double x1, v2bf &h1, v2bf &h2,
                                            v2bf &h3) {
    float f0 = (float)x0, f1 = (float)x1;
    __asm__("" : "+v"(f0));
    __asm__("" : "+v"(f1));
    const v2f f = {f0, f1};
    h1 = __builtin_convertvector(f, v2bf);
    const v2f r1 = f - __builtin_convertvector(h1, v2f);
    h2 = __builtin_convertvector(r1, v2bf);
    h3 = __builtin_convertvector(r1 - __builtin_convertvector(h2, v2f), v2bf);
}

// Small operands, split, in chunks of 32 k: S[ch][p][g][c][e] = part p of the operand's
// element (k, c) with k = 32 ch + 8 g + e over the concatenated k range of the nq operands
// (operand q covers k in [q Kp, q Kp + n) of (q ? Yr : Xr), row-major n x n; zero for
// k >= n within an operand; Kp = n rounded up to 64), c < nc.  With a second output
// (Zr != nullptr, nq = 2, nc = 2n) columns n .. 2n - 1 hold its operand [0; Zr]: the first
// big operand does not enter it.  A workgroup's columns of one (chunk, part, k group) are
// contiguous 16-byte pieces.
__global__ __launch_bounds__(256) void k_split3(const double *__restrict__ Xr,
                                                const double *__restrict__ Yr,
                                                const double *__restrict__ Zr, int n, int nc,
                                                int Kp, int nq, __bf16 *__restrict__ S) {
    const long total = (long)nc * nq * Kp;  // elements per part
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        // e = ((ch * 4 + g) * nc + c) * 8 + x, part-major afterwards
        const int x = (int)(e & 7);
        const long r = e >> 3;
        const int c = (int)(r % nc);
        const long cg = r / nc;
        const int g = (int)(cg & 3);
        const int ch = (int)(cg >> 2);
        const int kk = ch * 32 + g * 8 + x;
        const int q = kk >= Kp ? 1 : 0;
        const int k = kk - q * Kp;
        const bool second = c >= n;  // only with Zr
        const double *M = second ? (q ? Zr : nullptr) : (q ? Yr : Xr);
        const float f = (k < n && M) ? (float)M[(long)k * n + (second ? c - n : c)] : 0.0f;
        __bf16 b1, b2, b3;
        split3(f, b1, b2, b3);
        const long o = (((long)ch * 3 * 4 + g) * nc + c) * 8 + x;  // part 0
        const long ps = 4L * nc * 8;                                // part stride in a chunk
        S[o] = b1;
        S[o + ps] = b2;
        S[o + 2 * ps] = b3;
    }
}

// One workgroup: 64 grid rows from m0 x up to 128 columns (wave w: the 32-column tile
// c0 = 128 blockIdx.y' + 32 w).  The big operand passes through LDS in 32-k chunks: 64 rows
// x 32 FP64 values (512-byte coalesced rows), split and stored as the MFMA B operand (8
// consecutive k of one row per 16 bytes), shared by the four waves.  The small operand's
// split parts are read by each wave straight from global memory (L2) into its A fragments:
// no wave uses another's columns, so an LDS round trip would only add LDS traffic (the
// limit of this kernel).  Big-operand chunks are loaded three chunks ahead of their
// product and staged one ahead; a wave's A fragments two ahead.  Output layout (the 16x16
// FP32 accumulator): value v of lane l is row 4 (l/16) + v, column l%16 of Out^T.
constexpr int kB3Cols = 128;  // columns per workgroup

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_tsgemm_b3(
    double *__restrict__ Out, long ldo, const double *__restrict__ C0,
    const double *__restrict__ A, const double *__restrict__ B, const v8bf *__restrict__ S,
    int Kp, int nq, long ld, long ng, int n, __bf16 *__restrict__ Zb,
    double *__restrict__ Out2, int gn) {
    __shared__ __align__(16) v8bf sb[2][3][4][64];  // [buffer][part][k group][row]
    const int tid = threadIdx.x, lane = tid & 63;
    // the wave index is wave-uniform: in a scalar register, the big operand's k (and its
    // column address) is scalar arithmetic
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane & 15, lg = lane >> 4;
    // the column groups of one row panel on one XCD: they read the same big-operand rows
    const int L = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int rt = L / gridDim.y;
    const long m0 = (long)rt * 64;
    // Column groups gn and up (only with Out2) compute the second output B Zs: columns
    // n .. 2n - 1 of the split operand, and only the second big operand's chunks.
    const int gy = L - rt * (int)gridDim.y;
    const bool second = Out2 != nullptr && gy >= gn;
    const int nc = Out2 ? 2 * n : n;                           // columns of the split operand
    const int cbase = second ? n : 0;                          // this group's first of them
    const int cwg = (second ? gy - gn : gy) * kB3Cols;         // the group's first output column
    const int c0 = cwg + 32 * w;
    const bool wact = c0 < n;
    const int cpq = Kp >> 5;  // chunks per operand
    const int nch = nq * cpq;
    // With a second output every group of a row panel starts with the second big operand's
    // chunks, so that the panel's groups read its rows at about the same time (one HBM
    // read, the rest from L2); the first output's groups then take the first operand's.
    // Chunk i of the group is (rot + i) mod nch, for i < cnt (cnt even).
    const int rot = Out2 ? cpq : 0;
    const int cnt = second ? cpq : nch;
    // big-operand staging: thread -> row (lane) of the tile; wave w holds k group w
    const long mrow = min(m0 + lane, ng - 1);
    auto gload = [&](int ch, double (&v)[8]) {
        const int q = ch >= cpq ? 1 : 0;
        const int kc = (ch - q * cpq) * 32 + 8 * w;
        const double *T = q ? B : A;
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = T[(long)min(kc + u, n - 1) * ld + mrow];
    };
    // A fragments of chunk ch: parts p of columns c0 + 16 j + lr, k group lg (16 lanes read
    // 256 contiguous bytes).  Clamped columns past n reach only outputs never stored.
    const int ca0 = cbase + min(c0 + lr, n - 1), ca1 = cbase + min(c0 + 16 + lr, n - 1);
    auto aload = [&](int ch, v8bf (&a)[2][3]) {
        const v8bf *base = S + ((long)ch * 3 * 4 + lg) * nc;
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            a[0][p] = base[(long)p * 4 * nc + ca0];
            a[1][p] = base[(long)p * 4 * nc + ca1];
        }
    };
    auto sstore = [&](int buf, const double (&v)[8]) {
        v8bf p0, p1, p2;
#pragma unroll
        for (int u = 0; u < 8; u += 2) {
            v2bf h1, h2, h3;
            split3_pair(v[u], v[u + 1], h1, h2, h3);
            p0[u] = h1[0];
            p0[u + 1] = h1[1];
            p1[u] = h2[0];
            p1[u + 1] = h2[1];
            p2[u] = h3[0];
            p2[u + 1] = h3[1];
        }
        sb[buf][0][w][lane] = p0;
        sb[buf][1][w][lane] = p1;
        sb[buf][2][w][lane] = p2;
    };
    v4f acc[2][4];  // [column block j][row block i]
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[j][i] = v4f{0.f, 0.f, 0.f, 0.f};
    auto mma = [&](int buf, const v8bf (&a)[2][3]) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const v8bf b1 = sb[buf][0][lg][16 * i + lr];
            const v8bf b2 = sb[buf][1][lg][16 * i + lr];
            const v8bf b3 = sb[buf][2][lg][16 * i + lr];
#pragma unroll
            for (int j = 0; j < 2; ++j) {
                // smallest terms first
                v4f t = acc[j][i];
                t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j][2], b1, t, 0, 0, 0);
                t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j][1], b2, t, 0, 0, 0);
                t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j][0], b3, t, 0, 0, 0);
                t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j][1], b1, t, 0, 0, 0);
                t = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j][0], b2, t, 0, 0, 0);
                acc[j][i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[j][0], b1, t, 0, 0, 0);
            }
        }
    };
    {
        // Chunk ch is multiplied from LDS buffer ch & 1 with the A fragments of register
        // set ch & 1, while the big operand of chunk ch + 1 waits staged in the other
        // buffer and the big-operand registers of one set load chunk ch + 3 (issued before
        // the product); after the product its A set loads chunk ch + 2.  nch is even (Kp
        // is a multiple of 64); loads past the end re-read the last chunk, so that every
        // load and wait is unconditional.  The loop is entered unconditionally (nch >= 2),
        // so that the prologue's loads stay where they are issued.
        double v0[8], v1[8];
        v8bf a0[2][3], a1[2][3];
        const int last = cnt - 1;
        auto chk = [&](int i) {  // actual chunk of loop position i (past the end: the last)
            const int j = rot + min(i, last);
            return j >= nch ? j - nch : j;
        };
        gload(chk(0), v0);
        aload(chk(0), a0);
        gload(chk(1), v1);
        aload(chk(1), a1);
        __builtin_amdgcn_sched_barrier(0);
        sstore(0, v0);
        gload(chk(2), v0);
        __syncthreads();
        int ch = 0;
        do {
            // v1: chunk ch + 1, v0: chunk ch + 2 (loading)
            sstore(1, v1);
            gload(chk(ch + 3), v1);
            __builtin_amdgcn_sched_barrier(0);
            mma(0, a0);
            __builtin_amdgcn_sched_barrier(0);
            aload(chk(ch + 2), a0);
            __syncthreads();
            // v0: chunk ch + 2, v1: chunk ch + 3 (loading)
            sstore(0, v0);
            gload(chk(ch + 4), v0);
            __builtin_amdgcn_sched_barrier(0);
            mma(1, a1);
            __builtin_amdgcn_sched_barrier(0);
            aload(chk(ch + 3), a1);
            __syncthreads();
            ch += 2;
        } while (ch < cnt);
    }
    if (!wact) return;
    // C0 for every value of the tile first (clamped, unconditional loads issued together),
    // then the sums are stored: acc[j][i][v] = Out^T[c0 + 16j + 4lg + v][m0 + 16i + lr]
    double c0v[2][4][4];
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = c0 + 16 * j + 4 * lg + v;
                const long m = min(m0 + 16 * i + lr, ng - 1);
                c0v[j][i][v] = C0 ? (double)gptr(C0)[(long)(c < n ? c : n - 1) * ld + m] : 0.0;
            }
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const long m = m0 + 16 * i + lr;
            if (m >= ng) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = c0 + 16 * j + 4 * lg + v;
                if (c < n) {
                    const double o = c0v[j][i][v] + (double)acc[j][i][v];
                    if (second) {
                        Out2[(long)c * ldo + m] = o;
                    } else {
                        Out[(long)c * ldo + m] = o;
                        if (Zb) Zb[bf16_rowblock_index(m, c, n)] = dev::f64_to_bf16_rne(o);
                    }
                }
            }
        }
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_tsgemm(double *__restrict__ Out, long ldo,
                                               const double *__restrict__ C0,
                                               const double *__restrict__ A,
                                               const double *__restrict__ Xr,
                                               const double *__restrict__ B,
                                               const double *__restrict__ Yr, long ld, long ng,
                                               int n, double *__restrict__ Out2,
                                               const double *__restrict__ Zr, int tn) {
    // column tiles of one row panel on one XCD: they read the same rows of A and B; tiles
    // tn and up (only with Out2) compute the second output B Zr
    const int L = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int rt = L / gridDim.y;
    const int ct = L - rt * (int)gridDim.y;
    if (Out2 && ct >= tn)
        tsgemm_tile(Out2, ldo, nullptr, nullptr, nullptr, B, Zr, ld, ng, n, (long)rt * 64,
                    (ct - tn) * 64);
    else
        tsgemm_tile(Out, ldo, C0, A, Xr, B, Yr, ld, ng, n, (long)rt * 64, ct * 64,
                    Out2 != nullptr);
}

// Grouped batches: job blockIdx.z; row tile blockIdx.x, column tile blockIdx.y.
__global__ __launch_bounds__(64) void k_tsgemm_batch(const TsJob *__restrict__ jobs, long ld,
                                                     long ng) {
    const TsJob J = jobs[blockIdx.z];
    const int c0 = blockIdx.y * 64;
    if (c0 >= J.n) return;
    tsgemm_tile(J.Out, ld, J.C0, J.A, J.Xr, J.B, J.Yr, ld, ng, J.n, (long)blockIdx.x * 64, c0);
}

}  // namespace

hipError_t launch_tsgemm_batch(const TsJob *jobs, int njobs, int max_n, long ld, long ng,
                               hipStream_t st) {
    if (njobs <= 0 || ng <= 0) return hipSuccess;
    const dim3 grid((unsigned)((ng + 63) / 64), (unsigned)((max_n + 63) / 64), (unsigned)njobs);
    hipLaunchKernelGGL(k_tsgemm_batch, grid, dim3(64), 0, st, jobs, ld, ng);
    return hipGetLastError();
}

size_t tsgemm_split_elems(int n) { return (size_t)3 * (2 * n) * 2 * ((n + 63) / 64 * 64); }

hipError_t launch_tsgemm(double *Out, long ldo, const double *C0, const double *A,
                         const double *Xr, const double *B, const double *Yr, long ld, long ng,
                         int n, hipStream_t st, bool fp32, __bf16 *Zb, __bf16 *split,
                         double *Out2, const double *Zr) {
    if (n <= 0 || ng <= 0) return hipSuccess;
    // each big operand needs its small operand (and the reverse); the FP32-accurate path
    // needs its split scratch; a BF16 copy only from that path; a second output needs both
    // big operands, its small operand and no C0
    if ((A == nullptr) != (Xr == nullptr) || (B == nullptr) != (Yr == nullptr) || !Out ||
        (Zb && !fp32) || (fp32 && !split) || ((Out2 == nullptr) != (Zr == nullptr)) ||
        (Out2 && (!A || !B || C0)))
        return hipErrorInvalidValue;
    if (fp32) {
        // the split small operands (k padded with zeros to a multiple of 64: an even number
        // of 32-k chunks), then 128-column workgroups (twice as many with a second output)
        const int Kp = (n + 63) / 64 * 64;
        const int nq = (A ? 1 : 0) + (B ? 1 : 0);
        if (nq == 0) return hipErrorInvalidValue;
        const double *X1 = A ? Xr : Yr, *X2 = A ? Yr : nullptr;
        const double *T1 = A ? A : B, *T2 = A ? B : nullptr;
        const int nc = Out2 ? 2 * n : n;
        const long items = (long)nc * nq * Kp;
        const unsigned blocks = (unsigned)std::min<long>((items + 255) / 256, 4096);
        hipLaunchKernelGGL(k_split3, dim3(blocks), dim3(256), 0, st, X1, X2, Zr, n, nc, Kp, nq,
                           split);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        const int gn = (n + kB3Cols - 1) / kB3Cols;
        const dim3 g3((unsigned)((ng + 63) / 64), (unsigned)(Out2 ? 2 * gn : gn));
        hipLaunchKernelGGL(k_tsgemm_b3, g3, dim3(256), 0, st, Out, ldo, C0, T1, T2,
                           reinterpret_cast<const v8bf *>(split), Kp, nq, ld, ng, n, Zb, Out2,
                           gn);
    } else {
        const int tn = (n + 63) / 64;
        const dim3 grid((unsigned)((ng + 63) / 64), (unsigned)(Out2 ? 2 * tn : tn));
        hipLaunchKernelGGL(k_tsgemm, grid, dim3(64), 0, st, Out, ldo, C0, A, Xr, B, Yr, ld, ng, n,
                           Out2, Zr, tn);
    }
    return hipGetLastError();
}

}  // namespace qo
