// Tall-skinny block updates of the scheme of Sec. 4.1:
//   predictor   U_hat = U X + P Y          (P = G U_n)
//   warm start  x0    = P (X + C Y)        for the solve G U_hat
//   corrector   U_{n+1} = U_hat + Q (-tau O)   (Q = G U_hat, O = <U_hat,U_hat> - I)
// as one FP64 MFMA kernel Out = C0 + A Xs + B Ys (Ng x n), with an FP32-arithmetic twin
// for the mixed-precision path.
//
// Computed transposed, Out^T = Xs^T A^T + Ys^T B^T, so that the MFMA output
// rows run along the grid: lane l of a 16x16 block owns grid row m0 + l%16 of
// four output columns, and each store instruction writes 16 consecutive grid
// values per column.  The small operand is passed row-major (Xr[k*n + i] =
// Xs[k][i]) so that its loads are contiguous too.  One wavefront computes a
// 64 (grid rows) x 64 (columns) tile.
#include "qo_device.h"

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
                                            int n, long m0, int c0) {
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
    if (A) pass(A, Xr);
    if (B) pass(B, Yr);
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

// The same tile in FP32 arithmetic: operands rounded from FP64 to FP32 as they enter the
// MFMA (v_mfma_f32_16x16x4f32, twice the FP64 rate), FP32 accumulation, and C0 added in FP64
// when the tile is stored.  The prefetch keeps FP64 values, converted at their use, so
// that no conversion waits for a load still in flight.  Used by the mixed-precision path,
// whose Gram matrices are BF16: an FP32 block update (relative error ~1e-7 per entry, like
// the FP32 PCG) is well inside what that path tolerates.
__device__ __forceinline__ void tsgemm32_tile(double *__restrict__ Out, long ldo,
                                              const double *__restrict__ C0,
                                              const double *__restrict__ A,
                                              const double *__restrict__ Xr,
                                              const double *__restrict__ B,
                                              const double *__restrict__ Yr, long ld, long ng,
                                              int n, long m0, int c0, __bf16 *__restrict__ Zb) {
    const int lane = threadIdx.x;
    const int lr = lane & 15, lg = lane >> 4;

    v4f acc[4][4];  // [column block j][row block i]
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[j][i] = v4f{0.f, 0.f, 0.f, 0.f};

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
        // twice the MFMA rate of FP64: chunks of 16 k-values keep as much time between a
        // chunk's loads and their use as the FP64 kernel's chunks of 8
        constexpr int KSC = 2 * QO_TSG_KSC, KC = 4 * KSC;
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
                        acc[j][i] = __builtin_amdgcn_mfma_f32_16x16x4f32(
                            (float)sa[ks][j], (float)tb[ks][i], acc[j][i], 0, 0, 0);
        };
        const int nfull = n & ~(KC - 1);
        double sa0[KSC][4], tb0[KSC][4], sa1[KSC][4], tb1[KSC][4];
        if (nfull > 0) {
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
    if (A) pass(A, Xr);
    if (B) pass(B, Yr);
    // FP32 16x16 accumulator layout: value v of lane l is row 4 (l/16) + v, column l%16,
    // so acc[j][i][v] = Out^T[c0 + 16j + 4lg + v][m0 + 16i + lr]
    // C0 for every value of the tile first (clamped, unconditional loads issued together),
    // then the sums are stored
    double c0v[4][4][4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = c0 + 16 * j + 4 * lg + v;
                c0v[j][i][v] = C0 ? (double)gptr(C0)[(long)(c < n ? c : n - 1) * ld + moff[i]]
                                  : 0.0;
            }
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const long m = m0 + 16 * i + lr;
            if (m >= ng) continue;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int c = c0 + 16 * j + 4 * lg + v;
                if (c < n) {
                    const double o = c0v[j][i][v] + (double)acc[j][i][v];
                    Out[(long)c * ldo + m] = o;
                    if (Zb) Zb[(long)c * ldo + m] = dev::f64_to_bf16_rne(o);
                }
            }
        }
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_tsgemm32(
    double *__restrict__ Out, long ldo, const double *__restrict__ C0,
    const double *__restrict__ A, const double *__restrict__ Xr, const double *__restrict__ B,
    const double *__restrict__ Yr, long ld, long ng, int n, __bf16 *__restrict__ Zb) {
    const int L = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int rt = L / gridDim.y;
    tsgemm32_tile(Out, ldo, C0, A, Xr, B, Yr, ld, ng, n, (long)rt * 64,
                  (L - rt * gridDim.y) * 64, Zb);
}

__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(2))) void k_tsgemm(double *__restrict__ Out, long ldo,
                                               const double *__restrict__ C0,
                                               const double *__restrict__ A,
                                               const double *__restrict__ Xr,
                                               const double *__restrict__ B,
                                               const double *__restrict__ Yr, long ld, long ng,
                                               int n) {
    // column tiles of one row panel on one XCD: they read the same rows of A and B
    const int L = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int rt = L / gridDim.y;
    tsgemm_tile(Out, ldo, C0, A, Xr, B, Yr, ld, ng, n, (long)rt * 64, (L - rt * gridDim.y) * 64);
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

hipError_t launch_tsgemm(double *Out, long ldo, const double *C0, const double *A,
                         const double *Xr, const double *B, const double *Yr, long ld, long ng,
                         int n, hipStream_t st, bool fp32, __bf16 *Zb) {
    if (n <= 0 || ng <= 0) return hipSuccess;
    // each big operand needs its small operand (and the reverse); a BF16 copy only from the
    // FP32 kernel
    if ((A == nullptr) != (Xr == nullptr) || (B == nullptr) != (Yr == nullptr) || !Out ||
        (Zb && !fp32))
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)((ng + 63) / 64), (unsigned)((n + 63) / 64));
    if (fp32)
        hipLaunchKernelGGL(k_tsgemm32, grid, dim3(64), 0, st, Out, ldo, C0, A, Xr, B, Yr, ld, ng,
                           n, Zb);
    else
        hipLaunchKernelGGL(k_tsgemm, grid, dim3(64), 0, st, Out, ldo, C0, A, Xr, B, Yr, ld, ng, n);
    return hipGetLastError();
}

}  // namespace qo
