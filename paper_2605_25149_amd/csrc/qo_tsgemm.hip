// Tall-skinny block updates of the scheme of Sec. 4.1:
//   predictor   U_hat = U X + P Y          (P = G U_n)
//   warm start  x0    = P (X + C Y)        for the solve G U_hat
//   corrector   U_{n+1} = U_hat + Q (-tau O)   (Q = G U_hat, O = <U_hat,U_hat> - I)
// as one FP64 MFMA kernel Out = C0 + A Xs + B Ys (Ng x n).
//
// Computed transposed, Out^T = Xs^T A^T + Ys^T B^T, so that the MFMA output
// rows run along the grid: lane l of a 16x16 block owns grid row m0 + l%16 of
// four output columns, and each store instruction writes 16 consecutive grid
// values per column.  The small operand is passed row-major (Xr[k*n + i] =
// Xs[k][i]) so that its loads are contiguous too.  One wavefront computes a
// 64 (grid rows) x 64 (columns) tile.
#include "qo_internal.h"

namespace qo {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

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

    // One K range over [A | B] (length n, or 2n with B), in chunks of 16 k-values
    // (4 MFMA k-steps); the next chunk's loads are issued before the current chunk's
    // MFMAs, so the memory latency hides behind 64 MFMAs.
    // Operand pairs present: (A, Xr) and/or (B, Yr); either may be absent.  The K
    // range covers the present ones only, so no load ever goes through a null pointer.
    const double *T0 = A ? A : B, *S0 = A ? Xr : Yr;
    const double *T1 = A ? B : nullptr, *S1 = A ? Yr : nullptr;
    const int ktot = (T0 ? n : 0) + (T1 ? n : 0);
    auto load_chunk = [&](int kc, double (&sa)[4][4], double (&tb)[4][4]) {
#pragma unroll
        for (int ks = 0; ks < 4; ++ks) {
            const int kg = kc + 4 * ks + lg;
            const bool second = kg >= n;  // only reachable when T1 is present (ktot = 2n)
            const int k = second ? kg - n : kg;
            const double *T = second ? T1 : T0;
            const double *S = second ? S1 : S0;
            const bool kin = kg < ktot;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = c0 + 16 * j + lr;
                sa[ks][j] = (kin && c < n) ? S[(long)k * n + c] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long m = m0 + 16 * i + lr;
                tb[ks][i] = (kin && m < ng) ? T[(long)k * ld + m] : 0.0;
            }
        }
    };
    auto mma_chunk = [&](const double (&sa)[4][4], const double (&tb)[4][4]) {
#pragma unroll
        for (int ks = 0; ks < 4; ++ks)
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    acc[j][i] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[ks][j], tb[ks][i],
                                                                    acc[j][i], 0, 0, 0);
    };
    double sa0[4][4], tb0[4][4], sa1[4][4], tb1[4][4];
    load_chunk(0, sa0, tb0);
    for (int kc = 0; kc < ktot; kc += 32) {
        if (kc + 16 < ktot) load_chunk(kc + 16, sa1, tb1);
        mma_chunk(sa0, tb0);
        if (kc + 16 >= ktot) break;
        if (kc + 32 < ktot) load_chunk(kc + 32, sa0, tb0);
        mma_chunk(sa1, tb1);
    }
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

__global__ __launch_bounds__(64) void k_tsgemm(double *__restrict__ Out, long ldo,
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
                         int n, hipStream_t st) {
    if (n <= 0 || ng <= 0) return hipSuccess;
    // each big operand needs its small operand (and the reverse)
    if ((A == nullptr) != (Xr == nullptr) || (B == nullptr) != (Yr == nullptr) || !Out)
        return hipErrorInvalidValue;
    const dim3 grid((unsigned)((ng + 63) / 64), (unsigned)((n + 63) / 64));
    hipLaunchKernelGGL(k_tsgemm, grid, dim3(64), 0, st, Out, ldo, C0, A, Xr, B, Yr, ld, ng, n);
    return hipGetLastError();
}

}  // namespace qo
