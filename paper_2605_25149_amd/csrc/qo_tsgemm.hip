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

__global__ __launch_bounds__(64) void k_tsgemm(double *__restrict__ Out, long ldo,
                                               const double *__restrict__ C0,
                                               const double *__restrict__ A,
                                               const double *__restrict__ Xr,
                                               const double *__restrict__ B,
                                               const double *__restrict__ Yr, long ld, long ng,
                                               int n) {
    const int lane = threadIdx.x;
    const int lr = lane & 15, lg = lane >> 4;
    // column tiles of one row panel on one XCD: they read the same rows of A and B
    const int L = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int rt = L / gridDim.y;
    const long m0 = (long)rt * 64;
    const int c0 = (L - rt * gridDim.y) * 64;

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

    for (int pass = 0; pass < 2; ++pass) {
        const double *T = pass == 0 ? A : B;
        const double *S = pass == 0 ? Xr : Yr;
        if (!T) continue;
        for (int k0 = 0; k0 < n; k0 += 4) {
            const int k = k0 + lg;
            double sa[4], tb[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int c = c0 + 16 * j + lr;
                sa[j] = (k < n && c < n) ? S[(long)k * n + c] : 0.0;
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const long m = m0 + 16 * i + lr;
                tb[i] = (k < n && m < ng) ? T[(long)k * ld + m] : 0.0;
            }
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    acc[j][i] = __builtin_amdgcn_mfma_f64_16x16x4f64(sa[j], tb[i], acc[j][i], 0,
                                                                    0, 0);
        }
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

}  // namespace

hipError_t launch_tsgemm(double *Out, long ldo, const double *C0, const double *A,
                         const double *Xr, const double *B, const double *Yr, long ld, long ng,
                         int n, hipStream_t st) {
    if (n <= 0 || ng <= 0) return hipSuccess;
    const dim3 grid((unsigned)((ng + 63) / 64), (unsigned)((n + 63) / 64));
    hipLaunchKernelGGL(k_tsgemm, grid, dim3(64), 0, st, Out, ldo, C0, A, Xr, B, Yr, ld, ng, n);
    return hipGetLastError();
}

}  // namespace qo
