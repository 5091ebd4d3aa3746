// Device helpers shared by the stencil-family kernels: deterministic block
// reductions (wavefront shuffles, then a fixed-order sum over the waves), the
// per-column reduction of partial sums, and the FP64 -> BF16 rounding of the
// mixed-precision Gram operands.
#pragma once
#include "qo_internal.h"

namespace qo {
namespace dev {

struct Red {
    double v[4][kThreads / 64];
};

template <int NQ>
__device__ __forceinline__ void block_sums(double (&v)[NQ], Red &red) {
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int q = 0; q < NQ; ++q) red.v[q][wid] = v[q];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) s += red.v[q][w];
        v[q] = s;
    }
}

// Sum of part[c*tiles + t] over t, identical in every thread and every block.
__device__ __forceinline__ double col_sum(const double *__restrict__ part, int c, int tiles,
                                          Red &red) {
    double s[1] = {0.0};
    for (int t = threadIdx.x; t < tiles; t += kThreads) s[0] += part[(long)c * tiles + t];
    block_sums<1>(s, red);
    return s[0];
}

// Round an FP64 value to bfloat16, nearest-even on the 45 dropped mantissa bits (one
// rounding, no FP32 intermediate).  Magnitudes below the FP32 normal range flush to signed
// zero; beyond it saturate to infinity; NaN becomes the quiet NaN.  Straight-line form: the
// rounded magnitude's bits 45..59 are the exponent and the 7 kept mantissa bits, rebiased
// to BF16 with selects instead of branches.
__device__ __forceinline__ __bf16 f64_to_bf16_rne(double d) {
    const unsigned long long b = __double_as_longlong(d);
    const unsigned long long mag =
        (b & 0x7fffffffffffffffull) + 0xfffffffffffull + ((b >> 45) & 1ull);
    int v = (int)(unsigned int)(mag >> 45) - ((1023 - 127) << 7);
    v = v < 0x80 ? 0 : v;
    v = min(v, 0x7f80);
    v = __builtin_isnan(d) ? 0x7fc0 : v;
    const unsigned int s16 = (unsigned int)(b >> 48) & 0x8000u;
    return __builtin_bit_cast(__bf16, (unsigned short)(s16 | (unsigned int)v));
}

}  // namespace dev
}  // namespace qo
