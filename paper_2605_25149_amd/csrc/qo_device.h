// Device helpers shared by the stencil-family kernels: deterministic block
// reductions (wavefront shuffles, then a fixed-order sum over the waves) and
// the per-column reduction of partial sums.
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


}  // namespace dev
}  // namespace qo
