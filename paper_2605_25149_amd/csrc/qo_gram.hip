// Tall-skinny Gram matrices <Z,Z> = w Z^T Z of Z = [X | Y] (Ng x 2n): the
// inner-product matrices of Sec. 2.1 that the scheme of Sec. 4.1 needs
// (<U,U>, <U,GU>, <GU,GU> and <U_hat,U_hat>, <U_hat,GU_hat>, <GU_hat,GU_hat>).
//
// Split-K over the grid: one wavefront computes one 64x64 tile of the upper
// block triangle over one chunk of rows with MFMA, writes it as a partial,
// and a second kernel sums the partials of every entry in a fixed order and
// mirrors the upper triangle (deterministic, exactly symmetric).
//
// Operand trick: the sum over grid rows may visit the rows in any order as
// long as both operands use the same order, so lane l takes rows
// k0 + R*(l/16) + s (s < R) for its MFMA slot (l/16, l%16): each lane reads R
// consecutive doubles of one column instead of a strided gather.
//   FP64: v_mfma_f64_16x16x4f64, R = 4.
//   BF16: v_mfma_f32_16x16x32_bf16, R = 8, inputs rounded to nearest-even
//         from FP64, FP32 accumulation within a chunk, FP64 across chunks.
#include "qo_internal.h"
#include "qo_device.h"

#include <type_traits>


namespace qo {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int TM = 64;  // output tile edge per wavefront

// Global-address-space views.  Pointers read from a job table are generic; generic loads
// count on both the vector-memory and the LDS/scalar counters, and the compiler then
// waits for all of them before the MFMAs, which defeats the prefetch.
typedef const double __attribute__((address_space(1))) gdouble;
typedef double d2 __attribute__((ext_vector_type(2)));
typedef const d2 __attribute__((address_space(1))) gd2;
__device__ __forceinline__ gdouble *gptr(const double *p) { return (gdouble *)p; }

__device__ __forceinline__ const double *zcol(const double *X, const double *Y, long ld, int n,
                                              int c) {
    return c < n ? X + (long)c * ld : Y + (long)(c - n) * ld;
}

using dev::f64_to_bf16_rne;

// Decode the upper-triangular tile pair index.
__device__ __forceinline__ void tile_pair(int p, int nt, int &ti, int &tj) {
    int i = 0, rem = p;
    while (rem >= nt - i) {
        rem -= nt - i;
        ++i;
    }
    ti = i;
    tj = i + rem;
}

// One 64 x 64 tile pair of one K-chunk, FP64 MFMA (one wavefront).
// CROSS: the n x n block X^T Y alone (tile (ti, tj) = pair / ntn, pair % ntn over X
// columns x Y columns), partials n x n per split.
template <bool CROSS = false>
__device__ __forceinline__ void gram_f64_tile(const double *__restrict__ X,
                                              const double *__restrict__ Y, long ld, long ng,
                                              int n, long kchunk, double *__restrict__ part,
                                              int vec_ok, int pair, int split) {
    const int nn = CROSS ? n : 2 * n;
    const int nt = (nn + TM - 1) / TM;
    int ti, tj;
    if (CROSS) {
        ti = pair / nt;
        tj = pair - ti * nt;
    } else {
        tile_pair(pair, nt, ti, tj);
    }
    const long kb = (long)split * kchunk;
    const long ke = min(ng, kb + kchunk);
    const int lane = threadIdx.x;
    const int lr = lane & 15, lg = lane >> 4;

    // Columns beyond 2n read column 0: their products only reach entries that are never
    // stored, so the loads need no guard.  (Guarded loads become branches, and the
    // compiler then waits for every load in flight before the MFMAs.)
    gdouble *pa[4];
    gdouble *pb[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int ca = ti * TM + 16 * i + lr;
        const int cb = tj * TM + 16 * i + lr;
        if (CROSS) {
            pa[i] = gptr(X + (long)(ca < nn ? ca : 0) * ld);
            pb[i] = gptr(Y + (long)(cb < nn ? cb : 0) * ld);
        } else {
            pa[i] = gptr(ca < nn ? zcol(X, Y, ld, n, ca) : X);
            pb[i] = gptr(cb < nn ? zcol(X, Y, ld, n, cb) : X);
        }
    }
    v4d acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

    auto mma_chunk = [&](const double (&a)[4][4], const double (&b)[4][4]) {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i][s], b[j][s], acc[i][j],
                                                                    0, 0, 0);
    };
    // rows [kb, kend) in full chunks of 16, software-pipelined one chunk ahead (past the end
    // the prefetch re-reads the final chunk); the scheduling barriers keep the prefetch
    // ahead of the MFMAs it overlaps
    const long len = ke > kb ? ke - kb : 0;
    const long kend = kb + (len & ~15L);
    auto run = [&](auto vec) {
        auto load_chunk = [&](long k0, double (&a)[4][4], double (&b)[4][4]) {
            const long r0 = k0 + 4 * lg;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                if constexpr (decltype(vec)::value) {
                    gd2 *qa = (gd2 *)(pa[i] + r0);
                    gd2 *qb = (gd2 *)(pb[i] + r0);
                    const d2 a0 = qa[0], a1 = qa[1], b0 = qb[0], b1 = qb[1];
                    a[i][0] = a0.x; a[i][1] = a0.y; a[i][2] = a1.x; a[i][3] = a1.y;
                    b[i][0] = b0.x; b[i][1] = b0.y; b[i][2] = b1.x; b[i][3] = b1.y;
                } else {
#pragma unroll
                    for (int s = 0; s < 4; ++s) {
                        a[i][s] = pa[i][r0 + s];
                        b[i][s] = pb[i][r0 + s];
                    }
                }
            }
        };
        if (kend > kb) {
            double a0[4][4], b0[4][4], a1[4][4], b1[4][4];
            const long last = kend - 16;
            const long npairs = (kend - kb) >> 5;
            load_chunk(kb, a0, b0);
            for (long p = 0; p < npairs; ++p) {
                const long k0 = kb + (p << 5);
                load_chunk(k0 + 16, a1, b1);
                __builtin_amdgcn_sched_barrier(0);
                mma_chunk(a0, b0);
                __builtin_amdgcn_sched_barrier(0);
                load_chunk(min(k0 + 32, last), a0, b0);
                __builtin_amdgcn_sched_barrier(0);
                mma_chunk(a1, b1);
                __builtin_amdgcn_sched_barrier(0);
            }
            if ((kend - kb) & 16) mma_chunk(a0, b0);
        }
    };
    if (vec_ok) run(std::true_type{});
    else run(std::false_type{});
    // tail rows [kend, ke): rows past ke are zeroed (they belong to another chunk)
    if (kend < ke) {
        const long r0 = kend + 4 * lg;
        double a[4][4], b[4][4];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const bool in = r0 + s < ke;
                const long r = in ? r0 + s : ke - 1;
                const double x = pa[i][r], y = pb[i][r];
                a[i][s] = in ? x : 0.0;
                b[i][s] = in ? y : 0.0;
            }
        mma_chunk(a, b);
    }
    // FP64 16x16 accumulator layout: value v of lane l is row l/16 + 4v, column l%16
    double *out = part + (long)split * nn * nn;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = ti * TM + 16 * i + lg + 4 * v;
                const int c = tj * TM + 16 * j + lr;
                if (r < nn && c < nn) out[(long)c * nn + r] = acc[i][j][v];
            }
}

__global__ __launch_bounds__(64) void k_gram_f64(const double *__restrict__ X,
                                                 const double *__restrict__ Y, long ld, long ng,
                                                 int n, long kchunk, double *__restrict__ part,
                                                 int vec_ok) {
    // pairs of one K-chunk on one XCD: they read the same rows of the 2n columns
    const int nt = (2 * n + TM - 1) / TM;
    const int npairs = nt * (nt + 1) / 2;
    const int L = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int split = L / npairs;
    gram_f64_tile(X, Y, ld, ng, n, kchunk, part, vec_ok, L - split * npairs, split);
}

__global__ __launch_bounds__(64) void k_gram_cross_f64(const double *__restrict__ X,
                                                       const double *__restrict__ Y, long ld,
                                                       long ng, int n, long kchunk,
                                                       double *__restrict__ part, int vec_ok) {
    const int nt = (n + TM - 1) / TM;
    const int npairs = nt * nt;
    const int L = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int split = L / npairs;
    gram_f64_tile<true>(X, Y, ld, ng, n, kchunk, part, vec_ok, L - split * npairs, split);
}

// G = w sum_s part[s] (n x n, no mirroring)
__global__ void k_gram_cross_reduce(const double *__restrict__ part, int n, int nsplit, double w,
                                    double *__restrict__ G) {
    const long total = (long)n * n;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int k = 0; k < nsplit; ++k) s += part[(long)k * total + e];
        G[e] = w * s;
    }
}

// Grouped batches: job blockIdx.z, (pair, split) from blockIdx.x.
__global__ __launch_bounds__(64) void k_gram_f64_batch(const GramJob *__restrict__ jobs, long ld,
                                                       long ng, int vec_ok) {
    const GramJob J = jobs[blockIdx.z];
    const int nt = (2 * J.n + TM - 1) / TM;
    const int npairs = nt * (nt + 1) / 2;
    if ((int)blockIdx.x >= npairs * J.nsplit) return;
    const int split = blockIdx.x / npairs;
    gram_f64_tile(J.X, J.Y, ld, ng, J.n, J.kchunk, J.part, vec_ok, blockIdx.x - split * npairs,
                  split);
}

// One FP64 block (n columns, leading dimension ld) rounded to BF16 in the row-blocked
// layout of the BF16 Gram operands: element (r, c) at ((r / 32) n + c) 32 + r % 32, rows
// ng..ld-1 zero.  A 32-row step of any set of consecutive columns is then one contiguous
// run (64 bytes per column), which the Gram kernel reads with 16-byte loads.  One thread
// per 8 rows of a (row block, column): four consecutive threads read a column's 256
// contiguous bytes, and consecutive threads write consecutive 16 bytes.
__global__ __launch_bounds__(256) void k_pack_bf16(const double *__restrict__ X, long ld,
                                                   long ng, int n, __bf16 *__restrict__ Zb) {
    const long total = (ld >> 5) * n * 4;
    for (long it = (long)blockIdx.x * blockDim.x + threadIdx.x; it < total;
         it += (long)gridDim.x * blockDim.x) {
        const long bc = it >> 2;  // (row block, column)
        const int q = (int)(it & 3);
        const long rb = bc / n;
        const int c = (int)(bc - rb * n);
        const long r0 = rb * 32 + 8 * q;
        const double *src = X + (long)c * ld + r0;
        v8bf o;
        if (r0 + 8 <= ng) {
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const double2 v = reinterpret_cast<const double2 *>(src)[h];
                o[2 * h] = f64_to_bf16_rne(v.x);
                o[2 * h + 1] = f64_to_bf16_rne(v.y);
            }
        } else {
#pragma unroll
            for (int e = 0; e < 8; ++e) o[e] = f64_to_bf16_rne(r0 + e < ng ? src[e] : 0.0);
        }
        reinterpret_cast<v8bf *>(Zb)[it] = o;
    }
}

// Gram tiles of [X | Y] from the row-blocked BF16 copies ZX of X and ZY of Y, 256-column
// super-tiles: one 1024-thread workgroup per (super-tile pair, K-chunk) stages each 32-row
// step of its two super-tiles (a contiguous run per copy) in LDS (each thread copies 16
// rows of one column), and its 16 waves each run the 16
// MFMAs of one 64 x 64 tile pair from LDS.  A column is fetched by the super-tile pairs it
// belongs to (2 for 2n = 512) instead of by every tile pair (8 to 9), and two steps of
// loads are in flight beyond the one in LDS.
constexpr int kSuper = 256;  // columns per super-tile

__global__ __launch_bounds__(1024) void k_gram_bf16_super(const __bf16 *__restrict__ ZX,
                                                          const __bf16 *__restrict__ ZY, long ld,
                                                          long ng, int n, long kchunk,
                                                          double *__restrict__ part) {
    // [buffer][super-tile a/b][column][32 rows]: a column's step is 64 bytes
    __shared__ __align__(16) __bf16 sm[2][2][kSuper][32];
    const int nn = 2 * n;
    const int nst = (nn + kSuper - 1) / kSuper;
    const int nsp = nst * (nst + 1) / 2;
    const int L = xcd_remap(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
    const int split = L / nsp;
    int TI, TJ;
    tile_pair(L - split * nsp, nst, TI, TJ);
    // ZX and ZY are row-blocked (element (r, c) at ((r / 32) n + c) 32 + r % 32), rows
    // ng..ld-1 are zero and ld is a multiple of 64: whole 32-row steps
    const long kb = (long)split * kchunk;
    const long ke = min(ld, (min(ng, kb + kchunk) + 31) / 32 * 32);
    const int nsteps = ke > kb ? (int)((ke - kb) >> 5) : 0;
    const int tid = threadIdx.x;
    const bool two = TI != TJ;
    // copying: thread -> super-tile lt (the second one only off the diagonal), column lc,
    // rows 16 lh .. 16 lh + 15 of the step (two 16-byte loads)
    const int lt = tid >> 9, lc = (tid >> 1) & (kSuper - 1), lh = tid & 1;
    const bool loader = lt == 0 || two;
    typedef const v8bf __attribute__((address_space(1))) gv8bf;
    gv8bf *src;
    {
        const int c = (lt ? TJ : TI) * kSuper + lc;
        // columns past 2n read column 0: their products reach only entries never stored
        const __bf16 *col = c < n ? ZX + (long)c * 32 : c < nn ? ZY + (long)(c - n) * 32 : ZX;
        src = (gv8bf *)(col + (kb >> 5) * n * 32 + 16 * lh);
    }
    // steps past the end re-read the last one (their values are never stored)
    // one step is one row block: n 32-row column pieces further
    const long step = (long)n * 4;  // in 16-byte units
    auto gload = [&](int s, v8bf (&r)[2]) {
        const int sc = s < nsteps ? s : nsteps - 1;
        r[0] = src[step * sc];
        r[1] = src[step * sc + 1];
    };
    auto sstore = [&](int buf, const v8bf (&r)[2]) {
        if (loader) {
            *reinterpret_cast<v8bf *>(&sm[buf][lt][lc][16 * lh]) = r[0];
            *reinterpret_cast<v8bf *>(&sm[buf][lt][lc][16 * lh + 8]) = r[1];
        }
    };
    // compute: wave w -> tile pair (a, b) of the super-tile pair; on a diagonal super-tile
    // pair only a <= b is needed
    const int w = tid >> 6, lane = tid & 63, lr = lane & 15, lg = lane >> 4;
    const int a = w >> 2, b = w & 3;
    const int ti = TI * 4 + a, tj = TJ * 4 + b;
    const bool active = (two || a <= b) && ti * TM < nn && tj * TM < nn;
    const int sb = two ? 1 : 0;
    v4f acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
    auto mma = [&](int buf) {
        if (!active) return;
        v8bf fb[4];
#pragma unroll
        for (int j = 0; j < 4; ++j)
            fb[j] = *reinterpret_cast<const v8bf *>(&sm[buf][sb][b * 64 + 16 * j + lr][8 * lg]);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const v8bf fa =
                *reinterpret_cast<const v8bf *>(&sm[buf][0][a * 64 + 16 * i + lr][8 * lg]);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fa, fb[j], acc[i][j], 0, 0, 0);
        }
    };
    if (nsteps > 0) {
        // step s sits in LDS buffer s & 1 while steps s + 1 (in r0 or r1) and s + 2 load
        v8bf r0[2], r1[2];
        gload(0, r0);
        sstore(0, r0);
        gload(1, r0);
        __syncthreads();
        int s = 0;
        for (; s + 2 <= nsteps; s += 2) {
            gload(s + 2, r1);
            __builtin_amdgcn_sched_barrier(0);
            mma(0);
            __builtin_amdgcn_sched_barrier(0);
            sstore(1, r0);
            __syncthreads();
            gload(s + 3, r0);
            __builtin_amdgcn_sched_barrier(0);
            mma(1);
            __builtin_amdgcn_sched_barrier(0);
            sstore(0, r1);
            __syncthreads();
        }
        if (s < nsteps) mma(0);  // odd step count: the last step sits in buffer 0
    }
    if (!active) return;
    double *out = part + (long)split * nn * nn;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int r = ti * TM + 16 * i + 4 * lg + v;
                const int c = tj * TM + 16 * j + lr;
                if (r < nn && c < nn) out[(long)c * nn + r] = (double)acc[i][j][v];
            }
}

// G[r][c] = w * sum_s part[s][min(r,c)][max(r,c)]
__global__ void k_gram_reduce(const double *__restrict__ part, int nn, int nsplit, double w,
                              double *__restrict__ G) {
    // each partial entry (r <= c) is read once and gives both G[r][c] and G[c][r]
    const long total = (long)nn * nn;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int r = (int)(e % nn), c = (int)(e / nn);
        if (r > c) continue;
        double s = 0.0;
        for (int k = 0; k < nsplit; ++k) s += part[(long)k * total + e];
        G[e] = w * s;
        G[(long)r * nn + c] = w * s;
    }
}

__global__ void k_gram_reduce_batch(const GramJob *__restrict__ jobs, double w) {
    const GramJob J = jobs[blockIdx.z];
    const int nn = 2 * J.n;
    const long total = (long)nn * nn;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int r = (int)(e % nn), c = (int)(e / nn);
        const int a = min(r, c), b = max(r, c);
        const long o = (long)b * nn + a;
        double s = 0.0;
        for (int k = 0; k < J.nsplit; ++k) s += J.part[(long)k * total + o];
        J.G[e] = w * s;
    }
}

}  // namespace

hipError_t launch_gram_f64_batch(const GramJob *jobs, int njobs, int max_grid, long ld, long ng,
                                 double w, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gram_f64_batch, dim3((unsigned)max_grid, 1, (unsigned)njobs), dim3(64), 0,
                       st, jobs, ld, ng, 1);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_gram_reduce_batch, dim3(64, 1, (unsigned)njobs), dim3(256), 0, st, jobs,
                       w);
    return hipGetLastError();
}

int gram_pairs(int n) {
    const int nt = (2 * n + TM - 1) / TM;
    return nt * (nt + 1) / 2;
}

long gram_kchunk(long ng, int nsplit) {
    long kchunk = (ng + nsplit - 1) / nsplit;
    return (kchunk + 31) / 32 * 32;
}

int gram_nsplit(long ng, int n) {
    const int nt = (2 * n + TM - 1) / TM;
    const int npairs = nt * (nt + 1) / 2;
    long ns = 4096 / npairs;
    const long maxk = (ng + 255) / 256;
    if (ns > maxk) ns = maxk;
    // keep the partial buffer under 256 MiB
    const long per = (long)4 * n * n * 8;
    const long cap = (256L << 20) / per;
    if (ns > cap) ns = cap;
    if (ns < 1) ns = 1;
    return (int)ns;
}

size_t gram_part_elems(int n, int nsplit) { return (size_t)nsplit * 4 * n * n; }

static hipError_t gram_reduce(double *part, int nn, int nsplit, double w, double *G,
                              hipStream_t st) {
    const long total = (long)nn * nn;
    long blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_gram_reduce, dim3((unsigned)blocks), dim3(256), 0, st, part, nn, nsplit,
                       w, G);
    return hipGetLastError();
}

hipError_t launch_gram_f64(const double *X, const double *Y, long ld, long ng, int n, double w,
                           double *part, int nsplit, double *G, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int nt = (2 * n + TM - 1) / TM;
    const int npairs = nt * (nt + 1) / 2;
    long kchunk = (ng + nsplit - 1) / nsplit;
    kchunk = (kchunk + 31) / 32 * 32;
    const int vec_ok = (ld % 2 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0) &&
                       ((reinterpret_cast<uintptr_t>(Y) & 15) == 0);
    hipLaunchKernelGGL(k_gram_f64, dim3(npairs, nsplit), dim3(64), 0, st, X, Y, ld, ng, n, kchunk,
                       part, vec_ok);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return gram_reduce(part, 2 * n, nsplit, w, G, st);
}

hipError_t launch_gram_cross_f64(const double *X, const double *Y, long ld, long ng, int n,
                                 double w, double *part, int nsplit, double *G, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    const int nt = (n + TM - 1) / TM;
    long kchunk = (ng + nsplit - 1) / nsplit;
    kchunk = (kchunk + 31) / 32 * 32;
    const int vec_ok = (ld % 2 == 0) && ((reinterpret_cast<uintptr_t>(X) & 15) == 0) &&
                       ((reinterpret_cast<uintptr_t>(Y) & 15) == 0);
    hipLaunchKernelGGL(k_gram_cross_f64, dim3(nt * nt, nsplit), dim3(64), 0, st, X, Y, ld, ng, n,
                       kchunk, part, vec_ok);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long total = (long)n * n;
    long blocks = (total + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_gram_cross_reduce, dim3((unsigned)blocks), dim3(256), 0, st, part, n,
                       nsplit, w, G);
    return hipGetLastError();
}

hipError_t launch_gram_bf16(const double *X, const double *Y, long ld, long ng, int n, double w,
                            double *part, int nsplit, double *G, __bf16 *zx, __bf16 *zy,
                            bool pack_x, bool pack_y, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    // BF16 rows are read in whole 32-row steps of 16-byte loads: ld a multiple of 32,
    // 16-byte aligned operands
    if (ld % 32 != 0 || (reinterpret_cast<uintptr_t>(X) & 15) || (reinterpret_cast<uintptr_t>(Y) & 15) ||
        (reinterpret_cast<uintptr_t>(zx) & 15) || (reinterpret_cast<uintptr_t>(zy) & 15))
        return hipErrorInvalidValue;
    const long items = (long)n * (ld / 8);
    long blocks = (items + 255) / 256;
    if (blocks > 16384) blocks = 16384;
    hipError_t e;
    if (pack_x) {
        hipLaunchKernelGGL(k_pack_bf16, dim3((unsigned)blocks), dim3(256), 0, st, X, ld, ng, n, zx);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if (pack_y) {
        hipLaunchKernelGGL(k_pack_bf16, dim3((unsigned)blocks), dim3(256), 0, st, Y, ld, ng, n, zy);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    // one 1024-thread workgroup per CU: enough K-chunks for one round over 256 CUs
    const int nst = (2 * n + kSuper - 1) / kSuper;
    const int nsp = nst * (nst + 1) / 2;
    nsplit = max(1, min(nsplit, 256 / nsp));
    long kchunk = (ng + nsplit - 1) / nsplit;
    kchunk = (kchunk + 31) / 32 * 32;
    hipLaunchKernelGGL(k_gram_bf16_super, dim3(nsp, nsplit), dim3(1024), 0, st, zx, zy, ld, ng, n,
                       kchunk, part);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    return gram_reduce(part, 2 * n, nsplit, w, G, st);
}

}  // namespace qo
