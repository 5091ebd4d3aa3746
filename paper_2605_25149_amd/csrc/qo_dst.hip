// Fast-Poisson preconditioner for the inverse-operator solves of Sec. 3.1/4.1.
//
// The operator G = H_sigma^{-1} is applied by PCG (Sec. 4.1 leaves the linear
// solver open; the concluding section names a better preconditioner than the
// diagonal one as the way to cut solver cost).  Here M = kappa (-Lap_h) + vbar,
// the constant-coefficient part of H_sigma on the same Dirichlet grid with the
// potential replaced by a constant vbar >= 0, is inverted exactly:
// -Lap_h is diagonalised by the type-I discrete sine transform along each axis,
//   S_n[i][j] = sqrt(2/(n+1)) sin(pi (i+1)(j+1)/(n+1)),  S_n = S_n^T = S_n^{-1},
//   mu_n[j]   = (4/h^2) sin^2(pi (j+1) / (2(n+1)))   (eigenvalues of -d^2/dx^2),
// so M^{-1} r = S3 diag(1/lambda) S3 r with S3 = S_z (x) S_y (x) S_x and
// lambda = kappa (mu_x + mu_y + mu_z) + vbar.  The spectrum of M^{-1} H_sigma
// then no longer depends on h, and the iteration count stops growing with the
// grid.
//
// The transforms are dense contractions with the n x n matrices S (n <= 256),
// run on MFMA in FP16 with FP32 accumulation.  A preconditioner only has to be
// a fixed, nearly symmetric SPD operator: its rounding changes the iteration
// count, never the accuracy of the solve, which the FP64 (or reliable-update)
// residual decides.  Values are brought to O(1) before every FP16 rounding:
// r is scaled per column by sqrt(Ng)/||r||, the spectral division uses
// lambda_min/lambda <= 1, and the inverse transform undoes both.
//
// Three passes per application, each streaming the block once:
//   plane   (forward)  r (T) -> t1 (FP16): transform along x (and y in 3-D)
//   pencil             t1 -> t2 (FP16):    along the slowest axis, scale by
//                                          lambda_min/lambda, transform back; partial
//                                          sums of r.z = sum rhat^2 / lambda over the
//                                          spectral coefficients (Parseval: the
//                                          transforms are orthonormal)
//   plane   (inverse)  t2 -> z (FP32):     along x (and y), unscale.  z is FP32 in
//                                          the FP64 PCG too: its values carry FP32
//                                          precision (FP32 accumulation of FP16
//                                          transforms), so nothing is lost.
// r.z from the spectral coefficients differs from the product with the stored z only by
// the FP16 roundings of the transforms (about 1e-3 relative); PCG needs no more than a
// fixed, nearly symmetric preconditioner and a consistent step, and the iteration counts
// match those of the product with z.  The inverse pass then never reads r.
// "Plane" is one z-plane in 3-D and a batch of rows in 2-D; the slowest axis
// is z in 3-D and y in 2-D.
#include "qo_internal.h"
#include "qo_device.h"

#include <algorithm>
#include <climits>

#ifndef QO_PLANE_ALIAS
#define QO_PLANE_ALIAS 1
#endif

namespace qo {

namespace {

typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef unsigned v2u __attribute__((ext_vector_type(2)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef double v2d __attribute__((ext_vector_type(2)));

#ifndef QO_DST_NT
#define QO_DST_NT 1
#endif
// Global stores of the passes' outputs, non-temporal: each is read once, by the next
// pass, from HBM (a block of 96^3 x 256 values is far larger than the caches), and the
// stores then leave the cache to the inputs being read.
template <class V>
__device__ __forceinline__ void st_out(V *p, const V &v) {
#if QO_DST_NT
    __builtin_nontemporal_store(v, p);
#else
    *p = v;
#endif
}
typedef _Float16 v4h __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

constexpr int kMaxWaves = 16;

// Deterministic sum over the block (any multiple of 64 threads up to 1024).
__device__ __forceinline__ double block_sum(double v, double *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    return s;
}

// Sum of v over the 64 lanes of a wavefront, complete in lane 63, by DPP moves (no LDS
// traffic, no address registers): pairs and quads by quad permutations, rows of 16 by
// row shifts, then the row sums carried up by the row broadcasts of 15 and 31.  A lane
// a move has no source for adds 0.
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp_move(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v),
                                                                 CTRL, ROWS, 0xf, false));
}
__device__ __forceinline__ float wave_sum_lane63(float v) {
    v += dpp_move<0xb1>(v);          // quad_perm [1,0,3,2]
    v += dpp_move<0x4e>(v);          // quad_perm [2,3,0,1]
    v += dpp_move<0x114>(v);         // row_shr:4
    v += dpp_move<0x118>(v);         // row_shr:8
    v += dpp_move<0x142, 0xa>(v);    // row_bcast:15 into rows 1 and 3
    v += dpp_move<0x143, 0xc>(v);    // row_bcast:31 into rows 2 and 3
    return v;
}

template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp_move_d(double v) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, ROWS, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, ROWS, 0xf, false);
    return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double wave_sum_lane63(double v) {
    v += dpp_move_d<0xb1>(v);
    v += dpp_move_d<0x4e>(v);
    v += dpp_move_d<0x114>(v);
    v += dpp_move_d<0x118>(v);
    v += dpp_move_d<0x142, 0xa>(v);
    v += dpp_move_d<0x143, 0xc>(v);
    return v;
}

__device__ __forceinline__ v8h lds8(const _Float16 *p) {
    return *reinterpret_cast<const v8h *>(p);
}

__device__ __forceinline__ void st4h(_Float16 *p, v4f a, float f) {
    v4h h;
    h[0] = (_Float16)(a[0] * f);
    h[1] = (_Float16)(a[1] * f);
    h[2] = (_Float16)(a[2] * f);
    h[3] = (_Float16)(a[3] * f);
    *reinterpret_cast<v4h *>(p) = h;
}

__device__ __forceinline__ float mu_inplane(const DstPlan &p, int m) {
    if (p.dim == 3) {
        const int y = m / p.nx;
        return p.mux[m - y * p.nx] + p.muy[y];
    }
    return p.mux[m];
}

// S_n in FP16, zero-padded to NP x NP (row-major).
__global__ void k_dst_matrix(int n, int NP, _Float16 *__restrict__ S) {
    const double c = sqrt(2.0 / (n + 1));
    const long per = 2L * (n + 1);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < NP * NP; e += gridDim.x * blockDim.x) {
        const int i = e / NP, j = e - i * NP;
        double v = 0.0;
        if (i < n && j < n) {
            const long k = ((long)(i + 1) * (j + 1)) % per;  // exact argument reduction
            v = c * sin(M_PI * (double)k / (double)(n + 1));
        }
        S[e] = (_Float16)(float)v;
    }
}

// Sum of vs over the grid (one block), for the constant vbar of M.
__global__ void k_sum(const double *__restrict__ v, long n, double *__restrict__ out) {
    __shared__ double red[kMaxWaves];
    double s = 0.0;
    for (long i = threadIdx.x; i < n; i += blockDim.x) s += v[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) *out = s;
}

// The per-column scale is held in FP32; below ||r|| ~ 3e-39 sqrt(Ng) it is capped at
// 1e38 (the FP16 transform input r sc then falls below O(1) and loses digits to FP16
// subnormals: a weaker preconditioner, not a wrong solve).
constexpr double kMaxColScale = 1e38;

// pcs[c] = sqrt(Ng / ||r_c||^2), 0 for a zero (or non-finite) column.
__global__ __launch_bounds__(kThreads) void k_col_scale(const double *__restrict__ R, long ld,
                                                        long ng, float *__restrict__ pcs) {
    __shared__ double red[kMaxWaves];
    const int col = blockIdx.x;
    const double *r = R + (long)col * ld;
    double s = 0.0;
    for (long i = threadIdx.x; i < ng; i += blockDim.x) s += r[i] * r[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0)
        pcs[col] = (s > 0.0 && isfinite(s)) ? (float)fmin(sqrt((double)ng / s), kMaxColScale) : 0.f;
}

// Per-column scale of the forward transform for PCG iteration k, 0 for the
// columns that skip this iteration.  The activity and convergence decision is
// the one the first PCG sweep takes (same partial sums, same reduction code),
// so the preconditioner runs exactly on the columns that sweep then updates.
__global__ __launch_bounds__(kThreads) void k_pc_prep(int k, int ncols, const int *__restrict__ mask,
                                                      PcgState s, long qs, int tiles, double tol,
                                                      long ng, float *__restrict__ pcs) {
    __shared__ dev::Red red;
    const int col = blockIdx.x;
    const int prv = (k & 1) ^ 1;
    const int prev_active = (k == 0) ? (mask ? mask[col] : 1) : s.active[prv * ncols + col];
    if (!prev_active) {
        if (threadIdx.x == 0) pcs[col] = 0.f;
        return;
    }
    const double rr = dev::col_sum(s.part + qs, col, tiles, red);
    const double bb = (k == 0) ? dev::col_sum(s.part + 2 * qs, col, tiles, red) : s.bb[col];
    const double ctol = s.coltol ? s.coltol[col] : tol;
    if (threadIdx.x == 0) {
        float sc = 0.f;
        const bool fin = isfinite(rr) && isfinite(bb);
        if (fin && !(sqrt(rr) <= ctol * sqrt(bb)) && rr > 0.0)
            sc = (float)fmin(sqrt((double)ng / rr), kMaxColScale);
        pcs[col] = sc;
    }
}

// 3-D planes of more than 128 padded rows take the plane kernel's BIG form.
__host__ __device__ inline bool dst_plane_big(const DstPlan &p) { return p.dim == 3 && p.RP > 128; }

// Bytes of the plane pass's X (and, in 3-D, T^T) space in LDS, 16-byte aligned.
__host__ __device__ inline size_t dst_plane_xt_bytes(const DstPlan &p) {
    size_t b = (size_t)p.RP * (p.NXP + 8) * 2;
#if QO_PLANE_ALIAS
    if (p.dim == 3) b = b > (size_t)p.NXP * (p.NYP + 8) * 2 ? b : (size_t)p.NXP * (p.NYP + 8) * 2;
#else
    if (p.dim == 3) b += (size_t)p.NXP * (p.NYP + 8) * 2;
#endif
    return (b + 15) & ~(size_t)15;
}

// ---------------------------------------------------------------- plane pass
//
// Workgroup = one slab of one column: RP = 16 * waves padded rows of NXP
// padded x-points in LDS (FP16).  Wave w owns output rows [16w, 16w + 16).
//   GEMM1  T = X S_x     (A = X rows from LDS, B = rows of S_x: S symmetric)
//   GEMM2  Y = S_y T     (3-D only; T staged transposed in LDS)
// Forward: X = sc * r, output FP16.  Inverse: X = t2, output z = Y / (sc lmin) in FP32.
// VEC: rows are whole 16-byte groups (nx % 8 == 0): vector loads and stores throughout.
// FP32 3-D planes (NT <= 8) are held to 80 registers: 6 waves per SIMD, four 6-wave
// workgroups per CU, as many as their LDS allows.
// BIG (3-D planes of more than 128 padded rows, up to 256): up to 16 waves per workgroup,
// S_y fragments for up to 256 rows, and the inverse pass stages its FP32 output in two
// halves of the rows (the whole slab in FP32 would not fit the LDS).  SXB: the BIG form
// with the S_x copy in LDS for planes of 160 or 192 columns (where it fits).
// PF (inverse only): store the search direction P = z + beta[c] P_old (P = z when Pold is
// null) instead of z, and the partial sums of w z^2, w = V + sigma - vbar (vs holds
// V + sigma per grid point), one per wave: wzp[(c * nslab + slab) * RP / 16 + wave].
template <typename T, bool INV, int NT, bool VEC, bool PF = false, bool BIG = false,
          bool SXB = false>
__global__ __launch_bounds__(BIG ? 1024 : 512)
__attribute__((amdgpu_waves_per_eu(!BIG && sizeof(T) == 4 && NT <= 8 ? 6 : 1))) void k_dst_plane(DstPlan p, const T *__restrict__ R,
                                                   const _Float16 *__restrict__ Hin,
                                                   _Float16 *__restrict__ Hout,
                                                   float *__restrict__ Z, long ld,
                                                   const float *__restrict__ pcs,
                                                   const float *__restrict__ Pold = nullptr,
                                                   const float *__restrict__ beta = nullptr,
                                                   const float *__restrict__ vs = nullptr,
                                                   double *__restrict__ wzp = nullptr) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    int col, slab;
    plane_slab_of(L, p.nslab, col, slab);
    const float sc = pcs[col];
    if (sc == 0.f) return;  // column converged or inactive (uniform over the block)

    constexpr int NXP = 16 * NT, XP = NXP + 8;  // the launch dispatches NT = NXP / 16
    const int nx = p.nx;
    _Float16 *X = reinterpret_cast<_Float16 *>(smem);
#if QO_PLANE_ALIAS
    _Float16 *TT = X;  // T^T is written over X once every wave is past GEMM1
#else
    _Float16 *TT = X + p.RP * XP;
#endif
    const int TP = p.NYP + 8;

    const int row0 = slab * p.rows;
    const int rows = min(p.rows, (p.dim == 3 ? p.ny : p.ny - row0));
    const long base = (long)col * ld + (p.dim == 3 ? (long)slab * nx * p.ny : (long)row0 * nx);
    const int tid = threadIdx.x, nthr = blockDim.x;

    // ---- stage the slab into LDS as FP16 (zero padding).  With nthr = 4 RP threads each
    // thread owns exactly NT (forward, 4 values) or NT / 2 (inverse, 8 values) groups;
    // all their loads are issued before the first value is used (unconditional loads
    // from clamped addresses, out-of-grid groups zeroed at the conversion), so the slab
    // costs one memory round trip instead of one per group.
    constexpr int QF = NT, QI = NT / 2;
    // S_x is the B operand of every wave: up to 128 points (and with SXB) it is copied into
    // LDS once per workgroup (pitch NXP + 8, conflict-free 16-byte reads) instead of each
    // wave reading all of it through L2.  Its first four rows of loads per thread go out with the
    // slab's loads.  It sits after the X / T^T space; the inverse pass's FP32 staging may
    // later cover it (S_x is dead by then).
    constexpr bool kSxLds = NT <= 8 || (BIG && SXB);
    constexpr int kSxTotal = NXP * (NXP / 8);
    _Float16 *dstS = reinterpret_cast<_Float16 *>(smem + dst_plane_xt_bytes(p));
    v8h sxv[kSxLds ? 4 : 1];
    if constexpr (kSxLds) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int it = min(tid + u * nthr, kSxTotal - 1);
            const int r = it / (NXP / 8), c = (it - r * (NXP / 8)) * 8;
            sxv[u] = *reinterpret_cast<const v8h *>(p.Sx + r * NXP + c);
        }
    }
    T rv[INV ? 1 : QF][4];
    v8h hv[INV ? QI : 1];
    bool okq[INV ? QI : QF];
    if constexpr (!INV) {
        if constexpr (VEC) {
#pragma unroll
            for (int q = 0; q < QF; ++q) {
                const int it = tid + q * nthr;
                const int r = it / (NXP / 4);
                const int x = (it - r * (NXP / 4)) * 4;
                okq[q] = r < rows && x < nx;
                const T *src = R + (okq[q] ? base + (long)r * nx + x : base);
                if constexpr (sizeof(T) == 4) {
                    const float4 v = *reinterpret_cast<const float4 *>(src);
                    rv[q][0] = v.x; rv[q][1] = v.y; rv[q][2] = v.z; rv[q][3] = v.w;
                } else {
                    const double2 v0 = *reinterpret_cast<const double2 *>(src);
                    const double2 v1 = *reinterpret_cast<const double2 *>(src + 2);
                    rv[q][0] = v0.x; rv[q][1] = v0.y; rv[q][2] = v1.x; rv[q][3] = v1.y;
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < QF; ++q) {
                const int it = tid + q * nthr;
                const int r = it / (NXP / 4);
                const int x = (it - r * (NXP / 4)) * 4;
                okq[q] = r < rows && x < nx;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    rv[q][i] = (okq[q] && x + i < nx) ? R[base + (long)r * nx + x + i] : T(0);
            }
        }
    } else {
        if constexpr (VEC) {
#pragma unroll
            for (int q = 0; q < QI; ++q) {
                const int it = tid + q * nthr;
                const int r = it / (NXP / 8);
                const int x = (it - r * (NXP / 8)) * 8;
                okq[q] = r < rows && x < nx;
                hv[q] = *reinterpret_cast<const v8h *>(
                    Hin + (okq[q] ? base + (long)r * nx + x : base));
            }
        } else {
#pragma unroll
            for (int q = 0; q < QI; ++q) {
                const int it = tid + q * nthr;
                const int r = it / (NXP / 8);
                const int x = (it - r * (NXP / 8)) * 8;
                okq[q] = r < rows && x < nx;
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    hv[q][i] = (okq[q] && x + i < nx) ? Hin[base + (long)r * nx + x + i]
                                                      : (_Float16)0.f;
            }
        }
    }
    const _Float16 *SxL = nullptr;
    if constexpr (kSxLds) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int it = tid + u * nthr;
            if (it < kSxTotal) {
                const int r = it / (NXP / 8), c = (it - r * (NXP / 8)) * 8;
                *reinterpret_cast<v8h *>(dstS + r * XP + c) = sxv[u];
            }
        }
        for (int it = tid + 4 * nthr; it < kSxTotal; it += nthr) {  // small workgroups only
            const int r = it / (NXP / 8), c = (it - r * (NXP / 8)) * 8;
            *reinterpret_cast<v8h *>(dstS + r * XP + c) =
                *reinterpret_cast<const v8h *>(p.Sx + r * NXP + c);
        }
        SxL = dstS;  // the staging barrier below also covers this copy
    }

    if constexpr (!INV) {
#pragma unroll
        for (int q = 0; q < QF; ++q) {
            const int it = tid + q * nthr;
            const int r = it / (NXP / 4);
            const int x = (it - r * (NXP / 4)) * 4;
            v4h h;
#pragma unroll
            for (int i = 0; i < 4; ++i)
                h[i] = okq[q] ? (_Float16)((float)rv[q][i] * sc) : (_Float16)0.f;
            *reinterpret_cast<v4h *>(X + r * XP + x) = h;
        }
    } else {
#pragma unroll
        for (int q = 0; q < QI; ++q) {
            const int it = tid + q * nthr;
            const int r = it / (NXP / 8);
            const int x = (it - r * (NXP / 8)) * 8;
            v8h h;
#pragma unroll
            for (int i = 0; i < 8; ++i) h[i] = okq[q] ? hv[q][i] : (_Float16)0.f;
            *reinterpret_cast<v8h *>(X + r * XP + x) = h;
        }
    }
    __syncthreads();

    const int w = tid >> 6, lane = tid & 63, lr = lane & 15, lg = lane >> 4;
    const int KX = NXP / 32;
    // this wave's rows of S_y (the A operand of the y-transform; NYP <= 32 KYM in 3-D),
    // loaded now so that their latency overlaps the x-transform
    constexpr int KYM = BIG ? 8 : 4;
    v8h ay[KYM];
    if (p.dim == 3) {
#pragma unroll
        for (int ks = 0; ks < KYM; ++ks)
            ay[ks] = *reinterpret_cast<const v8h *>(
                p.Sy + (16 * w + lr) * p.NYP + 32 * min(ks, p.NYP / 32 - 1) + 8 * lg);
    }
    v4f acc[NT];
#pragma unroll
    for (int j = 0; j < NT; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
    for (int ks = 0; ks < KX; ++ks) {
        const v8h a = lds8(X + (16 * w + lr) * XP + 32 * ks + 8 * lg);
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            const v8h b = kSxLds ? lds8(SxL + (16 * j + lr) * XP + 32 * ks + 8 * lg)
                                 : *reinterpret_cast<const v8h *>(p.Sx + (16 * j + lr) * NXP +
                                                                  32 * ks + 8 * lg);
            acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, acc[j], 0, 0, 0);
        }
    }

    if (p.dim == 3) {
        // T^T into LDS, then Y = S_y T
#if QO_PLANE_ALIAS
        __syncthreads();
#endif
#pragma unroll
        for (int j = 0; j < NT; ++j) st4h(TT + (16 * j + lr) * TP + 16 * w + 4 * lg, acc[j], 1.f);
        __syncthreads();
        const int KY = p.NYP / 32;
#pragma unroll
        for (int j = 0; j < NT; ++j) acc[j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KYM; ++ks) {
            if (ks >= KY) break;
#pragma unroll
            for (int j = 0; j < NT; ++j) {
                const v8h b = lds8(TT + (16 * j + lr) * TP + 32 * ks + 8 * lg);
                acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ay[ks], b, acc[j], 0, 0, 0);
            }
        }
    }

    // ---- epilogue: lane values are rows 16w + 4lg + v, columns 16j + lr of the slab.
    // They are staged row-major in LDS, then each lane stores 16 contiguous bytes.
    __syncthreads();  // every wave is done reading X (and TT)
    if (!INV) {
        _Float16 *ST = X;  // RP x XP halves
#pragma unroll
        for (int j = 0; j < NT; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                ST[(16 * w + 4 * lg + v) * XP + 16 * j + lr] = (_Float16)acc[j][v];
        __syncthreads();
        const int g8 = NXP / 8;
        constexpr bool vec = VEC;
        for (int it = tid; it < rows * g8; it += nthr) {
            const int r = it / g8;
            const int x = (it - r * g8) * 8;
            if (x >= nx) continue;
            _Float16 *dst = Hout + base + (long)r * nx + x;
            const _Float16 *src = ST + r * XP + x;
            if constexpr (vec) {
                st_out(reinterpret_cast<v8h *>(dst), *reinterpret_cast<const v8h *>(src));
            } else {
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (x + i < nx) dst[i] = src[i];
            }
        }
    } else {
        const int FP = NXP + 4;
        float *SF = reinterpret_cast<float *>(smem);  // RP / NH x FP floats
        // in FP64: sc lmin exceeds the FP32 range for residuals below ~1e-37 sqrt(Ng)
        const float unscale =
            (float)(1.0 / ((double)sc * (double)(p.clmin ? p.clmin[col] : p.lmin)));
        const int g4 = NXP / 4;
        const bool first = !PF || Pold == nullptr;
        const float b = first ? 0.f : beta[col];
        float vb = 0.f;
        if constexpr (PF) vb = p.cvbar ? p.cvbar[col] : p.vbar;
        const long pbase = base - (long)col * ld;  // the slab's offset within a column
        double wz = 0.0;
        // the slab's rows are staged and stored in NH parts of RH rows (whole waves each)
        constexpr int NH = BIG ? 2 : 1;
        const int RH = p.RP / NH;
#pragma unroll
        for (int h = 0; h < NH; ++h) {
            const int r0 = h * RH;
            if (h) __syncthreads();  // every thread has stored the previous part
            if (NH == 1 || (16 * w >= r0 && 16 * w < r0 + RH)) {
#pragma unroll
                for (int j = 0; j < NT; ++j)
#pragma unroll
                    for (int v = 0; v < 4; ++v)
                        SF[(16 * w - r0 + 4 * lg + v) * FP + 16 * j + lr] = acc[j][v] * unscale;
            }
            __syncthreads();
            const int hrows = min(rows - r0, RH);
            if constexpr (PF && VEC) {
                // each thread owns at most QH groups of 4 (RH * NXP / 4 <= QH * nthr): the
                // P_old and V + sigma loads are issued together (clamped into the slab),
                // then P is stored and w z^2 summed
                constexpr int QH = QF / NH;
                float4 po[QH], v4[QH];
#pragma unroll
                for (int q = 0; q < QH; ++q) {
                    const int it = tid + q * nthr;
                    const int rl = it / g4, x = (it - rl * g4) * 4;
                    const bool ok = rl < hrows && x < nx;
                    const long off = ok ? (long)(r0 + rl) * nx + x : 0;
                    po[q] = first ? float4{0.f, 0.f, 0.f, 0.f}
                                  : *reinterpret_cast<const float4 *>(Pold + base + off);
                    v4[q] = *reinterpret_cast<const float4 *>(vs + pbase + off);
                }
#pragma unroll
                for (int q = 0; q < QH; ++q) {
                    const int it = tid + q * nthr;
                    const int rl = it / g4, x = (it - rl * g4) * 4;
                    if (rl >= hrows || x >= nx) continue;
                    const long i0 = base + (long)(r0 + rl) * nx + x;
                    const float4 z4 = *reinterpret_cast<const float4 *>(SF + rl * FP + x);
                    const v4f pv = first ? v4f{z4.x, z4.y, z4.z, z4.w}
                                         : v4f{z4.x + b * po[q].x, z4.y + b * po[q].y,
                                               z4.z + b * po[q].z, z4.w + b * po[q].w};
                    st_out(reinterpret_cast<v4f *>(Z + i0), pv);
                    wz += (double)((v4[q].x - vb) * z4.x * z4.x + (v4[q].y - vb) * z4.y * z4.y) +
                          (double)((v4[q].z - vb) * z4.z * z4.z + (v4[q].w - vb) * z4.w * z4.w);
                }
            } else {
                for (int it = tid; it < hrows * g4; it += nthr) {
                    const int rl = it / g4;
                    const int x = (it - rl * g4) * 4;
                    if (x >= nx) continue;
                    const long i0 = base + (long)(r0 + rl) * nx + x;
                    const float *src = SF + rl * FP + x;
                    if constexpr (VEC) {
                        const float4 z4 = *reinterpret_cast<const float4 *>(src);
                        st_out(reinterpret_cast<v4f *>(Z + i0), v4f{z4.x, z4.y, z4.z, z4.w});
                    } else {
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            if (x + i >= nx) break;
                            Z[i0 + i] = first ? src[i] : src[i] + b * Pold[i0 + i];
                            if constexpr (PF) {
                                const float wv = vs[pbase + (long)(r0 + rl) * nx + x + i] - vb;
                                wz += (double)(wv * src[i] * src[i]);
                            }
                        }
                    }
                }
            }
        }
        if constexpr (PF) {
            wz = wave_sum_lane63(wz);
            if ((tid & 63) == 63) wzp[((long)col * p.nslab + slab) * (nthr >> 6) + (tid >> 6)] = wz;
        }
    }
}

// ---------------------------------------------------------------- pencil pass
//
// Job = 64 consecutive in-plane positions m of one column, all ns slices along the
// slowest axis.  A workgroup of NSP / 32 waves works through jobs (persistent: the
// grid is sized to the resident workgroups); wave w owns slowest-axis rows
// [32w, 32w+32) as two blocks of 16 and keeps its rows of S_s (symmetric, so the same
// A operand serves both products) in registers across jobs.  Each B fragment read from
// LDS feeds both row blocks, so a product reads the staged tile once per 32 rows.  The
// 16 columns of position tile j are the positions 4 c + j (c = 0 .. 15): the tile index
// then moves an LDS address by a constant, so one address register serves every tile.
//   GEMM1  Yh = S_s X   (X staged m-major: slice index contiguous per position)
//   scale  Yh[s][m] *= lmin / (kappa (mu_f(m) + mu_s(s)) + vbar)
//   GEMM2  Z  = S_s Yh
// With A = S_s X = sc rhat and Yh its scaled FP16 copy, r.z = sum A Yh / (sc^2 lmin)
// = sum X Z / (sc^2 lmin) (S_s is symmetric), Z = S_s Yh the second product: every wave
// adds up its share of a job (FP32) as it replaces X by Z in LDS and writes it to
// rzp[job * NSP / 32 + wave], job = column * npen + position block, so a column's
// partials are reduced in a fixed order by the PCG sweep.
// Thread t moves slices 4 (t >> 3) .. + 3 of positions 8 (t & 7) .. + 7: four 16-byte
// row accesses (eight lanes cover a 128-byte row segment), transposed in registers into
// 8-byte LDS words.  The next job's rows are loaded during the current job's products.
// In the m-major LDS arrays the 16-byte blocks of row m are permuted by XOR with
// (m >> 3) & 3, which spreads the transposing writes of rows 8 apart over the banks and
// keeps the 16-byte operand reads contiguous.
constexpr int kPenMB = 64;

// Buffer resource of a byte range [base, base + bytes) for buffer loads and stores on
// gfx9-class chips (dword 3: 32-bit data format, no swizzle).  An access whose offset
// lies outside the range returns zeros (load) or is dropped (store), so a store that must
// not happen is given an out-of-range offset instead of a branch around it.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void *base, int bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, bytes,
                                             0x00020000);
}
constexpr int kBufOff = (int)0x80000000u;  // beyond every range used here
constexpr int kBufNT = 2;                  // cache policy: non-temporal

template <int KS, bool VEC>
__global__ __launch_bounds__(64 * KS) __attribute__((amdgpu_waves_per_eu(KS <= 3 ? 4 : KS <= 6 ? 3 : 2))) void k_dst_pencil(DstPlan p, const _Float16 *__restrict__ Hin,
                                                    _Float16 *__restrict__ Hout, long ld,
                                                    int ncols, const float *__restrict__ pcs,
                                                    double *__restrict__ rzp) {
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int NJ = kPenMB / 16;  // position tiles of 16
    constexpr int RB = 2;            // row blocks of 16 per wave
    constexpr int NSP = 32 * KS, SP = NSP + 8;
    constexpr int nw = KS;           // waves per workgroup (the launch uses 64 KS threads)
    const int ns = p.ns, nf = p.nf;
    _Float16 *XT = reinterpret_cast<_Float16 *>(smem);
    _Float16 *YT = XT + kPenMB * SP;
    // slowest-axis eigenvalues (-1 past ns), then the in-plane ones along x and y, copied
    // once (per-job lookups in global memory would each wait out a cache round trip)
    float *MUS = reinterpret_cast<float *>(YT + kPenMB * SP);
    float *MUX = MUS + NSP;
    float *MUY = MUX + ((p.nx + 3) & ~3);
    // per column: the forward scale sc (0: the column is skipped in this PCG iteration),
    // vbar and lmin, so that finding the next job and its constants needs no global load
    float *CSC = MUS + pen_mu_floats(NSP, p.nx, p.ny), *CVB = CSC + ncols, *CLM = CVB + ncols;
    const int tid = threadIdx.x;
    for (int i = tid; i < NSP; i += blockDim.x) MUS[i] = i < ns ? p.mus[i] : -1.f;
    for (int i = tid; i < p.nx; i += blockDim.x) MUX[i] = p.mux[i];
    if (p.dim == 3)
        for (int i = tid; i < p.ny; i += blockDim.x) MUY[i] = p.muy[i];
    for (int i = tid; i < ncols; i += blockDim.x) {
        CSC[i] = pcs[i];
        CVB[i] = p.cvbar ? p.cvbar[i] : p.vbar;
        CLM[i] = p.clmin ? p.clmin[i] : p.lmin;
    }
    __syncthreads();
    const int w = tid >> 6, lane = tid & 63, lr = lane & 15, lg = lane >> 4;
    const int mg = tid & 7, s0 = 4 * (tid >> 3);  // this thread's transfer item
    const long njobs = (long)ncols * p.npen;
    // LDS offsets (halves) of this lane's accesses at tile 0 / item 0; the tile index j,
    // the k-chunk ks and the item i add j SP, 32 ks and i SP (the swizzle depends on
    // bits of the position that these do not change)
    const int xg = pen_off(4 * lr, 8 * lg, SP);                   // product operands
    const int xw0 = pen_off(4 * lr, 32 * w + 4 * lg, SP);         // row block 0 results
    const int xw1 = pen_off(4 * lr, 32 * w + 16 + 4 * lg, SP);    // row block 1 results
    const int xs = pen_off(8 * mg, s0, SP);                       // transfer items

    // S_s rows 32w + 16rb + lr, k-chunks of 32: the A operands of both products
    v8h A[RB][KS];
#pragma unroll
    for (int rb = 0; rb < RB; ++rb)
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
            A[rb][ks] = *reinterpret_cast<const v8h *>(p.Ss + (32 * w + 16 * rb + lr) * NSP +
                                                       32 * ks + 8 * lg);

    // per-column constants from LDS into scalar registers (an LDS read does not wait for
    // the prefetch on the vector memory counter, and a job index that stays in scalar
    // registers keeps the loop's control flow uniform)
    auto sreg = [](float v) {
        return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, v)));
    };
    // Jobs are dealt round-robin, so the workgroups resident at one time work on
    // neighbouring positions of the same slices (DRAM pages stay open); columns the PCG
    // skips are passed over.
    auto next_active = [&](long job) {
        while (job < njobs && sreg(CSC[job / p.npen]) == 0.f) job += gridDim.x;
        const unsigned long u = (unsigned long)job;
        return (long)(((unsigned long)(unsigned)__builtin_amdgcn_readfirstlane((int)(u >> 32)) << 32) |
                      (unsigned)__builtin_amdgcn_readfirstlane((int)u));
    };
    // rows s0 .. s0 + 3 at positions m .. m + 7 of a job
    v8h h[4];
    auto job_m = [&](long job) {
        const int col = (int)(job / p.npen);
        return (int)(job - (long)col * p.npen) * kPenMB + 8 * mg;
    };
    // Vector case: buffer accesses relative to the job's first position, so that the
    // per-thread byte offsets (row s0 + r, positions 8 mg ..) stay fixed across jobs;
    // rows past ns lie outside the range (loads return 0, stores are dropped)
    auto row_off = [&](int r) { return ((s0 + r) * nf + 8 * mg) * (int)sizeof(_Float16); };
    auto job_rsrc = [&](const _Float16 *H, long job) {
        const int col = (int)(job / p.npen);
        const int m0 = (int)(job - (long)col * p.npen) * kPenMB;
        return buf_rsrc(H + (long)col * ld + m0, (ns * nf - m0) * (int)sizeof(_Float16));
    };
    auto load = [&](long job) {
        if constexpr (VEC) {
            const __amdgpu_buffer_rsrc_t ri = job_rsrc(Hin, job);
#pragma unroll
            for (int r = 0; r < 4; ++r)
                h[r] = __builtin_bit_cast(v8h, __builtin_amdgcn_raw_buffer_load_b128(ri, row_off(r), 0, 0));
        } else {
            const int col = (int)(job / p.npen);
            const int m = job_m(job);
            const _Float16 *src = Hin + (long)col * ld;
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    h[r][i] = (m + i < nf && s0 + r < ns) ? src[(long)(s0 + r) * nf + m + i]
                                                          : (_Float16)0.f;
        }
    };
    // transpose a job's rows into XT: slices s0 .. s0 + 3 of rows 8 mg + i
    auto stage = [&](long job) {
        const bool mok = job_m(job) < nf;  // nf % 8 == 0 in the vector case
        bool ok[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) ok[r] = mok && s0 + r < ns;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            v4h q;
#pragma unroll
            for (int r = 0; r < 4; ++r) q[r] = ok[r] ? h[r][i] : (_Float16)0.f;
            *reinterpret_cast<v4h *>(XT + xs + i * SP) = q;
        }
    };
    // the partial sums of r.z: one per (job, wave); lanes other than 63 store out of range
    const int offR = lane == 63 ? w * (int)sizeof(double) : kBufOff;

    long job = next_active(blockIdx.x);
    if (job >= njobs) return;
    load(job);
    // In the vector case every global access of the loop is unconditional: per job four
    // loads (the next job's rows) followed by five stores (an r.z partial, four rows of Z).
    // Five stores that the hardware drops (out-of-range offsets) follow the first loads
    // as well, so on every path into the staging the rows are followed by exactly five
    // stores and its wait leaves the previous job's stores in flight.
    if constexpr (VEC) {
        const v2u zero2 = {0u, 0u};
        const v4u zero4 = {0u, 0u, 0u, 0u};
        const __amdgpu_buffer_rsrc_t ro = buf_rsrc(Hout, 0);
        __builtin_amdgcn_raw_buffer_store_b64(zero2, ro, kBufOff, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r)
            __builtin_amdgcn_raw_buffer_store_b128(zero4, ro, kBufOff + 64 * (r + 1), 0, kBufNT);
    }
    while (true) {
        // the next job is found before the barrier, so the prefetch after it need not
        // wait for the activity flag
        const long nxt = next_active(job + gridDim.x);
        const int col = (int)(job / p.npen);
        const int m0 = (int)(job - (long)col * p.npen) * kPenMB;
        const float vbar = sreg(CVB[col]);
        const float lmin = sreg(CLM[col]);
        const float scj = sreg(CSC[col]);
        stage(job);
        __syncthreads();
        load(nxt < njobs ? nxt : job);  // in flight during the products below

        v4f acc[RB][NJ];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[rb][j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const v8h b = lds8(XT + xg + j * SP + 32 * ks);
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
                    acc[rb][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[rb][ks], b, acc[rb][j], 0, 0, 0);
            }
        // spectral scaling, then Yh m-major into YT
#pragma unroll
        for (int j = 0; j < NJ; ++j) {
            // in-plane eigenvalue sum of position m0 + 4 lr + j (-1 past nf)
            const int m = m0 + 4 * lr + j;
            float muf;
            if (p.dim == 3) {
                const int y = m / p.nx;
                muf = m < nf ? MUX[m - y * p.nx] + MUY[y] : -1.f;
            } else {
                muf = m < nf ? MUX[m] : -1.f;
            }
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) {
                const int sb = 32 * w + 16 * rb + 4 * lg;
                const v4f mus = *reinterpret_cast<const v4f *>(MUS + sb);
                v4h hv;
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    float f = 0.f;
                    // hardware reciprocal (about 1 ulp): the product is rounded to FP16 next
                    if (muf >= 0.f && mus[v] >= 0.f)
                        f = lmin * __builtin_amdgcn_rcpf(p.kap * (muf + mus[v]) + vbar);
                    hv[v] = (_Float16)(acc[rb][j][v] * f);
                }
                *reinterpret_cast<v4h *>(YT + (rb ? xw1 : xw0) + j * SP) = hv;
            }
        }
        __syncthreads();
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int j = 0; j < NJ; ++j) acc[rb][j] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks)
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                const v8h b = lds8(YT + xg + j * SP + 32 * ks);
#pragma unroll
                for (int rb = 0; rb < RB; ++rb)
                    acc[rb][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(A[rb][ks], b, acc[rb][j], 0, 0, 0);
            }
        // Z m-major into XT (every wave finished GEMM1 before the barrier above), each
        // element after its product with the X it replaces: this lane's share of r.z
        float rzl = 0.f;
#pragma unroll
        for (int rb = 0; rb < RB; ++rb)
#pragma unroll
            for (int j = 0; j < NJ; ++j) {
                typedef _Float16 v2h __attribute__((ext_vector_type(2)));
                _Float16 *q = XT + (rb ? xw1 : xw0) + j * SP;
                const v4h x = *reinterpret_cast<const v4h *>(q);
                v4h hv;
#pragma unroll
                for (int v = 0; v < 4; ++v) hv[v] = (_Float16)acc[rb][j][v];
                // products of FP16 pairs summed in FP32 (v_dot2_f32_f16)
                rzl = __builtin_amdgcn_fdot2(v2h{x[0], x[1]}, v2h{hv[0], hv[1]}, rzl, false);
                rzl = __builtin_amdgcn_fdot2(v2h{x[2], x[3]}, v2h{hv[2], hv[3]}, rzl, false);
                *reinterpret_cast<v4h *>(q) = hv;
            }
        {
            rzl = wave_sum_lane63(rzl);
            // in FP64: sc^2 leaves the FP32 range once ||r|| < ~5e-20 sqrt(Ng)
            const double rz = (double)rzl / ((double)scj * (double)scj * (double)lmin);
            const __amdgpu_buffer_rsrc_t rr = buf_rsrc(rzp + job * nw, nw * (int)sizeof(double));
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(v2u, rz), rr, offR, 0, 0);
        }
        __syncthreads();
        {
            // rows s0 .. s0 + 3 of Z at positions m .. m + 7
            const int m = m0 + 8 * mg;
            v8h z[4];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const v4h q = *reinterpret_cast<const v4h *>(XT + xs + i * SP);
#pragma unroll
                for (int r = 0; r < 4; ++r) z[r][i] = q[r];
            }
            if constexpr (VEC) {
                // positions past nf (a ragged last job) would land in the next row
                const __amdgpu_buffer_rsrc_t ro = job_rsrc(Hout, job);
#pragma unroll
                for (int r = 0; r < 4; ++r)
                    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(v4u, z[r]), ro,
                                                           m < nf ? row_off(r) : kBufOff, 0, kBufNT);
            } else {
                _Float16 *dst = Hout + (long)col * ld + m;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    if (m + i >= nf) break;
#pragma unroll
                    for (int r = 0; r < 4; ++r)
                        if (s0 + r < ns) dst[(long)(s0 + r) * nf + i] = z[r][i];
                }
            }
        }
        if (nxt >= njobs) break;
        job = nxt;
        // no barrier: the next staging writes exactly the XT words this thread has just read
        // (the same transfer item), and every other access to XT and YT of this job came
        // before the barrier above
    }
}


}  // namespace

// ---------------------------------------------------------------- host side

static int pad32(int n) { return (n + 31) / 32 * 32; }


void dst_plan_geometry(DstPlan &p, int dim, int nx, int ny, int nz) {
    p.dim = dim;
    p.nx = nx;
    p.ny = ny;
    p.nz = dim == 3 ? nz : 1;
    p.NXP = pad32(nx);
    p.NYP = pad32(ny);
    if (dim == 3) {
        p.ns = nz;
        p.nf = nx * ny;
        p.NSP = pad32(nz);
        p.RP = p.NYP;
        p.rows = ny;
        p.nslab = nz;
    } else {
        p.ns = ny;
        p.nf = nx;
        p.NSP = p.NYP;
        p.RP = 64;
        p.rows = 64;
        p.nslab = (ny + 63) / 64;
    }
    p.npen = (p.nf + kPenMB - 1) / kPenMB;
    p.rzparts = p.npen * (p.NSP / 32);
}

constexpr size_t kLdsBytes = 160 * 1024;  // LDS of one CU (gfx950)

// The plane pass copies S_x into LDS up to 128 points, and in the BIG form up to 192
// points where the copy fits beside X / T^T.
static bool dst_plane_sx_lds(const DstPlan &p) {
    if (p.NXP <= 128) return true;
    return dst_plane_big(p) && p.NXP <= 192 &&
           dst_plane_xt_bytes(p) + (size_t)p.NXP * (p.NXP + 8) * 2 <= kLdsBytes;
}

// X (RP x (NXP+8) halves) and, in 3-D, TT (NXP x (NYP+8) halves), then the S_x copy; the
// inverse pass also stages its FP32 output (RP x (NXP+4) floats) over the same space.
size_t dst_plane_lds(const DstPlan &p, bool inv) {
    size_t b = dst_plane_xt_bytes(p);
    if (dst_plane_sx_lds(p)) b += (size_t)p.NXP * (p.NXP + 8) * 2;  // S_x copy
    if (inv) b = std::max(b, (size_t)(p.RP / (dst_plane_big(p) ? 2 : 1)) * (p.NXP + 4) * 4);
    return b;
}

// A 3-D z-plane is transformed by one workgroup of 4 NYP threads with the plane in LDS: the
// LDS of both plane passes must fit the CU's 160 KiB.
const char *dst_plan_check(int dim, const int n[3]) {
    if (n[0] > 256 || n[1] > 256) return "DST preconditioner: nx, ny must be <= 256";
    if (dim == 3) {
        if (n[2] > 256) return "DST preconditioner: nz must be <= 256";
        DstPlan p{};
        dst_plan_geometry(p, dim, n[0], n[1], n[2]);
        if (std::max(dst_plane_lds(p, false), dst_plane_lds(p, true)) > kLdsBytes)
            return "DST preconditioner: a 3-D z-plane (nx x ny, padded to multiples of 32) "
                   "does not fit the LDS of one workgroup";
    }
    return nullptr;
}

// XT and YT (64 x (NSP + 8) halves each), the slowest-axis, x and y eigenvalues, then
// three floats per column (sc, vbar, lmin)
static size_t dst_pencil_lds(const DstPlan &p, int ncols) {
    return 2 * (size_t)kPenMB * (p.NSP + 8) * 2 +
           sizeof(float) * ((size_t)pen_mu_floats(p.NSP, p.nx, p.ny) + 3 * (size_t)ncols);
}

hipError_t launch_dst_matrix(int n, int NP, _Float16 *S, hipStream_t st) {
    hipLaunchKernelGGL(k_dst_matrix, dim3(64), dim3(256), 0, st, n, NP, S);
    return hipGetLastError();
}

hipError_t launch_sum(const double *v, long n, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_sum, dim3(1), dim3(1024), 0, st, v, n, out);
    return hipGetLastError();
}

hipError_t launch_col_scale(const double *R, long ld, long ng, int ncols, float *pcs,
                            hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_col_scale, dim3(ncols), dim3(kThreads), 0, st, R, ld, ng, pcs);
    return hipGetLastError();
}

hipError_t launch_pc_prep(int k, int ncols, const int *mask, PcgState s, long qs, int tiles,
                          double tol, long ng, float *pcs, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_pc_prep, dim3(ncols), dim3(kThreads), 0, st, k, ncols, mask, s, qs,
                       tiles, tol, ng, pcs);
    return hipGetLastError();
}

#define QO_DISPATCH_NT(NTV, ...)                              \
    switch (NTV) {                                            \
        case 2: { constexpr int NT = 2; __VA_ARGS__; } break;   \
        case 4: { constexpr int NT = 4; __VA_ARGS__; } break;   \
        case 6: { constexpr int NT = 6; __VA_ARGS__; } break;   \
        case 8: { constexpr int NT = 8; __VA_ARGS__; } break;   \
        case 10: { constexpr int NT = 10; __VA_ARGS__; } break; \
        case 12: { constexpr int NT = 12; __VA_ARGS__; } break; \
        case 14: { constexpr int NT = 14; __VA_ARGS__; } break; \
        case 16: { constexpr int NT = 16; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;                 \
    }

// One plane-pass launch: a workgroup of 4 RP threads per (column, slab); the row-vector
// form when rows are whole 16-byte groups, the BIG form for 3-D planes of more than 128 rows.
template <typename T, bool INV, bool PF, typename... A>
static hipError_t launch_plane(const DstPlan &p, int ncols, size_t lds, hipStream_t st, A... args) {
    const dim3 grid((unsigned)(ncols * p.nslab)), block((unsigned)(64 * (p.RP / 16)));
    const bool vec = p.nx % 8 == 0, big = dst_plane_big(p);
#define QO_PLANE_GO(V, B)                                                                  \
    QO_DISPATCH_NT(p.NXP / 16, hipLaunchKernelGGL((k_dst_plane<T, INV, NT, V, PF, B>), grid, \
                                                  block, lds, st, p, args...))
#define QO_PLANE_SX(V)                                                                     \
    if (p.NXP == 160)                                                                      \
        hipLaunchKernelGGL((k_dst_plane<T, INV, 10, V, PF, true, true>), grid, block, lds,  \
                           st, p, args...);                                                \
    else                                                                                   \
        hipLaunchKernelGGL((k_dst_plane<T, INV, 12, V, PF, true, true>), grid, block, lds,  \
                           st, p, args...);
    // the BIG form with the S_x copy: 160 or 192 columns where it fits (dst_plane_sx_lds)
    const bool sxb = big && p.NXP > 128 && dst_plane_sx_lds(p);
    if (vec) {
        if (sxb) { QO_PLANE_SX(true) } else if (big) QO_PLANE_GO(true, true) else QO_PLANE_GO(true, false)
    } else {
        if (sxb) { QO_PLANE_SX(false) } else if (big) QO_PLANE_GO(false, true) else QO_PLANE_GO(false, false)
    }
#undef QO_PLANE_SX
#undef QO_PLANE_GO
    return hipGetLastError();
}

template <typename T>
hipError_t launch_dst_fwd(const DstPlan &p, const T *R, long ld, int ncols, _Float16 *t1,
                          const float *pcs, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    return launch_plane<T, false, false>(p, ncols, dst_plane_lds(p, false), st, R,
                                         (const _Float16 *)nullptr, t1, (float *)nullptr, ld, pcs);
}

// Persistent grid: as many workgroups as are resident at once (the runtime's occupancy for
// this kernel and LDS size, times the CUs), cached per instantiation.
template <int KS>
static hipError_t launch_pencil_ks(const DstPlan &p, const _Float16 *t1, _Float16 *t2, long ld,
                                   int ncols, const float *pcs, double *rzp, hipStream_t st) {
    static int resident[2] = {0, 0};  // {dynamic LDS bytes it was taken for, workgroups}
    const size_t lds = dst_pencil_lds(p, ncols);
    const int block = 64 * KS;
    if (resident[0] != (int)lds || resident[1] <= 0) {
        int dev = 0, cus = 0, per_cu = 0;
        hipError_t e = hipGetDevice(&dev);
        if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        if (e == hipSuccess)
            e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_dst_pencil<KS, true>, block,
                                                             lds);
        if (e != hipSuccess) return e;
        resident[0] = (int)lds;
        resident[1] = std::max(1, per_cu) * std::max(1, cus);
    }
    const long njobs = (long)ncols * p.npen;
    // the kernel's buffer ranges (a column of the output, the r.z partials) are addressed
    // with 32-bit byte offsets
    if ((long)p.ns * p.nf * (long)sizeof(_Float16) > INT_MAX ||
        njobs * (block / 64) * (long)sizeof(double) > INT_MAX)
        return hipErrorInvalidValue;
    const unsigned grid = (unsigned)std::min<long>(njobs, resident[1]);
    if (p.nf % 8 == 0)
        hipLaunchKernelGGL((k_dst_pencil<KS, true>), dim3(grid), dim3(block), lds, st, p, t1, t2,
                           ld, ncols, pcs, rzp);
    else
        hipLaunchKernelGGL((k_dst_pencil<KS, false>), dim3(grid), dim3(block), lds, st, p, t1,
                           t2, ld, ncols, pcs, rzp);
    return hipGetLastError();
}

hipError_t launch_dst_pencil(const DstPlan &p, const _Float16 *t1, _Float16 *t2, long ld,
                             int ncols, const float *pcs, double *rzp, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    switch (p.NSP / 32) {
        case 1: return launch_pencil_ks<1>(p, t1, t2, ld, ncols, pcs, rzp, st);
        case 2: return launch_pencil_ks<2>(p, t1, t2, ld, ncols, pcs, rzp, st);
        case 3: return launch_pencil_ks<3>(p, t1, t2, ld, ncols, pcs, rzp, st);
        case 4: return launch_pencil_ks<4>(p, t1, t2, ld, ncols, pcs, rzp, st);
        case 5: return launch_pencil_ks<5>(p, t1, t2, ld, ncols, pcs, rzp, st);
        case 6: return launch_pencil_ks<6>(p, t1, t2, ld, ncols, pcs, rzp, st);
        case 7: return launch_pencil_ks<7>(p, t1, t2, ld, ncols, pcs, rzp, st);
        case 8: return launch_pencil_ks<8>(p, t1, t2, ld, ncols, pcs, rzp, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_dst_inv(const DstPlan &p, const _Float16 *t2, float *Z, long ld, int ncols,
                          const float *pcs, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    return launch_plane<float, true, false>(p, ncols, dst_plane_lds(p, true), st,
                                            (const float *)nullptr, t2, (_Float16 *)nullptr, Z, ld,
                                            pcs);
}

namespace {
// rzc[c] = rho_k = r.z from the pencil's partials (the first sweep takes it from here) and
// beta[c] = rho_k / rho_{k-1}, 0 at k = 0; columns with pcs[c] == 0 skipped.
__global__ __launch_bounds__(kThreads) void k_rho_beta(int k, int ncols,
                                                       const float *__restrict__ pcs,
                                                       const double *__restrict__ rzp, int rzt,
                                                       PcgState s, float *__restrict__ beta,
                                                       double *__restrict__ rzc) {
    __shared__ dev::Red red;
    const int col = blockIdx.x;
    if (pcs[col] == 0.f) return;
    const double rz = dev::col_sum(rzp, col, rzt, red);
    if (threadIdx.x == 0) {
        rzc[col] = rz;
        beta[col] = k == 0 ? 0.f : (float)(rz / s.rho[((k & 1) ^ 1) * ncols + col]);
    }
}

// Z (FP64) = Z32 for columns with pcs[c] != 0, else 0.
__global__ void k_z_expand(const float *__restrict__ Z32, const float *__restrict__ pcs,
                           double *__restrict__ Z, long ld, long ng) {
    const int c = blockIdx.y;
    const bool on = pcs[c] != 0.f;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < ng;
         i += (long)gridDim.x * blockDim.x)
        Z[(long)c * ld + i] = on ? (double)Z32[(long)c * ld + i] : 0.0;
}
}  // namespace

hipError_t launch_rho_beta(int k, int ncols, const float *pcs, const double *rzp, int rzt,
                           PcgState s, float *beta, double *rzc, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_rho_beta, dim3(ncols), dim3(kThreads), 0, st, k, ncols, pcs, rzp, rzt, s,
                       beta, rzc);
    return hipGetLastError();
}

hipError_t launch_dst_inv_p(const DstPlan &p, const _Float16 *t2, const float *Pold,
                            const float *beta, float *P, long ld, int ncols, const float *pcs,
                            const float *vs, double *wzp, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    return launch_plane<float, true, true>(p, ncols, dst_plane_lds(p, true), st,
                                           (const float *)nullptr, t2, (_Float16 *)nullptr, P, ld,
                                           pcs, Pold, beta, vs, wzp);
}

hipError_t launch_z_expand(const float *Z32, const float *pcs, double *Z, long ld, long ng,
                           int ncols, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    long bx = (ng + 255) / 256;
    if (bx > 1024) bx = 1024;
    hipLaunchKernelGGL(k_z_expand, dim3((unsigned)bx, (unsigned)ncols), dim3(256), 0, st, Z32,
                       pcs, Z, ld, ng);
    return hipGetLastError();
}

template hipError_t launch_dst_fwd<double>(const DstPlan &, const double *, long, int,
                                           _Float16 *, const float *, hipStream_t);
template hipError_t launch_dst_fwd<float>(const DstPlan &, const float *, long, int, _Float16 *,
                                          const float *, hipStream_t);

}  // namespace qo
