// Small dense FP64 linear algebra on the N x N inner-product matrices of the
// scheme (Sec. 4.1): products, Gauss-Jordan solves (with the SPD test of the
// Gram matrix <U,U>), cyclic Jacobi eigen-decomposition for the eigenvalue
// read-out of Sec. 5, and the scalar diagnostics.  N is at most a few
// hundred, so these kernels are latency-bound; the solves and the Jacobi
// sweeps run in one workgroup with the matrices resident in L2.
#include "qo_internal.h"

namespace qo {

namespace {

constexpr int TB = 16;

__global__ __launch_bounds__(256) void k_gemm(double *__restrict__ C, int ldc,
                                              const double *__restrict__ A, int lda, int ta,
                                              const double *__restrict__ B, int ldb, int tb,
                                              int m, int n, int k, double alpha, double beta,
                                              double gamma) {
    __shared__ double As[TB][TB + 1], Bs[TB][TB + 1];
    const int tx = threadIdx.x % TB, ty = threadIdx.x / TB;
    const int row = blockIdx.x * TB + tx;  // output row
    const int col = blockIdx.y * TB + ty;  // output column
    double s = 0.0;
    for (int kk = 0; kk < k; kk += TB) {
        // As[tx][j] = op(A)[blockrow + tx][kk + j]; thread (tx, ty) loads j = ty
        {
            const int r = blockIdx.x * TB + tx, c = kk + ty;
            double v = 0.0;
            if (r < m && c < k) v = ta ? A[(long)r * lda + c] : A[(long)c * lda + r];
            As[tx][ty] = v;
        }
        {
            const int r = kk + tx, c = blockIdx.y * TB + ty;
            double v = 0.0;
            if (r < k && c < n) v = tb ? B[(long)r * ldb + c] : B[(long)c * ldb + r];
            Bs[tx][ty] = v;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < TB; ++j) s += As[tx][j] * Bs[j][ty];
        __syncthreads();
    }
    if (row < m && col < n) {
        double c = alpha * s;
        if (beta != 0.0) c += beta * C[(long)col * ldc + row];
        if (gamma != 0.0 && row == col) c += gamma;
        C[(long)col * ldc + row] = c;
    }
}

__global__ void k_axpby(double *__restrict__ C, int ldc, double a, const double *__restrict__ A,
                        int lda, double b, const double *__restrict__ B, int ldb, int tb,
                        double g, int m, int n) {
    const long total = (long)m * n;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (long)gridDim.x * blockDim.x) {
        const int r = (int)(e % m), c = (int)(e / m);
        double v = 0.0;
        if (A && a != 0.0) v += a * A[(long)c * lda + r];
        if (B && b != 0.0) v += b * (tb ? B[(long)r * ldb + c] : B[(long)c * ldb + r]);
        if (r == c) v += g;
        C[(long)c * ldc + r] = v;
    }
}

// In-place transpose-safe variant is not needed: nn_axpby with tb requires C != B.

constexpr int GJT = 1024;

__global__ __launch_bounds__(GJT) void k_gj(double *__restrict__ A, int lda,
                                            double *__restrict__ B, int ldb, int n, int m,
                                            int spd, int *__restrict__ status) {
    __shared__ double sval[GJT / 64];
    __shared__ int sidx[GJT / 64];
    __shared__ int piv_sh;
    __shared__ int fail_sh;
    __shared__ double scale_sh;
    extern __shared__ double gj_smem[];  // f[n], prow[n + m]
    double *f = gj_smem;
    double *prow = gj_smem + n;
    const int tid = threadIdx.x;
    if (tid == 0) {
        fail_sh = 0;
        // SPD test threshold: a pivot below 1e-13 of the largest diagonal entry
        // means the matrix is (numerically) not positive definite
        double md = 0.0;
        if (spd)
            for (int i = 0; i < n; ++i) md = fmax(md, fabs(A[(long)i * lda + i]));
        scale_sh = 1e-13 * md;
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        // pivot
        if (spd) {
            if (tid == 0) {
                piv_sh = k;
                const double d = A[(long)k * lda + k];
                if (!(d > scale_sh) || !isfinite(d)) fail_sh = isfinite(d) ? 5 : 7;
            }
        } else {
            double best = -1.0;
            int bi = k;
            for (int i = k + tid; i < n; i += GJT) {
                const double v = fabs(A[(long)k * lda + i]);
                if (v > best || (v == best && i < bi)) { best = v; bi = i; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(best, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
            }
            if ((tid & 63) == 0) { sval[tid >> 6] = best; sidx[tid >> 6] = bi; }
            __syncthreads();
            if (tid == 0) {
                double bv = sval[0];
                int bix = sidx[0];
                for (int w = 1; w < GJT / 64; ++w)
                    if (sval[w] > bv || (sval[w] == bv && sidx[w] < bix)) { bv = sval[w]; bix = sidx[w]; }
                piv_sh = bix;
                if (!(bv > 0.0) || !isfinite(bv)) fail_sh = isfinite(bv) ? 5 : 7;
            }
        }
        __syncthreads();
        if (fail_sh) break;
        const int p = piv_sh;
        if (p != k) {
            for (int j = tid; j < n + m; j += GJT) {
                double *base = j < n ? A + (long)j * lda : B + (long)(j - n) * ldb;
                const double t = base[k];
                base[k] = base[p];
                base[p] = t;
            }
            __syncthreads();
        }
        const double inv = 1.0 / A[(long)k * lda + k];
        for (int i = tid; i < n; i += GJT) f[i] = A[(long)k * lda + i];
        for (int j = tid; j < n + m; j += GJT) {
            if (j < n && j <= k) continue;
            double *base = j < n ? A + (long)j * lda : B + (long)(j - n) * ldb;
            const double v = base[k] * inv;
            prow[j] = v;
            base[k] = v;
        }
        __syncthreads();
        // eliminate rows i != k over columns j > k (A) and all of B
        const int w0 = k + 1;
        const int W = (n - w0) + m;
        const long tot = (long)W * n;
        for (long e = tid; e < tot; e += GJT) {
            const int i = (int)(e % n);
            const int jj = (int)(e / n);
            if (i == k) continue;
            const int j = jj + w0;
            double *base = j < n ? A + (long)j * lda : B + (long)(j - n) * ldb;
            base[i] -= f[i] * prow[j];
        }
        __syncthreads();
    }
    if (tid == 0 && fail_sh) atomicMax(status, fail_sh);
}

// ---- blocked Gauss-Jordan on [A | B] (n <= 512) ----------------------------
//
// Panels of b pivot columns (32 for n <= 256, else 16).  The panel kernel (one workgroup, panel in LDS)
// chooses the pivots of columns [k0, k0+b) by eliminating inside the panel
// only, records the row swaps, and hands out the panel columns after the swaps
// (O = A[:, K], n x b) and the inverse of their pivot block P = O[K, :].  The
// update kernel then applies the same elimination to every column x still to
// be reduced (columns >= k0+b of A, all of B): swaps, y = P^{-1} x_K,
// x_K = y, x_i -= O[i, :] y for the other rows i.  Same pivots and SPD test as
// the unblocked kernel above; a column's updates are grouped per panel.
constexpr int GB = 32;
constexpr int GPT = 512;
constexpr int GCW = 4;  // columns per update workgroup (many workgroups: the update is spread over the CUs)

__global__ __launch_bounds__(GPT) void k_gjb_panel(double *__restrict__ A, int lda, int n, int k0,
                                                   int b, int spd, double *__restrict__ work,
                                                   int *__restrict__ piv,
                                                   int *__restrict__ status) {
    extern __shared__ double gsm[];
    double *W = gsm;          // working panel, column kk at W + kk * n
    double *O = gsm + n * b;  // original panel after the row swaps
    __shared__ double sval[GPT / 64];
    __shared__ int sidx[GPT / 64];
    __shared__ int piv_sh, fail_sh;
    __shared__ double thr_sh;
    const int tid = threadIdx.x;
    if (*status) return;  // an earlier panel failed
    // elimination: thread -> row eri, columns ecg, ecg + encg, ... of the panel (n <= GPT)
    const int eri = tid % n, ecg = tid / n, encg = GPT / n;
    double *scal = work + (size_t)n * GB + GB * GB;
    // The panel's loads (n b <= 8192 values: at most 16 per thread) are all issued before
    // any is used, so the panel costs one memory round trip, not one per value.
    constexpr int PQ = (GB * kGjBlockedMax / 2) / GPT;
    const int nb = n * b;
    double pv[PQ];
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
        const int e = min(tid + q * GPT, nb - 1);
        const int kk = e / n, i = e - kk * n;
        pv[q] = A[(long)(k0 + kk) * lda + i];
    }
    // SPD test threshold: 1e-13 of the largest diagonal entry of the input, reduced over
    // the workgroup on the first panel and kept for the later ones
    double md = 0.0;
    if (k0 == 0 && spd) {
        for (int i = tid; i < n; i += GPT) md = fmax(md, fabs(A[(long)i * lda + i]));
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) md = fmax(md, __shfl_xor(md, off, 64));
        if ((tid & 63) == 0) sval[tid >> 6] = md;
    }
#pragma unroll
    for (int q = 0; q < PQ; ++q) {
        const int e = tid + q * GPT;
        if (e < nb) {
            W[e] = pv[q];
            O[e] = pv[q];
        }
    }
    __syncthreads();
    if (tid == 0) {
        fail_sh = 0;
        if (k0 == 0) {
            double m = 0.0;
            if (spd)
                for (int w = 0; w < GPT / 64; ++w) m = fmax(m, sval[w]);
            scal[0] = 1e-13 * m;
            thr_sh = 1e-13 * m;
        } else {
            thr_sh = scal[0];
        }
    }
    __syncthreads();
    for (int kk = 0; kk < b; ++kk) {
        const int k = k0 + kk;
        const double *wc = W + kk * n;
        if (spd) {
            if (tid == 0) {
                piv_sh = k;
                const double d = wc[k];
                if (!(d > thr_sh) || !isfinite(d)) fail_sh = isfinite(d) ? 5 : 7;
            }
        } else {
            double best = -1.0;
            int bi = k;
            for (int i = k + tid; i < n; i += GPT) {
                const double v = fabs(wc[i]);
                if (v > best || (v == best && i < bi)) { best = v; bi = i; }
            }
            for (int off = 32; off > 0; off >>= 1) {
                const double ov = __shfl_xor(best, off, 64);
                const int oi = __shfl_xor(bi, off, 64);
                if (ov > best || (ov == best && oi < bi)) { best = ov; bi = oi; }
            }
            if ((tid & 63) == 0) { sval[tid >> 6] = best; sidx[tid >> 6] = bi; }
            __syncthreads();
            if (tid == 0) {
                double bv = sval[0];
                int bix = sidx[0];
                for (int w = 1; w < GPT / 64; ++w)
                    if (sval[w] > bv || (sval[w] == bv && sidx[w] < bix)) { bv = sval[w]; bix = sidx[w]; }
                piv_sh = bix;
                if (!(bv > 0.0) || !isfinite(bv)) fail_sh = isfinite(bv) ? 5 : 7;
            }
        }
        __syncthreads();
        if (fail_sh) break;
        const int p = piv_sh;
        if (p != k) {
            for (int j = tid; j < b; j += GPT) {
                double t = W[j * n + k];
                W[j * n + k] = W[j * n + p];
                W[j * n + p] = t;
                t = O[j * n + k];
                O[j * n + k] = O[j * n + p];
                O[j * n + p] = t;
            }
        }
        if (tid == 0) piv[k] = p;
        __syncthreads();
        // scale the pivot row of the later panel columns, then eliminate
        const double inv = 1.0 / W[kk * n + k];
        for (int j = kk + 1 + tid; j < b; j += GPT) W[j * n + k] *= inv;
        __syncthreads();
        if (ecg < encg && eri != k) {
            const double f = W[kk * n + eri];
            for (int j = kk + 1 + ecg; j < b; j += encg) W[j * n + eri] -= f * W[j * n + k];
        }
        __syncthreads();
    }
    if (fail_sh) {
        if (tid == 0) atomicMax(status, fail_sh);
        return;
    }
    // P^{-1} for the pivot block P[r][c] = O[c * n + k0 + r]: Gauss-Jordan on [P | I]
    // in the pivot order the panel used (no further pivoting), in LDS (reuses W)
    double *G = gsm + 2 * n * b;  // b x 2b, column-major with leading dimension b
    for (int e = tid; e < b * 2 * b; e += GPT) {
        const int c = e / b, r = e - c * b;
        G[e] = c < b ? O[c * n + k0 + r] : (c - b == r ? 1.0 : 0.0);
    }
    __syncthreads();
    for (int kk = 0; kk < b; ++kk) {
        const double inv = 1.0 / G[kk * b + kk];
        __syncthreads();
        for (int c = kk + tid; c < 2 * b; c += GPT) G[c * b + kk] *= inv;
        __syncthreads();
        for (int e = tid; e < b * 2 * b; e += GPT) {
            const int c = e / b, r = e - c * b;
            if (r == kk || c <= kk) continue;
            G[c * b + r] -= G[kk * b + r] * G[c * b + kk];
        }
        __syncthreads();
    }
    for (int e = tid; e < n * b; e += GPT) work[e] = O[e];
    for (int e = tid; e < b * b; e += GPT) {
        const int c = e / b, r = e - c * b;
        work[(size_t)n * GB + e] = G[(b + c) * b + r];  // P^{-1}[r][c], column-major b x b
    }
}

__global__ __launch_bounds__(256) void k_gjb_update(double *__restrict__ A, int lda,
                                                    double *__restrict__ B, int ldb, int n,
                                                    int m, int k0, int b,
                                                    const double *__restrict__ work,
                                                    const int *__restrict__ piv,
                                                    const int *__restrict__ status) {
    extern __shared__ double usm[];
    double *X = usm;              // n x GCW, column c at X + c * n
    double *Y = usm + n * GCW;    // b x GCW
    double *OL = Y + b * GCW;     // the panel O (n x b), then P^{-1} (b x b)
    double *PL = OL + n * b;
    if (*status) return;
    const int tid = threadIdx.x;
    const int jbeg = k0 + b;
    const int ncol = (n - jbeg) + m;
    const int c0 = blockIdx.x * GCW;
    const int cw = min(GCW, ncol - c0);
    auto colp = [&](int c) -> double * {
        const int j = jbeg + c0 + c;
        return j < n ? A + (long)j * lda : B + (long)(j - n) * ldb;
    };
    // Copies into LDS with eight loads per thread in flight before their stores (a load
    // used at once would cost a memory round trip per value).  O and P^{-1} come from L2
    // once per workgroup instead of once per product term.
    auto stage = [&](double *dst, int count, auto src) {
        for (int e0 = tid; e0 < count; e0 += 8 * 256) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = src(min(e0 + u * 256, count - 1));
#pragma unroll
            for (int u = 0; u < 8; ++u)
                if (e0 + u * 256 < count) dst[e0 + u * 256] = v[u];
        }
    };
    stage(X, n * cw, [&](int e) { const int c = e / n; return colp(c)[e - c * n]; });
    stage(OL, n * b, [&](int e) { return work[e]; });
    stage(PL, b * b, [&](int e) { return work[(size_t)n * GB + e]; });
    __syncthreads();
    if (tid < cw) {
        double *x = X + tid * n;
        for (int kk = 0; kk < b; ++kk) {
            const int p = piv[k0 + kk];
            if (p != k0 + kk) {
                const double t = x[k0 + kk];
                x[k0 + kk] = x[p];
                x[p] = t;
            }
        }
    }
    __syncthreads();
    for (int e = tid; e < b * cw; e += 256) {
        const int c = e / b, r = e - c * b;
        const double *x = X + c * n + k0;
        double s = 0.0;
        for (int q = 0; q < b; ++q) s += PL[q * b + r] * x[q];
        Y[c * b + r] = s;
    }
    __syncthreads();
    for (int e = tid; e < n * cw; e += 256) {
        const int c = e / n, i = e - c * n;
        const double *y = Y + c * b;
        double v;
        if (i >= k0 && i < k0 + b) {
            v = y[i - k0];
        } else {
            double s = 0.0;
            for (int q = 0; q < b; ++q) s += OL[q * n + i] * y[q];
            v = X[c * n + i] - s;
        }
        colp(c)[i] = v;
    }
}

// Cyclic Jacobi with round-robin (circle) ordering: each round rotates n/2
// disjoint pairs.  A <- J^T A J with J the Givens rotation zeroing A_pq.
constexpr int JT = 1024;

__global__ __launch_bounds__(JT) void k_jacobi(double *__restrict__ A, int lda, int n,
                                               double *__restrict__ evals,
                                               double *__restrict__ V, int ldv) {
    extern __shared__ double jsm[];
    const int m = (n + 1) & ~1;  // even number of players; index n is a dummy
    const int np = m / 2;
    double *cs = jsm;            // [np] c
    double *sn = jsm + np;       // [np] s
    int *pp = reinterpret_cast<int *>(jsm + 2 * np);  // [np] p
    int *qq = pp + np;                                // [np] q
    __shared__ double red[JT / 64];
    __shared__ double off_sh, tot_sh;
    const int tid = threadIdx.x;
    for (long e = tid; e < (long)n * n; e += JT) {
        const int r = (int)(e % n), c = (int)(e / n);
        V[(long)c * ldv + r] = (r == c) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 60; ++sweep) {
        // convergence: off-diagonal mass relative to the total
        double off = 0.0, tot = 0.0;
        for (long e = tid; e < (long)n * n; e += JT) {
            const int r = (int)(e % n), c = (int)(e / n);
            const double v = A[(long)c * lda + r];
            tot += v * v;
            if (r != c) off += v * v;
        }
        for (int o = 32; o > 0; o >>= 1) off += __shfl_xor(off, o, 64);
        if ((tid & 63) == 0) red[tid >> 6] = off;
        __syncthreads();
        if (tid == 0) { double s = 0; for (int w = 0; w < JT / 64; ++w) s += red[w]; off_sh = s; }
        __syncthreads();
        for (int o = 32; o > 0; o >>= 1) tot += __shfl_xor(tot, o, 64);
        if ((tid & 63) == 0) red[tid >> 6] = tot;
        __syncthreads();
        if (tid == 0) { double s = 0; for (int w = 0; w < JT / 64; ++w) s += red[w]; tot_sh = s; }
        __syncthreads();
        if (!(off_sh > 1e-32 * tot_sh)) break;
        for (int rnd = 0; rnd < m - 1; ++rnd) {
            for (int i = tid; i < np; i += JT) {
                int p, q;
                if (i == 0) {
                    p = rnd % (m - 1);
                    q = m - 1;
                } else {
                    p = (rnd + i) % (m - 1);
                    q = (rnd - i + (m - 1)) % (m - 1);
                }
                if (p > q) { const int t = p; p = q; q = t; }
                double c = 1.0, s = 0.0;
                if (q < n) {
                    const double apq = A[(long)q * lda + p];
                    const double app = A[(long)p * lda + p];
                    const double aqq = A[(long)q * lda + q];
                    if (apq != 0.0 && fabs(apq) > 1e-300) {
                        const double th = (aqq - app) / (2.0 * apq);
                        double t;
                        if (fabs(th) > 1e150) t = 0.5 / th;
                        else t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(t * t + 1.0);
                        s = t * c;
                    }
                }
                cs[i] = c; sn[i] = s; pp[i] = p; qq[i] = q;
            }
            __syncthreads();
            // rows: A <- J^T A
            for (long e = tid; e < (long)np * n; e += JT) {
                const int i = (int)(e / n), j = (int)(e % n);
                const int p = pp[i], q = qq[i];
                if (q >= n) continue;
                const double c = cs[i], s = sn[i];
                const double ap = A[(long)j * lda + p], aq = A[(long)j * lda + q];
                A[(long)j * lda + p] = c * ap - s * aq;
                A[(long)j * lda + q] = s * ap + c * aq;
            }
            __syncthreads();
            // columns: A <- A J, V <- V J
            for (long e = tid; e < (long)np * n; e += JT) {
                const int i = (int)(e / n), j = (int)(e % n);
                const int p = pp[i], q = qq[i];
                if (q >= n) continue;
                const double c = cs[i], s = sn[i];
                const double ap = A[(long)p * lda + j], aq = A[(long)q * lda + j];
                A[(long)p * lda + j] = c * ap - s * aq;
                A[(long)q * lda + j] = s * ap + c * aq;
                const double vp = V[(long)p * ldv + j], vq = V[(long)q * ldv + j];
                V[(long)p * ldv + j] = c * vp - s * vq;
                V[(long)q * ldv + j] = s * vp + c * vq;
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < n; i += JT) evals[i] = A[(long)i * lda + i];
}

// Rank sort (stable) of evals with the matching column permutation of V.
__global__ __launch_bounds__(1024) void k_sort(double *__restrict__ ev, double *__restrict__ V,
                                               int ldv, int n, int desc,
                                               double *__restrict__ work) {
    const int tid = threadIdx.x;
    // work: [n] values, [n*n] vectors
    for (int i = tid; i < n; i += blockDim.x) {
        const double vi = ev[i];
        int rank = 0;
        for (int j = 0; j < n; ++j) {
            const double vj = ev[j];
            const bool before = desc ? (vj > vi) : (vj < vi);
            if (before || (vj == vi && j < i)) ++rank;
        }
        work[rank] = vi;
        if (V)
            for (int r = 0; r < n; ++r) work[n + (long)rank * n + r] = V[(long)i * ldv + r];
    }
    __syncthreads();
    for (int i = tid; i < n; i += blockDim.x) ev[i] = work[i];
    if (V)
        for (long e = tid; e < (long)n * n; e += blockDim.x) {
            const int r = (int)(e % n), c = (int)(e / n);
            V[(long)c * ldv + r] = work[n + e];
        }
}

__device__ double block_sum_1024(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x / 64); ++w) s += red[w];
    return s;
}

__global__ __launch_bounds__(1024) void k_grad2(const double *__restrict__ S,
                                                const double *__restrict__ M,
                                                const double *__restrict__ R, int ld, int n,
                                                const double *__restrict__ MS, int ldms,
                                                double *__restrict__ out) {
    __shared__ double red[16];
    double tr = 0.0, tmm = 0.0, tmsm = 0.0;
    for (long e = threadIdx.x; e < (long)n * n; e += blockDim.x) {
        const int r = (int)(e % n), c = (int)(e / n);
        const double mrc = M[(long)c * ld + r];
        tmm += mrc * M[(long)r * ld + c];
        tmsm += MS[(long)c * ldms + r] * mrc;
        if (r == c) tr += R[(long)c * ld + r];
    }
    tr = block_sum_1024(tr, red);
    tmm = block_sum_1024(tmm, red);
    tmsm = block_sum_1024(tmsm, red);
    if (threadIdx.x == 0) out[0] = tr - 2.0 * tmm + tmsm;
    (void)S;
}

__global__ __launch_bounds__(1024) void k_fro(const double *__restrict__ A, int lda, int n,
                                              double *__restrict__ out) {
    __shared__ double red[16];
    double s = 0.0;
    for (long e = threadIdx.x; e < (long)n * n; e += blockDim.x) {
        const int r = (int)(e % n), c = (int)(e / n);
        const double v = A[(long)c * lda + r];
        s += v * v;
    }
    s = block_sum_1024(s, red);
    if (threadIdx.x == 0) out[0] = sqrt(s);
}

__global__ void k_scale_cols(double *__restrict__ F, const double *__restrict__ V, int ld,
                             const double *__restrict__ ev, int n, int *__restrict__ status) {
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < (long)n * n;
         e += (long)gridDim.x * blockDim.x) {
        const int r = (int)(e % n), c = (int)(e / n);
        const double l = ev[c];
        if (!(l > 0.0)) {
            if (r == 0) atomicMax(status, 5);
            F[(long)c * ld + r] = 0.0;
        } else {
            F[(long)c * ld + r] = V[(long)c * ld + r] / sqrt(l);
        }
    }
}

__global__ void k_eval_map(double *__restrict__ out, const double *__restrict__ ev, int n,
                           int invert, double sigma) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        out[i] = (invert ? 1.0 / ev[i] : ev[i]) - sigma;
}

__global__ __launch_bounds__(1024) void k_energy_finish(const double *__restrict__ sums,
                                                        int ncols, double w,
                                                        double *__restrict__ out) {
    __shared__ double red[16];
    double a = 0.0, b = 0.0;
    for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
        a += sums[c];
        b += sums[ncols + c];
    }
    a = block_sum_1024(a, red);
    b = block_sum_1024(b, red);
    if (threadIdx.x == 0) {
        out[0] = 0.5 * w * a;
        out[1] = w * b;
    }
}

inline unsigned nblk(long total, int bs) {
    long b = (total + bs - 1) / bs;
    if (b < 1) b = 1;
    if (b > 4096) b = 4096;
    return (unsigned)b;
}

}  // namespace

hipError_t nn_gemm(double *C, int ldc, const double *A, int lda, bool ta, const double *B,
                   int ldb, bool tb, int m, int n, int k, double alpha, double beta, double gamma,
                   hipStream_t st) {
    if (m <= 0 || n <= 0) return hipSuccess;
    const dim3 grid((m + TB - 1) / TB, (n + TB - 1) / TB);
    hipLaunchKernelGGL(k_gemm, grid, dim3(TB * TB), 0, st, C, ldc, A, lda, (int)ta, B, ldb,
                       (int)tb, m, n, k, alpha, beta, gamma);
    return hipGetLastError();
}

hipError_t nn_axpby(double *C, int ldc, double a, const double *A, int lda, double b,
                    const double *B, int ldb, bool tb, double g, int m, int n, hipStream_t st) {
    if (m <= 0 || n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_axpby, dim3(nblk((long)m * n, 256)), dim3(256), 0, st, C, ldc, a, A,
                       lda, b, B, ldb, (int)tb, g, m, n);
    return hipGetLastError();
}

hipError_t nn_gj_solve(double *A, int lda, double *B, int ldb, int n, int m, bool spd,
                       int *status, hipStream_t st, double *work, int *piv) {
    if (n <= 0) return hipSuccess;
    if (n > kGjBlockedMax || !work || !piv) {
        const size_t smem = sizeof(double) * (size_t)(n + n + m);
        hipLaunchKernelGGL(k_gj, dim3(1), dim3(GJT), smem, st, A, lda, B, ldb, n, m, (int)spd,
                           status);
        return hipGetLastError();
    }
    // LDS of the panel kernel: 2 n b + 2 b^2 doubles (<= 144 KiB)
    const int bw = n <= 256 ? GB : GB / 2;
    for (int k0 = 0; k0 < n; k0 += bw) {
        const int b = min(bw, n - k0);
        hipLaunchKernelGGL(k_gjb_panel, dim3(1), dim3(GPT),
                           sizeof(double) * (2 * (size_t)n * b + 2 * (size_t)b * b), st,
                           A, lda, n, k0, b, (int)spd, work, piv, status);
        const int ncol = (n - k0 - b) + m;
        if (ncol > 0)
            hipLaunchKernelGGL(k_gjb_update, dim3((ncol + GCW - 1) / GCW), dim3(256),
                               sizeof(double) * ((size_t)(n + b) * GCW + (size_t)n * b +
                                                 (size_t)b * b),
                               st, A, lda, B, ldb, n, m, k0, b, work, piv, status);
    }
    return hipGetLastError();
}

size_t nn_gj_work_elems(int n) { return (size_t)n * GB + GB * GB + 8; }

hipError_t nn_jacobi(double *A, int lda, int n, double *evals, double *V, int ldv, double *work,
                     hipStream_t st) {
    (void)work;
    if (n <= 0) return hipSuccess;
    const int m = (n + 1) & ~1;
    const size_t smem = (size_t)m / 2 * (2 * sizeof(double) + 2 * sizeof(int));
    hipLaunchKernelGGL(k_jacobi, dim3(1), dim3(JT), smem, st, A, lda, n, evals, V, ldv);
    return hipGetLastError();
}

hipError_t nn_sort(double *evals, double *V, int ldv, int n, bool descending, double *work,
                   hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sort, dim3(1), dim3(1024), 0, st, evals, V, ldv, n, (int)descending,
                       work);
    return hipGetLastError();
}

hipError_t nn_grad2(const double *S, const double *M, const double *R, int ld, int n, double *MS,
                    int ldms, double *out, hipStream_t st) {
    hipError_t e = nn_gemm(MS, ldms, M, ld, false, S, ld, false, n, n, n, 1.0, 0.0, 0.0, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_grad2, dim3(1), dim3(1024), 0, st, S, M, R, ld, n, MS, ldms, out);
    return hipGetLastError();
}

hipError_t nn_fro(const double *A, int lda, int n, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_fro, dim3(1), dim3(1024), 0, st, A, lda, n, out);
    return hipGetLastError();
}

hipError_t nn_scale_cols_rsqrt(double *F, const double *V, int ld, const double *ev, int n,
                               int *status, hipStream_t st) {
    hipLaunchKernelGGL(k_scale_cols, dim3(nblk((long)n * n, 256)), dim3(256), 0, st, F, V, ld,
                       ev, n, status);
    return hipGetLastError();
}

hipError_t nn_eval_map(double *out, const double *ev, int n, bool invert, double sigma,
                       hipStream_t st) {
    hipLaunchKernelGGL(k_eval_map, dim3(nblk(n, 256)), dim3(256), 0, st, out, ev, n, (int)invert,
                       sigma);
    return hipGetLastError();
}

hipError_t nn_energy_finish(const double *sums, int ncols, double w, double *out,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_energy_finish, dim3(1), dim3(1024), 0, st, sums, ncols, w, out);
    return hipGetLastError();
}

}  // namespace qo
