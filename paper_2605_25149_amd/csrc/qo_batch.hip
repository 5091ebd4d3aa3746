// N x N algebra of the scheme of Sec. 4.1 for grouped batches: one workgroup per
// instance runs the whole predictor algebra (after the first Gram) or the corrector
// algebra (after the second Gram), so a batch of independent problems needs one launch
// per phase instead of dozens of tiny launches per instance.  The sequence and formulas
// are those of the single-instance step:
//
//   predictor  g2 = tr R - 2 tr M^2 + tr M S M^T        (squared gradient norm, Sec. 3.1)
//              C = S^{-1} M (SPD Gauss-Jordan), R_W = sym(R - M^T C), D = C S - M^T,
//              (I + a^2 R_W S - a D) b = D - a R_W S     (a = tau/2, partial pivoting)
//              A = S + a S b, X = I + tau b - tau C A, Y = tau A, Z = X + C Y,
//              and the transposes X^T, Y^T, Z^T for the block updates
//   corrector  O = sym <U_hat,U_hat> - I, O_R = -tau O, ||O||_F, and ||O_{n+1}||_F from
//              O_{n+1} = O - tau (A_n O + O A_n) + tau^2 O B_n O
//
// Matrices live in global memory (L2-resident, a few KiB to MiB per instance).
#include "qo_internal.h"

#include <algorithm>

namespace qo {

namespace {

enum {
    BP_SW, BP_C, BP_RW, BP_D, BP_RWS, BP_MAT, BP_RHS, BP_A, BP_X, BP_Y, BP_Z, BP_XR, BP_YR,
    BP_ZR, BP_O, BP_OR, BP_MS, BP_T1, BP_T2, BP_T3, BP_COUNT
};

constexpr int kWgThreads = 1024;

__device__ __forceinline__ double wg_sum(double v, double *red) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    __syncthreads();
    return s;
}

// C = alpha op(A) op(B) + beta C + gamma I  (m x n, inner k; C must not alias A or B)
__device__ void wg_gemm(double *C, int ldc, const double *A, int lda, bool ta, const double *B,
                        int ldb, bool tb, int m, int n, int k, double alpha, double beta,
                        double gamma) {
    for (int e = threadIdx.x; e < m * n; e += blockDim.x) {
        const int r = e % m, c = e / m;
        double s = 0.0;
        for (int q = 0; q < k; ++q) {
            const double a = ta ? A[(long)r * lda + q] : A[(long)q * lda + r];
            const double b = tb ? B[(long)q * ldb + c] : B[(long)c * ldb + q];
            s += a * b;
        }
        double v = alpha * s;
        if (beta != 0.0) v += beta * C[(long)c * ldc + r];
        if (gamma != 0.0 && r == c) v += gamma;
        C[(long)c * ldc + r] = v;
    }
    __syncthreads();
}

// C = a A + b op(B) + g I  (elementwise; C may alias A, not a transposed B)
__device__ void wg_axpby(double *C, int ldc, double a, const double *A, int lda, double b,
                         const double *B, int ldb, bool tb, double g, int m, int n) {
    for (int e = threadIdx.x; e < m * n; e += blockDim.x) {
        const int r = e % m, c = e / m;
        double v = 0.0;
        if (A && a != 0.0) v += a * A[(long)c * lda + r];
        if (B && b != 0.0) v += b * (tb ? B[(long)r * ldb + c] : B[(long)c * ldb + r]);
        if (r == c) v += g;
        C[(long)c * ldc + r] = v;
    }
    __syncthreads();
}

// B <- A^{-1} B by Gauss-Jordan (A destroyed): spd -> no pivoting, fail (5) when a pivot
// is not above 1e-13 of the largest diagonal entry; else partial pivoting.  Returns the
// status (0 ok, 5 singular / not SPD, 7 non-finite), identical in every thread.
__device__ int wg_gj(double *A, int lda, double *B, int ldb, int n, int m, bool spd, double *f,
                     double *prow, double *sval, int *sidx, int *ish) {
    const int tid = threadIdx.x, nthr = blockDim.x;
    if (tid == 0) {
        double md = 0.0;
        if (spd)
            for (int i = 0; i < n; ++i) md = fmax(md, fabs(A[(long)i * lda + i]));
        sval[0] = 1e-13 * md;
        ish[1] = 0;
    }
    __syncthreads();
    const double thr = sval[0];
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        if (spd) {
            if (tid == 0) {
                ish[0] = k;
                const double d = A[(long)k * lda + k];
                if (!(d > thr) || !isfinite(d)) ish[1] = isfinite(d) ? 5 : 7;
            }
        } else {
            double best = -1.0;
            int bi = k;
            for (int i = k + tid; i < n; i += nthr) {
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
                for (int w = 1; w < nthr / 64; ++w)
                    if (sval[w] > bv || (sval[w] == bv && sidx[w] < bix)) { bv = sval[w]; bix = sidx[w]; }
                ish[0] = bix;
                if (!(bv > 0.0) || !isfinite(bv)) ish[1] = isfinite(bv) ? 5 : 7;
            }
        }
        __syncthreads();
        if (ish[1]) break;
        const int p = ish[0];
        if (p != k) {
            for (int j = tid; j < n + m; j += nthr) {
                double *base = j < n ? A + (long)j * lda : B + (long)(j - n) * ldb;
                const double t = base[k];
                base[k] = base[p];
                base[p] = t;
            }
            __syncthreads();
        }
        const double inv = 1.0 / A[(long)k * lda + k];
        for (int i = tid; i < n; i += nthr) f[i] = A[(long)k * lda + i];
        __syncthreads();
        for (int j = tid; j < n + m; j += nthr) {
            if (j < n && j <= k) continue;
            double *base = j < n ? A + (long)j * lda : B + (long)(j - n) * ldb;
            const double v = base[k] * inv;
            prow[j] = v;
            base[k] = v;
        }
        __syncthreads();
        const int w0 = k + 1;
        const int W = (n - w0) + m;
        for (int e = tid; e < W * n; e += nthr) {
            const int i = e % n;
            const int j = e / n + w0;
            if (i == k) continue;
            double *base = j < n ? A + (long)j * lda : B + (long)(j - n) * ldb;
            base[i] -= f[i] * prow[j];
        }
        __syncthreads();
    }
    const int st = ish[1];
    __syncthreads();
    return st;
}

__device__ double wg_fro(const double *A, int lda, int n, double *red) {
    double s = 0.0;
    for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
        const double v = A[(long)(e / n) * lda + e % n];
        s += v * v;
    }
    return sqrt(wg_sum(s, red));
}

__global__ __launch_bounds__(kWgThreads) void k_nn_predict(const NnJob *__restrict__ jobs) {
    extern __shared__ double nsm[];  // f[n], prow[2n]
    __shared__ double red[kWgThreads / 64], sval[kWgThreads / 64];
    __shared__ int sidx[kWgThreads / 64], ish[2];
    const NnJob J = jobs[blockIdx.x];
    const int N = J.n, N2 = 2 * N;
    const double tau = J.tau, al = 0.5 * tau;
    double *P = J.pool;
    auto mp = [&](int i) { return P + (size_t)i * N * N; };
    const double *S = J.G1;
    const double *M = J.G1 + (size_t)N * N2;
    const double *R = J.G1 + (size_t)N * N2 + N;
    // squared gradient norm: tr R - 2 tr M^2 + tr M S M^T
    wg_gemm(mp(BP_MS), N, M, N2, false, S, N2, false, N, N, N, 1.0, 0.0, 0.0);
    {
        double tr = 0.0, tmm = 0.0, tmsm = 0.0;
        const double *MS = mp(BP_MS);
        for (int e = threadIdx.x; e < N * N; e += blockDim.x) {
            const int r = e % N, c = e / N;
            const double mrc = M[(long)c * N2 + r];
            tmm += mrc * M[(long)r * N2 + c];
            tmsm += MS[(long)c * N + r] * mrc;
            if (r == c) tr += R[(long)c * N2 + r];
        }
        tr = wg_sum(tr, red);
        tmm = wg_sum(tmm, red);
        tmsm = wg_sum(tmsm, red);
        if (threadIdx.x == 0) J.scal[0] = tr - 2.0 * tmm + tmsm;
    }
    // C = S^{-1} M
    wg_axpby(mp(BP_SW), N, 1.0, S, N2, 0.0, nullptr, N, false, 0.0, N, N);
    wg_axpby(mp(BP_C), N, 1.0, M, N2, 0.0, nullptr, N, false, 0.0, N, N);
    int st = wg_gj(mp(BP_SW), N, mp(BP_C), N, N, N, true, nsm, nsm + N, sval, sidx, ish);
    if (st) {
        if (threadIdx.x == 0) *J.status = st;
        return;
    }
    // R_W = sym(R - M^T C)
    wg_axpby(mp(BP_T1), N, 1.0, R, N2, 0.0, nullptr, N, false, 0.0, N, N);
    wg_gemm(mp(BP_T1), N, M, N2, true, mp(BP_C), N, false, N, N, N, -1.0, 1.0, 0.0);
    wg_axpby(mp(BP_RW), N, 0.5, mp(BP_T1), N, 0.5, mp(BP_T1), N, true, 0.0, N, N);
    // D = C S - M^T
    wg_gemm(mp(BP_D), N, mp(BP_C), N, false, S, N2, false, N, N, N, 1.0, 0.0, 0.0);
    wg_axpby(mp(BP_D), N, 1.0, mp(BP_D), N, -1.0, M, N2, true, 0.0, N, N);
    // RWS = R_W S; (I + a^2 RWS - a D) b = D - a RWS
    wg_gemm(mp(BP_RWS), N, mp(BP_RW), N, false, S, N2, false, N, N, N, 1.0, 0.0, 0.0);
    wg_axpby(mp(BP_MAT), N, al * al, mp(BP_RWS), N, -al, mp(BP_D), N, false, 1.0, N, N);
    wg_axpby(mp(BP_RHS), N, 1.0, mp(BP_D), N, -al, mp(BP_RWS), N, false, 0.0, N, N);
    st = wg_gj(mp(BP_MAT), N, mp(BP_RHS), N, N, N, false, nsm, nsm + N, sval, sidx, ish);
    if (st) {
        if (threadIdx.x == 0) *J.status = st;
        return;
    }
    const double *bm = mp(BP_RHS);
    // A = S + a S b ; X = I + tau b - tau C A ; Y = tau A ; Z = X + C Y
    wg_axpby(mp(BP_A), N, 1.0, S, N2, 0.0, nullptr, N, false, 0.0, N, N);
    wg_gemm(mp(BP_A), N, S, N2, false, bm, N, false, N, N, N, al, 1.0, 0.0);
    wg_axpby(mp(BP_X), N, tau, bm, N, 0.0, nullptr, N, false, 1.0, N, N);
    wg_gemm(mp(BP_X), N, mp(BP_C), N, false, mp(BP_A), N, false, N, N, N, -tau, 1.0, 0.0);
    wg_axpby(mp(BP_Y), N, tau, mp(BP_A), N, 0.0, nullptr, N, false, 0.0, N, N);
    wg_axpby(mp(BP_Z), N, 1.0, mp(BP_X), N, 0.0, nullptr, N, false, 0.0, N, N);
    wg_gemm(mp(BP_Z), N, mp(BP_C), N, false, mp(BP_Y), N, false, N, N, N, 1.0, 1.0, 0.0);
    // row-major copies for the block updates
    wg_axpby(mp(BP_XR), N, 0.0, nullptr, N, 1.0, mp(BP_X), N, true, 0.0, N, N);
    wg_axpby(mp(BP_YR), N, 0.0, nullptr, N, 1.0, mp(BP_Y), N, true, 0.0, N, N);
    wg_axpby(mp(BP_ZR), N, 0.0, nullptr, N, 1.0, mp(BP_Z), N, true, 0.0, N, N);
}

__global__ __launch_bounds__(kWgThreads) void k_nn_correct(const NnJob *__restrict__ jobs) {
    __shared__ double red[kWgThreads / 64];
    const NnJob J = jobs[blockIdx.x];
    const int N = J.n, N2 = 2 * N;
    const double tau = J.tau;
    double *P = J.pool;
    auto mp = [&](int i) { return P + (size_t)i * N * N; };
    const double *G2 = J.G2;
    // O = sym <U_hat,U_hat> - I ; O_R = -tau O
    wg_axpby(mp(BP_O), N, 0.5, G2, N2, 0.5, G2, N2, true, -1.0, N, N);
    wg_axpby(mp(BP_OR), N, -tau, mp(BP_O), N, 0.0, nullptr, N, false, 0.0, N, N);
    const double fo = wg_fro(mp(BP_O), N, N, red);
    // O_{n+1} = O - tau (A O + O A) + tau^2 O B O with A = sym <U_hat,Q>, B = <Q,Q>
    double *Am = mp(BP_T1), *T2 = mp(BP_T2), *On = mp(BP_T3);
    wg_axpby(Am, N, 0.5, G2 + (size_t)N * N2, N2, 0.5, G2 + (size_t)N * N2, N2, true, 0.0, N, N);
    wg_axpby(On, N, 1.0, mp(BP_O), N, 0.0, nullptr, N, false, 0.0, N, N);
    wg_gemm(On, N, Am, N, false, mp(BP_O), N, false, N, N, N, -tau, 1.0, 0.0);
    wg_gemm(On, N, mp(BP_O), N, false, Am, N, false, N, N, N, -tau, 1.0, 0.0);
    wg_gemm(T2, N, G2 + (size_t)N * N2 + N, N2, false, mp(BP_O), N, false, N, N, N, 1.0, 0.0, 0.0);
    wg_gemm(On, N, mp(BP_O), N, false, T2, N, false, N, N, N, tau * tau, 1.0, 0.0);
    const double fn = wg_fro(On, N, N, red);
    if (threadIdx.x == 0) {
        J.scal[1] = fo;
        J.scal[2] = fn;
    }
}

// Reverse mode of the predictor algebra (one instance, one workgroup): given the
// adjoints Xb, Yb of X, Y (N x N, column-major), return Sb, Mb, Rb, the adjoints of
// S = <U,U>, M = <U,P>, R = <P,P> (the forward intermediates are recomputed from S, M, R):
//   Ab = tau Yb - tau C^T Xb,  Cb = -tau Xb A^T,  bb = tau Xb + a S Ab,  Sb = Ab + a Ab b^T,
//   MAT^T RHSb = bb,  MATb = -RHSb b^T,  Kb = a^2 MATb - a RHSb,  Db = RHSb - a MATb,
//   RWb = Kb S, Sb += RW Kb, Cb += Db S, Sb += C^T Db, Mb = -Db^T,
//   Tb = sym(RWb), Rb = Tb, Mb -= C Tb, Cb -= M Tb,
//   Z = S^{-1} Cb, Mb += Z, Sb -= Z C^T.
// Work slots AD_* (N x N each); status as in the forward.
enum {
    AD_SW, AD_C, AD_T, AD_RW, AD_D, AD_K, AD_MAT, AD_MATT, AD_B, AD_A, AD_AB, AD_CB, AD_BB, AD_SB,
    AD_RHSB, AD_MATB, AD_KB, AD_DB, AD_RWB, AD_TB, AD_MB, AD_RB, AD_Z, AD_COUNT
};

__global__ __launch_bounds__(kWgThreads) void k_nn_adjoint(const double *__restrict__ G1, int N,
                                                           double tau, const double *__restrict__ Xb,
                                                           const double *__restrict__ Yb,
                                                           double *__restrict__ pool,
                                                           double *__restrict__ out,
                                                           int *__restrict__ status) {
    extern __shared__ double nsm[];  // f[n], prow[2n]
    __shared__ double sval[kWgThreads / 64];
    __shared__ int sidx[kWgThreads / 64], ish[2];
    const int N2 = 2 * N;
    const double al = 0.5 * tau;
    auto mp = [&](int i) { return pool + (size_t)i * N * N; };
    const double *S = G1;
    const double *M = G1 + (size_t)N * N2;
    const double *R = G1 + (size_t)N * N2 + N;
    // forward intermediates
    wg_axpby(mp(AD_SW), N, 1.0, S, N2, 0.0, nullptr, N, false, 0.0, N, N);
    wg_axpby(mp(AD_C), N, 1.0, M, N2, 0.0, nullptr, N, false, 0.0, N, N);
    int st = wg_gj(mp(AD_SW), N, mp(AD_C), N, N, N, true, nsm, nsm + N, sval, sidx, ish);
    if (st) {
        if (threadIdx.x == 0) *status = st;
        return;
    }
    double *C = mp(AD_C);
    wg_axpby(mp(AD_T), N, 1.0, R, N2, 0.0, nullptr, N, false, 0.0, N, N);
    wg_gemm(mp(AD_T), N, M, N2, true, C, N, false, N, N, N, -1.0, 1.0, 0.0);
    wg_axpby(mp(AD_RW), N, 0.5, mp(AD_T), N, 0.5, mp(AD_T), N, true, 0.0, N, N);
    wg_gemm(mp(AD_D), N, C, N, false, S, N2, false, N, N, N, 1.0, 0.0, 0.0);
    wg_axpby(mp(AD_D), N, 1.0, mp(AD_D), N, -1.0, M, N2, true, 0.0, N, N);
    wg_gemm(mp(AD_K), N, mp(AD_RW), N, false, S, N2, false, N, N, N, 1.0, 0.0, 0.0);
    wg_axpby(mp(AD_MAT), N, al * al, mp(AD_K), N, -al, mp(AD_D), N, false, 1.0, N, N);
    wg_axpby(mp(AD_MATT), N, 0.0, nullptr, N, 1.0, mp(AD_MAT), N, true, 0.0, N, N);
    wg_axpby(mp(AD_B), N, 1.0, mp(AD_D), N, -al, mp(AD_K), N, false, 0.0, N, N);
    st = wg_gj(mp(AD_MAT), N, mp(AD_B), N, N, N, false, nsm, nsm + N, sval, sidx, ish);
    if (st) {
        if (threadIdx.x == 0) *status = st;
        return;
    }
    double *b = mp(AD_B);
    wg_axpby(mp(AD_A), N, 1.0, S, N2, 0.0, nullptr, N, false, 0.0, N, N);
    wg_gemm(mp(AD_A), N, S, N2, false, b, N, false, N, N, N, al, 1.0, 0.0);
    // reverse sweep
    double *Ab = mp(AD_AB), *Cb = mp(AD_CB), *bb = mp(AD_BB), *Sb = mp(AD_SB);
    wg_axpby(Ab, N, tau, Yb, N, 0.0, nullptr, N, false, 0.0, N, N);
    wg_gemm(Ab, N, C, N, true, Xb, N, false, N, N, N, -tau, 1.0, 0.0);
    wg_gemm(Cb, N, Xb, N, false, mp(AD_A), N, true, N, N, N, -tau, 0.0, 0.0);
    wg_axpby(bb, N, tau, Xb, N, 0.0, nullptr, N, false, 0.0, N, N);
    wg_gemm(bb, N, S, N2, false, Ab, N, false, N, N, N, al, 1.0, 0.0);
    wg_axpby(Sb, N, 1.0, Ab, N, 0.0, nullptr, N, false, 0.0, N, N);
    wg_gemm(Sb, N, Ab, N, false, b, N, true, N, N, N, al, 1.0, 0.0);
    // RHSb = MAT^{-T} bb
    double *RHSb = mp(AD_RHSB);
    wg_axpby(RHSb, N, 1.0, bb, N, 0.0, nullptr, N, false, 0.0, N, N);
    st = wg_gj(mp(AD_MATT), N, RHSb, N, N, N, false, nsm, nsm + N, sval, sidx, ish);
    if (st) {
        if (threadIdx.x == 0) *status = st;
        return;
    }
    double *MATb = mp(AD_MATB), *Kb = mp(AD_KB), *Db = mp(AD_DB);
    wg_gemm(MATb, N, RHSb, N, false, b, N, true, N, N, N, -1.0, 0.0, 0.0);
    wg_axpby(Kb, N, al * al, MATb, N, -al, RHSb, N, false, 0.0, N, N);
    wg_axpby(Db, N, 1.0, RHSb, N, -al, MATb, N, false, 0.0, N, N);
    double *RWb = mp(AD_RWB);
    wg_gemm(RWb, N, Kb, N, false, S, N2, false, N, N, N, 1.0, 0.0, 0.0);
    wg_gemm(Sb, N, mp(AD_RW), N, false, Kb, N, false, N, N, N, 1.0, 1.0, 0.0);
    wg_gemm(Cb, N, Db, N, false, S, N2, false, N, N, N, 1.0, 1.0, 0.0);
    wg_gemm(Sb, N, C, N, true, Db, N, false, N, N, N, 1.0, 1.0, 0.0);
    double *Mb = mp(AD_MB), *Tb = mp(AD_TB), *Rb = mp(AD_RB);
    wg_axpby(Mb, N, 0.0, nullptr, N, -1.0, Db, N, true, 0.0, N, N);
    wg_axpby(Tb, N, 0.5, RWb, N, 0.5, RWb, N, true, 0.0, N, N);
    wg_axpby(Rb, N, 1.0, Tb, N, 0.0, nullptr, N, false, 0.0, N, N);
    wg_gemm(Mb, N, C, N, false, Tb, N, false, N, N, N, -1.0, 1.0, 0.0);
    wg_gemm(Cb, N, M, N2, false, Tb, N, false, N, N, N, -1.0, 1.0, 0.0);
    // C = S^{-1} M
    double *Z = mp(AD_Z);
    wg_axpby(Z, N, 1.0, Cb, N, 0.0, nullptr, N, false, 0.0, N, N);
    wg_axpby(mp(AD_SW), N, 1.0, S, N2, 0.0, nullptr, N, false, 0.0, N, N);
    st = wg_gj(mp(AD_SW), N, Z, N, N, N, true, nsm, nsm + N, sval, sidx, ish);
    if (st) {
        if (threadIdx.x == 0) *status = st;
        return;
    }
    wg_axpby(Mb, N, 1.0, Mb, N, 1.0, Z, N, false, 0.0, N, N);
    wg_gemm(Sb, N, Z, N, false, C, N, true, N, N, N, -1.0, 1.0, 0.0);
    // outputs: [Sb | Mb | Rb], each N x N column-major
    wg_axpby(out, N, 1.0, Sb, N, 0.0, nullptr, N, false, 0.0, N, N);
    wg_axpby(out + (size_t)N * N, N, 1.0, Mb, N, 0.0, nullptr, N, false, 0.0, N, N);
    wg_axpby(out + (size_t)2 * N * N, N, 1.0, Rb, N, 0.0, nullptr, N, false, 0.0, N, N);
}

// Per-instance energy from the quadratic-form partials of the group's columns:
// out[i] = {E_sigma = 1/2 w sum x.Hx, w sum x.x} over the columns [coff[i], coff[i+1]).
__global__ __launch_bounds__(256) void k_instance_energy(const double *__restrict__ part, long qs,
                                                         int tiles, const int *__restrict__ coff,
                                                         double w, double *__restrict__ out) {
    __shared__ double red[4];
    const int i = blockIdx.x;
    const long a = (long)coff[i] * tiles, b = (long)coff[i + 1] * tiles;
    double e = 0.0, t = 0.0;
    for (long k = a + threadIdx.x; k < b; k += blockDim.x) {
        e += part[k];
        t += part[qs + k];
    }
    e = wg_sum(e, red);
    t = wg_sum(t, red);
    if (threadIdx.x == 0) {
        out[2 * i] = 0.5 * w * e;
        out[2 * i + 1] = w * t;
    }
}

// V + sigma and 1 / diag(H_sigma); with vs32 also their FP32 copies (the FP32 stencil
// forms its diagonal from the FP32 c0 and V + sigma, so 1/diag is taken from those).
__global__ void k_batch_potential(const double *__restrict__ V, long ng, double sigma, double c0,
                                  double *__restrict__ vs, double *__restrict__ dinv,
                                  float *__restrict__ vs32, float *__restrict__ dinv32,
                                  int *__restrict__ status) {
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < ng;
         i += (long)gridDim.x * blockDim.x) {
        const double v = V[i] + sigma;
        const double d = c0 + v;
        if (!isfinite(v)) atomicMax(status, 7);
        else if (!(d > 0.0)) atomicMax(status, 5);
        vs[i] = v;
        dinv[i] = 1.0 / d;
        if (vs32) {
            vs32[i] = (float)v;
            dinv32[i] = (float)(1.0 / ((double)(float)c0 + (double)(float)v));
        }
    }
}

// Bookkeeping of one FP32 refinement round (one workgroup): per column total += its and
// rounds += mask (columns outside the mask ran no iteration); rstat[0] = the round's
// largest iteration count, rstat[1] = the number of columns that took part.
__global__ __launch_bounds__(256) void k_its_accum(const int *__restrict__ its,
                                                   const int *__restrict__ mask, int n,
                                                   int *__restrict__ total,
                                                   int *__restrict__ rounds,
                                                   int *__restrict__ rstat) {
    __shared__ int smax[4], scnt[4];
    int mk = 0, cnt = 0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int m = mask[i] ? 1 : 0;
        const int k = m ? its[i] : 0;
        total[i] += k;
        rounds[i] += m;
        mk = k > mk ? k : mk;
        cnt += m;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const int o = __shfl_xor(mk, off, 64);
        mk = o > mk ? o : mk;
        cnt += __shfl_xor(cnt, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        smax[threadIdx.x >> 6] = mk;
        scnt[threadIdx.x >> 6] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int a = 0, c = 0;
        for (int w = 0; w < 4; ++w) {
            a = smax[w] > a ? smax[w] : a;
            c += scnt[w];
        }
        rstat[0] = a;
        rstat[1] = c;
    }
}

__global__ void k_fill_int(int *__restrict__ p, int n, int v) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = v;
}

__global__ void k_noconv_check(const int *__restrict__ active, int n, int *__restrict__ err) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        if (active[i]) {
            atomicMax(&err[0], 6);
            atomicMin(&err[1], i);
        }
}

}  // namespace

hipError_t launch_its_accum(const int *its, const int *mask, int n, int *total, int *rounds,
                            int *rstat, hipStream_t st) {
    hipLaunchKernelGGL(k_its_accum, dim3(1), dim3(256), 0, st, its, mask, n, total, rounds, rstat);
    return hipGetLastError();
}

hipError_t launch_batch_potential(const double *V, long ng, double sigma, double c0, double *vs,
                                  double *dinv, float *vs32, float *dinv32, int *status,
                                  hipStream_t st) {
    long blocks = (ng + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_batch_potential, dim3((unsigned)blocks), dim3(256), 0, st, V, ng, sigma,
                       c0, vs, dinv, vs32, dinv32, status);
    return hipGetLastError();
}

hipError_t launch_fill_int(int *p, int n, int v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_int, dim3((unsigned)std::min(1024, (n + 255) / 256)), dim3(256), 0,
                       st, p, n, v);
    return hipGetLastError();
}

hipError_t launch_noconv_check(const int *active, int n, int *err, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_noconv_check, dim3((unsigned)std::min(1024, (n + 255) / 256)), dim3(256),
                       0, st, active, n, err);
    return hipGetLastError();
}

size_t nn_pool_elems(int n) { return (size_t)BP_COUNT * n * n; }

size_t nn_adjoint_pool_elems(int n) { return (size_t)AD_COUNT * n * n; }

hipError_t launch_nn_adjoint(const double *G1, int n, double tau, const double *Xb,
                             const double *Yb, double *pool, double *out, int *status,
                             hipStream_t st) {
    hipLaunchKernelGGL(k_nn_adjoint, dim3(1), dim3(kWgThreads), sizeof(double) * 3 * (size_t)n, st,
                       G1, n, tau, Xb, Yb, pool, out, status);
    return hipGetLastError();
}

hipError_t launch_nn_predict(const NnJob *jobs, int njobs, int max_n, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_nn_predict, dim3((unsigned)njobs), dim3(kWgThreads),
                       sizeof(double) * 3 * (size_t)max_n, st, jobs);
    return hipGetLastError();
}

hipError_t launch_nn_correct(const NnJob *jobs, int njobs, hipStream_t st) {
    if (njobs <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_nn_correct, dim3((unsigned)njobs), dim3(kWgThreads), 0, st, jobs);
    return hipGetLastError();
}

hipError_t launch_instance_energy(const double *part, long qs, int tiles, const int *coff,
                                  int ninst, double w, double *out, hipStream_t st) {
    if (ninst <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_instance_energy, dim3((unsigned)ninst), dim3(256), 0, st, part, qs,
                       tiles, coff, w, out);
    return hipGetLastError();
}

// slot index of the row-major update coefficients in an instance pool
int nn_slot_xr() { return BP_XR; }
int nn_slot_yr() { return BP_YR; }
int nn_slot_zr() { return BP_ZR; }
int nn_slot_or() { return BP_OR; }

}  // namespace qo
