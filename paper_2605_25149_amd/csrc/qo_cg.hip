// One PCG iteration per sweep: the Chronopoulos-Gear form of Jacobi-PCG for the
// inverse operator G = H_sigma^{-1} of Sec. 3.1, on many columns at once.
//
// Per column, iteration k (alpha, beta from the inner products of the previous
// sweep, reduced in this kernel's prologue):
//     p   = D r + beta p_old                   (beta = 0 at k = 0)
//     s   = H p;   r' = r - alpha s;   x += alpha p
//     u   = D r';  w = H u
//     gamma' = r'.u,  delta' = w.u,  ||r'||^2   (partials for the next sweep)
//     next: beta' = gamma'/gamma, alpha' = gamma' / (delta' - beta' gamma' / alpha)
// Global traffic per grid point and column: read r, p_old, x; write r', p, x
// (6 values; the two-sweep Hestenes-Stiefel form needs 8).  The stop test
// ||r|| <= tol ||b|| is taken in the prologue, so a column freezes at the same
// iteration as in the two-sweep form.
//
// Tiling: one workgroup streams TY full x-rows of ZC z-planes of one column.
// Three stages run skewed over z, each with a 3-plane LDS ring:
//   P-stage, plane t:    p on rows [-2, TY+1]           -> LDS-P[t % 3]
//   U-stage, plane t-1:  s = H p, r', u on rows [-1, TY] -> LDS-U[(t-1) % 3];
//                        own rows: store r', p, x; gamma', ||r'||^2
//   W-stage, plane t-2:  w = H u on own rows; delta'
// Two barriers per plane; all global loads are issued one plane ahead.
#include "qo_device.h"
#include "qo_internal.h"

namespace qo {

namespace {

using dev::block_sums;
using dev::col_sum;
using dev::Red;

template <typename T>
struct CgArgs {
    Grid g;
    const T *vs, *dinv;
    const T *Rin;
    T *Rout;
    const T *Pold;
    T *Pnew;
    T *X;
    long ld;
    int ncols, k;
    double tol;
    const int *mask;
    PcgState s;
    const double *pin;  // partial sums read  [4][ncols*tiles]
    double *pout;       // partial sums written
    long qs;
};

template <typename T>
__device__ __forceinline__ T *smem_ptr() {
    extern __shared__ __align__(16) unsigned char qo_cg_smem[];
    return reinterpret_cast<T *>(qo_cg_smem);
}

template <typename T, int PPT>
__global__ __launch_bounds__(kThreads) void k_cg_step(CgArgs<T> a) {
    __shared__ Red red;
    __shared__ int sh_flag;
    __shared__ double sh_alpha, sh_beta;
    const Grid &g = a.g;
    const int tiles = g.tiles();
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    int col, tile;
    stencil_tile_of(L, (int)(gridDim.x / tiles), tiles, col, tile);
    const TileExtent te = g.extent(tile);
    const bool lead = tile == 0;
    const int k = a.k;
    const int cur = k & 1, prv = cur ^ 1;
    const int ncols = a.ncols;
    PcgState &s = a.s;

    // ---- prologue: this column's scalars
    const int prev_active = (k == 0) ? (a.mask ? a.mask[col] : 1) : s.active[prv * ncols + col];
    if (!prev_active) {
        if (lead && threadIdx.x == 0) s.active[cur * ncols + col] = 0;
        return;
    }
    const double gam = col_sum(a.pin, col, tiles, red);
    const double rr = col_sum(a.pin + a.qs, col, tiles, red);
    const double del = col_sum(a.pin + 3 * a.qs, col, tiles, red);
    double bb;
    if (k == 0) {
        bb = col_sum(a.pin + 2 * a.qs, col, tiles, red);
        if (lead && threadIdx.x == 0) s.bb[col] = bb;
    } else {
        bb = s.bb[col];
    }
    const double ctol = s.coltol ? s.coltol[col] : a.tol;
    if (threadIdx.x == 0) {
        int flag = 0;  // 0 run, 1 converged, 5 not SPD, 7 non-finite
        double beta = 0.0, alpha = 0.0;
        if (!isfinite(gam) || !isfinite(rr) || !isfinite(bb) || !isfinite(del)) {
            flag = 7;
        } else if (sqrt(rr) <= ctol * sqrt(bb)) {
            flag = 1;
        } else {
            double den = del;
            if (k > 0) {
                beta = gam / s.rho[prv * ncols + col];
                den = del - beta * gam / s.alpha[prv * ncols + col];
            }
            if (!isfinite(den)) flag = 7;
            else if (!(den > 0.0)) flag = 5;
            else alpha = gam / den;
        }
        sh_flag = flag;
        sh_alpha = alpha;
        sh_beta = beta;
        if (lead) {
            s.its[col] = k;
            s.active[cur * ncols + col] = flag == 0 ? 1 : 0;
            if (flag == 0) {
                s.rho[cur * ncols + col] = gam;
                s.alpha[cur * ncols + col] = alpha;
            }
            if (flag >= 5) {
                atomicMax(&s.err[0], flag);
                atomicMin(&s.err[1], col);
            }
        }
    }
    __syncthreads();
    if (sh_flag != 0) return;
    const T alpha = (T)sh_alpha, beta = (T)sh_beta;
    const bool first = k == 0;

    // ---- geometry
    const int tid = threadIdx.x;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const int TY = g.TY;
    const int y0 = te.y0, ty = te.ty, z0 = te.z0, z1 = te.z1;
    const long plane = (long)nx * ny;
    const int nP = (ty + 4) * nx, nU = (ty + 2) * nx, nO = ty * nx;
    const int slotP = (TY + 4) * nx, slotU = (TY + 2) * nx;
    T *ldsP = smem_ptr<T>();
    T *ldsU = ldsP + 3 * slotP;
    const T kap = (T)g.kappa, c0 = (T)g.c0;
    const T ihx2 = (T)g.ihx2, ihy2 = (T)g.ihy2, ihz2 = (T)g.ihz2;
    const long cb = (long)col * a.ld;
    const T *__restrict__ Rin = a.Rin + cb;
    T *__restrict__ Rout = a.Rout + cb;
    const T *__restrict__ Pold = a.Pold + cb;
    T *__restrict__ Pnew = a.Pnew + cb;
    T *__restrict__ X = a.X + cb;
    const T *__restrict__ vs = a.vs;
    const T *__restrict__ dinv = a.dinv;

    // in-plane offsets (row-major within the plane) of this thread's points;
    // -1 marks a point outside the grid (Dirichlet zero) or outside the set
    int offP[PPT], offU[PPT], offO[PPT];
    int xU[PPT], xO[PPT];
    bool ownU[PPT];
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        const int j = tid + m * kThreads;
        offP[m] = -2;  // not in set
        if (j < nP) {
            const int row = y0 + j / nx - 2;
            offP[m] = (row >= 0 && row < ny) ? row * nx + j % nx : -1;
        }
        offU[m] = -2;
        xU[m] = 0;
        ownU[m] = false;
        if (j < nU) {
            const int rrel = j / nx - 1;
            const int row = y0 + rrel;
            xU[m] = j % nx;
            offU[m] = (row >= 0 && row < ny) ? row * nx + xU[m] : -1;
            ownU[m] = rrel >= 0 && rrel < ty;
        }
        offO[m] = -2;
        xO[m] = 0;
        if (j < nO) {
            xO[m] = j % nx;
            offO[m] = (y0 + j / nx) * nx + xO[m];
        }
    }

    // prefetched raw values
    T pd[PPT], pr[PPT], pp[PPT];             // P-stage: D, r, p_old of the next P plane
    T ur[PPT], ud[PPT], uv[PPT], ux[PPT];    // U-stage: r, D, V+sigma, x of the next U plane
    T wv[PPT];                               // W-stage: V+sigma of the next W plane
    auto loadP = [&](int t) {
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            pd[m] = pr[m] = pp[m] = T(0);
            if (t >= 0 && t < nz && offP[m] >= 0) {
                const long i = (long)t * plane + offP[m];
                pd[m] = dinv[i];
                pr[m] = Rin[i];
                if (!first) pp[m] = Pold[i];
            }
        }
    };
    auto loadU = [&](int t) {
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            ur[m] = ud[m] = uv[m] = ux[m] = T(0);
            if (t >= 0 && t < nz && offU[m] >= 0) {
                const long i = (long)t * plane + offU[m];
                ur[m] = Rin[i];
                ud[m] = dinv[i];
                uv[m] = vs[i];
                if (ownU[m] && t >= z0 && t < z1) ux[m] = X[i];
            }
        }
    };
    auto loadW = [&](int t) {
#pragma unroll
        for (int m = 0; m < PPT; ++m) {
            wv[m] = T(0);
            if (t >= z0 && t < z1 && offO[m] >= 0) wv[m] = vs[(long)t * plane + offO[m]];
        }
    };

    double acc[3] = {0.0, 0.0, 0.0};  // gamma', ||r'||^2, delta'
    loadP(z0 - 2);
    loadU(z0 - 1);
    for (int t = z0 - 2; t <= z1 + 1; ++t) {
        // ---------------- P-stage: plane t
        {
            T *P = ldsP + ((t + 3) % 3) * slotP;
#pragma unroll
            for (int m = 0; m < PPT; ++m) {
                const int j = tid + m * kThreads;
                if (j < nP) {
                    const T z = pd[m] * pr[m];
                    P[j] = first ? z : z + beta * pp[m];
                }
            }
            if (t + 1 <= z1 + 1) loadP(t + 1);
        }
        __syncthreads();
        // ---------------- U-stage: plane t-1
        if (t >= z0) {
            const int kU = t - 1;
            const T *Pm = ldsP + ((kU + 2) % 3) * slotP;  // plane kU-1
            const T *Pc = ldsP + ((kU + 3) % 3) * slotP;  // plane kU
            const T *Pp = ldsP + ((kU + 4) % 3) * slotP;  // plane kU+1
            T *U = ldsU + ((kU + 3) % 3) * slotU;
            const bool kin = kU >= 0 && kU < nz;
            const bool kown = kU >= z0 && kU < z1;
#pragma unroll
            for (int m = 0; m < PPT; ++m) {
                const int j = tid + m * kThreads;
                if (j >= nU) continue;
                T u = T(0);
                if (kin && offU[m] >= 0) {
                    const int pi = j + nx;
                    const int x = xU[m];
                    const T pc = Pc[pi];
                    const T xm = x > 0 ? Pc[pi - 1] : T(0);
                    const T xp = x < nx - 1 ? Pc[pi + 1] : T(0);
                    const T sv = (c0 + uv[m]) * pc -
                                 kap * (ihx2 * (xm + xp) + ihy2 * (Pc[pi - nx] + Pc[pi + nx]) +
                                        ihz2 * (Pm[pi] + Pp[pi]));
                    const T rn = ur[m] - alpha * sv;
                    u = ud[m] * rn;
                    if (ownU[m] && kown) {
                        const long i = (long)kU * plane + offU[m];
                        Rout[i] = rn;
                        Pnew[i] = pc;
                        X[i] = ux[m] + alpha * pc;
                        const double rd = (double)rn;
                        acc[0] += rd * (double)u;
                        acc[1] += rd * rd;
                    }
                }
                U[j] = u;
            }
            if (t <= z1) loadU(t);
        }
        __syncthreads();
        // ---------------- W-stage: plane t-2
        if (t >= z0 + 2) {
            const int kW = t - 2;
            const T *Um = ldsU + ((kW + 2) % 3) * slotU;
            const T *Uc = ldsU + ((kW + 3) % 3) * slotU;
            const T *Up = ldsU + ((kW + 4) % 3) * slotU;
#pragma unroll
            for (int m = 0; m < PPT; ++m) {
                const int j = tid + m * kThreads;
                if (j >= nO) continue;
                const int ui = j + nx;
                const int x = xO[m];
                const T uc = Uc[ui];
                const T xm = x > 0 ? Uc[ui - 1] : T(0);
                const T xp = x < nx - 1 ? Uc[ui + 1] : T(0);
                const T wvv = (c0 + wv[m]) * uc -
                              kap * (ihx2 * (xm + xp) + ihy2 * (Uc[ui - nx] + Uc[ui + nx]) +
                                     ihz2 * (Um[ui] + Up[ui]));
                acc[2] += (double)wvv * (double)uc;
            }
        }
        loadW(t - 1);
    }
    block_sums<3>(acc, red);
    if (threadIdx.x == 0) {
        const long o = (long)col * tiles + tile;
        a.pout[o] = acc[0];
        a.pout[a.qs + o] = acc[1];
        a.pout[3 * a.qs + o] = acc[2];
    }
}

}  // namespace

size_t cg_lds_bytes(const Grid &g, size_t elem) {
    return 3 * (size_t)(g.TY + 4) * g.nx * elem + 3 * (size_t)(g.TY + 2) * g.nx * elem;
}

template <typename T>
hipError_t launch_cg_step(const Grid &g, const T *vs, const T *dinv, const T *Rin, T *Rout,
                          const T *Pold, T *Pnew, T *X, long ld, int ncols, int k, double tol,
                          const int *mask, PcgState s, const double *pin, double *pout,
                          hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    CgArgs<T> a{g, vs, dinv, Rin, Rout, Pold, Pnew, X, ld, ncols, k, tol, mask, s, pin, pout,
                (long)ncols * g.tiles()};
    const dim3 grid(ncols * g.tiles());
    const size_t smem = cg_lds_bytes(g, sizeof(T));
    switch (g.ppt) {
        case 2: hipLaunchKernelGGL((k_cg_step<T, 2>), grid, dim3(kThreads), smem, st, a); break;
        case 3: hipLaunchKernelGGL((k_cg_step<T, 3>), grid, dim3(kThreads), smem, st, a); break;
        case 4: hipLaunchKernelGGL((k_cg_step<T, 4>), grid, dim3(kThreads), smem, st, a); break;
        case 5: hipLaunchKernelGGL((k_cg_step<T, 5>), grid, dim3(kThreads), smem, st, a); break;
        case 6: hipLaunchKernelGGL((k_cg_step<T, 6>), grid, dim3(kThreads), smem, st, a); break;
        case 8: hipLaunchKernelGGL((k_cg_step<T, 8>), grid, dim3(kThreads), smem, st, a); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template hipError_t launch_cg_step<double>(const Grid &, const double *, const double *,
                                           const double *, double *, const double *, double *,
                                           double *, long, int, int, double, const int *,
                                           PcgState, const double *, double *, hipStream_t);
template hipError_t launch_cg_step<float>(const Grid &, const float *, const float *,
                                          const float *, float *, const float *, float *,
                                          float *, long, int, int, double, const int *,
                                          PcgState, const double *, double *, hipStream_t);

}  // namespace qo
