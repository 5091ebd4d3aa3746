// Stencil family: the discrete operator H_sigma = -kappa Lap_h + V + sigma
// (5-point in 2-D, 7-point in 3-D, Dirichlet) applied to many columns, and the
// batched Jacobi-PCG sweeps that apply the inverse operator G = H_sigma^{-1}
// of Sec. 3.1 to a block.
//
// One workgroup (256 threads) streams one tile of one column: TY full x-rows
// of ZC z-planes.  The operand of the stencil is formed on the fly for the
// tile plus one halo row on each side and written to a double-buffered LDS
// plane; the z-neighbours live in registers (z-marching), so every value is
// read from HBM once per sweep up to the halo rows shared with the
// neighbouring band.  Per-column dot products are reduced per workgroup with
// wavefront shuffles and written as partial sums; the next kernel reduces a
// column's partials in a fixed order, so results are deterministic.
//
// PCG per column (Hestenes-Stiefel form, Jacobi preconditioner D = diag(H)^-1):
//   sweep1(k): from r and the previous p form p = D r + beta p_old on the fly
//              (beta = rho_k / rho_{k-1}, p = D r at k = 0), store p,
//              gamma = p . H p  (q = H p is not stored)
//   sweep2(k): alpha = rho_k / gamma;  x += alpha p;  r -= alpha H p (H p
//              recomputed from p);  partials of r . D r and r . r
// The per-column stop test ||r|| <= tol ||b|| is evaluated at the start of
// sweep1, so a column freezes at the first iteration that passes it.
#include "qo_internal.h"
#include "qo_device.h"

#ifndef QO_SWEEP2_NT
#define QO_SWEEP2_NT 1
#endif
#ifndef QO_RESID_NT
#define QO_RESID_NT 1
#endif
#ifndef QO_SWEEP1_NT
#define QO_SWEEP1_NT 1
#endif

namespace qo {

namespace {

using dev::Red;
using dev::block_sums;
using dev::col_sum;

// The engine for wide tiles (PPT >= 4: the 2-D grids, one plane per tile).  Its prefetch
// is issued under the tile's own bounds, which keeps the registers of those many points
// per thread low; with one plane per tile the loop below runs once and nothing is
// carried across planes.
template <typename T, int PPT, class Ld, class Ep>
__device__ __forceinline__ void engine_wide(const Grid &g, int band, int zc,
                                            const T *__restrict__ vs, Ld &ld, Ep &ep,
                                            T *__restrict__ lds) {
    using LR = typename Ld::Raw;
    using ER = typename Ep::Raw;
    const int tid = threadIdx.x;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const TileExtent te = g.extent(band * g.nzc + zc);
    const int y0 = te.y0, ty = te.ty, z0 = te.z0, z1 = te.z1;
    const int npts = ty * nx;
    const long plane = (long)nx * ny;
    const int ldsz = (g.TY + 2) * nx;
    const bool has_lo = y0 > 0, has_hi = (y0 + ty) < ny;
    const bool hown = tid < nx;  // this thread owns halo column tid (prefetched)
    const T kap = (T)g.kappa, c0 = (T)g.c0;
    const T ihx2 = (T)g.ihx2, ihy2 = (T)g.ihy2, ihz2 = (T)g.ihz2;
    const long lo_off = -(long)nx, hi_off = (long)ty * nx;

    int xs[PPT];
    bool val[PPT];
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
        const int t = tid + s * kThreads;
        val[s] = t < npts;
        xs[s] = val[s] ? t % nx : 0;
    }
    T om[PPT], oc[PPT], op[PPT], vsr[PPT];
    LR rq[PPT];
    ER er[PPT];
    LR hlo = Ld::zero(), hhi = Ld::zero();
    const long b0 = (long)z0 * plane + (long)y0 * nx;
    // prologue: operands of planes z0-1, z0 (with halo rows), z0+1
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
        const int t = tid + s * kThreads;
        om[s] = (val[s] && z0 > 0) ? ld.make(ld.load(b0 - plane + t)) : T(0);
        oc[s] = val[s] ? ld.make(ld.load(b0 + t)) : T(0);
        op[s] = (val[s] && z0 + 1 < nz) ? ld.make(ld.load(b0 + plane + t)) : T(0);
        if (val[s]) lds[nx + t] = oc[s];
    }
    for (int hh = tid; hh < nx; hh += kThreads) {
        lds[hh] = has_lo ? ld.make(ld.load(b0 + lo_off + hh)) : T(0);
        lds[(ty + 1) * nx + hh] = has_hi ? ld.make(ld.load(b0 + hi_off + hh)) : T(0);
    }
    // prefetch for the first iteration
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
        const int t = tid + s * kThreads;
        vsr[s] = val[s] ? vs[b0 + t] : T(0);
        er[s] = val[s] ? ep.load(b0 + t) : Ep::zero();
        rq[s] = (val[s] && z0 + 2 < nz && z0 + 1 < z1) ? ld.load(b0 + 2 * plane + t) : Ld::zero();
    }
    if (hown && z0 + 1 < z1) {
        if (has_lo) hlo = ld.load(b0 + plane + lo_off + tid);
        if (has_hi) hhi = ld.load(b0 + plane + hi_off + tid);
    }
    __syncthreads();
    for (int z = z0; z < z1; ++z) {
        const int cur = (z - z0) & 1;
        const T *__restrict__ L = lds + cur * ldsz;
        const long b = (long)z * plane + (long)y0 * nx;
#pragma unroll
        for (int s = 0; s < PPT; ++s) {
            if (!val[s]) continue;
            const int t = tid + s * kThreads;
            const int x = xs[s];
            const T xm = x > 0 ? L[nx + t - 1] : T(0);
            const T xp = x < nx - 1 ? L[nx + t + 1] : T(0);
            const T ym = L[t];
            const T yp = L[t + 2 * nx];
            const T hv = (c0 + vsr[s]) * oc[s] -
                         kap * (ihx2 * (xm + xp) + ihy2 * (ym + yp) + ihz2 * (om[s] + op[s]));
            ep(s, b + t, oc[s], hv, er[s]);
        }
        if (z + 1 < z1) {
            T *__restrict__ Ln = lds + (cur ^ 1) * ldsz;
            const long bn = b + plane;
#pragma unroll
            for (int s = 0; s < PPT; ++s) {
                const int t = tid + s * kThreads;
                if (val[s]) Ln[nx + t] = op[s];
            }
            if (hown) {
                Ln[tid] = has_lo ? ld.make(hlo) : T(0);
                Ln[(ty + 1) * nx + tid] = has_hi ? ld.make(hhi) : T(0);
            }
            for (int hh = tid + kThreads; hh < nx; hh += kThreads) {  // nx > 256 only
                Ln[hh] = has_lo ? ld.make(ld.load(bn + lo_off + hh)) : T(0);
                Ln[(ty + 1) * nx + hh] = has_hi ? ld.make(ld.load(bn + hi_off + hh)) : T(0);
            }
#pragma unroll
            for (int s = 0; s < PPT; ++s) {
                const int t = tid + s * kThreads;
                om[s] = oc[s];
                oc[s] = op[s];
                op[s] = (val[s] && z + 2 < nz) ? ld.make(rq[s]) : T(0);
            }
            // issue the loads the next iterations consume
#pragma unroll
            for (int s = 0; s < PPT; ++s) {
                const int t = tid + s * kThreads;
                vsr[s] = val[s] ? vs[bn + t] : T(0);
                er[s] = val[s] ? ep.load(bn + t) : Ep::zero();
                rq[s] = (val[s] && z + 3 < nz && z + 2 < z1) ? ld.load(bn + 2 * plane + t)
                                                              : Ld::zero();
            }
            if (hown && z + 2 < z1) {
                if (has_lo) hlo = ld.load(bn + plane + lo_off + tid);
                if (has_hi) hhi = ld.load(bn + plane + hi_off + tid);
            }
        }
        __syncthreads();
    }
}

// The streaming engine.
//
//   Ld: stencil operand.   Ld::Raw raw = ld.load(i);  T v = ld.make(raw)
//   Ep: per-point epilogue. Ep::Raw e = ep.load(i);   ep(s, i, centre, Hv, e)
//
// Software pipeline over z-planes: while plane z is computed, the raw global
// loads of the operand of plane z+3 (own points), of the halo rows of plane
// z+2, and of V+sigma and the epilogue inputs of plane z+1 are in flight.  The
// per-plane barrier waits on LDS only, so those loads overlap the barrier and
// the next plane's arithmetic instead of stalling each plane.
template <typename T, int PPT, bool PP = true, class Ld, class Ep>
__device__ __forceinline__ void engine(const Grid &g, int band, int zc,
                                       const T *__restrict__ vs, Ld &ld, Ep &ep,
                                       T *__restrict__ lds) {
    if constexpr (PPT >= 4) {
        engine_wide<T, PPT>(g, band, zc, vs, ld, ep, lds);
        return;
    }
    using LR = typename Ld::Raw;
    using ER = typename Ep::Raw;
    const int tid = threadIdx.x;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const TileExtent te = g.extent(band * g.nzc + zc);
    const int y0 = te.y0, ty = te.ty, z0 = te.z0, z1 = te.z1;
    const int npts = ty * nx;
    const long plane = (long)nx * ny;
    const int ldsz = (g.TY + 2) * nx;
    const bool has_lo = y0 > 0, has_hi = (y0 + ty) < ny;
    const bool hown = tid < nx;  // this thread owns halo column tid (prefetched)
    const T kap = (T)g.kappa, c0 = (T)g.c0;
    const T ihx2 = (T)g.ihx2, ihy2 = (T)g.ihy2, ihz2 = (T)g.ihz2;
    const long lo_off = -(long)nx, hi_off = (long)ty * nx;

    int xs[PPT];
    bool val[PPT];
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
        const int t = tid + s * kThreads;
        val[s] = t < npts;
        xs[s] = val[s] ? t % nx : 0;
    }
    T om[PPT], oc[PPT], op[PPT];
    // Prefetched values.  PP: two sets used in turn by even and odd planes, so that no
    // loop-carried register is ever copied (a copy would wait for the load still in
    // flight); otherwise one set (fewer registers, higher occupancy).
    struct Pf {
        T vsr[PPT];   // V + sigma of the next plane
        ER er[PPT];   // epilogue inputs of the next plane
        LR rq[PPT];   // operand of the plane after the one staged next
        LR hlo, hhi;  // halo rows of the plane staged next
    } pa, pb;
    const long b0 = (long)z0 * plane + (long)y0 * nx;
    // prologue: operands of planes z0-1, z0 (with halo rows), z0+1
#pragma unroll
    for (int s = 0; s < PPT; ++s) {
        const int t = tid + s * kThreads;
        om[s] = (val[s] && z0 > 0) ? ld.make(ld.load(b0 - plane + t)) : T(0);
        oc[s] = val[s] ? ld.make(ld.load(b0 + t)) : T(0);
        op[s] = (val[s] && z0 + 1 < nz) ? ld.make(ld.load(b0 + plane + t)) : T(0);
        if (val[s]) lds[nx + t] = oc[s];
    }
    for (int hh = tid; hh < nx; hh += kThreads) {
        lds[hh] = has_lo ? ld.make(ld.load(b0 + lo_off + hh)) : T(0);
        lds[(ty + 1) * nx + hh] = has_hi ? ld.make(ld.load(b0 + hi_off + hh)) : T(0);
    }
    // Every load from here on is unconditional: a point past the tile's end reads the
    // tile's first point, a plane past the column's end reads the last plane, a halo row
    // that does not exist reads the tile's own row (halo columns past nx: column 0), and
    // the value is dropped at its use.  (Lane offsets below 256 * PPT let the loads take
    // a scalar base plus a 32-bit lane offset.)  Loads under a branch would end in registers
    // merged at the join, and the copies of such a merge wait for the loads in flight.
    int tc[PPT];
#pragma unroll
    for (int s = 0; s < PPT; ++s) tc[s] = val[s] ? tid + s * kThreads : 0;
    const int hx = hown ? tid : 0;
    const long hlo_off = has_lo ? lo_off : 0, hhi_off = has_hi ? hi_off : 0;
    const long yb = (long)y0 * nx;
    // loads for the iteration after plane z: V + sigma and epilogue inputs of plane z+1,
    // the operand of plane z+3 and the halo rows of plane z+2
    auto prefetch = [&](int z, Pf &f) {
        const long bv = (long)min(z + 1, nz - 1) * plane + yb;
        const long bq = (long)min(z + 3, nz - 1) * plane + yb;
        const long bh = (long)min(z + 2, nz - 1) * plane + yb;
#pragma unroll
        for (int s = 0; s < PPT; ++s) {
            f.vsr[s] = vs[bv + tc[s]];
            f.er[s] = ep.load(bv + tc[s]);
            f.rq[s] = ld.load(bq + tc[s]);
        }
        f.hlo = ld.load(bh + hlo_off + hx);
        f.hhi = ld.load(bh + hhi_off + hx);
    };
    prefetch(z0 - 1, pa);
    __syncthreads();
    // the stencil at plane z from LDS buffer L and the z-registers, and the epilogue
    auto plane_out = [&](int z, const T *__restrict__ L, const Pf &cu) {
        const long b = (long)z * plane + yb;
#pragma unroll
        for (int s = 0; s < PPT; ++s) {
            if (!val[s]) continue;
            const int t = tid + s * kThreads;
            const int x = xs[s];
            const T xm = x > 0 ? L[nx + t - 1] : T(0);
            const T xp = x < nx - 1 ? L[nx + t + 1] : T(0);
            const T ym = L[t];
            const T yp = L[t + 2 * nx];
            const T hv = (c0 + cu.vsr[s]) * oc[s] -
                         kap * (ihx2 * (xm + xp) + ihy2 * (ym + yp) + ihz2 * (om[s] + op[s]));
            ep(s, b + t, oc[s], hv, cu.er[s]);
        }
    };
    if (z1 - z0 == 1) {  // a single plane (2-D grids)
        plane_out(z0, lds, pa);
        __syncthreads();
        return;
    }
    // Plane z (epilogue only when live), then plane z+1 staged into the other LDS buffer,
    // the z-registers moved on, and the next loads issued into set nx_.
    auto step = [&](int z, bool live, const Pf &cu, Pf &nx_) {
        const int cur = (z - z0) & 1;
        const long b = (long)z * plane + yb;
        if (live) plane_out(z, lds + cur * ldsz, cu);
        // stage plane z+1 (past the last plane: into a buffer not read again)
        T *__restrict__ Ln = lds + (cur ^ 1) * ldsz;
#pragma unroll
        for (int s = 0; s < PPT; ++s) {
            const int t = tid + s * kThreads;
            if (val[s]) Ln[nx + t] = op[s];
        }
        if (hown) {
            Ln[tid] = has_lo ? ld.make(cu.hlo) : T(0);
            Ln[(ty + 1) * nx + tid] = has_hi ? ld.make(cu.hhi) : T(0);
        }
#pragma unroll
        for (int s = 0; s < PPT; ++s) {
            om[s] = oc[s];
            oc[s] = op[s];
            op[s] = (val[s] && z + 2 < nz) ? ld.make(cu.rq[s]) : T(0);
        }
        if (z + 1 < z1) {
            const long bn = b + plane;
            for (int hh = tid + kThreads; hh < nx; hh += kThreads) {  // nx > 256 only
                Ln[hh] = has_lo ? ld.make(ld.load(bn + lo_off + hh)) : T(0);
                Ln[(ty + 1) * nx + hh] = has_hi ? ld.make(ld.load(bn + hi_off + hh)) : T(0);
            }
        }
        // one set: the loads must not be moved above the last uses of the old values
        if constexpr (!PP) __builtin_amdgcn_sched_barrier(0);
        prefetch(z, nx_);
        __syncthreads();
    };
    if constexpr (!PP) {
        // One prefetch set, refilled in every iteration (the last one too: clamped,
        // unused), so the back edge is reached only with freshly loaded registers.
        for (int z = z0; z < z1; ++z) step(z, true, pa, pa);
    } else {
        // Two sets in turn: one plane's loads go to the set the previous plane has
        // finished with.  Planes in pairs; an odd count ends with a pass whose epilogue is
        // off (its loads are clamped, its staging goes to a buffer not read again).
        for (int z = z0; z < z1; z += 2) {
            step(z, true, pa, pb);
            step(z + 1, z + 1 < z1, pb, pa);
        }
    }
}

// ---- operand loaders and epilogue building blocks

template <typename T>
struct LdPlain {  // operand x[i]
    struct Raw { T x; };
    const T *__restrict__ x;
    __device__ static Raw zero() { return {T(0)}; }
    __device__ Raw load(long i) const { return {x[i]}; }
    __device__ T make(const Raw &r) const { return r.x; }
};

template <typename T>
struct LdZero {  // operand 0 (no loads)
    struct Raw {};
    __device__ static Raw zero() { return {}; }
    __device__ Raw load(long) const { return {}; }
    __device__ T make(const Raw &) const { return T(0); }
};

template <typename T>
struct LdPcgP {  // p = D r + beta p_old  (beta = 0: p = D r, p_old not read)
    struct Raw { T d, r, p; };
    const T *__restrict__ dinv;
    const T *__restrict__ r;
    const T *__restrict__ po;
    T beta;
    bool first;
    __device__ static Raw zero() { return {T(0), T(0), T(0)}; }
    __device__ Raw load(long i) const { return {dinv[i], r[i], first ? T(0) : po[i]}; }
    __device__ T make(const Raw &a) const {
        const T z = a.d * a.r;
        return first ? z : z + beta * a.p;
    }
};

template <typename T>
struct LdPcgZ {  // p = z + beta p_old with an explicit preconditioned residual z (FP32)
    struct Raw { float z; T p; };
    const float *__restrict__ z;
    const T *__restrict__ po;
    T beta;
    bool first;
    __device__ static Raw zero() { return {0.f, T(0)}; }
    __device__ Raw load(long i) const { return {z[i], first ? T(0) : po[i]}; }
    __device__ T make(const Raw &a) const { return first ? (T)a.z : (T)a.z + beta * a.p; }
};

struct NoRaw {};

// Workgroup -> (column, tile) of an ncols x tiles launch (stencil_tile_of).
__device__ __forceinline__ void tile_of(const Grid &g, int &col, int &tile, int &band, int &zc) {
    const int tiles = g.tiles();
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    stencil_tile_of(L, (int)(gridDim.x / tiles), tiles, col, tile);
    const TileExtent e = g.extent(tile);
    band = e.band;
    zc = e.zc;
}

// Per-point array of a column's instance (see Grid::cinst).
template <typename T>
__device__ __forceinline__ const T *col_pt(const Grid &g, const T *p, int col) {
    return (g.cinst && p) ? p + (long)g.cinst[col] * g.ng : p;
}

template <typename T>
__device__ __forceinline__ T *lds_ptr() {
    extern __shared__ __align__(16) unsigned char qo_smem[];
    return reinterpret_cast<T *>(qo_smem);
}

// ---------------------------------------------------------------- kernels

template <int PPT>
__global__ __launch_bounds__(kThreads) void k_apply(Grid g, const double *__restrict__ vs,
                                                    const double *__restrict__ X,
                                                    double *__restrict__ Y, long ld) {
    int col, tile, band, zc;
    tile_of(g, col, tile, band, zc);
    vs = col_pt(g, vs, col);
    struct Ep {
        using Raw = NoRaw;
        double *__restrict__ y;
        __device__ static Raw zero() { return {}; }
        __device__ Raw load(long) const { return {}; }
        __device__ void operator()(int, long i, double, double hv, const Raw &) { y[i] = hv; }
    } ep{Y + (long)col * ld};
    LdPlain<double> l{X + (long)col * ld};
    engine<double, PPT>(g, band, zc, vs, l, ep, lds_ptr<double>());
}

template <int PPT>
__global__ __launch_bounds__(kThreads) void k_quad(Grid g, const double *__restrict__ vs,
                                                   const double *__restrict__ X, long ld,
                                                   double *__restrict__ part, long qs) {
    __shared__ Red red;
    int col, tile, band, zc;
    tile_of(g, col, tile, band, zc);
    vs = col_pt(g, vs, col);
    struct Ep {
        using Raw = NoRaw;
        double acc[2];
        __device__ static Raw zero() { return {}; }
        __device__ Raw load(long) const { return {}; }
        __device__ void operator()(int, long, double c, double hv, const Raw &) {
            acc[0] += c * hv;
            acc[1] += c * c;
        }
    } ep{{0.0, 0.0}};
    LdPlain<double> l{X + (long)col * ld};
    engine<double, PPT>(g, band, zc, vs, l, ep, lds_ptr<double>());
    block_sums<2>(ep.acc, red);
    if (threadIdx.x == 0) {
        const long o = (long)col * g.tiles() + tile;
        part[o] = ep.acc[0];
        part[qs + o] = ep.acc[1];
    }
}

template <int PPT>
__global__ __launch_bounds__(kThreads) void k_resid(Grid g, const double *__restrict__ vs,
                                                    const double *__restrict__ B,
                                                    const double *__restrict__ X, long ld,
                                                    float *__restrict__ R32, long ld32,
                                                    const int *__restrict__ mask,
                                                    double *__restrict__ part, long qs) {
    __shared__ Red red;
    int col, tile, band, zc;
    tile_of(g, col, tile, band, zc);
    vs = col_pt(g, vs, col);
    const long o = (long)col * g.tiles() + tile;
    if (mask && !mask[col]) {
        if (threadIdx.x == 0) part[qs + o] = part[2 * qs + o] = 0.0;
        return;
    }
    struct Ep {
        struct Raw { double b; };
        const double *__restrict__ b;
        float *__restrict__ r32;
        double acc[2];
        __device__ static Raw zero() { return {0.0}; }
        __device__ Raw load(long i) const { return {b[i]}; }
        __device__ void operator()(int, long i, double, double hv, const Raw &e) {
            const double r = e.b - hv;
            r32[i] = (float)r;
            acc[0] += r * r;
            acc[1] += e.b * e.b;
        }
    } ep{B + (long)col * ld, R32 + (long)col * ld32, {0.0, 0.0}};
    LdPlain<double> l{X + (long)col * ld};
    engine<double, PPT>(g, band, zc, vs, l, ep, lds_ptr<double>());
    block_sums<2>(ep.acc, red);
    if (threadIdx.x == 0) {
        part[qs + o] = ep.acc[0];
        part[2 * qs + o] = ep.acc[1];
    }
}

// The refinement update and the next residual in one pass, out of place: for every column
// x_new = x + d where the last inner solve updated d (upd: mask[c] and its[c] > 0), else
// x_new = x; then r = b - H x_new in FP64, r32 = (float) r, partials rr, bb.  x and d are
// only read (the stencil forms x + d at the halo points too), x_new goes to its own block,
// so no workgroup reads a value another one is changing.
// With zb, x_new rounded to BF16 (nearest-even) also goes to the row-blocked BF16 copy of
// an zn-column block (the Gram operand of the solution block: the last pass of a solve
// leaves it holding the solution).
template <int PPT, bool ZB>
__global__ __launch_bounds__(kThreads) void k_resid_next(Grid g, const double *__restrict__ vs,
                                                         const double *__restrict__ B,
                                                         const double *__restrict__ X,
                                                         const float *__restrict__ D,
                                                         double *__restrict__ Xn, long ld,
                                                         float *__restrict__ R32,
                                                         const int *__restrict__ mask,
                                                         const int *__restrict__ its,
                                                         double *__restrict__ part, long qs,
                                                         __bf16 *__restrict__ zb, int zn) {
    __shared__ Red red;
    int col, tile, band, zc;
    tile_of(g, col, tile, band, zc);
    vs = col_pt(g, vs, col);
    const long o = (long)col * g.tiles() + tile;
    struct LdNext {  // operand x + d (d dropped in the columns left alone; loaded anyway)
        struct Raw { double x; float d; };
        const double *__restrict__ x;
        const float *__restrict__ d;
        bool upd;
        __device__ static Raw zero() { return {0.0, 0.f}; }
        __device__ Raw load(long i) const { return {x[i], d[i]}; }
        // a select, not a product with 0: d of a column left alone may hold anything
        __device__ double make(const Raw &r) const { return r.x + (upd ? (double)r.d : 0.0); }
    };
    struct Ep {
        struct Raw { double b; };
        const double *__restrict__ b;
        double *__restrict__ xn;
        float *__restrict__ r32;
        __bf16 *__restrict__ zb;
        int col, zn;
        double acc[2];
        __device__ static Raw zero() { return {0.0}; }
        __device__ Raw load(long i) const { return {b[i]}; }
        __device__ void operator()(int, long i, double c, double hv, const Raw &e) {
            const double r = e.b - hv;
#if QO_RESID_NT  // x' and r32 are read again only after the next passes over the block
            __builtin_nontemporal_store(c, xn + i);
            __builtin_nontemporal_store((float)r, r32 + i);
#else
            xn[i] = c;
            r32[i] = (float)r;
#endif
            if constexpr (ZB) zb[bf16_rowblock_index(i, col, zn)] = dev::f64_to_bf16_rne(c);
            acc[0] += r * r;
            acc[1] += e.b * e.b;
        }
    } ep{B + (long)col * ld, Xn + (long)col * ld, R32 + (long)col * ld, zb, col, zn, {0.0, 0.0}};
    const bool upd = mask[col] != 0 && its[col] > 0;
    LdNext l{X + (long)col * ld, D + (long)col * ld, upd};
    engine<double, PPT>(g, band, zc, vs, l, ep, lds_ptr<double>());
    block_sums<2>(ep.acc, red);
    if (threadIdx.x == 0) {
        part[qs + o] = ep.acc[0];
        part[2 * qs + o] = ep.acc[1];
    }
}

// Residual replacement of the mixed-precision solve (reliable update): for the
// columns with mask != 0, r = b - H x in FP64, r32 = (float) r.  Partials in the
// FP32 PCG layout: q0 = r32 . D32 r32, q1 = q2 = ||r32||^2; and in `outer`:
// [0] ||r||^2 (FP64), [1] ||b||^2.  Unmasked columns are untouched.
template <int PPT>
__global__ __launch_bounds__(kThreads) void k_resid_rel(Grid g, const double *__restrict__ vs,
                                                        const float *__restrict__ dinv32,
                                                        const double *__restrict__ B,
                                                        const double *__restrict__ X, long ld,
                                                        float *__restrict__ R32,
                                                        const int *__restrict__ mask,
                                                        double *__restrict__ part, long qs,
                                                        double *__restrict__ outer) {
    __shared__ Red red;
    int col, tile, band, zc;
    tile_of(g, col, tile, band, zc);
    vs = col_pt(g, vs, col);
    dinv32 = col_pt(g, dinv32, col);
    if (!mask[col]) return;
    struct Ep {
        struct Raw { double b; float d; };
        const double *__restrict__ b;
        const float *__restrict__ dinv;
        float *__restrict__ r32;
        double acc[4];
        __device__ static Raw zero() { return {0.0, 0.f}; }
        __device__ Raw load(long i) const { return {b[i], dinv[i]}; }
        __device__ void operator()(int, long i, double, double hv, const Raw &e) {
            const double r = e.b - hv;
            const float rf = (float)r;
            r32[i] = rf;
            acc[0] += (double)rf * (double)(e.d * rf);
            acc[1] += (double)rf * (double)rf;
            acc[2] += r * r;
            acc[3] += e.b * e.b;
        }
    } ep{B + (long)col * ld, dinv32, R32 + (long)col * ld, {0.0, 0.0, 0.0, 0.0}};
    LdPlain<double> l{X + (long)col * ld};
    engine<double, PPT>(g, band, zc, vs, l, ep, lds_ptr<double>());
    block_sums<4>(ep.acc, red);
    if (threadIdx.x == 0) {
        const long o = (long)col * g.tiles() + tile;
        part[o] = ep.acc[0];
        part[qs + o] = ep.acc[1];
        part[2 * qs + o] = ep.acc[1];
        outer[o] = ep.acc[2];
        outer[qs + o] = ep.acc[3];
    }
}

// r = b - H x0 (or r = b, x = 0); partials rz (q0), rr (q1), bb (q2)
template <typename T>
struct EpInit {
    struct Raw { T b, d; };
    const T *__restrict__ b;
    const T *__restrict__ dinv;
    T *__restrict__ x;
    T *__restrict__ r;
    bool use_x0;
    double acc[3];
    __device__ static Raw zero() { return {T(0), T(0)}; }
    __device__ Raw load(long i) const { return {b[i], dinv[i]}; }
    __device__ void operator()(int, long i, T, T hv, const Raw &e) {
        T ri;
        if (use_x0) {
            ri = e.b - hv;
        } else {
            ri = e.b;
            x[i] = T(0);
        }
        r[i] = ri;
        const double rd = (double)ri;
        acc[0] += rd * (double)(e.d * ri);
        acc[1] += rd * rd;
        acc[2] += (double)e.b * (double)e.b;
    }
};

template <typename T, int PPT>
__global__ __launch_bounds__(kThreads) void k_pcg_init(Grid g, const T *__restrict__ vs,
                                                       const T *__restrict__ dinv,
                                                       const T *__restrict__ B,
                                                       T *__restrict__ X, T *__restrict__ R,
                                                       long ld, int use_x0,
                                                       double *__restrict__ part, long qs) {
    __shared__ Red red;
    int col, tile, band, zc;
    tile_of(g, col, tile, band, zc);
    vs = col_pt(g, vs, col);
    dinv = col_pt(g, dinv, col);
    EpInit<T> ep{B + (long)col * ld, dinv, X + (long)col * ld, R + (long)col * ld,
                 use_x0 != 0, {0.0, 0.0, 0.0}};
    if (use_x0) {
        LdPlain<T> l{X + (long)col * ld};
        engine<T, PPT>(g, band, zc, vs, l, ep, lds_ptr<T>());
    } else {
        LdZero<T> l;
        engine<T, PPT>(g, band, zc, vs, l, ep, lds_ptr<T>());
    }
    block_sums<3>(ep.acc, red);
    if (threadIdx.x == 0) {
        const long o = (long)col * g.tiles() + tile;
        part[o] = ep.acc[0];
        part[qs + o] = ep.acc[1];
        part[2 * qs + o] = ep.acc[2];
    }
}

// store p, gamma = p . H p.  p is stored non-temporally: the next kernel reads it from
// HBM anyway, and the store then leaves the cache to the halo rows of this sweep's operand.
template <typename T>
struct EpSweep1 {
    using Raw = NoRaw;
    T *__restrict__ pn;
    double acc[1];
    __device__ static Raw zero() { return {}; }
    __device__ Raw load(long) const { return {}; }
    __device__ void operator()(int, long i, T c, T hv, const Raw &) {
#if QO_SWEEP1_NT
        __builtin_nontemporal_store(c, pn + i);
#else
        pn[i] = c;
#endif
        acc[0] += (double)c * (double)hv;
    }
};

// MODE 0: Jacobi, z = D r formed on the fly, r.z from sweep2's partials.
// MODE 1: the preconditioned residual z is an input (fast-Poisson preconditioner) and
//         r.z comes from the preconditioner's partials rzp (rzt per column).
// MODE 2: as 1, but the inverse preconditioner pass has already formed p = z + beta p_old
//         (in Pnew) and r.z per column is rzp[c] (rzt == 1): the sweep only reads p for
//         gamma and the bookkeeping; nothing is stored.
// FP32 with z as input at 3 points per thread: capped to six waves per SIMD, which spills
// a few registers of the two prefetch sets and is still faster than the five waves that
// fit without spills (96^3 x 256: 423 against 456 us).
template <typename T, int PPT, int MODE>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && MODE == 1 && PPT == 3 ? 6 : 1))) void k_pcg_sweep1(Grid g, const T *__restrict__ vs,
                                                         const T *__restrict__ dinv,
                                                         const T *__restrict__ R,
                                                         const T *__restrict__ Pold,
                                                         T *__restrict__ Pnew, long ld, int ncols,
                                                         int k, double tol,
                                                         const int *__restrict__ mask,
                                                         PcgState s, long qs,
                                                         const float *__restrict__ Z,
                                                         const double *__restrict__ rzp, int rzt) {
    __shared__ Red red;
    __shared__ int sh_flag;
    int col, tile, band, zc;
    tile_of(g, col, tile, band, zc);
    vs = col_pt(g, vs, col);
    dinv = col_pt(g, dinv, col);
    const bool lead = tile == 0;
    const int cur = k & 1, prv = cur ^ 1;
    const int tiles = g.tiles();
    int prev_active = (k == 0) ? (mask ? mask[col] : 1) : s.active[prv * ncols + col];
    if (!prev_active) {
        if (lead && threadIdx.x == 0) s.active[cur * ncols + col] = 0;
        return;
    }
    const double rr = col_sum(s.part + qs, col, tiles, red);
    double bb;
    if (k == 0) {
        bb = col_sum(s.part + 2 * qs, col, tiles, red);
        if (lead && threadIdx.x == 0) s.bb[col] = bb;
    } else {
        bb = s.bb[col];
    }
    const double ctol = s.coltol ? s.coltol[col] : tol;
    // the convergence test first: a converged column's z is not computed
    const bool conv = sqrt(rr) <= ctol * sqrt(bb);
    constexpr bool XZ = MODE != 0;
    const double rz = (XZ && conv) ? 0.0
                      : MODE == 2 ? rzp[col]
                      : (XZ ? col_sum(rzp, col, rzt, red) : col_sum(s.part, col, tiles, red));
    if (threadIdx.x == 0) {
        int flag = 0;  // 0 run, 1 converged, 2 non-finite
        if (!isfinite(rz) || !isfinite(rr) || !isfinite(bb)) flag = 2;
        else if (conv) flag = 1;
        sh_flag = flag;
        if (lead) {
            s.its[col] = k;
            s.active[cur * ncols + col] = flag == 0 ? 1 : 0;
            if (flag == 0) s.rho[cur * ncols + col] = rz;
            if (flag == 2) {
                atomicMax(&s.err[0], 7);
                atomicMin(&s.err[1], col);
            }
        }
    }
    __syncthreads();
    if (sh_flag != 0) return;
    if constexpr (MODE == 2) {
        struct Ep {
            using Raw = NoRaw;
            double acc[1];
            __device__ static Raw zero() { return {}; }
            __device__ Raw load(long) const { return {}; }
            __device__ void operator()(int, long, T c, T hv, const Raw &) {
                acc[0] += (double)c * (double)hv;
            }
        } ep{{0.0}};
        LdPlain<T> l{Pnew + (long)col * ld};
        engine<T, PPT>(g, band, zc, vs, l, ep, lds_ptr<T>());
        block_sums<1>(ep.acc, red);
        if (threadIdx.x == 0) s.part[3 * qs + (long)col * tiles + tile] = ep.acc[0];
        return;
    }
    const T beta = (k == 0) ? T(0) : (T)(rz / s.rho[prv * ncols + col]);
    EpSweep1<T> ep{Pnew + (long)col * ld, {0.0}};
    if constexpr (XZ) {
        LdPcgZ<T> l{Z + (long)col * ld, Pold + (long)col * ld, beta, k == 0};
        engine<T, PPT>(g, band, zc, vs, l, ep, lds_ptr<T>());
    } else {
        LdPcgP<T> l{dinv, R + (long)col * ld, Pold + (long)col * ld, beta, k == 0};
        engine<T, PPT>(g, band, zc, vs, l, ep, lds_ptr<T>());
    }
    block_sums<1>(ep.acc, red);
    if (threadIdx.x == 0) s.part[3 * qs + (long)col * tiles + tile] = ep.acc[0];
}

// The first sweep's work for the FP32 PCG whose preconditioner pass has formed
// p = z + beta p_old, without a pass over the grid: one block per column takes the stop
// test, the iteration count and activity flag, rho = r.z (rzc, from the preconditioner), and
// gamma = p.Hp from identities of the iteration:
//   H p_old = (r_old - r) / alpha_old (the residual recurrence), z.r_old = 0 (successive
//   residuals are M^{-1}-orthogonal), z.M z = r.z (z = M^{-1} r) and H - M = diag(w),
//   w = V + sigma - vbar, so that
//   gamma = rho + sum w z^2 - 2 beta rho / alpha_old + beta^2 gamma_old,
// with sum w z^2 from the preconditioner's inverse pass (wzp, nslab partials per column) and
// gamma_old = p_old.H p_old from the previous second sweep (partials in section 0).  The
// identities hold up to the preconditioner's FP16 rounding (about 1e-3 relative), like
// the spectral r.z; the second sweep's update uses gamma as given.  gamma is written to
// slot 0 of the column's partials (the others zero), so the second sweep's reduction
// returns it unchanged, and alpha = rho / gamma is kept for the next iteration.
__global__ __launch_bounds__(kThreads) void k_pcg_gamma(int k, int ncols, double tol,
                                                        const int *__restrict__ mask,
                                                        PcgState s, long qs, int tiles,
                                                        const double *__restrict__ rzc,
                                                        const double *__restrict__ wzp,
                                                        int nslab) {
    __shared__ Red red;
    const int col = blockIdx.x;
    const int cur = k & 1, prv = cur ^ 1;
    const int prev_active = (k == 0) ? (mask ? mask[col] : 1) : s.active[prv * ncols + col];
    if (!prev_active) {
        if (threadIdx.x == 0) s.active[cur * ncols + col] = 0;
        return;
    }
    const double rr = col_sum(s.part + qs, col, tiles, red);
    double bb;
    if (k == 0) {
        bb = col_sum(s.part + 2 * qs, col, tiles, red);
        if (threadIdx.x == 0) s.bb[col] = bb;
    } else {
        bb = s.bb[col];
    }
    const double ctol = s.coltol ? s.coltol[col] : tol;
    const bool conv = sqrt(rr) <= ctol * sqrt(bb);
    const double wz = conv ? 0.0 : col_sum(wzp, col, nslab, red);
    const double gold = (conv || k == 0) ? 0.0 : col_sum(s.part, col, tiles, red);
    if (threadIdx.x == 0) {
        const double rz = conv ? 0.0 : rzc[col];
        int flag = 0;  // 0 run, 1 converged, 2 non-finite
        if (!isfinite(rz) || !isfinite(rr) || !isfinite(bb)) flag = 2;
        else if (conv) flag = 1;
        s.its[col] = k;
        s.active[cur * ncols + col] = flag == 0 ? 1 : 0;
        if (flag == 2) {
            atomicMax(&s.err[0], 7);
            atomicMin(&s.err[1], col);
        }
        if (flag == 0) {
            double gam = rz + wz;
            if (k > 0) {
                const double b = rz / s.rho[prv * ncols + col];
                gam += -2.0 * b * rz / s.alpha[prv * ncols + col] + b * b * gold;
            }
            s.rho[cur * ncols + col] = rz;
            s.alpha[cur * ncols + col] = rz / gam;
            double *g = s.part + 3 * qs + (long)col * tiles;
            g[0] = gam;
            for (int t = 1; t < tiles; ++t) g[t] = 0.0;
        }
    }
}

// x += alpha p; r -= alpha H p; partials r.D r (JAC: Jacobi form; else p.Hp) and r.r.
// x and r are each read and written once per sweep: non-temporal accesses keep
// them from evicting the stencil operand's halo rows from the caches.
// XZ: x is known to be zero (the first iteration of a solve that starts from x = 0 without
// an init pass): it is written, not read.
template <typename T, bool JAC, bool XZ = false>
struct EpSweep2 {
    struct Raw { T x, r, d; };
    T *__restrict__ x;
    T *__restrict__ r;
    const T *__restrict__ dinv;
    T alpha;
    double acc[2];
    __device__ static Raw zero() { return {T(0), T(0), T(0)}; }
    __device__ Raw load(long i) const {
#if QO_SWEEP2_NT
        return {XZ ? T(0) : __builtin_nontemporal_load(x + i), __builtin_nontemporal_load(r + i),
                JAC ? dinv[i] : T(0)};
#else
        return {XZ ? T(0) : x[i], r[i], JAC ? dinv[i] : T(0)};
#endif
    }
    __device__ void operator()(int, long i, T c, T hv, const Raw &e) {
        const T ri = e.r - alpha * hv;
#if QO_SWEEP2_NT
        __builtin_nontemporal_store(e.x + alpha * c, x + i);
        __builtin_nontemporal_store(ri, r + i);
#else
        x[i] = e.x + alpha * c;
        r[i] = ri;
#endif
        const double rd = (double)ri;
        // Jacobi form: r.D r; preconditioned form: p.Hp with the Hp of this update, the
        // exact gamma of the iteration (the next one's gamma identity uses it)
        if (JAC) acc[0] += rd * (double)(e.d * ri);
        else acc[0] += (double)c * (double)hv;
        acc[1] += rd * rd;
    }
};

// FP32 without the Jacobi term at 3 points per thread: one prefetch set, capped to six
// waves per SIMD (80 registers; one spill).
template <typename T, int PPT, bool JAC, bool XZ = false>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 && !JAC && PPT == 3 ? 6 : 1))) void k_pcg_sweep2(Grid g, const T *__restrict__ vs,
                                                         const T *__restrict__ dinv,
                                                         const T *__restrict__ Pn,
                                                         T *__restrict__ X, T *__restrict__ R,
                                                         long ld, int ncols, int k, PcgState s,
                                                         long qs) {
    __shared__ Red red;
    __shared__ int sh_flag;
    int col, tile, band, zc;
    tile_of(g, col, tile, band, zc);
    vs = col_pt(g, vs, col);
    dinv = col_pt(g, dinv, col);
    const int cur = k & 1;
    const int tiles = g.tiles();
    if (!s.active[cur * ncols + col]) return;
    const double gam = col_sum(s.part + 3 * qs, col, tiles, red);
    if (threadIdx.x == 0) {
        int flag = 0;
        if (!isfinite(gam)) flag = 7;
        else if (!(gam > 0.0)) flag = 5;
        sh_flag = flag;
        if (flag && tile == 0) {
            atomicMax(&s.err[0], flag);
            atomicMin(&s.err[1], col);
        }
    }
    __syncthreads();
    if (sh_flag) return;
    const T alpha = (T)(s.rho[cur * ncols + col] / gam);
    LdPlain<T> l{Pn + (long)col * ld};
    EpSweep2<T, JAC, XZ> ep{X + (long)col * ld, R + (long)col * ld, dinv, alpha, {0.0, 0.0}};
    // FP32: one prefetch set (measured faster here: the second set costs occupancy)
    engine<T, PPT, sizeof(T) == 8>(g, band, zc, vs, l, ep, lds_ptr<T>());
    block_sums<2>(ep.acc, red);
    if (threadIdx.x == 0) {
        const long o = (long)col * tiles + tile;
        s.part[o] = ep.acc[0];
        s.part[qs + o] = ep.acc[1];
    }
}

// delta0 = u . H u with u = D r0 (one-reduction PCG start)
template <typename T, int PPT>
__global__ __launch_bounds__(kThreads) void k_cg_delta0(Grid g, const T *__restrict__ vs,
                                                        const T *__restrict__ dinv,
                                                        const T *__restrict__ R, long ld,
                                                        double *__restrict__ part, long qs) {
    __shared__ Red red;
    int col, tile, band, zc;
    tile_of(g, col, tile, band, zc);
    vs = col_pt(g, vs, col);
    dinv = col_pt(g, dinv, col);
    LdPcgP<T> l{dinv, R + (long)col * ld, nullptr, T(0), true};
    struct Ep {
        using Raw = NoRaw;
        double acc[1];
        __device__ static Raw zero() { return {}; }
        __device__ Raw load(long) const { return {}; }
        __device__ void operator()(int, long, T c, T hv, const Raw &) {
            acc[0] += (double)c * (double)hv;
        }
    } ep{{0.0}};
    engine<T, PPT>(g, band, zc, vs, l, ep, lds_ptr<T>());
    block_sums<1>(ep.acc, red);
    if (threadIdx.x == 0) part[3 * qs + (long)col * g.tiles() + tile] = ep.acc[0];
}

__global__ void k_colsum(const double *__restrict__ part, int tiles, int ncols, int nq, long qs,
                         double *__restrict__ out) {
    __shared__ Red red;
    const int c = blockIdx.x;
    for (int q = 0; q < nq; ++q) {
        const double v = col_sum(part + q * qs, c, tiles, red);
        if (threadIdx.x == 0) out[q * ncols + c] = v;
    }
}

__global__ void k_refine_axpy(double *__restrict__ X, long ld, float *__restrict__ D,
                              long ld32, long ng, const int *__restrict__ mask, int zero_d) {
    const int c = blockIdx.y;
    if (!mask[c]) return;
    double *x = X + (long)c * ld;
    float *d = D + (long)c * ld32;
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < ng;
         i += (long)gridDim.x * blockDim.x) {
        x[i] += (double)d[i];
        if (zero_d) d[i] = 0.f;
    }
}

// Reliable-update bookkeeping, one thread per column.
//   check:    need[c] = active[c] && (||r32|| < delta rref[c] || ||r32|| <= tol ||b||)
//   finalize: for need[c]: rref[c] = ||r||; ||r|| <= tol ||b|| -> active[c] = 0 (done)
__global__ void k_rel_check(const double *__restrict__ part, int tiles, long qs, int ncols,
                            const int *__restrict__ active, const double *__restrict__ rref,
                            const double *__restrict__ bb64, double delta, double tol,
                            int *__restrict__ need, int *__restrict__ nneed) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncols;
         c += gridDim.x * blockDim.x) {
        int m = 0;
        if (active[c]) {
            double rr = 0.0;
            for (int t = 0; t < tiles; ++t) rr += part[qs + (long)c * tiles + t];
            const double rn = sqrt(rr);
            m = (rn < delta * rref[c] || rn <= tol * sqrt(bb64[c]) || !isfinite(rn)) ? 1 : 0;
        }
        need[c] = m;
        if (m) atomicAdd(nneed, 1);
    }
}

__global__ void k_rel_finalize(const double *__restrict__ outer, int tiles, long qs, int ncols,
                               const int *__restrict__ need, int *__restrict__ active,
                               double *__restrict__ rref, double *__restrict__ bb64, double tol,
                               int init, int *__restrict__ nactive, int *__restrict__ err) {
    for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < ncols;
         c += gridDim.x * blockDim.x) {
        if (need[c]) {
            double rr = 0.0, bb = 0.0;
            for (int t = 0; t < tiles; ++t) {
                rr += outer[(long)c * tiles + t];
                bb += outer[qs + (long)c * tiles + t];
            }
            if (!isfinite(rr) || !isfinite(bb)) {
                atomicMax(&err[0], 7);
                atomicMin(&err[1], c);
            }
            rref[c] = sqrt(rr);
            if (init) bb64[c] = bb;
            const bool done = sqrt(rr) <= tol * sqrt(bb64[c]);
            active[c] = done ? 0 : 1;
        }
        if (active[c]) atomicAdd(nactive, 1);
    }
}

// sums: [0..ncols) = rr, [ncols..2ncols) = bb.  For active columns the inner
// tolerance is what the column still needs (with a safety factor), but no
// tighter than the FP32 floor tol_in: coltol = clamp(0.3 tol ||b|| / ||r||, tol_in, 0.5).
// tol is ctol[c] per column when ctol is given, else tol_all.
__global__ void k_refine_mask(const double *__restrict__ sums, int ncols, double tol_all,
                              double tol_in, int *__restrict__ mask,
                              double *__restrict__ coltol, int *__restrict__ nactive,
                              int *__restrict__ err, const double *__restrict__ ctol) {
    __shared__ int cnt;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    for (int c = threadIdx.x; c < ncols; c += blockDim.x) {
        const double rr = sums[c], bb = sums[ncols + c];
        const double tol = ctol ? ctol[c] : tol_all;
        int m = 0;
        if (!isfinite(rr) || !isfinite(bb)) {
            atomicMax(&err[0], 7);
            atomicMin(&err[1], c);
        } else {
            m = sqrt(rr) > tol * sqrt(bb) ? 1 : 0;
        }
        mask[c] = m;
        if (coltol) {
            double t = m ? 0.3 * tol * sqrt(bb) / sqrt(rr) : tol_in;
            coltol[c] = fmin(0.5, fmax(tol_in, t));
        }
        if (m) atomicAdd(&cnt, 1);
    }
    __syncthreads();
    if (threadIdx.x == 0) *nactive = cnt;
}

inline size_t lds_bytes(const Grid &g, size_t elem) { return 2 * (size_t)(g.TY + 2) * g.nx * elem; }

#define QO_DISPATCH_PPT(PPTV, ...)                        \
    switch (PPTV) {                                       \
        case 1: { constexpr int P = 1; __VA_ARGS__; } break; \
        case 2: { constexpr int P = 2; __VA_ARGS__; } break; \
        case 3: { constexpr int P = 3; __VA_ARGS__; } break; \
        case 4: { constexpr int P = 4; __VA_ARGS__; } break; \
        case 5: { constexpr int P = 5; __VA_ARGS__; } break; \
        case 6: { constexpr int P = 6; __VA_ARGS__; } break; \
        case 8: { constexpr int P = 8; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;               \
    }

}  // namespace

// Points per thread per plane of a band of `pts` points (the instantiated set), -1 if none.
int pick_ppt(int pts) {
    const int raw = (pts + kThreads - 1) / kThreads;
    const int opts[6] = {1, 2, 3, 4, 6, 8};
    for (int o : opts)
        if (o >= raw) return o;
    return -1;
}

hipError_t launch_apply(const Grid &g, const double *vs, const double *X, double *Y, long ld,
                        int ncols, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    const dim3 grid(ncols * g.tiles());
    QO_DISPATCH_PPT(g.ppt, hipLaunchKernelGGL(k_apply<P>, grid, dim3(kThreads),
                                               lds_bytes(g, 8), st, g, vs, X, Y, ld));
    return hipGetLastError();
}

hipError_t launch_quad(const Grid &g, const double *vs, const double *X, long ld, int ncols,
                       double *part, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    const long qs = (long)ncols * g.tiles();
    const dim3 grid(ncols * g.tiles());
    QO_DISPATCH_PPT(g.ppt, hipLaunchKernelGGL(k_quad<P>, grid, dim3(kThreads),
                                               lds_bytes(g, 8), st, g, vs, X, ld, part, qs));
    return hipGetLastError();
}

hipError_t launch_resid(const Grid &g, const double *vs, const double *B, const double *X,
                        long ld, float *R32, long ld32, int ncols, const int *mask, double *part,
                        hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    const long qs = (long)ncols * g.tiles();
    const dim3 grid(ncols * g.tiles());
    QO_DISPATCH_PPT(g.ppt, hipLaunchKernelGGL(k_resid<P>, grid, dim3(kThreads),
                                               lds_bytes(g, 8), st, g, vs, B, X, ld, R32, ld32,
                                               mask, part, qs));
    return hipGetLastError();
}

hipError_t launch_resid_next(const Grid &g, const double *vs, const double *B, const double *X,
                             const float *D, double *Xn, long ld, float *R32, int ncols,
                             const int *mask, const int *its, double *part, hipStream_t st,
                             __bf16 *zb, int zn) {
    if (ncols <= 0) return hipSuccess;
    if (zb && zn < ncols) return hipErrorInvalidValue;
    const long qs = (long)ncols * g.tiles();
    const dim3 grid(ncols * g.tiles());
    if (zb) {
        QO_DISPATCH_PPT(g.ppt, hipLaunchKernelGGL((k_resid_next<P, true>), grid, dim3(kThreads),
                                                   lds_bytes(g, 8), st, g, vs, B, X, D, Xn, ld,
                                                   R32, mask, its, part, qs, zb, zn));
    } else {
        QO_DISPATCH_PPT(g.ppt, hipLaunchKernelGGL((k_resid_next<P, false>), grid, dim3(kThreads),
                                                   lds_bytes(g, 8), st, g, vs, B, X, D, Xn, ld,
                                                   R32, mask, its, part, qs, zb, zn));
    }
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pcg_init(const Grid &g, const T *vs, const T *dinv, const T *B, T *X, T *R,
                           long ld, int ncols, int use_x0, double *part, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    const long qs = (long)ncols * g.tiles();
    const dim3 grid(ncols * g.tiles());
    QO_DISPATCH_PPT(g.ppt, hipLaunchKernelGGL((k_pcg_init<T, P>), grid, dim3(kThreads),
                                               lds_bytes(g, sizeof(T)), st, g, vs, dinv, B, X, R,
                                               ld, use_x0, part, qs));
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pcg_sweep1(const Grid &g, const T *vs, const T *dinv, const T *R,
                             const T *Pold, T *Pnew, long ld, int ncols, int k, double tol,
                             const int *mask, PcgState s, hipStream_t st, const float *Z,
                             const double *rzp, int rzt, bool p_given) {
    if (ncols <= 0) return hipSuccess;
    const long qs = (long)ncols * g.tiles();
    const dim3 grid(ncols * g.tiles());
    if (p_given) {
        QO_DISPATCH_PPT(g.ppt, hipLaunchKernelGGL((k_pcg_sweep1<T, P, 2>), grid,
                                                   dim3(kThreads), lds_bytes(g, sizeof(T)), st,
                                                   g, vs, dinv, R, Pold, Pnew, ld, ncols, k, tol,
                                                   mask, s, qs, Z, rzp, rzt));
    } else if (Z) {
        QO_DISPATCH_PPT(g.ppt, hipLaunchKernelGGL((k_pcg_sweep1<T, P, 1>), grid,
                                                   dim3(kThreads), lds_bytes(g, sizeof(T)), st,
                                                   g, vs, dinv, R, Pold, Pnew, ld, ncols, k, tol,
                                                   mask, s, qs, Z, rzp, rzt));
    } else {
        QO_DISPATCH_PPT(g.ppt, hipLaunchKernelGGL((k_pcg_sweep1<T, P, 0>), grid,
                                                   dim3(kThreads), lds_bytes(g, sizeof(T)), st,
                                                   g, vs, dinv, R, Pold, Pnew, ld, ncols, k, tol,
                                                   mask, s, qs, Z, rzp, rzt));
    }
    return hipGetLastError();
}

hipError_t launch_pcg_gamma(const Grid &g, int k, int ncols, double tol, const int *mask,
                            PcgState s, const double *rzc, const double *wzp, int nslab,
                            hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    const long qs = (long)ncols * g.tiles();
    hipLaunchKernelGGL(k_pcg_gamma, dim3(ncols), dim3(kThreads), 0, st, k, ncols, tol, mask, s, qs,
                       g.tiles(), rzc, wzp, nslab);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_pcg_sweep2(const Grid &g, const T *vs, const T *dinv, const T *Pn, T *X, T *R,
                             long ld, int ncols, int k, PcgState s, hipStream_t st, bool jac,
                             bool xzero) {
    if (ncols <= 0) return hipSuccess;
    const long qs = (long)ncols * g.tiles();
    const dim3 grid(ncols * g.tiles());
    if (xzero && !jac) {
        QO_DISPATCH_PPT(g.ppt, hipLaunchKernelGGL((k_pcg_sweep2<T, P, false, true>), grid,
                                                   dim3(kThreads), lds_bytes(g, sizeof(T)), st,
                                                   g, vs, dinv, Pn, X, R, ld, ncols, k, s, qs));
        return hipGetLastError();
    }
    if (xzero) return hipErrorInvalidValue;  // only the preconditioned form is instantiated
    if (jac) {
        QO_DISPATCH_PPT(g.ppt, hipLaunchKernelGGL((k_pcg_sweep2<T, P, true>), grid,
                                                   dim3(kThreads), lds_bytes(g, sizeof(T)), st,
                                                   g, vs, dinv, Pn, X, R, ld, ncols, k, s, qs));
    } else {
        QO_DISPATCH_PPT(g.ppt, hipLaunchKernelGGL((k_pcg_sweep2<T, P, false>), grid,
                                                   dim3(kThreads), lds_bytes(g, sizeof(T)), st,
                                                   g, vs, dinv, Pn, X, R, ld, ncols, k, s, qs));
    }
    return hipGetLastError();
}

template hipError_t launch_pcg_init<double>(const Grid &, const double *, const double *,
                                            const double *, double *, double *, long, int, int,
                                            double *, hipStream_t);
template hipError_t launch_pcg_init<float>(const Grid &, const float *, const float *,
                                           const float *, float *, float *, long, int, int,
                                           double *, hipStream_t);
template hipError_t launch_pcg_sweep1<double>(const Grid &, const double *, const double *,
                                              const double *, const double *, double *, long,
                                              int, int, double, const int *, PcgState,
                                              hipStream_t, const float *, const double *, int,
                                              bool);
template hipError_t launch_pcg_sweep1<float>(const Grid &, const float *, const float *,
                                             const float *, const float *, float *, long, int,
                                             int, double, const int *, PcgState, hipStream_t,
                                             const float *, const double *, int, bool);
template hipError_t launch_pcg_sweep2<double>(const Grid &, const double *, const double *,
                                              const double *, double *, double *, long, int, int,
                                              PcgState, hipStream_t, bool, bool);
template hipError_t launch_pcg_sweep2<float>(const Grid &, const float *, const float *,
                                             const float *, float *, float *, long, int, int,
                                             PcgState, hipStream_t, bool, bool);

template <typename T>
hipError_t launch_cg_delta0(const Grid &g, const T *vs, const T *dinv, const T *R, long ld,
                            int ncols, double *part, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    const long qs = (long)ncols * g.tiles();
    const dim3 grid(ncols * g.tiles());
    QO_DISPATCH_PPT(g.ppt, hipLaunchKernelGGL((k_cg_delta0<T, P>), grid, dim3(kThreads),
                                              lds_bytes(g, sizeof(T)), st, g, vs, dinv, R, ld,
                                              part, qs));
    return hipGetLastError();
}
template hipError_t launch_cg_delta0<double>(const Grid &, const double *, const double *,
                                             const double *, long, int, double *, hipStream_t);
template hipError_t launch_cg_delta0<float>(const Grid &, const float *, const float *,
                                            const float *, long, int, double *, hipStream_t);

hipError_t launch_colsum(const double *part, int tiles, int ncols, int nq, long qstride,
                         double *out, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_colsum, dim3(ncols), dim3(kThreads), 0, st, part, tiles, ncols, nq,
                       qstride, out);
    return hipGetLastError();
}

hipError_t launch_refine_axpy(double *X, long ld, float *D, long ld32, long ng, int ncols,
                              const int *mask, int zero_d, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    long blocks = (ng + 1023) / 1024;
    if (blocks > 1024) blocks = 1024;
    hipLaunchKernelGGL(k_refine_axpy, dim3((unsigned)blocks, ncols), dim3(256), 0, st, X, ld, D,
                       ld32, ng, mask, zero_d);
    return hipGetLastError();
}

hipError_t launch_resid_rel(const Grid &g, const double *vs, const float *dinv32, const double *B,
                            const double *X, long ld, float *R32, int ncols, const int *mask,
                            double *part, double *outer, hipStream_t st) {
    if (ncols <= 0) return hipSuccess;
    const long qs = (long)ncols * g.tiles();
    const dim3 grid(ncols * g.tiles());
    QO_DISPATCH_PPT(g.ppt, hipLaunchKernelGGL(k_resid_rel<P>, grid, dim3(kThreads),
                                              lds_bytes(g, 8), st, g, vs, dinv32, B, X, ld, R32,
                                              mask, part, qs, outer));
    return hipGetLastError();
}

hipError_t launch_rel_check(const double *part, int tiles, int ncols, const int *active,
                            const double *rref, const double *bb64, double delta, double tol,
                            int *need, int *nneed, hipStream_t st) {
    hipLaunchKernelGGL(k_rel_check, dim3((ncols + 255) / 256), dim3(256), 0, st, part, tiles,
                       (long)ncols * tiles, ncols, active, rref, bb64, delta, tol, need, nneed);
    return hipGetLastError();
}

hipError_t launch_rel_finalize(const double *outer, int tiles, int ncols, const int *need,
                               int *active, double *rref, double *bb64, double tol, int init,
                               int *nactive, int *err, hipStream_t st) {
    hipLaunchKernelGGL(k_rel_finalize, dim3((ncols + 255) / 256), dim3(256), 0, st, outer, tiles,
                       (long)ncols * tiles, ncols, need, active, rref, bb64, tol, init, nactive,
                       err);
    return hipGetLastError();
}

hipError_t launch_refine_mask(const double *sums, int ncols, double tol, double tol_in,
                              int *mask, double *coltol, int *nactive, int *err,
                              hipStream_t st, const double *ctol) {
    hipLaunchKernelGGL(k_refine_mask, dim3(1), dim3(256), 0, st, sums, ncols, tol, tol_in, mask,
                       coltol, nactive, err, ctol);
    return hipGetLastError();
}

}  // namespace qo
