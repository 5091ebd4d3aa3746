// CPU check of the index arithmetic of the HIP kernels (no GPU needed): the workgroup ->
// work-item maps and tilings the kernels use, taken from the library's own headers and
// planners, for every launch shape the API admits (and more).
//
//  * xcd_remap is a bijection of [0, B) that gives each of the 8 XCDs one contiguous range.
//  * stencil_tile_of and plane_slab_of are bijections onto (column, tile) / (column, slab).
//  * plan_grid (the stencil family's tiling): the tiles of a column partition its grid
//    exactly (bands x z-chunks), every point of a tile plane has a thread (points per thread
//    x 256), halo rows lie in [-1, ny], the LDS of a tile fits 64 KiB, the engine for fewer
//    than 4 points per thread (one halo column per thread) only meets rows of at most 256
//    points when a tile has several planes; the same for the one-sweep PCG tiling.
//  * dst_plan_geometry: slabs cover the rows, pencil jobs cover the in-plane positions,
//    padded lengths are multiples of 32 and cover the grid, the LDS of both passes fits.
//  * pen_off (the pencil pass's swizzled LDS tiles): one to one within a row, contiguous
//    over 8 indices, and equal to the per-lane base offsets plus the constant steps the
//    kernel adds for its position tiles, k-chunks and transfer items.
//  * bf16_rowblock_index is a bijection of [0, ld) x [0, n) onto [0, ld n).
// Exit status 0 when every check holds; the first failures are printed.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "qo_internal.h"

using namespace qo;

static long fails = 0;
#define CHECK(c, ...)                         \
    do {                                      \
        if (!(c)) {                           \
            if (fails < 20) {                 \
                std::fprintf(stderr, __VA_ARGS__); \
                std::fputc('\n', stderr);     \
            }                                 \
            ++fails;                          \
        }                                     \
    } while (0)

static void check_remap(int B) {
    std::vector<char> seen(B, 0);
    const int q = B / 8, r = B % 8;
    for (int b = 0; b < B; ++b) {
        const int L = xcd_remap(b, B);
        CHECK(L >= 0 && L < B, "xcd_remap(%d, %d) = %d out of range", b, B, L);
        if (L < 0 || L >= B) continue;
        CHECK(!seen[L], "xcd_remap(., %d) hits %d twice", B, L);
        seen[L] = 1;
        // XCD x = b % 8 owns [x q + min(x, r), ... + q + (x < r))
        const int x = b & 7;
        const int lo = x * q + (x < r ? x : r), hi = lo + q + (x < r ? 1 : 0);
        CHECK(L >= lo && L < hi, "xcd_remap(%d, %d) = %d leaves XCD %d's range", b, B, L, x);
    }
}

static void check_tile_map(int ncols, int tiles) {
    std::vector<char> seen((size_t)ncols * tiles, 0);
    for (int L = 0; L < ncols * tiles; ++L) {
        int col = -1, tile = -1;
        stencil_tile_of(L, ncols, tiles, col, tile);
        const bool ok = col >= 0 && col < ncols && tile >= 0 && tile < tiles;
        CHECK(ok, "stencil_tile_of(%d; %d x %d) = (%d, %d)", L, ncols, tiles, col, tile);
        if (!ok) continue;
        CHECK(!seen[(size_t)col * tiles + tile], "stencil_tile_of: (%d, %d) twice", col, tile);
        seen[(size_t)col * tiles + tile] = 1;
    }
    std::vector<char> seen2((size_t)ncols * tiles, 0);
    for (int L = 0; L < ncols * tiles; ++L) {
        int col = -1, slab = -1;
        plane_slab_of(L, tiles, col, slab);
        const bool ok = col >= 0 && col < ncols && slab >= 0 && slab < tiles;
        CHECK(ok, "plane_slab_of(%d; %d x %d) = (%d, %d)", L, ncols, tiles, col, slab);
        if (!ok) continue;
        CHECK(!seen2[(size_t)col * tiles + slab], "plane_slab_of: (%d, %d) twice", col, slab);
        seen2[(size_t)col * tiles + slab] = 1;
    }
}

static void check_tiling(const Grid &g, const char *what, int N, bool cg) {
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    CHECK(g.TY >= 1 && g.TY <= ny && g.ZC >= 1 && g.ZC <= nz, "%s %dx%dx%d N=%d: TY %d ZC %d",
          what, nx, ny, nz, N, g.TY, g.ZC);
    CHECK(g.nbands * g.TY >= ny && (g.nbands - 1) * g.TY < ny, "%s: %d bands of %d rows for %d",
          what, g.nbands, g.TY, ny);
    CHECK(g.nzc * g.ZC >= nz && (g.nzc - 1) * g.ZC < nz, "%s: %d z-chunks of %d for %d", what,
          g.nzc, g.ZC, nz);
    std::vector<int> cover((size_t)ny * nz, 0);
    for (int t = 0; t < g.tiles(); ++t) {
        const TileExtent e = g.extent(t);
        CHECK(e.ty >= 1 && e.y0 >= 0 && e.y0 + e.ty <= ny && e.z0 >= 0 && e.z1 <= nz &&
                  e.z0 < e.z1,
              "%s %dx%dx%d: tile %d rows [%d,%d) planes [%d,%d)", what, nx, ny, nz, t, e.y0,
              e.y0 + e.ty, e.z0, e.z1);
        // halo rows y0 - 1 and y0 + ty: inside the grid or the zero boundary row
        CHECK(e.y0 - 1 >= -1 && e.y0 + e.ty <= ny, "%s: halo rows of tile %d", what, t);
        for (int z = e.z0; z < e.z1; ++z)
            for (int y = e.y0; y < e.y0 + e.ty; ++y)
                if (y >= 0 && y < ny && z >= 0 && z < nz) ++cover[(size_t)z * ny + y];
    }
    for (size_t i = 0; i < cover.size(); ++i)
        CHECK(cover[i] == 1, "%s %dx%dx%d: row %zu covered %d times", what, nx, ny, nz, i,
              cover[i]);
    if (!cg) {
        CHECK(g.ppt >= 1 && (long)g.ppt * kThreads >= (long)g.TY * nx,
              "%s %dx%dx%d: %d points per thread for %d x %d", what, nx, ny, nz, g.ppt, g.TY, nx);
        const int opts[6] = {1, 2, 3, 4, 6, 8};
        bool disp = false;
        for (int o : opts) disp = disp || o == g.ppt;
        CHECK(disp, "%s: points per thread %d is not dispatched", what, g.ppt);
        // the engine below 4 points per thread stages one halo column per thread
        CHECK(g.ppt >= 4 || nz == 1 || g.ZC == 1 || nx <= kThreads,
              "%s %dx%dx%d: narrow engine with %d-point rows", what, nx, ny, nz, nx);
        CHECK(2L * (g.TY + 2) * nx * 8 <= 65536, "%s %dx%dx%d: LDS %ld bytes", what, nx, ny, nz,
              2L * (g.TY + 2) * nx * 8);
    } else {
        CHECK(g.ppt >= 1 && (long)g.ppt * kThreads >= (long)(g.TY + 4) * nx,
              "%s %dx%dx%d: %d points per thread for %d + 4 rows", what, nx, ny, nz, g.ppt,
              g.TY);
        CHECK((3L * (g.TY + 4) + 3L * (g.TY + 2)) * nx * 8 <= 65536, "%s: LDS", what);
    }
}

static void check_dst(int dim, int nx, int ny, int nz, int ncols) {
    DstPlan p{};
    dst_plan_geometry(p, dim, nx, ny, nz);
    CHECK(p.NXP % 32 == 0 && p.NXP >= nx && p.NXP - nx < 32, "dst NXP %d for %d", p.NXP, nx);
    CHECK(p.NYP % 32 == 0 && p.NYP >= ny && p.NYP - ny < 32, "dst NYP %d for %d", p.NYP, ny);
    CHECK(p.NSP % 32 == 0 && p.NSP >= p.ns, "dst NSP %d for %d", p.NSP, p.ns);
    CHECK(p.rows <= p.RP && p.RP % 16 == 0, "dst rows %d RP %d", p.rows, p.RP);
    CHECK((long)p.nslab * p.rows >= (dim == 3 ? (long)ny * nz : ny) / (dim == 3 ? ny : 1),
          "dst slabs %d x %d rows", p.nslab, p.rows);
    if (dim == 2) CHECK((p.nslab - 1) * p.rows < ny && p.nslab * p.rows >= ny, "dst 2-D slabs");
    if (dim == 3) CHECK(p.nslab == nz && p.rows == ny, "dst 3-D slabs");
    CHECK((long)p.npen * 64 >= p.nf && (long)(p.npen - 1) * 64 < p.nf, "dst pencils %d for %d",
          p.npen, p.nf);
    CHECK(p.rzparts == p.npen * (p.NSP / 32), "dst rzparts");
    // LDS: plane pass (X, T^T, S_x copy; FP32 staging of the inverse), pencil pass
    size_t xt = (size_t)p.RP * (p.NXP + 8) * 2;
    const size_t tt = (size_t)p.NXP * (p.NYP + 8) * 2;
    if (dim == 3) xt = xt > tt ? xt : tt;
    // planes of more than 128 rows (3-D) stage the inverse's FP32 output in two halves;
    // S_x is copied into LDS up to 128 points, and for such planes up to 192 where it fits
    const bool big = dim == 3 && p.RP > 128;
    xt = (xt + 15) / 16 * 16;
    const size_t sx = (size_t)p.NXP * (p.NXP + 8) * 2;
    size_t pl = xt + (p.NXP <= 128 || (big && p.NXP <= 192 && xt + sx <= 163840) ? sx : 0);
    const size_t inv = (size_t)(p.RP / (big ? 2 : 1)) * (p.NXP + 4) * 4;
    pl = pl > inv ? pl : inv;
    CHECK(pl <= 163840, "dst plane LDS %zu bytes (%dx%dx%d)", pl, nx, ny, nz);
    CHECK(4 * p.RP <= (big ? 1024 : 512) && (!big || (p.RP / 2) % 16 == 0),
          "dst plane workgroup of %d threads (%dx%dx%d)", 4 * p.RP, nx, ny, nz);
    const size_t pen = 2 * 64 * (size_t)(p.NSP + 8) * 2 +
                       4 * ((size_t)pen_mu_floats(p.NSP, nx, ny) + 3 * (size_t)ncols);
    CHECK(pen <= 163840, "dst pencil LDS %zu bytes (%dx%dx%d, %d columns)", pen, nx, ny, nz,
          ncols);
    check_tile_map(ncols < 40 ? ncols : 40, p.nslab);
}

// The pencil pass's LDS tiles (64 positions x NSP slowest-axis indices, pitch NSP + 8):
// pen_off maps row m onto [m SP, m SP + NSP) one to one, keeps 8 consecutive indices from
// a multiple of 8 contiguous, and the kernel's per-lane base offsets plus constant steps
// (tile j: positions 4 c + j; k-chunk ks; transfer item i) equal pen_off of the element.
static void check_pencil_lds(int KS) {
    const int NSP = 32 * KS, SP = NSP + 8;
    for (int m = 0; m < 64; ++m) {
        std::vector<char> seen(NSP, 0);
        for (int s = 0; s < NSP; ++s) {
            const int o = pen_off(m, s, SP) - m * SP;
            const bool ok = o >= 0 && o < NSP;
            CHECK(ok, "pen_off(%d, %d; NSP %d) leaves its row", m, s, NSP);
            if (!ok) continue;
            CHECK(!seen[o], "pen_off(%d, .; NSP %d) hits %d twice", m, NSP, o);
            seen[o] = 1;
            if (s % 8 == 0)
                for (int t = 1; t < 8; ++t)
                    CHECK(pen_off(m, s + t, SP) == pen_off(m, s, SP) + t,
                          "pen_off(%d, %d..+7; NSP %d) not contiguous", m, s, NSP);
        }
    }
    for (int lane = 0; lane < 64; ++lane) {
        const int lr = lane & 15, lg = lane >> 4;
        for (int j = 0; j < 4; ++j) {
            for (int ks = 0; ks < KS; ++ks)
                CHECK(pen_off(4 * lr, 8 * lg, SP) + j * SP + 32 * ks ==
                          pen_off(4 * lr + j, 32 * ks + 8 * lg, SP),
                      "pencil operand offset (lane %d, j %d, ks %d; NSP %d)", lane, j, ks, NSP);
            for (int w = 0; w < KS; ++w)
                for (int rb = 0; rb < 2; ++rb)
                    CHECK(pen_off(4 * lr, 32 * w + 16 * rb + 4 * lg, SP) + j * SP ==
                              pen_off(4 * lr + j, 32 * w + 16 * rb + 4 * lg, SP),
                          "pencil result offset (lane %d, j %d, w %d, rb %d; NSP %d)", lane, j,
                          w, rb, NSP);
        }
    }
    for (int tid = 0; tid < 64 * KS; ++tid) {
        const int mg = tid & 7, s0 = 4 * (tid >> 3);
        CHECK(s0 + 3 < NSP, "pencil transfer rows (tid %d; NSP %d)", tid, NSP);
        for (int i = 0; i < 8; ++i)
            CHECK(pen_off(8 * mg, s0, SP) + i * SP == pen_off(8 * mg + i, s0, SP) &&
                      pen_off(8 * mg + i, s0 + 3, SP) == pen_off(8 * mg + i, s0, SP) + 3,
                  "pencil transfer offset (tid %d, i %d; NSP %d)", tid, i, NSP);
    }
}

static void check_bf16(long ld, int n) {
    std::vector<char> seen((size_t)ld * n, 0);
    for (int c = 0; c < n; ++c)
        for (long m = 0; m < ld; ++m) {
            const long i = bf16_rowblock_index(m, c, n);
            const bool ok = i >= 0 && i < ld * n;
            CHECK(ok, "bf16 index (%ld, %d; ld %ld, n %d) = %ld", m, c, ld, n, i);
            if (!ok) continue;
            CHECK(!seen[i], "bf16 index %ld twice", i);
            seen[i] = 1;
        }
}

int main() {
    for (int B = 1; B <= 4200; ++B) check_remap(B);
    for (int B : {24576, 36864, 98304, 131071}) check_remap(B);
    for (int ncols = 1; ncols <= 70; ++ncols)
        for (int tiles = 1; tiles <= 40; ++tiles) check_tile_map(ncols, tiles);
    check_tile_map(256, 12);
    check_tile_map(4470, 5);

    const double L1[3] = {1.0, 1.0, 1.0};
    // 3-D grids: ragged, anisotropic, the benchmark sizes, rows wider than a workgroup
    const int g3[][3] = {{4, 3, 2},    {6, 5, 4},     {13, 11, 10},  {24, 20, 18}, {32, 32, 32},
                         {48, 40, 36}, {64, 64, 64},  {96, 96, 96},  {100, 7, 9},  {128, 128, 200},
                         {255, 3, 5},  {257, 4, 6},   {300, 5, 17},  {384, 2, 40}, {500, 3, 8},
                         {768, 2, 20}, {769, 3, 4},   {1000, 1, 33}, {1024, 2, 3}, {17, 1, 1},
                         {1, 1, 40},   {2, 300, 2}};
    const int Ns[] = {1, 3, 8, 64, 256, 1000};
    for (const auto &n : g3)
        for (int N : Ns) {
            Grid g{}, q{};
            plan_grid(3, n, L1, 0.5, N, g, q);
            check_tiling(g, "3-D", N, false);
            if (n[0] <= 256) check_tiling(q, "3-D one-sweep", N, true);
        }
    // 2-D grids
    for (int nx : {1, 2, 5, 31, 32, 33, 64, 96, 100, 128, 192, 199, 255, 256, 257, 383, 512, 700,
                   1000, 1024})
        for (int ny : {1, 2, 7, 64, 65, 199, 256, 300}) {
            const int n[3] = {nx, ny, 1};
            for (int N : {1, 7, 64}) {
                Grid g{}, q{};
                plan_grid(2, n, L1, 0.5, N, g, q);
                check_tiling(g, "2-D", N, false);
                if (nx <= 256) check_tiling(q, "2-D one-sweep", N, true);
            }
        }
    // fast-Poisson plans over every admitted size class.  3-D: admitted exactly when every
    // axis has at most 256 points and both plane passes fit the LDS, by the padded sizes
    // (workgroup = 4 padded rows of threads; X and T^T share their space; the S_x copy up to
    // 128 points, above 128 rows up to 192 where it fits; the inverse's FP32 output staged
    // in halves above 128 rows).
    auto pad32 = [](int v) { return (v + 31) / 32 * 32; };
    auto lds3 = [&](int nx, int ny) {
        const size_t X = (size_t)pad32(nx), Y = (size_t)pad32(ny);
        size_t xt = std::max(Y * (X + 8) * 2, X * (Y + 8) * 2);
        xt = (xt + 15) / 16 * 16;
        const size_t sx = X * (X + 8) * 2;
        xt += X <= 128 || (Y > 128 && X <= 192 && xt + sx <= 163840) ? sx : 0;
        return std::max(xt, (Y > 128 ? Y / 2 : Y) * (X + 4) * 4);
    };
    for (int nx : {1, 2, 7, 31, 32, 33, 64, 96, 100, 127, 128, 129, 160, 192, 193, 224, 256, 257})
        for (int ny : {1, 5, 32, 96, 128, 129, 160, 192, 193, 224, 256, 257})
            for (int nz : {1, 3, 32, 96, 200, 256, 257}) {
                const int n[3] = {nx, ny, nz};
                const bool want = nx <= 256 && ny <= 256 && nz <= 256 && lds3(nx, ny) <= 163840;
                const bool got = dst_plan_check(3, n) == nullptr;
                CHECK(want == got, "3-D %dx%dx%d: admitted %d, expected %d", nx, ny, nz, got, want);
                if (got) check_dst(3, nx, ny, nz, 256);
            }
    CHECK(lds3(256, 256) <= 163840, "a 256 x 256 plane exceeds the LDS");
    for (int nx : {1, 31, 64, 65, 199, 256})
        for (int ny : {1, 2, 63, 64, 65, 199, 256}) check_dst(2, nx, ny, 1, 4096);
    check_dst(3, 96, 96, 96, 4096);
    for (int KS = 1; KS <= 8; ++KS) check_pencil_lds(KS);
    // row-blocked BF16 operands
    for (long ld : {64L, 128L, 640L, 4096L})
        for (int n : {1, 2, 3, 31, 64, 100}) check_bf16(ld, n);

    if (fails) {
        std::fprintf(stderr, "%ld check(s) failed\n", fails);
        return 1;
    }
    std::printf("index checks: all passed\n");
    return 0;
}
