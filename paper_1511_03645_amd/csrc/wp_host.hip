// Host side of the C ABI (include/wp.h): handles, device memory, tile
// tables, time stepping, the adjoint run and its snapshot store, flagging
// and functionals.  Kernels live in acoustics.hip, swe.hip, flag_reduce.hip
// and amr.hip; Berger-Rigoutsos clustering in cluster.cpp.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "abi_guard.h"
#include "richardson_level.h"
#include "wp_ctx.h"

using namespace wp;

// ---------------------------------------------------------------------------
// errors and memory
// ---------------------------------------------------------------------------
int wp_fail(wp_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        ctx->err = buf;
    }
    return code;
}

void *wp_dalloc(wp_ctx *ctx, size_t bytes)
{
    if (bytes == 0) bytes = 256;
    void *p = nullptr;
    if (ctx->has_alloc) {
        p = ctx->alloc.alloc(bytes, ctx->alloc.user);
    } else if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
    }
    if (p) ctx->owned.push_back(p);
    return p;
}

void wp_dfree(wp_ctx *ctx, void *p)
{
    if (!p) return;
    auto it = std::find(ctx->owned.begin(), ctx->owned.end(), p);
    if (it != ctx->owned.end()) ctx->owned.erase(it);
    // work already queued may still read the block; a caller's allocator may
    // hand it out again at once
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->has_alloc)
        ctx->alloc.free(p, ctx->alloc.user);
    else
        (void)hipFree(p);
}

static size_t state_bytes(const wp_ctx *ctx, long long cells)
{
    if (ctx->prob.precision == WP_MIXED) return (size_t)cells * (8 + 4 + 4);
    return (size_t)cells * ctx->m * ctx->esz;
}

// ---------------------------------------------------------------------------
// tiles
// ---------------------------------------------------------------------------
// Tiles of the 2D step kernels: strips of STRIP columns and `rows` rows over
// every patch.  Ordered so that the workgroups the hardware places on one XCD
// (workgroup ids congruent mod 8) receive one contiguous, column-major run of
// tiles, keeping vertically adjacent tiles -- which share halo rows -- in the
// same L2.
std::vector<Tile> wp_make_tiles(const std::vector<wp_patch> &patches, int inst, int rows, int width, bool xcd_order)
{
    std::vector<Tile> t;
    for (const auto &p : patches)
        for (int i = 0; i < p.nx; i += width)
            for (int j = 0; j < p.ny; j += rows)
                t.push_back(Tile{inst, p.ilo + i, p.jlo + j, std::min(width, p.nx - i), std::min(rows, p.ny - j), -1,
                                 (j / rows) & 1});
    if (xcd_order) wp_xcd_order(t);
    return t;
}

// Reorder a spatially ordered tile list so that workgroups k, k+8, k+16, ...
// (the ones the hardware places on one XCD) take one contiguous run of it.
void wp_xcd_order(std::vector<Tile> &t)
{
    if (t.size() < 16) return;
    const size_t n = t.size(), nx = 8;
    std::vector<Tile> o(n);
    const size_t chunk = (n + nx - 1) / nx;
    size_t k = 0;
    for (size_t r = 0; r < chunk; ++r)
        for (size_t x = 0; x < nx; ++x) {
            const size_t src = x * chunk + r;
            if (src < n) o[k++] = t[src];
        }
    o.resize(k);
    t.swap(o);
}

static int host_resolve(int i, int n, int lo, int hi)
{
    i = std::min(std::max(i, -2), n + 1);
    if (i < 0) return lo == WP_BC_PERIODIC ? i + n : (lo == WP_BC_WALL ? -1 - i : 0);
    if (i >= n) return hi == WP_BC_PERIODIC ? i - n : (hi == WP_BC_WALL ? 2 * n - 1 - i : n - 1);
    return i;
}

// Material of a level cell: that of the level-0 cell containing it.
uint8_t wp_level_mat(const wp_ctx *ctx, const Level &lv, int i, int j)
{
    const int r = lv.nx / ctx->grid.nx0;
    const int ry = ctx->kind2d ? lv.ny / ctx->grid.ny0 : 1;
    return ctx->mat0[(size_t)(j / ry) * ctx->grid.nx0 + i / r];
}

// Mark tiles whose whole read footprint (`halo` cells around the tile, ghost
// cells resolved by the boundary rules as the loaders do) holds one
// material, and cut the others (mixed) into pieces acou_mixed_rows(rows)
// high.
void wp_classify_tiles(const wp_ctx *ctx, const Level &lv, std::vector<Tile> &tiles, int rows, int halo)
{
    if (!ctx->is_acoustics || !ctx->kind2d) return;
    std::vector<Tile> out;
    out.reserve(tiles.size());
    const int *bc = ctx->prob.bc;
    // a level cell's material is that of the level-0 cell containing it, so
    // the footprint's materials are those of the level-0 rows and columns
    // its resolved rows and columns fall in
    const int r = lv.nx / ctx->grid.nx0, ry = lv.ny / ctx->grid.ny0;
    // the level-0 indices of the footprint [lo, hi] on an axis of n cells
    // (ratio q): the in-domain part is one contiguous range, the ghost cells
    // are resolved one by one
    auto footprint = [](int lo, int hi, int n, int q, int blo, int bhi, std::vector<int> &out) {
        out.clear();
        const int a = std::max(lo, 0), b = std::min(hi, n - 1);
        for (int k = a / q; a <= b && k <= b / q; ++k) out.push_back(k);
        for (int i = lo; i < std::min(0, hi + 1); ++i) out.push_back(host_resolve(i, n, blo, bhi) / q);
        for (int i = std::max(n, lo); i <= hi; ++i) out.push_back(host_resolve(i, n, blo, bhi) / q);
        std::sort(out.begin(), out.end());
        out.erase(std::unique(out.begin(), out.end()), out.end());
    };
    std::vector<int> cols, rws;
    for (auto &t : tiles) {
        footprint(t.i0 - halo, t.i0 + t.ni + halo - 1, lv.nx, r, bc[0], bc[1], cols);
        footprint(t.j0 - halo, t.j0 + t.nj + halo - 1, lv.ny, ry, bc[2], bc[3], rws);
        int m0 = -1;
        bool uni = true;
        for (size_t b = 0; b < rws.size() && uni; ++b)
            for (size_t a = 0; a < cols.size(); ++a) {
                const int m = ctx->mat0[(size_t)rws[b] * ctx->grid.nx0 + cols[a]];
                if (m0 < 0) m0 = m;
                else if (m != m0) { uni = false; break; }
            }
        t.mat = uni ? m0 : -1;
        if (uni) {
            out.push_back(t);
            continue;
        }
        const int hm = acou_mixed_rows(rows);
        for (int j = 0; j < t.nj; j += hm)
            out.push_back(Tile{t.inst, t.i0, t.j0 + j, t.ni, std::min(hm, t.nj - j), -1, ((t.j0 + j) / hm) & 1});
    }
    tiles.swap(out);
}

// Whether a level can take two steps per launch: a 2D acoustics canvas
// covered by one patch, the full method (second order, MC limiter,
// transverse terms), no periodic boundary.
bool wp_pair_capable(const wp_ctx *ctx, const Level &lv)
{
    if (!ctx->is_acoustics || !ctx->kind2d || ctx->pair_rows == 0) return false;
    if (!(ctx->prob.order == 2 && ctx->prob.limiter == 1 && ctx->prob.transverse == 1)) return false;
    for (int k = 0; k < 4; ++k)
        if (ctx->prob.bc[k] == WP_BC_PERIODIC) return false;
    if (lv.nx < 8 || lv.ny < 8 || lv.patches.size() != 1) return false;
    const wp_patch &p = lv.patches[0];
    return p.ilo == 0 && p.jlo == 0 && p.nx == lv.nx && p.ny == lv.ny;
}

// Two-step tiles: PAIR_STRIP columns by pair_rows rows (4..64; mixed tiles
// cut to acou_mixed_rows of that, so every tile starts on row 0 or at least
// 4 rows above it), classified with the four-cell footprint; mixed ones
// first, each group in XCD order.
static int upload_pair_tiles(wp_ctx *ctx, Level &lv)
{
    lv.nptiles = lv.npuni = lv.pair_rows = 0;
    if (!wp_pair_capable(ctx, lv)) return WP_OK;
    const long long cells = (long long)lv.nx * lv.ny;
    const int rows = ctx->pair_rows > 0 ? ctx->pair_rows : (cells <= (1LL << 19) ? 8 : 12);
    std::vector<Tile> t = wp_make_tiles(lv.patches, 0, rows, PAIR_STRIP, false);
    wp_classify_tiles(ctx, lv, t, rows, 4);
    std::vector<Tile> mixed, uni;
    for (Tile &x : t) {
        x.down = 0;
        (x.mat < 0 ? mixed : uni).push_back(x);
    }
    wp_xcd_order(mixed);
    wp_xcd_order(uni);
    t = mixed;
    t.insert(t.end(), uni.begin(), uni.end());
    void *d = lv.ptiles_dev;
    const int rc = wp_upload(ctx, t.data(), sizeof(Tile) * t.size(), d, lv.ptiles_cap, "pair tile table");
    lv.ptiles_dev = (Tile *)d;
    if (rc != WP_OK) return rc;
    lv.nptiles = (int)t.size();
    lv.npuni = (int)uni.size();
    lv.pair_rows = rows;
    return WP_OK;
}

bool wp_pair_ready(const wp_ctx *ctx, const Level &lv)
{
    return ctx->pair_rows != 0 && lv.ptiles_dev && lv.nptiles > 0;
}

// Tiles of the same material and march direction share a wave two by two
// when their columns fit side by side (at most TWO_TILE_COLS together); true
// if any did.
static bool pair_narrow(std::vector<Tile> &t)
{
    // per (material, direction), widest first: each tile is paired with the
    // narrowest one left if that fits beside it; a pair takes the place of
    // its wider tile in the list
    std::map<std::pair<int, int>, std::vector<size_t>> groups;
    for (size_t k = 0; k < t.size(); ++k)
        if (t[k].ni < TWO_TILE_COLS) groups[std::make_pair(t[k].mat, t[k].down)].push_back(k);
    std::vector<long long> partner(t.size(), -1);   // index of the tile riding with k, or -2 if k rides
    bool any = false;
    for (auto &g : groups) {
        std::vector<size_t> &v = g.second;
        std::stable_sort(v.begin(), v.end(), [&](size_t a, size_t b) { return t[a].ni > t[b].ni; });
        size_t lo = 0, hi = v.size();
        while (lo + 1 < hi) {
            if (t[v[lo]].ni + t[v[hi - 1]].ni <= TWO_TILE_COLS) {
                const size_t a = std::min(v[lo], v[hi - 1]), b = std::max(v[lo], v[hi - 1]);
                // the wider of the two takes the lower lanes
                const bool wide_first = t[a].ni >= t[b].ni;
                partner[wide_first ? a : b] = (long long)(wide_first ? b : a);
                partner[wide_first ? b : a] = -2;
                --hi;
                any = true;
            }
            ++lo;
        }
    }
    std::vector<Tile> out;
    out.reserve(t.size());
    for (size_t k = 0; k < t.size(); ++k) {
        if (partner[k] == -2) continue;
        Tile x = t[k];
        if (partner[k] >= 0) {
            const Tile &y = t[(size_t)partner[k]];
            x.i0b = y.i0;
            x.j0b = y.j0;
            x.nib = y.ni;
            x.njb = y.nj;
        }
        out.push_back(x);
    }
    t.swap(out);
    return any;
}

static int upload_tiles(wp_ctx *ctx, Level &lv);

int wp_upload_tiles(wp_ctx *ctx, Level &lv)
{
    ctx->host_ms[HT_TILES] -= wp_now_ms();
    const int rc = upload_tiles(ctx, lv);
    ctx->host_ms[HT_TILES] += wp_now_ms();
    lv.tables_ok = rc == WP_OK;
    if (rc != WP_OK) lv.ntiles = lv.nftiles = lv.nptiles = lv.nuni = lv.npuni = 0;
    return rc;
}

static int upload_tiles(wp_ctx *ctx, Level &lv)
{
    int rc;
    const bool is_1d = ctx->prob.kind == WP_ACOUSTICS_1D;
    const int rows = ctx->tile_rows > 0 ? ctx->tile_rows : wp_default_rows(ctx, lv);
    lv.tiles_host = wp_make_tiles(lv.patches, 0, is_1d ? 1 : rows, STRIP, false);
    lv.tile_rows = rows;
    wp_classify_tiles(ctx, lv, lv.tiles_host, rows);
    // mixed-material tiles (the slower march) first, so they are dispatched
    // at the start rather than forming the tail; each group in XCD-aware
    // order
    std::vector<Tile> mixed, uni;
    for (const Tile &t : lv.tiles_host) (t.mat < 0 ? mixed : uni).push_back(t);
    // levels of several patches (refined levels, forward steps only): two
    // narrow tiles per wave where the unrolled march runs them
    lv.dual = false;
    const bool full = ctx->prob.order == 2 && ctx->prob.limiter == 1 && ctx->prob.transverse == 1;
    if (ctx->is_acoustics && ctx->kind2d && full && ctx->equation == 0 && lv.patches.size() > 1 &&
        (rows == 4 || rows == 6 || rows == 8 || rows == 12 || rows == 16)) {
        const bool a = pair_narrow(mixed), b = pair_narrow(uni);
        lv.dual = a || b;
    }
    wp_xcd_order(mixed);
    wp_xcd_order(uni);
    lv.nuni = (int)uni.size();
    lv.tiles_host = mixed;
    lv.tiles_host.insert(lv.tiles_host.end(), uni.begin(), uni.end());
    if ((rc = upload_pair_tiles(ctx, lv)) != WP_OK) return rc;
    // flag / reduction tiles: larger blocks of whole patches
    std::vector<Tile> ft = wp_make_tiles(lv.patches, 0, 16, 64, false);
    // captured sequences hold the old table pointers and sizes (the new
    // tables may reuse the blocks; the copies follow earlier work on the stream)
    ++ctx->topo_gen;
    lv.ntiles = (int)lv.tiles_host.size();
    lv.nftiles = (int)ft.size();
    void *t = lv.tiles_dev, *f = lv.ftiles_dev;
    rc = wp_upload(ctx, lv.tiles_host.data(), sizeof(Tile) * lv.ntiles, t, lv.tiles_cap, "tile table");
    lv.tiles_dev = (Tile *)t;
    if (rc != WP_OK) return rc;
    rc = wp_upload(ctx, ft.data(), sizeof(Tile) * lv.nftiles, f, lv.ftiles_cap, "flag tile table");
    lv.ftiles_dev = (Tile *)f;
    return rc;
}

int wp_default_rows(const wp_ctx *ctx, const Level &lv)
{
    // enough strips to give every SIMD several waves on small grids, long
    // marches (little halo re-read) on large ones
    long long cells = 0;   // cells the level's patches hold
    for (const wp_patch &p : lv.patches) cells += (long long)p.nx * p.ny;
    if (cells <= (1LL << 18)) return 4;
    // FP64 shallow water on large grids: the forward march (a rolled loop)
    // gains from longer tiles, the adjoint from shorter ones (2048^2: 24 and
    // 8 rows, 122 and 61 us per step against 129 and 63 at 12)
    if (!ctx->is_acoustics && ctx->prob.precision == WP_FP64 && cells > (1LL << 21))
        return &lv == &ctx->adj ? 8 : 24;
    // refined levels of many patches: shorter tiles balance the narrow
    // two-per-wave tiles against the full ones (8 rows measured 3% faster
    // than 12 on a level of 1 600 patches and 2.3 M cells)
    if (cells <= (1LL << 21) || lv.patches.size() > 1) return 8;
    return 12;
}

// ---------------------------------------------------------------------------
// creation
// ---------------------------------------------------------------------------
static int build_materials(wp_ctx *ctx, const wp_coefficients *coef)
{
    const int nx = ctx->grid.nx0, ny = ctx->kind2d ? ctx->grid.ny0 : 1;
    std::map<std::pair<double, double>, int> ids;
    std::vector<uint8_t> mat((size_t)nx * ny);
    for (long long k = 0; k < (long long)nx * ny; ++k) {
        const double r = coef->rho[k], K = coef->K[k];
        if (!(r > 0.0) || !(K > 0.0) || !std::isfinite(r) || !std::isfinite(K))
            return wp_fail(ctx, WP_EINVAL, "rho and K must be positive and finite (cell %lld)", k);
        auto key = std::make_pair(r, K);
        auto it = ids.find(key);
        int id;
        if (it == ids.end()) {
            id = (int)ids.size();
            if (id >= MAXMAT) return wp_fail(ctx, WP_EINVAL, "more than %d distinct (rho, K) pairs", MAXMAT);
            ids[key] = id;
            ctx->rho.push_back(r);
            ctx->K.push_back(K);
        } else {
            id = it->second;
        }
        mat[k] = (uint8_t)id;
    }
    ctx->nmat = (int)ids.size();
    ctx->mat0 = mat;
    ctx->cmax = 0.0;
    for (int a = 0; a < ctx->nmat; ++a) ctx->cmax = std::max(ctx->cmax, std::sqrt(ctx->K[a] / ctx->rho[a]));
    // material and pair tables in the state precision
    const int nm = ctx->nmat;
    std::vector<double> mt(nm * 4), pt(nm * nm * 3);
    std::vector<double> Z(nm), c(nm);
    for (int a = 0; a < nm; ++a) {
        Z[a] = std::sqrt(ctx->rho[a] * ctx->K[a]);
        c[a] = std::sqrt(ctx->K[a] / ctx->rho[a]);
        mt[a * 4 + 0] = Z[a];
        mt[a * 4 + 1] = c[a];
        mt[a * 4 + 2] = ctx->K[a];
        mt[a * 4 + 3] = 1.0 / ctx->rho[a];
    }
    for (int a = 0; a < nm; ++a)
        for (int b = 0; b < nm; ++b) {
            double *p = &pt[(a * nm + b) * 3];
            p[0] = 1.0 / (Z[a] + Z[b]);
            p[1] = (Z[a] * Z[b] + 1.0) / (Z[a] * Z[a] + 1.0);   // wave 1, upwind edge to the right
            p[2] = (Z[a] * Z[b] + 1.0) / (Z[b] * Z[b] + 1.0);   // wave 2, upwind edge to the left
        }
    {
        std::vector<double> m64(nm * 4);
        for (int a = 0; a < nm; ++a) {
            m64[a * 4 + 0] = Z[a];
            m64[a * 4 + 1] = c[a];
            m64[a * 4 + 2] = ctx->rho[a];
            m64[a * 4 + 3] = ctx->K[a];
        }
        ctx->mtab64 = (double *)wp_dalloc(ctx, m64.size() * 8);
        if (!ctx->mtab64) return wp_fail(ctx, WP_ENOMEM, "material tables");
        if (hipMemcpy(ctx->mtab64, m64.data(), m64.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
            return wp_fail(ctx, WP_EDEVICE, "material table upload");
    }
    ctx->mtab = wp_dalloc(ctx, mt.size() * ctx->esz);
    ctx->ptab = wp_dalloc(ctx, pt.size() * ctx->esz);
    if (!ctx->mtab || !ctx->ptab) return wp_fail(ctx, WP_ENOMEM, "material tables");
    if (ctx->esz == 8) {
        if (hipMemcpy(ctx->mtab, mt.data(), mt.size() * 8, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(ctx->ptab, pt.data(), pt.size() * 8, hipMemcpyHostToDevice) != hipSuccess)
            return wp_fail(ctx, WP_EDEVICE, "material table upload");
    } else {
        std::vector<float> mf(mt.begin(), mt.end()), pf(pt.begin(), pt.end());
        if (hipMemcpy(ctx->mtab, mf.data(), mf.size() * 4, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(ctx->ptab, pf.data(), pf.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
            return wp_fail(ctx, WP_EDEVICE, "material table upload");
    }
    return WP_OK;
}

int wp_alloc_level(wp_ctx *ctx, Level &lv)
{
    const long long cells = (long long)lv.nx * lv.ny;
    for (int b = 0; b < 2; ++b) {
        lv.q[b] = wp_dalloc(ctx, state_bytes(ctx, cells));
        if (!lv.q[b]) return wp_fail(ctx, WP_ENOMEM, "state canvas (%lld cells)", cells);
        if (hipMemsetAsync(lv.q[b], 0, state_bytes(ctx, cells), ctx->stream) != hipSuccess)
            return wp_fail(ctx, WP_EDEVICE, "state clear");
    }
    lv.flags = (uint8_t *)wp_dalloc(ctx, (size_t)cells);
    if (!lv.flags) return wp_fail(ctx, WP_ENOMEM, "flag canvas");
    if (hipMemsetAsync(lv.flags, 0, (size_t)cells, ctx->stream) != hipSuccess)
        return wp_fail(ctx, WP_EDEVICE, "flag clear");
    if (ctx->is_acoustics) {
        // material of each level cell: that of the level-0 cell containing it
        lv.mat = (uint8_t *)wp_dalloc(ctx, (size_t)cells);
        if (!lv.mat) return wp_fail(ctx, WP_ENOMEM, "material canvas");
        std::vector<uint8_t> m((size_t)cells);
        const int r = lv.nx / ctx->grid.nx0;
        const int ry = ctx->kind2d ? lv.ny / ctx->grid.ny0 : 1;
        for (int j = 0; j < lv.ny; ++j)
            for (int i = 0; i < lv.nx; ++i) m[(size_t)j * lv.nx + i] = ctx->mat0[(size_t)(j / ry) * ctx->grid.nx0 + i / r];
        if (hipMemcpy(lv.mat, m.data(), m.size(), hipMemcpyHostToDevice) != hipSuccess)
            return wp_fail(ctx, WP_EDEVICE, "material upload");
    }
    return WP_OK;
}

extern "C" int wp_create(const wp_problem *problem, const wp_coefficients *coef, const wp_grid *grid,
                         const wp_allocator *alloc, void *stream, wp_ctx **out)
{
    WP_ABI_TRY
    if (!out) return WP_EINVAL;
    *out = nullptr;
    if (!problem || !coef || !grid) return WP_EINVAL;
    wp_ctx *ctx = new wp_ctx();
    *out = ctx;   // handed back on failure too, for wp_last_error; the caller destroys it
    ctx->prob = *problem;
    ctx->grid = *grid;
    ctx->stream = (hipStream_t)stream;
    if (alloc && alloc->alloc && alloc->free) {
        ctx->alloc = *alloc;
        ctx->has_alloc = true;
    }
    const wp_problem &P = ctx->prob;
    int rc = WP_OK;
    auto bail = [&](int code) {
        *out = ctx;   // hand back for wp_last_error, caller destroys
        return code;
    };
    if (P.kind != WP_ACOUSTICS_1D && P.kind != WP_ACOUSTICS_2D && P.kind != WP_SWE_2D)
        return bail(wp_fail(ctx, WP_EINVAL, "unknown kind %d", P.kind));
    ctx->kind2d = P.kind != WP_ACOUSTICS_1D;
    ctx->is_acoustics = P.kind != WP_SWE_2D;
    ctx->m = P.kind == WP_ACOUSTICS_1D ? 2 : 3;
    if (P.precision == WP_FP64) ctx->esz = 8;
    else if (P.precision == WP_FP32 && ctx->is_acoustics) ctx->esz = 4;
    else if (P.precision == WP_MIXED && !ctx->is_acoustics) ctx->esz = 4;
    else if (P.precision == WP_FP32 && !ctx->is_acoustics) ctx->esz = 4;
    else return bail(wp_fail(ctx, WP_EINVAL, "precision %d not available for kind %d", P.precision, P.kind));
    if (P.order < 1 || P.order > 2 || P.limiter < 0 || P.limiter > 1 || P.transverse < 0 || P.transverse > 1)
        return bail(wp_fail(ctx, WP_EINVAL, "order must be 1|2, limiter 0|1, transverse 0|1"));
    for (int k = 0; k < 4; ++k)
        if (P.bc[k] < 0 || P.bc[k] > 2) return bail(wp_fail(ctx, WP_EINVAL, "bad boundary type"));
    if ((P.bc[0] == WP_BC_PERIODIC) != (P.bc[1] == WP_BC_PERIODIC) ||
        (ctx->kind2d && (P.bc[2] == WP_BC_PERIODIC) != (P.bc[3] == WP_BC_PERIODIC)))
        return bail(wp_fail(ctx, WP_EINVAL, "periodic boundaries must be paired"));
    if (!(P.cfl_max > 0.0)) return bail(wp_fail(ctx, WP_EINVAL, "cfl_max must be positive"));
    const wp_grid &G = ctx->grid;
    if (G.nx0 < 4 || (ctx->kind2d && G.ny0 < 4)) return bail(wp_fail(ctx, WP_EINVAL, "grid must be at least 4 cells per side"));
    if (!(G.xhi > G.xlo) || (ctx->kind2d && !(G.yhi > G.ylo))) return bail(wp_fail(ctx, WP_EINVAL, "empty domain"));
    if (G.num_levels < 1 || G.num_levels > WP_MAX_LEVELS) return bail(wp_fail(ctx, WP_EINVAL, "num_levels out of range"));
    if (G.num_levels > 1 && P.kind == WP_ACOUSTICS_1D)
        return bail(wp_fail(ctx, WP_EINVAL, "refinement levels are supported in 2D"));
    long long cells_l = (long long)G.nx0 * (ctx->kind2d ? G.ny0 : 1);
    for (int l = 0; l + 1 < G.num_levels; ++l) {
        if (G.ratio[l] < 2 || G.ratio[l] > 16)
            return bail(wp_fail(ctx, WP_EINVAL, "refinement ratios must be between 2 and 16"));
        cells_l *= (long long)G.ratio[l] * G.ratio[l];
    }
    // kernels address a canvas with 32-bit byte offsets; a dropped store
    // goes just past the three components, plus a component offset
    const long long esz_max = P.precision == WP_FP32 ? 4 : 8;
    if (cells_l * 5 * esz_max >= (1LL << 32))
        return bail(wp_fail(ctx, WP_EINVAL, "finest level canvas of %lld cells is above the %lld-cell limit", cells_l,
                            ((1LL << 32) - 1) / (5 * esz_max)));
    if (G.num_levels > 1)
        for (int k = 0; k < 4; ++k)
            if (P.bc[k] == WP_BC_PERIODIC)
                return bail(wp_fail(ctx, WP_EINVAL, "refinement levels need extrapolation or wall boundaries"));
    if (ctx->is_acoustics) {
        if (!coef->rho || !coef->K) return bail(wp_fail(ctx, WP_EINVAL, "acoustics needs rho and K"));
        if ((rc = build_materials(ctx, coef)) != WP_OK) return bail(rc);
    } else {
        if (!coef->B) return bail(wp_fail(ctx, WP_EINVAL, "shallow water needs B"));
        if (!(P.g > 0.0)) return bail(wp_fail(ctx, WP_EINVAL, "g must be positive"));
    }
    // status words and reduction scratch
    ctx->status = (int *)wp_dalloc(ctx, 256);
    ctx->count = (unsigned long long *)wp_dalloc(ctx, sizeof(unsigned long long) * COUNT_SPAN);
    ctx->partials = (double *)wp_dalloc(ctx, sizeof(double) * 2 * RED_BLOCKS);
    ctx->red_out = (double *)wp_dalloc(ctx, 256);
    ctx->cflbits = (unsigned *)wp_dalloc(ctx, 256);
    if (!ctx->status || !ctx->count || !ctx->partials || !ctx->red_out || !ctx->cflbits)
        return bail(wp_fail(ctx, WP_ENOMEM, "scratch"));
    if (hipMemsetAsync(ctx->status, 0, 256, ctx->stream) != hipSuccess ||
        hipMemsetAsync(ctx->cflbits, 0, 256, ctx->stream) != hipSuccess)
        return bail(wp_fail(ctx, WP_EDEVICE, "status clear"));
    // levels
    int nxl = G.nx0, nyl = ctx->kind2d ? G.ny0 : 1;
    for (int l = 0; l < G.num_levels; ++l) {
        Level lv;
        lv.nx = nxl;
        lv.ny = nyl;
        lv.dx = (G.xhi - G.xlo) / nxl;
        lv.dy = ctx->kind2d ? (G.yhi - G.ylo) / nyl : 1.0;
        lv.ratio = l == 0 ? 1 : G.ratio[l - 1];
        ctx->L.push_back(lv);
        if (l + 1 < G.num_levels) {
            nxl *= G.ratio[l];
            nyl *= G.ratio[l];
        }
    }
    for (int l = 0; l < G.num_levels; ++l)
        if ((rc = wp_alloc_level(ctx, ctx->L[l])) != WP_OK) return bail(rc);
    ctx->L[0].patches.push_back(wp_patch{0, 0, ctx->L[0].nx, ctx->L[0].ny});
    if ((rc = wp_upload_tiles(ctx, ctx->L[0])) != WP_OK) return bail(rc);
    if (!ctx->is_acoustics && (rc = wp_swe_init(ctx, coef)) != WP_OK) return bail(rc);
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return bail(wp_fail(ctx, WP_EDEVICE, "create sync"));
    *out = ctx;
    return WP_OK;
    WP_ABI_CATCH(out && *out ? &(*out)->err : nullptr)
}

extern "C" void wp_destroy(wp_ctx *ctx)
{
    if (!ctx) return;
    (void)hipStreamSynchronize(ctx->stream);
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->adj_exec) (void)hipGraphExecDestroy(ctx->adj_exec);
    if (ctx->bo_exec) (void)hipGraphExecDestroy(ctx->bo_exec);
    if (ctx->ff_exec) (void)hipGraphExecDestroy(ctx->ff_exec);
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->pin) (void)hipHostFree(ctx->pin);
    for (wp_ctx *h : ctx->rich) wp_destroy(h);
    std::vector<void *> all = ctx->owned;
    for (void *p : all) wp_dfree(ctx, p);
    delete ctx;
}

extern "C" const char *wp_last_error(const wp_ctx *ctx) { return ctx ? ctx->err.c_str() : "null handle"; }

extern "C" const char *wp_status_string(int s)
{
    switch (s) {
    case WP_OK: return "ok";
    case WP_EINVAL: return "invalid argument";
    case WP_ENOMEM: return "out of device memory";
    case WP_EDEVICE: return "HIP runtime error";
    case WP_ECFL: return "Courant number above the limit";
    case WP_ENONFINITE: return "non-finite value";
    case WP_ERANGE: return "outside the stored adjoint snapshots";
    case WP_ESTATE: return "call out of order";
    default: return "unknown status";
    }
}

extern "C" int wp_set_stream(wp_ctx *ctx, void *stream)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    (void)hipStreamSynchronize(ctx->stream);
    ctx->stream = (hipStream_t)stream;
    return WP_OK;
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

extern "C" int wp_level_info(const wp_ctx *ctx, int level, int *nx, int *ny, int *npatches)
{
    if (!ctx) return WP_EINVAL;
    if (level < 0 || level >= (int)ctx->L.size()) return wp_fail_get(ctx, WP_EINVAL, "level out of range");
    if (nx) *nx = ctx->L[level].nx;
    if (ny) *ny = ctx->L[level].ny;
    if (npatches) *npatches = (int)ctx->L[level].patches.size();
    return WP_OK;
}

// ---------------------------------------------------------------------------
// state transfer
// ---------------------------------------------------------------------------
// Copy between a caller buffer [m][h][w] and box (i0, j0, w, h) of a level
// canvas.  Component k of the canvas sits at k * cells elements of size esz
// (mixed precision: eta doubles, then hu, hv floats).
constexpr size_t WP_PIN_CAP = 32u << 20;

// Pinned staging for host transfers: asynchronous copies to or from pageable
// memory are not reliably complete at the stream's synchronisation (seen
// under a profiler's interception), copies to or from pinned memory are.
static int ensure_pin(wp_ctx *ctx, size_t want)
{
    want = std::min(std::max(want, (size_t)4096), WP_PIN_CAP);
    if (ctx->pin_bytes >= want) return WP_OK;
    if (ctx->pin) (void)hipHostFree(ctx->pin);
    ctx->pin = nullptr;
    ctx->pin_bytes = 0;
    if (hipHostMalloc(&ctx->pin, want, hipHostMallocDefault) != hipSuccess || !ctx->pin)
        return wp_fail(ctx, WP_ENOMEM, "pinned staging buffer (%zu bytes)", want);
    ctx->pin_bytes = want;
    return WP_OK;
}

int wp_host_copy2d(wp_ctx *ctx, void *dst, size_t dpitch, const void *src, size_t spitch, size_t width, size_t rows,
                   bool to_device)
{
    if (rows == 0 || width == 0) return WP_OK;
    int rc;
    if ((rc = ensure_pin(ctx, width * rows)) != WP_OK) return rc;
    if (width > ctx->pin_bytes) {
        // rows wider than the staging buffer: one row at a time, in pieces
        for (size_t r = 0; r < rows; ++r)
            for (size_t o = 0; o < width; o += ctx->pin_bytes) {
                const size_t n = std::min(ctx->pin_bytes, width - o);
                if ((rc = wp_host_copy2d(ctx, (char *)dst + r * dpitch + o, n, (const char *)src + r * spitch + o, n,
                                         n, 1, to_device)) != WP_OK)
                    return rc;
            }
        return WP_OK;
    }
    const size_t chunk = ctx->pin_bytes / width;
    char *pin = (char *)ctx->pin;
    for (size_t r0 = 0; r0 < rows; r0 += chunk) {
        const size_t n = std::min(chunk, rows - r0);
        hipError_t e;
        if (to_device) {
            for (size_t r = 0; r < n; ++r) memcpy(pin + r * width, (const char *)src + (r0 + r) * spitch, width);
            e = hipMemcpy2DAsync((char *)dst + r0 * dpitch, dpitch, pin, width, width, n, hipMemcpyHostToDevice,
                                 ctx->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
        } else {
            e = hipMemcpy2DAsync(pin, width, (const char *)src + r0 * spitch, spitch, width, n, hipMemcpyDeviceToHost,
                                 ctx->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
            if (e == hipSuccess)
                for (size_t r = 0; r < n; ++r) memcpy((char *)dst + (r0 + r) * dpitch, pin + r * width, width);
        }
        if (e != hipSuccess) return wp_fail(ctx, WP_EDEVICE, "host transfer: %s", hipGetErrorString(e));
    }
    return WP_OK;
}

// Counters spread over slots (see COUNT_SLOTS): clear n of them, and read
// them back as their slot sums.
int wp_clear_counts(wp_ctx *ctx, unsigned long long *dev, int n, hipStream_t s)
{
    if (hipMemsetAsync(dev, 0, sizeof(unsigned long long) * COUNT_SPAN * (size_t)n, s) != hipSuccess)
        return wp_fail(ctx, WP_EDEVICE, "count clear");
    return WP_OK;
}

int wp_read_counts(wp_ctx *ctx, const unsigned long long *dev, int n, int64_t *out)
{
    std::vector<unsigned long long> v((size_t)COUNT_SPAN * n);
    int rc;
    if ((rc = wp_host_copy(ctx, v.data(), dev, v.size() * sizeof(unsigned long long), false)) != WP_OK) return rc;
    for (int k = 0; k < n; ++k) {
        unsigned long long c = 0;
        for (int q = 0; q < COUNT_SLOTS; ++q) c += v[(size_t)k * COUNT_SPAN + (size_t)q * COUNT_STRIDE];
        out[k] = (int64_t)c;
    }
    return WP_OK;
}

int wp_upload(wp_ctx *ctx, const void *src, size_t bytes, void *&dev, size_t &cap, const char *what)
{
    if (bytes > cap || !dev) {
        if (dev) wp_dfree(ctx, dev);
        const size_t want = std::max(bytes + bytes / 2, (size_t)256);
        dev = wp_dalloc(ctx, want);
        cap = dev ? want : 0;
        if (!dev) return wp_fail(ctx, WP_ENOMEM, "%s allocation failed", what);
    }
    if (bytes == 0) return WP_OK;
    ctx->host_ms[HT_H2D] -= wp_now_ms();
    const int rc = wp_host_copy(ctx, dev, src, bytes, true);
    ctx->host_ms[HT_H2D] += wp_now_ms();
    return rc;
}

int wp_host_copy(wp_ctx *ctx, void *dst, const void *src, size_t bytes, bool to_device)
{
    if (bytes == 0) return WP_OK;
    // as rows of at most 1 MiB
    const size_t width = std::min(bytes, (size_t)1 << 20);
    const size_t rows = bytes / width, tail = bytes - rows * width;
    int rc = wp_host_copy2d(ctx, dst, width, src, width, width, rows, to_device);
    if (rc == WP_OK && tail)
        rc = wp_host_copy2d(ctx, (char *)dst + rows * width, tail, (const char *)src + rows * width, tail, tail, 1,
                            to_device);
    return rc;
}

static int copy_box(wp_ctx *ctx, Level &lv, int i0, int j0, int w, int h, void *user, int on_device, bool to_canvas)
{
    const long long cells = (long long)lv.nx * lv.ny;
    char *canvas = (char *)lv.q[lv.cur];
    const hipMemcpyKind kind = on_device ? hipMemcpyDeviceToDevice
                                         : (to_canvas ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost);
    size_t uoff = 0;
    size_t coff = 0;
    for (int k = 0; k < ctx->m; ++k) {
        const size_t es = ctx->prob.precision == WP_MIXED ? (k == 0 ? 8 : 4) : (size_t)ctx->esz;
        char *cbase = canvas + coff + ((size_t)j0 * lv.nx + i0) * es;
        char *ubase = (char *)user + uoff;
        if (!on_device) {
            // host memory: through the pinned staging buffer
            const int rc = to_canvas ? wp_host_copy2d(ctx, cbase, (size_t)lv.nx * es, ubase, (size_t)w * es,
                                                      (size_t)w * es, h, true)
                                     : wp_host_copy2d(ctx, ubase, (size_t)w * es, cbase, (size_t)lv.nx * es,
                                                      (size_t)w * es, h, false);
            if (rc != WP_OK) return rc;
            uoff += (size_t)w * h * es;
            coff += (size_t)cells * es;
            continue;
        }
        hipError_t e;
        if (to_canvas)
            e = hipMemcpy2DAsync(cbase, (size_t)lv.nx * es, ubase, (size_t)w * es, (size_t)w * es, h, kind, ctx->stream);
        else
            e = hipMemcpy2DAsync(ubase, (size_t)w * es, cbase, (size_t)lv.nx * es, (size_t)w * es, h, kind, ctx->stream);
        if (e != hipSuccess) return wp_fail(ctx, WP_EDEVICE, "state copy: %s", hipGetErrorString(e));
        uoff += (size_t)w * h * es;
        coff += (size_t)cells * es;
    }
    if (hipStreamSynchronize(ctx->stream) != hipSuccess) return wp_fail(ctx, WP_EDEVICE, "state copy sync");
    return WP_OK;
}

static int box_of(wp_ctx *ctx, int level, int patch, int &i0, int &j0, int &w, int &h)
{
    if (level < 0 || level >= (int)ctx->L.size()) return wp_fail(ctx, WP_EINVAL, "level %d out of range", level);
    Level &lv = ctx->L[level];
    if (patch < 0) {
        i0 = j0 = 0;
        w = lv.nx;
        h = lv.ny;
        return WP_OK;
    }
    if (patch >= (int)lv.patches.size()) return wp_fail(ctx, WP_EINVAL, "patch %d out of range", patch);
    const wp_patch &p = lv.patches[patch];
    i0 = p.ilo;
    j0 = p.jlo;
    w = p.nx;
    h = p.ny;
    return WP_OK;
}

extern "C" int wp_set_state(wp_ctx *ctx, int level, int patch, const void *src, int on_device)
{
    WP_ABI_TRY
    if (!ctx || !src) return ctx ? wp_fail(ctx, WP_EINVAL, "null source") : WP_EINVAL;
    int i0, j0, w, h, rc;
    if ((rc = box_of(ctx, level, patch, i0, j0, w, h)) != WP_OK) return rc;
    ctx->L[level].prev_valid = false;   // the other canvas no longer precedes this state
    return copy_box(ctx, ctx->L[level], i0, j0, w, h, const_cast<void *>(src), on_device, true);
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

extern "C" int wp_get_state(wp_ctx *ctx, int level, int patch, void *dst, int on_device)
{
    WP_ABI_TRY
    if (!ctx || !dst) return ctx ? wp_fail(ctx, WP_EINVAL, "null destination") : WP_EINVAL;
    int i0, j0, w, h, rc;
    if ((rc = box_of(ctx, level, patch, i0, j0, w, h)) != WP_OK) return rc;
    if ((rc = copy_box(ctx, ctx->L[level], i0, j0, w, h, dst, on_device, false)) != WP_OK) return rc;
    return wp_check_status(ctx);
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

int wp_check_status(wp_ctx *ctx)
{
    int st = 0, rc;
    if ((rc = wp_host_copy(ctx, &st, ctx->status, sizeof(int), false)) != WP_OK) return rc;
    if (st) {
        (void)hipMemsetAsync(ctx->status, 0, sizeof(int), ctx->stream);
        (void)hipStreamSynchronize(ctx->stream);
        if (st & ST_NONFINITE) return wp_fail(ctx, WP_ENONFINITE, "a step produced a non-finite value");
        if (st & ST_CFL) return wp_fail(ctx, WP_ECFL, "a step exceeded the Courant limit %g", ctx->prob.cfl_max);
    }
    return WP_OK;
}

extern "C" int wp_sync(wp_ctx *ctx)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    if (hipStreamSynchronize(ctx->stream) != hipSuccess)
        return wp_fail(ctx, WP_EDEVICE, "sync: %s", hipGetErrorString(hipGetLastError()));
    return wp_check_status(ctx);
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

extern "C" int wp_get_time(const wp_ctx *ctx, int level, double *t)
{
    if (!ctx) return WP_EINVAL;
    if (!t) return wp_fail_get(ctx, WP_EINVAL, "null output");
    if (level < 0 || level >= (int)ctx->L.size()) return wp_fail_get(ctx, WP_EINVAL, "level out of range");
    *t = ctx->L[level].t;
    return WP_OK;
}

extern "C" int wp_set_time(wp_ctx *ctx, int level, double t)
{
    WP_ABI_TRY
    if (!ctx || level < 0 || level >= (int)ctx->L.size()) return WP_EINVAL;
    ctx->L[level].t = t;
    ctx->L[level].prev_valid = false;
    return WP_OK;
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

extern "C" int wp_set_tile_rows(wp_ctx *ctx, int rows)
{
    WP_ABI_TRY
    if (!ctx || rows < 0 || rows > 4096) return WP_EINVAL;
    ctx->tile_rows = rows;
    int rc;
    for (auto &lv : ctx->L)
        if (!lv.patches.empty() && (rc = wp_upload_tiles(ctx, lv)) != WP_OK) return rc;
    if (ctx->adj_ready && (rc = wp_upload_tiles(ctx, ctx->adj)) != WP_OK) return rc;
    return WP_OK;
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

extern "C" int wp_get_tile_rows(const wp_ctx *ctx, int *rows)
{
    if (!ctx) return WP_EINVAL;
    if (!rows) return wp_fail_get(ctx, WP_EINVAL, "null output");
    *rows = ctx->tile_rows > 0 ? ctx->tile_rows : wp_default_rows(ctx, ctx->L[0]);
    return WP_OK;
}

// ---------------------------------------------------------------------------
// acoustics stepping
// ---------------------------------------------------------------------------
template <typename T>
static int ensure_acou_inst(wp_ctx *ctx, Level &lv, double dt)
{
    if (lv.inst && lv.inst_dt == dt && lv.inst_snap == lv.snap_base) return WP_OK;
    AcouInst<T> I;
    memset(&I, 0, sizeof I);
    I.q[0] = (T *)lv.q[0];
    I.q[1] = (T *)lv.q[1];
    I.mat = lv.mat;
    I.cs = (long long)lv.nx * lv.ny;
    I.nx = lv.nx;
    I.ny = lv.ny;
    for (int k = 0; k < 4; ++k) I.bc[k] = ctx->prob.bc[k];
    I.nux = (T)(dt / lv.dx);
    I.nuy = (T)(ctx->kind2d ? dt / lv.dy : 0.0);
    I.mtab = (const T *)ctx->mtab;
    I.ptab = (const T *)ctx->ptab;
    I.nmat = ctx->nmat;
    I.order = ctx->prob.order;
    I.limiter = ctx->prob.limiter;
    I.transverse = ctx->kind2d ? ctx->prob.transverse : 0;
    I.snap = (T *)lv.snap_base;
    I.snap_stride = (long long)lv.nx * lv.ny * ctx->m;
    if (!lv.inst) lv.inst = wp_dalloc(ctx, sizeof(AcouInst<T>));
    if (!lv.inst) return wp_fail(ctx, WP_ENOMEM, "instance");
    if (hipMemcpyAsync(lv.inst, &I, sizeof I, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        return wp_fail(ctx, WP_EDEVICE, "instance upload");
    lv.inst_dt = dt;
    lv.inst_snap = lv.snap_base;
    memcpy(lv.inst_host, &I, sizeof I);
    return WP_OK;
}

template <typename T>
static int acou_step(wp_ctx *ctx, Level &lv, double dt, int adjoint, hipStream_t stream, int snap_index)
{
    int rc;
    if ((rc = ensure_acou_inst<T>(ctx, lv, dt)) != WP_OK) return rc;
    if (stream != ctx->stream && lv.inst_dt != dt) return wp_fail(ctx, WP_ESTATE, "descriptor not prepared before capture");
    if (ctx->kind2d) {
        const bool full = ctx->prob.order == 2 && ctx->prob.limiter == 1 && ctx->prob.transverse == 1;
        const AcouInst<T> *I = (const AcouInst<T> *)lv.inst;
        // one launch: a single-material level runs the lean kernel, any other
        // the kernel that picks the path per tile
        if (lv.dual && adjoint) return wp_fail(ctx, WP_ESTATE, "adjoint step on a level with two tiles per wave");
        // the average onto the level below, when asked and the launch can
        AvgTo<T> avg{nullptr, 0, 0};
        lv.averaged = false;
        if (lv.avg_onto && !adjoint && acou2d_can_average(lv.dual, full, lv.tile_rows, lv.ratio)) {
            avg = AvgTo<T>{(T *)lv.avg_onto->q[lv.avg_onto->cur], lv.avg_onto->nx,
                           (long long)lv.avg_onto->nx * lv.avg_onto->ny};
            lv.averaged = true;
        }
        lv.avg_onto = nullptr;
        launch_acou2d<T>(I, lv.tiles_dev, lv.ntiles, lv.cur, adjoint, ctx->nmat, full, lv.tile_rows,
                         lv.nuni == lv.ntiles ? 1 : 0, snap_index, ctx->status, stream, ctx->stamp_next, lv.dual,
                         lv.averaged ? &avg : nullptr);
        ctx->stamp_next = nullptr;   // consumed by this launch only
    }
    else
        launch_acou1d<T>((const AcouInst<T> *)lv.inst, *(const AcouInst<T> *)lv.inst_host, lv.cur, adjoint, snap_index,
                         ctx->status, stream);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return wp_fail(ctx, WP_EDEVICE, "step launch: %s", hipGetErrorString(e));
    lv.cur ^= 1;
    return WP_OK;
}

// Two steps of a level in one launch; snap1 / snap2: snapshot slots of the
// first / second step (-1: none).  The result lands in the other canvas.
template <typename T>
static int acou_pair(wp_ctx *ctx, Level &lv, double dt, int adjoint, hipStream_t stream, int snap1, int snap2,
                     const PairFlag *flag)
{
    int rc;
    if ((rc = ensure_acou_inst<T>(ctx, lv, dt)) != WP_OK) return rc;
    if (stream != ctx->stream && lv.inst_dt != dt) return wp_fail(ctx, WP_ESTATE, "descriptor not prepared before capture");
    launch_acou2d_pair<T>((const AcouInst<T> *)lv.inst, lv.ptiles_dev, lv.nptiles, lv.cur, adjoint, ctx->nmat,
                          lv.pair_rows, lv.npuni == lv.nptiles ? 1 : 0, snap1, snap2, ctx->status, stream,
                          ctx->stamp_next, flag);
    ctx->stamp_next = nullptr;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return wp_fail(ctx, WP_EDEVICE, "step launch: %s", hipGetErrorString(e));
    lv.cur ^= 1;
    return WP_OK;
}

int wp_step_pair(wp_ctx *ctx, Level &lv, double dt, int adjoint, hipStream_t s, int snap1, int snap2,
                 const PairFlag *flag)
{
    if (!lv.tables_ok || !wp_pair_ready(ctx, lv))
        return wp_fail(ctx, WP_ESTATE, "level cannot take two steps per launch");
    if (ctx->esz == 8) return acou_pair<double>(ctx, lv, dt, adjoint, s, snap1, snap2, flag);
    return acou_pair<float>(ctx, lv, dt, adjoint, s, snap1, snap2, flag);
}

extern "C" int wp_set_step_pairs(wp_ctx *ctx, int rows)
{
    WP_ABI_TRY
    if (!ctx || !(rows == -1 || rows == 0 || (rows >= 4 && rows <= 64))) return WP_EINVAL;
    ctx->pair_rows = rows;
    int rc;
    for (auto &lv : ctx->L)
        if (!lv.patches.empty() && (rc = wp_upload_tiles(ctx, lv)) != WP_OK) return rc;
    if (ctx->adj_ready && (rc = wp_upload_tiles(ctx, ctx->adj)) != WP_OK) return rc;
    return WP_OK;
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

extern "C" int wp_get_step_pairs(const wp_ctx *ctx, int *rows)
{
    if (!ctx) return WP_EINVAL;
    if (!rows) return wp_fail_get(ctx, WP_EINVAL, "null output");
    *rows = ctx->L.empty() ? 0 : ctx->L[0].pair_rows;
    return WP_OK;
}

int wp_courant_check(wp_ctx *ctx, const Level &lv, double dt)
{
    if (!(dt > 0.0) || !std::isfinite(dt)) return wp_fail(ctx, WP_EINVAL, "dt must be positive");
    if (ctx->is_acoustics || &lv == &ctx->adj) {
        const double nu = ctx->cmax * dt / (ctx->kind2d ? std::min(lv.dx, lv.dy) : lv.dx);
        if (nu > ctx->prob.cfl_max * (1.0 + 1e-12))
            return wp_fail(ctx, WP_ECFL, "Courant number %.6g above %.6g", nu, ctx->prob.cfl_max);
    }
    return WP_OK;
}

// Make the level's instance descriptor current for step size dt (an upload
// when dt changed), so that a following capture records launches only.
int wp_prepare_level(wp_ctx *ctx, Level &lv, double dt)
{
    if (ctx->is_acoustics) return ctx->esz == 8 ? ensure_acou_inst<double>(ctx, lv, dt) : ensure_acou_inst<float>(ctx, lv, dt);
    return wp_swe_prepare(ctx, lv, dt);
}

int wp_step_level(wp_ctx *ctx, Level &lv, double dt, int adjoint, hipStream_t s, int snap_index)
{
    if (!lv.tables_ok) return wp_fail(ctx, WP_ESTATE, "tile tables missing after a failed rebuild");
    if (ctx->is_acoustics) {
        if (ctx->esz == 8) return acou_step<double>(ctx, lv, dt, adjoint, s, snap_index);
        return acou_step<float>(ctx, lv, dt, adjoint, s, snap_index);
    }
    return wp_swe_step(ctx, lv, dt, adjoint, s, snap_index);
}

// ---------------------------------------------------------------------------
// graphs: captured on an internal stream, replayed on the handle stream
// ---------------------------------------------------------------------------
double wp_now_ms()
{
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

extern "C" int wp_host_times(wp_ctx *ctx, double *ms, int n, int reset)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    if (n < 0 || (n > 0 && !ms)) return wp_fail(ctx, WP_EINVAL, "bad output");
    for (int k = 0; k < n && k < WP_HOST_TIMES; ++k) ms[k] = ctx->host_ms[k];
    for (int k = WP_HOST_TIMES; k < n; ++k) ms[k] = 0.0;
    if (reset)
        for (double &v : ctx->host_ms) v = 0.0;
    return WP_OK;
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

int wp_graph_begin(wp_ctx *ctx, hipStream_t &s)
{
    ctx->host_ms[HT_CAPTURE] -= wp_now_ms();
    if (!ctx->cap_stream) {
        if (hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking) != hipSuccess)
            return wp_fail(ctx, WP_EDEVICE, "capture stream creation failed");
    }
    s = ctx->cap_stream;
    if (hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return wp_fail(ctx, WP_EDEVICE, "stream capture begin: %s", hipGetErrorString(hipGetLastError()));
    return WP_OK;
}

// A sequence captured again with the same launches (new tile tables, sizes
// or time weights after a regrid) updates the instantiated graph in place;
// another shape of sequence is instantiated anew.
int wp_graph_end(wp_ctx *ctx, hipStream_t s, hipGraphExec_t &exec)
{
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(s, &g) != hipSuccess || !g) {
        ctx->host_ms[HT_CAPTURE] += wp_now_ms();
        return wp_fail(ctx, WP_EDEVICE, "stream capture end: %s", hipGetErrorString(hipGetLastError()));
    }
    ctx->host_ms[HT_NCAPTURE] += 1.0;
    if (exec) {
        hipGraphNode_t bad = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        if (hipGraphExecUpdate(exec, g, &bad, &res) == hipSuccess && res == hipGraphExecUpdateSuccess) {
            (void)hipGraphDestroy(g);
            ctx->host_ms[HT_NUPDATE] += 1.0;
            ctx->host_ms[HT_CAPTURE] += wp_now_ms();
            return WP_OK;
        }
        (void)hipGetLastError();
        (void)hipGraphExecDestroy(exec);
        exec = nullptr;
    }
    hipError_t e = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    ctx->host_ms[HT_CAPTURE] += wp_now_ms();
    if (e != hipSuccess) {
        exec = nullptr;
        return wp_fail(ctx, WP_EDEVICE, "graph instantiate: %s", hipGetErrorString(e));
    }
    return WP_OK;
}

// A captured sequence runs on the handle's stream, ordered with the rest of
// its work like any launch.
int wp_graph_launch(wp_ctx *ctx, hipGraphExec_t exec)
{
    if (hipGraphLaunch(exec, ctx->stream) != hipSuccess)
        return wp_fail(ctx, WP_EDEVICE, "graph launch: %s", hipGetErrorString(hipGetLastError()));
    return WP_OK;
}

extern "C" int wp_run_graph(wp_ctx *ctx, int nsteps, double dt, int replays)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    if (nsteps < 1 || replays < 0) return wp_fail(ctx, WP_EINVAL, "nsteps must be >= 1 and replays >= 0");
    if (ctx->L.size() != 1) return wp_fail(ctx, WP_EINVAL, "graph replay is for single-level instances (use wp_advance)");
    Level &lv = ctx->L[0];
    int rc;
    if ((rc = wp_courant_check(ctx, lv, dt)) != WP_OK) return rc;
    if (!ctx->graph_exec || ctx->graph_steps != nsteps || ctx->graph_dt != dt || ctx->graph_parity != lv.cur ||
        ctx->graph_gen != ctx->topo_gen) {
        if ((rc = wp_prepare_level(ctx, lv, dt)) != WP_OK) return rc;
        hipStream_t s;
        if ((rc = wp_graph_begin(ctx, s)) != WP_OK) return rc;
        int par = lv.cur;
        // two steps per launch where the level allows it
        const bool pairs = wp_pair_ready(ctx, lv);
        for (int k = 0; k < nsteps && rc == WP_OK;) {
            if (pairs && k + 1 < nsteps) {
                rc = wp_step_pair(ctx, lv, dt, ctx->equation, s, -1, -1);
                k += 2;
            } else {
                rc = wp_step_level(ctx, lv, dt, ctx->equation, s, -1);
                k += 1;
            }
        }
        ctx->graph_flip = lv.cur ^ par;
        lv.cur = par;
        int rc2 = wp_graph_end(ctx, s, ctx->graph_exec);
        if (rc != WP_OK) return rc;
        if (rc2 != WP_OK) return rc2;
        ctx->graph_steps = nsteps;
        ctx->graph_gen = ctx->topo_gen;
        ctx->graph_dt = dt;
        ctx->graph_parity = lv.cur;
    }
    // the other canvas ends two steps back when the last launch took two
    const double back = wp_pair_ready(ctx, lv) && nsteps % 2 == 0 ? 2.0 * dt : dt;
    for (int r = 0; r < replays; ++r) {
        if ((rc = wp_graph_launch(ctx, ctx->graph_exec)) != WP_OK) return rc;
        if (ctx->graph_flip) {
            // a sequence that ends on the other buffer: later replays need the
            // graph captured for that parity
            lv.cur ^= 1;
            lv.t += nsteps * dt;
            lv.t_prev = lv.t - back;
            lv.prev_valid = true;
            if (r + 1 < replays) return wp_run_graph(ctx, nsteps, dt, replays - r - 1);
            return WP_OK;
        }
        lv.t += nsteps * dt;
        lv.t_prev = lv.t - back;
        lv.prev_valid = true;
    }
    return WP_OK;
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

extern "C" int wp_step_patches(wp_ctx *ctx, int level, double dt)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    if (level < 0 || level >= (int)ctx->L.size()) return wp_fail(ctx, WP_EINVAL, "level %d out of range", level);
    Level &lv = ctx->L[level];
    int rc;
    if ((rc = wp_courant_check(ctx, lv, dt)) != WP_OK) return rc;
    if (lv.patches.empty()) {
        lv.t += dt;
        return WP_OK;
    }
    if (level > 0 && (rc = wp_fill_coarse_ghosts(ctx, level, lv.t)) != WP_OK) return rc;
    if ((rc = wp_step_level(ctx, lv, dt, ctx->equation, ctx->stream, -1)) != WP_OK) return rc;
    lv.t_prev = lv.t;
    lv.prev_valid = true;
    lv.t += dt;
    return WP_OK;
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

// The system the level hierarchy steps.  The adjoint acoustics update uses
// the same tiles except the two-tile waves of the forward kernel, so the
// tables are rebuilt (which also re-captures every cached sequence).
extern "C" int wp_set_equation(wp_ctx *ctx, int adjoint)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    if (adjoint != 0 && adjoint != 1) return wp_fail(ctx, WP_EINVAL, "equation must be 0 (forward) or 1 (adjoint)");
    if (!ctx->is_acoustics) return wp_fail(ctx, WP_EINVAL, "the adjoint hierarchy is for acoustics");
    if (ctx->equation == adjoint) return WP_OK;
    ctx->equation = adjoint;
    if (!adjoint) ctx->reflux = false;
    int rc;
    for (Level &lv : ctx->L)
        if (!lv.patches.empty() && (rc = wp_upload_tiles(ctx, lv)) != WP_OK) return rc;
    return WP_OK;
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

extern "C" int wp_set_reflux(wp_ctx *ctx, int on)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    if (on != 0 && on != 1) return wp_fail(ctx, WP_EINVAL, "on must be 0 or 1");
    if (on && !ctx->kind2d) return wp_fail(ctx, WP_EINVAL, "refluxing is for 2D hierarchies");
    if (on && ctx->is_acoustics && ctx->equation != 1)
        return wp_fail(ctx, WP_ESTATE, "refluxing needs the adjoint system (the forward one is not conservative)");
    if (ctx->reflux != (on == 1)) {
        ctx->reflux = on == 1;
        ++ctx->topo_gen;   // captured Berger-Oliger sequences gain or lose the correction
    }
    return WP_OK;
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

extern "C" int wp_get_reflux(const wp_ctx *ctx, int *on)
{
    if (!ctx || !on) return ctx ? wp_fail_get(ctx, WP_EINVAL, "null output") : WP_EINVAL;
    *on = ctx->reflux ? 1 : 0;
    return WP_OK;
}

extern "C" int wp_get_equation(const wp_ctx *ctx, int *adjoint)
{
    if (!ctx) return WP_EINVAL;
    if (!adjoint) return wp_fail_get(ctx, WP_EINVAL, "null output");
    *adjoint = ctx->equation;
    return WP_OK;
}

// ---------------------------------------------------------------------------
// adjoint run and snapshot store
// ---------------------------------------------------------------------------
static bool in_target(const wp_functional *J, double x, double y, bool is2d)
{
    switch (J->kind) {
    case WP_FUNC_INTERVAL: return x >= J->x0 && x <= J->x1;
    case WP_FUNC_BOX: return x >= J->x0 && x <= J->x1 && (!is2d || (y >= J->y0 && y <= J->y1));
    case WP_FUNC_DISC: {
        const double dx = x - J->cx, dy = y - J->cy;
        return dx * dx + dy * dy <= J->r * J->r;
    }
    }
    return false;
}

// indicator of the target region at level-0 cell centres (closed set)
int wp_build_indicator(wp_ctx *ctx, const wp_functional *J, std::vector<uint8_t> &ind)
{
    if (!J || J->kind < 0 || J->kind > 2 || J->component < 0 || J->component >= ctx->m)
        return wp_fail(ctx, WP_EINVAL, "bad functional");
    const Level &l0 = ctx->L[0];
    ind.assign((size_t)l0.nx * l0.ny, 0);
    for (int j = 0; j < l0.ny; ++j)
        for (int i = 0; i < l0.nx; ++i) {
            const double x = ctx->grid.xlo + (i + 0.5) * l0.dx;
            const double y = ctx->kind2d ? ctx->grid.ylo + (j + 0.5) * l0.dy : 0.0;
            ind[(size_t)j * l0.nx + i] = in_target(J, x, y, ctx->kind2d) ? 1 : 0;
        }
    return WP_OK;
}

// Release every block a level holds and reset it.
static void release_level(wp_ctx *ctx, Level &lv)
{
    void *blocks[] = {lv.q[0], lv.q[1], lv.mat, lv.flags, lv.tiles_dev, lv.ptiles_dev, lv.ftiles_dev, lv.inst,
                      lv.ring_dev, lv.ringb_dev, lv.cover_dev};
    for (void *p : blocks) wp_dfree(ctx, p);
    lv = Level();
}

// The adjoint grid, built on first use; a failed build releases what it
// allocated so that the next call starts again from nothing.
int wp_ensure_adjoint_level(wp_ctx *ctx)
{
    Level &a = ctx->adj;
    if (ctx->adj_ready) return WP_OK;
    release_level(ctx, a);
    const Level &l0 = ctx->L[0];
    a.nx = l0.nx;
    a.ny = l0.ny;
    a.dx = l0.dx;
    a.dy = l0.dy;
    a.ratio = 1;
    int rc = wp_alloc_level(ctx, a);
    if (rc == WP_OK) {
        a.patches.push_back(wp_patch{0, 0, a.nx, a.ny});
        if (!ctx->is_acoustics) rc = wp_swe_adj_init(ctx);
    }
    if (rc == WP_OK) rc = wp_upload_tiles(ctx, a);
    if (rc != WP_OK) {
        release_level(ctx, a);
        return rc;
    }
    ctx->adj_ready = true;
    return WP_OK;
}

// Everything of an adjoint run but the stepping: snapshot store, phi on the
// device, qtilde(x, 0) = phi in the adjoint canvas and in snapshot 0, and a
// descriptor whose steps write the store.  Shared by wp_adjoint_run and the
// batched adjoint run.
int wp_adjoint_setup(wp_ctx *ctx, const wp_functional *J, const wp_snapshot_spec *sp)
{
    if (!sp || sp->nsteps < 0 || sp->snap_every < 1 || sp->nsteps % sp->snap_every != 0)
        return wp_fail(ctx, WP_EINVAL, "snapshot spec: nsteps must be a non-negative multiple of snap_every >= 1");
    int rc;
    if (!J || J->kind < 0 || J->kind > 2 || J->component < 0 || J->component >= ctx->m)
        return wp_fail(ctx, WP_EINVAL, "bad functional");
    if ((rc = wp_ensure_adjoint_level(ctx)) != WP_OK) return rc;
    Level &a = ctx->adj;
    if ((rc = wp_courant_check(ctx, a, sp->dt)) != WP_OK) return rc;
    const long long cells = (long long)a.nx * a.ny;
    const int nsnap = sp->nsteps / sp->snap_every + 1;
    const size_t snap_bytes = (size_t)cells * ctx->m * ctx->snap_esz();
    if (ctx->snaps_cap < (size_t)nsnap * snap_bytes) {
        if (ctx->snaps) wp_dfree(ctx, ctx->snaps);
        ctx->snaps = wp_dalloc(ctx, (size_t)nsnap * snap_bytes);
        if (!ctx->snaps) {
            ctx->snaps_cap = 0;
            ctx->nsnap = 0;
            return wp_fail(ctx, WP_ENOMEM, "snapshot store (%d x %zu bytes)", nsnap, snap_bytes);
        }
        ctx->snaps_cap = (size_t)nsnap * snap_bytes;
    }
    // qtilde(x, 0) = phi = I(x) e_component, kept on the device per functional
    if (!ctx->phi_valid || memcmp(&ctx->phi_key, J, sizeof *J) != 0) {
        std::vector<uint8_t> ind;
        if ((rc = wp_build_indicator(ctx, J, ind)) != WP_OK) return rc;
        const size_t es = ctx->snap_esz();
        std::vector<char> host(snap_bytes, 0);
        for (long long k = 0; k < cells; ++k)
            if (ind[k]) {
                char *dst = host.data() + ((size_t)J->component * cells + k) * es;
                if (es == 8) { double one = 1.0; memcpy(dst, &one, 8); }
                else { float one = 1.0f; memcpy(dst, &one, 4); }
            }
        if (!ctx->phi_dev) ctx->phi_dev = wp_dalloc(ctx, snap_bytes);
        if (!ctx->phi_dev) return wp_fail(ctx, WP_ENOMEM, "adjoint initial data");
        if (hipMemcpy(ctx->phi_dev, host.data(), snap_bytes, hipMemcpyHostToDevice) != hipSuccess)
            return wp_fail(ctx, WP_EDEVICE, "adjoint initial data upload");
        ctx->phi_key = *J;
        ctx->phi_valid = true;
    }
    ctx->nsnap = 0;
    a.snap_base = ctx->snaps;
    if ((rc = wp_prepare_level(ctx, a, sp->dt)) != WP_OK) return rc;
    a.cur = 0;
    if (hipMemcpyAsync(a.q[0], ctx->phi_dev, snap_bytes, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess ||
        hipMemcpyAsync(ctx->snaps, ctx->phi_dev, snap_bytes, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess)
        return wp_fail(ctx, WP_EDEVICE, "adjoint initial data copy");
    ctx->snap_bytes = snap_bytes;
    return WP_OK;
}

void wp_adjoint_finish(wp_ctx *ctx, const wp_snapshot_spec *sp)
{
    ctx->nsnap = sp->nsteps / sp->snap_every + 1;
    ctx->snap_ds = sp->dt * sp->snap_every;
    ctx->adj_tf = sp->dt * sp->nsteps;
    ctx->adj.t = ctx->adj_tf;
}

extern "C" int wp_adjoint_run(wp_ctx *ctx, const wp_functional *J, const wp_snapshot_spec *sp)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    int rc;
    if ((rc = wp_adjoint_setup(ctx, J, sp)) != WP_OK) return rc;
    Level &a = ctx->adj;
    // the whole run is one captured graph, re-captured only when the step
    // count, interval, dt or store change; the stencil writes each snapshot
    // itself on its snapshot steps
    if (!ctx->adj_exec || ctx->adj_steps != sp->nsteps || ctx->adj_every != sp->snap_every || ctx->adj_dt != sp->dt ||
        ctx->adj_snaps != ctx->snaps || ctx->adj_gen != ctx->topo_gen) {
        hipStream_t cs;
        if ((rc = wp_graph_begin(ctx, cs)) != WP_OK) return rc;
        auto snap_of = [&](int s) { return s % sp->snap_every == 0 ? s / sp->snap_every : -1; };
        const bool pairs = wp_pair_ready(ctx, a);
        for (int s = 1; s <= sp->nsteps && rc == WP_OK;) {
            if (pairs && s + 1 <= sp->nsteps) {
                rc = wp_step_pair(ctx, a, sp->dt, 1, cs, snap_of(s), snap_of(s + 1));
                s += 2;
            } else {
                rc = wp_step_level(ctx, a, sp->dt, 1, cs, snap_of(s));
                s += 1;
            }
        }
        int rc2 = wp_graph_end(ctx, cs, ctx->adj_exec);
        if (rc != WP_OK) return rc;
        if (rc2 != WP_OK) return rc2;
        ctx->adj_end = a.cur;
        ctx->adj_steps = sp->nsteps;
        ctx->adj_gen = ctx->topo_gen;
        ctx->adj_every = sp->snap_every;
        ctx->adj_dt = sp->dt;
        ctx->adj_snaps = ctx->snaps;
    } else {
        a.cur = ctx->adj_end;
    }
    if ((rc = wp_graph_launch(ctx, ctx->adj_exec)) != WP_OK) return rc;
    wp_adjoint_finish(ctx, sp);
    return wp_sync(ctx);
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

extern "C" int wp_num_snapshots(const wp_ctx *ctx) { return ctx ? ctx->nsnap : 0; }

extern "C" int wp_get_snapshot(wp_ctx *ctx, int n, void *dst, int on_device)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    if (n < 0 || n >= ctx->nsnap) return wp_fail(ctx, WP_ERANGE, "snapshot %d of %d", n, ctx->nsnap);
    if (!dst) return wp_fail(ctx, WP_EINVAL, "null destination");
    const char *src = (const char *)ctx->snaps + (size_t)n * ctx->snap_bytes;
    if (!on_device) return wp_host_copy(ctx, dst, src, ctx->snap_bytes, false);
    if (hipMemcpyAsync(dst, src, ctx->snap_bytes, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess)
        return wp_fail(ctx, WP_EDEVICE, "snapshot read");
    return WP_OK;
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

// A snapshot store computed elsewhere (e.g. the level-0 composite of an
// adjoint solved with refinement) replaces the store of the last adjoint run.
extern "C" int wp_set_snapshots(wp_ctx *ctx, const void *src, int nsnap, double ds, int on_device)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    if (!src) return wp_fail(ctx, WP_EINVAL, "null source");
    if (nsnap < 1) return wp_fail(ctx, WP_EINVAL, "at least one snapshot is needed");
    if (!(ds > 0.0) || !std::isfinite(ds)) return wp_fail(ctx, WP_EINVAL, "ds must be positive");
    int rc;
    if ((rc = wp_ensure_adjoint_level(ctx)) != WP_OK) return rc;
    const Level &a = ctx->adj;
    const size_t snap_bytes = (size_t)a.nx * a.ny * ctx->m * ctx->snap_esz();
    const size_t bytes = (size_t)nsnap * snap_bytes;
    if (ctx->snaps_cap < bytes) {
        if (ctx->snaps) wp_dfree(ctx, ctx->snaps);
        ctx->snaps_cap = 0;
        ctx->nsnap = 0;
        ctx->snaps = wp_dalloc(ctx, bytes);
        if (!ctx->snaps) return wp_fail(ctx, WP_ENOMEM, "snapshot store (%d x %zu bytes)", nsnap, snap_bytes);
        ctx->snaps_cap = bytes;
    }
    ctx->nsnap = 0;   // no store until the copy is complete
    if (on_device) {
        if (hipMemcpyAsync(ctx->snaps, src, bytes, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess ||
            hipStreamSynchronize(ctx->stream) != hipSuccess)
            return wp_fail(ctx, WP_EDEVICE, "snapshot store copy");
    } else if ((rc = wp_host_copy(ctx, ctx->snaps, src, bytes, true)) != WP_OK) {
        return rc;
    }
    ctx->snap_bytes = snap_bytes;
    ctx->nsnap = nsnap;
    ctx->snap_ds = ds;
    ctx->adj_tf = ds * (nsnap - 1);
    return WP_OK;
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

// ---------------------------------------------------------------------------
// flagging
// ---------------------------------------------------------------------------
int wp_window(wp_ctx *ctx, double t, double t_s, double t_f, int &n_lo, int &n_hi)
{
    if (ctx->nsnap <= 0) return wp_fail(ctx, WP_ESTATE, "no adjoint snapshots (run wp_adjoint_run first)");
    if (!(t_s <= t_f)) return wp_fail(ctx, WP_EINVAL, "t_s must not exceed t_f");
    const double ds = ctx->snap_ds, slack = 1e-9;
    const double T = std::min(t + t_f - t_s, t_f);
    long long hi = (long long)std::ceil((t_f - t) / ds - slack);
    long long lo = (long long)std::floor((t_f - T) / ds + slack);
    lo = std::max(lo, 0LL);
    hi = std::max(hi, lo);
    if (hi > ctx->nsnap - 1)
        return wp_fail(ctx, WP_ERANGE, "window at t=%g reaches snapshot %lld of %d", t, hi, ctx->nsnap);
    n_lo = (int)lo;
    n_hi = (int)hi;
    return WP_OK;
}

// Enqueue the flag of `level` for snapshot window [n_lo, n_hi] on stream s,
// adding the number of flagged cells to *count (which the caller clears).
static int flag_launch(wp_ctx *ctx, int level, double tol, int n_lo, int n_hi, unsigned long long *count,
                       hipStream_t s)
{
    Level &lv = ctx->L[level];
    if (!lv.tables_ok) return wp_fail(ctx, WP_ESTATE, "tile tables missing after a failed rebuild");
    const long long cells = (long long)lv.nx * lv.ny;
    int ratio = 1;
    for (int l = 1; l <= level; ++l) ratio *= ctx->L[l].ratio;
    // cells outside the patches read 0 (a level covered by one patch has none)
    const bool full = lv.patches.size() == 1 && lv.patches[0].nx == lv.nx && lv.patches[0].ny == lv.ny;
    if (!full) launch_fill_u8(lv.flags, cells, 0, s);
    const Level &a0 = ctx->adj;
    const long long hcs = (long long)a0.nx * a0.ny;
    const long long sstride = hcs * ctx->m;
    if (ctx->prob.precision == WP_MIXED) {
        launch_flag_mixed((const double *)lv.q[lv.cur], (const float *)((char *)lv.q[lv.cur] + cells * 8),
                          (const float *)((char *)lv.q[lv.cur] + cells * 12), cells, lv.nx, lv.ny,
                          (const float *)ctx->snaps, sstride, hcs, a0.nx, a0.ny, ratio, n_lo, n_hi, tol,
                          lv.ftiles_dev, lv.nftiles, lv.flags, count, s);
    } else if (ctx->esz == 8) {
        launch_flag<double, double>((const double *)lv.q[lv.cur], cells, lv.nx, lv.ny, ctx->m,
                                    (const double *)ctx->snaps, sstride, hcs, a0.nx, a0.ny, ratio, n_lo, n_hi, tol,
                                    lv.ftiles_dev, lv.nftiles, lv.flags, count, s);
    } else {
        launch_flag<float, float>((const float *)lv.q[lv.cur], cells, lv.nx, lv.ny, ctx->m, (const float *)ctx->snaps,
                                  sstride, hcs, a0.nx, a0.ny, ratio, n_lo, n_hi, tol, lv.ftiles_dev, lv.nftiles,
                                  lv.flags, count, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return wp_fail(ctx, WP_EDEVICE, "flag launch: %s", hipGetErrorString(e));
    lv.flags_valid = true;
    return WP_OK;
}

extern "C" int wp_flag_adjoint(wp_ctx *ctx, int level, double tol, double t, double t_s, double t_f, uint8_t *flags,
                               int on_device, int64_t *nflagged)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    if (level < 0 || level >= (int)ctx->L.size()) return wp_fail(ctx, WP_EINVAL, "level out of range");
    int n_lo, n_hi, rc;
    if ((rc = wp_window(ctx, t, t_s, t_f, n_lo, n_hi)) != WP_OK) return rc;
    Level &lv = ctx->L[level];
    const long long cells = (long long)lv.nx * lv.ny;
    if ((rc = wp_clear_counts(ctx, ctx->count, 1, ctx->stream)) != WP_OK) return rc;
    if ((rc = flag_launch(ctx, level, tol, n_lo, n_hi, ctx->count, ctx->stream)) != WP_OK) return rc;
    if (flags && on_device &&
        hipMemcpyAsync(flags, lv.flags, (size_t)cells, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess)
        return wp_fail(ctx, WP_EDEVICE, "flag copy");
    if (flags && !on_device && (rc = wp_host_copy(ctx, flags, lv.flags, (size_t)cells, false)) != WP_OK) return rc;
    if (nflagged && (rc = wp_read_counts(ctx, ctx->count, 1, nflagged)) != WP_OK) return rc;
    return WP_OK;
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

extern "C" int wp_get_flags(wp_ctx *ctx, int level, uint8_t *dst, int on_device)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    if (level < 0 || level >= (int)ctx->L.size()) return wp_fail(ctx, WP_EINVAL, "level out of range");
    if (!dst) return wp_fail(ctx, WP_EINVAL, "null destination");
    Level &lv = ctx->L[level];
    if (!lv.flags_valid) return wp_fail(ctx, WP_ESTATE, "level %d has no flags", level);
    const size_t cells = (size_t)lv.nx * lv.ny;
    if (on_device) {
        if (hipMemcpyAsync(dst, lv.flags, cells, hipMemcpyDeviceToDevice, ctx->stream) != hipSuccess)
            return wp_fail(ctx, WP_EDEVICE, "flag copy");
        return WP_OK;
    }
    return wp_host_copy(ctx, dst, lv.flags, cells, false);
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

// The comparison flags (Sec. 5.2.4, Sec. 5.3) on every patch of a level, with
// the count and the copy-out of wp_flag_adjoint.  A refined level's ghost
// ring is filled from the level below at the level's time first, so that the
// cells along a patch edge see their neighbours.
static int flag_standard(wp_ctx *ctx, int level, bool surface, double tol, uint8_t *flags, int on_device,
                         int64_t *nflagged)
{
    if (!ctx) return WP_EINVAL;
    if (level < 0 || level >= (int)ctx->L.size()) return wp_fail(ctx, WP_EINVAL, "level out of range");
    if (surface && ctx->is_acoustics) return wp_fail(ctx, WP_EINVAL, "the surface flag is for shallow water");
    if (!(tol >= 0.0)) return wp_fail(ctx, WP_EINVAL, "tolerance must be non-negative");
    Level &lv = ctx->L[level];
    if (!lv.tables_ok) return wp_fail(ctx, WP_ESTATE, "tile tables missing after a failed rebuild");
    const long long cells = (long long)lv.nx * lv.ny;
    hipStream_t s = ctx->stream;
    int rc;
    if (!surface && level > 0 && !lv.patches.empty() && (rc = wp_fill_coarse_ghosts(ctx, level, lv.t)) != WP_OK)
        return rc;
    if ((rc = wp_clear_counts(ctx, ctx->count, 1, s)) != WP_OK) return rc;
    const bool full = lv.patches.size() == 1 && lv.patches[0].nx == lv.nx && lv.patches[0].ny == lv.ny;
    if (!full) launch_fill_u8(lv.flags, cells, 0, s);
    const char *q = (const char *)lv.q[lv.cur];
    const int m = ctx->m;
    if (surface) {
        if (ctx->esz == 8 || ctx->prob.precision == WP_MIXED)
            launch_flag_surface<double>((const double *)q, lv.nx, tol, lv.ftiles_dev, lv.nftiles, lv.flags, ctx->count,
                                        s);
        else
            launch_flag_surface<float>((const float *)q, lv.nx, tol, lv.ftiles_dev, lv.nftiles, lv.flags, ctx->count,
                                       s);
    } else if (ctx->prob.precision == WP_MIXED) {
        launch_flag_difference<double, float>((const double *)q, (const float *)(q + cells * 8),
                                              (const float *)(q + cells * 12), lv.nx, lv.ny, ctx->prob.bc, tol,
                                              lv.ftiles_dev, lv.nftiles, lv.flags, ctx->count, s);
    } else if (ctx->esz == 8) {
        const double *c = (const double *)q;
        launch_flag_difference<double, double>(c, c + cells, m > 2 ? c + 2 * cells : nullptr, lv.nx, lv.ny,
                                               ctx->prob.bc, tol, lv.ftiles_dev, lv.nftiles, lv.flags, ctx->count, s);
    } else {
        const float *c = (const float *)q;
        launch_flag_difference<float, float>(c, c + cells, m > 2 ? c + 2 * cells : nullptr, lv.nx, lv.ny,
                                             ctx->prob.bc, tol, lv.ftiles_dev, lv.nftiles, lv.flags, ctx->count, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return wp_fail(ctx, WP_EDEVICE, "flag launch: %s", hipGetErrorString(e));
    lv.flags_valid = true;
    if (flags && on_device &&
        hipMemcpyAsync(flags, lv.flags, (size_t)cells, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return wp_fail(ctx, WP_EDEVICE, "flag copy");
    if (flags && !on_device && (rc = wp_host_copy(ctx, flags, lv.flags, (size_t)cells, false)) != WP_OK) return rc;
    if (nflagged && (rc = wp_read_counts(ctx, ctx->count, 1, nflagged)) != WP_OK) return rc;
    return WP_OK;
}

extern "C" int wp_flag_difference(wp_ctx *ctx, int level, double tol, uint8_t *flags, int on_device,
                                  int64_t *nflagged)
{
    WP_ABI_TRY
    return flag_standard(ctx, level, false, tol, flags, on_device, nflagged);
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

extern "C" int wp_flag_surface(wp_ctx *ctx, int level, double tol, uint8_t *flags, int on_device, int64_t *nflagged)
{
    WP_ABI_TRY
    return flag_standard(ctx, level, true, tol, flags, on_device, nflagged);
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

// Richardson error estimate and flag (the estimator that Sec. 1 describes
// and the Future Work section proposes to weight by the adjoint).  Two steps
// of dt from the level-0 state on a copy of the problem at the same
// resolution, one step of 2 dt from its 2 x 2 block means on a copy at half
// the resolution (each coarse cell with the medium of its lower-left fine
// cell); E = (coarse - block mean of fine) / (2^(p+1) - 2).
// Single-level copy of the problem at the resolution of `level` (which 0) or
// half of it (which 1), made on first use and kept per level; cell (i, j)
// takes the medium of the level cell (f i, f j), itself that of the level-0
// cell containing it.
static int rich_helper(wp_ctx *ctx, int which, int level, wp_ctx *&out)
{
    if (out) return out->stream == ctx->stream ? WP_OK : wp_set_stream(out, ctx->stream);
    int R = 1;
    for (int l = 1; l <= level; ++l) R *= ctx->L[l].ratio;
    const int nx0 = ctx->grid.nx0, nx = ctx->L[level].nx, ny = ctx->L[level].ny;
    const int f = which == 0 ? 1 : 2;
    const int hx = nx / f, hy = ny / f;
    std::vector<double> rho((size_t)hx * hy), K((size_t)hx * hy);
    for (int j = 0; j < hy; ++j)
        for (int i = 0; i < hx; ++i) {
            const uint8_t m = ctx->mat0[(size_t)(f * j / R) * nx0 + f * i / R];
            rho[(size_t)j * hx + i] = ctx->rho[m];
            K[(size_t)j * hx + i] = ctx->K[m];
        }
    wp_grid g = ctx->grid;
    g.nx0 = hx;
    g.ny0 = hy;
    g.num_levels = 1;
    const wp_coefficients coef{rho.data(), K.data(), nullptr};
    const int rc = wp_create(&ctx->prob, &coef, &g, ctx->has_alloc ? &ctx->alloc : nullptr, ctx->stream, &out);
    if (rc != WP_OK) return wp_fail(ctx, rc, "Richardson estimate: helper instance: %s", wp_status_string(rc));
    return WP_OK;
}

// Coarse cells (half the resolution of a refined level) whose estimate only
// reads cells of the level's patches: the 2 x 2 block of fine cells and
// every fine cell within `margin` of it (square neighbourhood, clipped to
// the domain) lie in the patches.  Two fine steps and one coarse step of the
// 2D update reach two cells per step, four fine cells in all.
static void rich_valid(const Level &lv, int margin, std::vector<uint8_t> &valid)
{
    const int nx = lv.nx, ny = lv.ny;
    std::vector<uint8_t> outside((size_t)nx * ny, 1), bad;
    for (const wp_patch &p : lv.patches)
        for (int j = p.jlo; j < p.jlo + p.ny; ++j) std::fill_n(&outside[(size_t)j * nx + p.ilo], p.nx, (uint8_t)0);
    wp_dilate(outside, nx, ny, margin, bad);
    const int NX = nx / 2, NY = ny / 2;
    valid.assign((size_t)NX * NY, 0);
    for (int J = 0; J < NY; ++J)
        for (int I = 0; I < NX; ++I) {
            bool ok = true;
            for (int b = 0; b < 2 && ok; ++b)
                for (int a = 0; a < 2 && ok; ++a) ok = !bad[(size_t)(2 * J + b) * nx + 2 * I + a];
            valid[(size_t)J * NX + I] = ok;
        }
}

extern "C" int wp_flag_richardson(wp_ctx *ctx, int level, double dt, int weighted, double tol, double t, double t_s,
                                  double t_f, uint8_t *flags, int on_device, int64_t *nflagged, double *estimate)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    if (level < 0 || level >= (int)ctx->L.size()) return wp_fail(ctx, WP_EINVAL, "level %d out of range", level);
    if (ctx->L[level].patches.empty()) return wp_fail(ctx, WP_EINVAL, "level %d has no patches", level);
    if (ctx->equation != 0)
        return wp_fail(ctx, WP_ESTATE, "the Richardson estimate is for the forward system");
    if (!ctx->is_acoustics || !ctx->kind2d) return wp_fail(ctx, WP_EINVAL, "the Richardson estimate is for 2D acoustics");
    if (ctx->L[level].nx % 2 || ctx->L[level].ny % 2 || ctx->L[level].nx < 4 || ctx->L[level].ny < 4)
        return wp_fail(ctx, WP_EINVAL, "the Richardson estimate needs even grid sizes of at least 4");
    if (!(dt > 0.0)) return wp_fail(ctx, WP_EINVAL, "dt must be positive");
    if (!(tol >= 0.0)) return wp_fail(ctx, WP_EINVAL, "tolerance must be non-negative");
    int rc, n_lo = 0, n_hi = -1;
    if (weighted && (rc = wp_window(ctx, t, t_s, t_f, n_lo, n_hi)) != WP_OK) return rc;
    Level &lv = ctx->L[level];
    if ((rc = wp_courant_check(ctx, lv, dt)) != WP_OK) return rc;
    if (ctx->rich.size() < 2 * ctx->L.size()) ctx->rich.resize(2 * ctx->L.size(), nullptr);
    for (int k = 0; k < 2; ++k)
        if ((rc = rich_helper(ctx, k, level, ctx->rich[2 * level + k])) != WP_OK) return rc;
    wp_ctx *F = ctx->rich[2 * level], *C = ctx->rich[2 * level + 1];
    Level &fl = F->L[0], &cl = C->L[0];
    const int nx = lv.nx, ny = lv.ny, NX = nx / 2, NY = ny / 2, m = ctx->m;
    const long long cs = (long long)nx * ny, ccs = (long long)NX * NY;
    hipStream_t s = ctx->stream;
    if (hipMemcpyAsync(fl.q[fl.cur], lv.q[lv.cur], (size_t)cs * m * ctx->esz, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return wp_fail(ctx, WP_EDEVICE, "Richardson estimate: state copy");
    if (ctx->esz == 8)
        launch_coarsen2<double>((const double *)lv.q[lv.cur], cs, nx, (double *)cl.q[cl.cur], ccs, NX, NY, m, s);
    else
        launch_coarsen2<float>((const float *)lv.q[lv.cur], cs, nx, (float *)cl.q[cl.cur], ccs, NX, NY, m, s);
    fl.prev_valid = cl.prev_valid = false;
    for (int k = 0; k < 2 && rc == WP_OK; ++k) rc = wp_step_patches(F, 0, dt);
    if (rc == WP_OK) rc = wp_step_patches(C, 0, 2.0 * dt);
    if (rc != WP_OK) return wp_fail(ctx, rc, "Richardson estimate: %s", F->err.empty() ? C->err.c_str() : F->err.c_str());
    const size_t ebytes = sizeof(double) * (size_t)ccs * m;
    if (ctx->richE_cap < ebytes) {
        if (ctx->richE) wp_dfree(ctx, ctx->richE);
        ctx->richE = (double *)wp_dalloc(ctx, ebytes);
        ctx->richE_cap = ctx->richE ? ebytes : 0;
        if (!ctx->richE) return wp_fail(ctx, WP_ENOMEM, "Richardson estimate buffer");
    }
    if ((rc = wp_clear_counts(ctx, ctx->count, 1, s)) != WP_OK) return rc;
    const double denom = (double)((1 << (ctx->prob.order + 1)) - 2);
    const long long hcs = cs, sstride = cs * m;
    const void *snaps = weighted ? ctx->snaps : nullptr;
    if (level > 0) {
        std::vector<uint8_t> valid;
        rich_valid(lv, 4, valid);
        void *vd = ctx->rich_valid;
        rc = wp_upload(ctx, valid.data(), valid.size(), vd, ctx->rich_valid_cap, "Richardson mask");
        ctx->rich_valid = (uint8_t *)vd;
        if (rc != WP_OK) return rc;
        launch_fill_u8(lv.flags, cs, 0, s);
        // weighted: the estimate alone here, its flag below
        const int nt = weighted ? 0 : lv.nftiles;
        if (ctx->esz == 8)
            launch_richardson_masked<double>((const double *)cl.q[cl.cur], ccs, (const double *)fl.q[fl.cur], cs, nx,
                                             NX, NY, m, denom, ctx->richE, ctx->rich_valid, tol, lv.ftiles_dev, nt,
                                             lv.flags, ctx->count, s);
        else
            launch_richardson_masked<float>((const float *)cl.q[cl.cur], ccs, (const float *)fl.q[fl.cur], cs, nx, NX,
                                            NY, m, denom, ctx->richE, ctx->rich_valid, tol, lv.ftiles_dev, nt,
                                            lv.flags, ctx->count, s);
        if (weighted) {
            // each fine cell carries its parent's E; the adjoint flag then
            // interpolates the snapshots to the level's cells
            const size_t fbytes = sizeof(double) * (size_t)cs * m;
            if (ctx->richEf_cap < fbytes) {
                if (ctx->richEf) wp_dfree(ctx, ctx->richEf);
                ctx->richEf = (double *)wp_dalloc(ctx, fbytes);
                ctx->richEf_cap = ctx->richEf ? fbytes : 0;
                if (!ctx->richEf) return wp_fail(ctx, WP_ENOMEM, "Richardson estimate on the level's cells");
            }
            launch_expand_estimate(ctx->richE, NX, NY, m, ctx->richEf, nx, ny, s);
            int R = 1;
            for (int l = 1; l <= level; ++l) R *= ctx->L[l].ratio;
            const Level &a0 = ctx->adj;
            const long long acs = (long long)a0.nx * a0.ny;
            if (ctx->esz == 8)
                launch_flag<double, double>(ctx->richEf, cs, nx, ny, m, (const double *)ctx->snaps, acs * m, acs, a0.nx,
                                            a0.ny, R, n_lo, n_hi, tol, lv.ftiles_dev, lv.nftiles, lv.flags, ctx->count,
                                            s);
            else
                launch_flag<double, float>(ctx->richEf, cs, nx, ny, m, (const float *)ctx->snaps, acs * m, acs, a0.nx,
                                           a0.ny, R, n_lo, n_hi, tol, lv.ftiles_dev, lv.nftiles, lv.flags, ctx->count,
                                           s);
        }
    } else if (ctx->esz == 8) {
        launch_richardson<double>((const double *)cl.q[cl.cur], ccs, (const double *)fl.q[fl.cur], cs, nx, NX, NY, m,
                                  denom, ctx->richE, snaps, sstride, hcs, n_lo, n_hi, tol, lv.ftiles_dev, lv.nftiles,
                                  lv.flags, ctx->count, s);
    } else {
        launch_richardson<float>((const float *)cl.q[cl.cur], ccs, (const float *)fl.q[fl.cur], cs, nx, NX, NY, m,
                                 denom, ctx->richE, snaps, sstride, hcs, n_lo, n_hi, tol, lv.ftiles_dev, lv.nftiles,
                                 lv.flags, ctx->count, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return wp_fail(ctx, WP_EDEVICE, "Richardson launch: %s", hipGetErrorString(e));
    lv.flags_valid = true;
    if (flags && on_device &&
        hipMemcpyAsync(flags, lv.flags, (size_t)cs, hipMemcpyDeviceToDevice, s) != hipSuccess)
        return wp_fail(ctx, WP_EDEVICE, "flag copy");
    if (flags && !on_device && (rc = wp_host_copy(ctx, flags, lv.flags, (size_t)cs, false)) != WP_OK) return rc;
    if (estimate && (rc = wp_host_copy(ctx, estimate, ctx->richE, ebytes, false)) != WP_OK) return rc;
    if (nflagged && (rc = wp_read_counts(ctx, ctx->count, 1, nflagged)) != WP_OK) return rc;
    return WP_OK;
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

// The flagged forward run as one captured sequence: a clear of the event
// counters, then per event the flag at the block's start time and the
// block's steps, the first two of which record their workgroups' start and
// end times on the device clock.  Re-captured when any parameter,
// the start time, the canvas parity or a tile table changes.
extern "C" int wp_forward_flagged(wp_ctx *ctx, double dt, int nsteps, int flag_every, double tol, double t_s,
                                  double t_f, int64_t *counts, float *step_ms)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    if (ctx->L.size() != 1) return wp_fail(ctx, WP_EINVAL, "flagged forward runs are for single-level instances");
    if (ctx->equation != 0) return wp_fail(ctx, WP_ESTATE, "flagged forward run on a hierarchy set to the adjoint system");
    if (flag_every < 1 || nsteps < 0 || nsteps % flag_every != 0)
        return wp_fail(ctx, WP_EINVAL, "nsteps must be a non-negative multiple of flag_every >= 1");
    Level &lv = ctx->L[0];
    int rc;
    if ((rc = wp_courant_check(ctx, lv, dt)) != WP_OK) return rc;
    const int nev = nsteps / flag_every;
    if (nev == 0) return WP_OK;
    // every window is checked before anything is enqueued
    std::vector<int> lo(nev), hi(nev);
    for (int k = 0; k < nev; ++k)
        if ((rc = wp_window(ctx, lv.t + (double)k * flag_every * dt, t_s, t_f, lo[k], hi[k])) != WP_OK) return rc;
    if ((int)ctx->ev_counts_cap < nev) {
        if (ctx->ev_counts) wp_dfree(ctx, ctx->ev_counts);
        ctx->ev_counts = (unsigned long long *)wp_dalloc(ctx, sizeof(unsigned long long) * COUNT_SPAN * nev);
        if (!ctx->ev_counts) {
            ctx->ev_counts_cap = 0;
            return wp_fail(ctx, WP_ENOMEM, "flag counters");
        }
        ctx->ev_counts_cap = nev;
        ctx->ff_gen = 0;   // pointer changed
    }
    // launch clocks: one (start, end) slot per workgroup of the first two
    // launches of every block (a launch takes two steps where the level
    // allows it)
    // A block's first launch takes the block's flag as well when it takes two
    // steps (acoustics, level 0 on the adjoint grid); the timed launches are
    // then the two after it where the block has them.
    const bool pairs = wp_pair_ready(ctx, lv);
    const bool fuse = pairs && flag_every >= 2;
    const int nlaunch = pairs ? flag_every / 2 + (flag_every & 1) : flag_every;
    const int tfirst = fuse && nlaunch >= 3 ? 1 : 0;
    const int ntimed = std::min(nlaunch - tfirst, 2);
    auto is_pair = [&](int l) { return pairs && 2 * l + 1 < flag_every; };
    const int nblk[2] = {is_pair(tfirst) ? lv.nptiles : lv.ntiles, is_pair(tfirst + 1) ? lv.nptiles : lv.ntiles};
    const int first_steps = is_pair(tfirst) ? 2 : 1;
    const size_t nslot = 2 * (size_t)std::max(std::max(lv.ntiles, lv.nptiles), 1);
    if (ctx->stamps_cap < (size_t)nev * ntimed * nslot) {
        if (ctx->stamps) wp_dfree(ctx, ctx->stamps);
        ctx->stamps = (unsigned long long *)wp_dalloc(ctx, sizeof(unsigned long long) * nslot * ntimed * nev);
        if (!ctx->stamps) {
            ctx->stamps_cap = 0;
            return wp_fail(ctx, WP_ENOMEM, "launch clocks");
        }
        ctx->stamps_cap = (size_t)nev * ntimed * nslot;
        ctx->ff_gen = 0;   // pointer changed
    }
    const double key[6] = {dt, (double)nsteps, (double)flag_every, tol, t_s, t_f};
    if (!ctx->ff_exec || memcmp(key, ctx->ff_key, sizeof key) != 0 || ctx->ff_t0 != lv.t ||
        ctx->ff_parity != lv.cur || ctx->ff_gen != ctx->topo_gen || ctx->ff_snaps != ctx->snaps ||
        ctx->ff_store[0] != ctx->snap_ds || ctx->ff_store[1] != (double)ctx->nsnap) {
        if ((rc = wp_prepare_level(ctx, lv, dt)) != WP_OK) return rc;
        hipStream_t s;
        if ((rc = wp_graph_begin(ctx, s)) != WP_OK) return rc;
        const int par = lv.cur;
        launch_fill_u8((uint8_t *)ctx->ev_counts, (long long)sizeof(unsigned long long) * COUNT_SPAN * nev, 0, s);
        const Level &a0 = ctx->adj;
        for (int k = 0; k < nev && rc == WP_OK; ++k) {
            if (!fuse) rc = flag_launch(ctx, 0, tol, lo[k], hi[k], ctx->ev_counts + (size_t)k * COUNT_SPAN, s);
            // the block's steps, two per launch where the level allows it
            for (int st = 0, launch = 0; st < flag_every && rc == WP_OK; ++launch) {
                if (launch >= tfirst && launch < tfirst + ntimed && ctx->is_acoustics && ctx->kind2d)
                    ctx->stamp_next = ctx->stamps + nslot * ((size_t)ntimed * k + (launch - tfirst));
                if (pairs && st + 1 < flag_every) {
                    const PairFlag fl{ctx->snaps, (long long)a0.nx * a0.ny * ctx->m, lo[k], hi[k], tol, lv.flags,
                                      ctx->ev_counts + (size_t)k * COUNT_SPAN};
                    rc = wp_step_pair(ctx, lv, dt, 0, s, -1, -1, fuse && launch == 0 ? &fl : nullptr);
                    st += 2;
                } else {
                    rc = wp_step_level(ctx, lv, dt, 0, s, -1);
                    st += 1;
                }
            }
        }
        lv.flags_valid = true;
        ctx->stamp_next = nullptr;
        ctx->ff_flip = lv.cur ^ par;
        lv.cur = par;
        const int rc2 = wp_graph_end(ctx, s, ctx->ff_exec);
        if (rc != WP_OK) return rc;
        if (rc2 != WP_OK) return rc2;
        memcpy(ctx->ff_key, key, sizeof key);
        ctx->ff_t0 = lv.t;
        ctx->ff_parity = par;
        ctx->ff_gen = ctx->topo_gen;
        ctx->ff_snaps = ctx->snaps;
        ctx->ff_store[0] = ctx->snap_ds;
        ctx->ff_store[1] = (double)ctx->nsnap;
    }
    if ((rc = wp_graph_launch(ctx, ctx->ff_exec)) != WP_OK) return rc;
    lv.cur ^= ctx->ff_flip;
    lv.t_prev = lv.t + (double)(nsteps - (pairs && flag_every % 2 == 0 ? 2 : 1)) * dt;
    lv.prev_valid = true;
    lv.t += (double)nsteps * dt;
    if (counts || step_ms) {
        if (hipStreamSynchronize(ctx->stream) != hipSuccess) return wp_fail(ctx, WP_EDEVICE, "flagged run sync");
        if (counts && (rc = wp_read_counts(ctx, ctx->ev_counts, nev, counts)) != WP_OK) return rc;
        if (step_ms) {
            if (!(ctx->is_acoustics && ctx->kind2d)) return wp_fail(ctx, WP_EINVAL, "launch times are for 2D acoustics");
            std::vector<unsigned long long> st(nslot * ntimed * nev);
            int khz = 0, dev = 0;
            if ((rc = wp_host_copy(ctx, st.data(), ctx->stamps, sizeof(unsigned long long) * st.size(), false)) !=
                WP_OK)
                return rc;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
                return wp_fail(ctx, WP_EDEVICE, "launch clock read");
            // earliest workgroup start and latest end of timed launch i (the
            // l-th of its block)
            auto window = [&](size_t i, int l, unsigned long long &t0, unsigned long long &t1) {
                t0 = ~0ULL;
                t1 = 0;
                for (size_t b = 0; b < (size_t)nblk[l]; ++b) {
                    t0 = std::min(t0, st[nslot * i + 2 * b]);
                    t1 = std::max(t1, st[nslot * i + 2 * b + 1]);
                }
            };
            for (int k = 0; k < nev; ++k) {
                unsigned long long a0, a1, b0, b1;
                window((size_t)ntimed * k, 0, a0, a1);
                // launch duration: from its first workgroup start to that of
                // the next launch (dispatch and completion included); the
                // workgroup window alone when a block has one launch; per
                // step of that launch
                unsigned long long d = a1 - a0;
                if (ntimed == 2) {
                    window((size_t)ntimed * k + 1, 1, b0, b1);
                    d = b0 - a0;
                }
                step_ms[k] = (float)((double)d / (double)khz / first_steps);
            }
        }
    }
    return wp_check_status(ctx);
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

// ---------------------------------------------------------------------------
// functionals
// ---------------------------------------------------------------------------
extern "C" int wp_functional_value(wp_ctx *ctx, const wp_functional *J, int which, int snapshot, double *out)
{
    WP_ABI_TRY
    if (!ctx || !out) return ctx ? wp_fail(ctx, WP_EINVAL, "null output") : WP_EINVAL;
    Level &l0 = ctx->L[0];
    const long long cells = (long long)l0.nx * l0.ny;
    const double dA = l0.dx * (ctx->kind2d ? l0.dy : 1.0);
    const int nb = (int)std::min<long long>(RED_BLOCKS, (cells + 255) / 256);
    const void *q = l0.q[l0.cur];
    int rc;
    if (which == 0) {
        if (!ctx->ind_valid || memcmp(&ctx->ind_key, J, sizeof *J) != 0) {
            std::vector<uint8_t> ind;
            if ((rc = wp_build_indicator(ctx, J, ind)) != WP_OK) return rc;
            if (!ctx->ind_dev) ctx->ind_dev = (uint8_t *)wp_dalloc(ctx, (size_t)cells);
            if (!ctx->ind_dev) return wp_fail(ctx, WP_ENOMEM, "indicator");
            if (hipMemcpy(ctx->ind_dev, ind.data(), (size_t)cells, hipMemcpyHostToDevice) != hipSuccess)
                return wp_fail(ctx, WP_EDEVICE, "indicator upload");
            ctx->ind_key = *J;
            ctx->ind_valid = true;
        }
        if (ctx->prob.precision == WP_MIXED) {
            if (J->component == 0)
                launch_sum_indicator<double>((const double *)q, cells, cells, 0, ctx->ind_dev, ctx->partials, nb,
                                             ctx->red_out, ctx->stream);
            else
                launch_sum_indicator<float>((const float *)((char *)q + cells * 8), cells, cells, J->component - 1,
                                            ctx->ind_dev, ctx->partials, nb, ctx->red_out, ctx->stream);
        } else if (ctx->esz == 8) {
            launch_sum_indicator<double>((const double *)q, cells, cells, J->component, ctx->ind_dev, ctx->partials,
                                         nb, ctx->red_out, ctx->stream);
        } else {
            launch_sum_indicator<float>((const float *)q, cells, cells, J->component, ctx->ind_dev, ctx->partials, nb,
                                        ctx->red_out, ctx->stream);
        }
    } else if (which == 1) {
        if (snapshot < 0 || snapshot >= ctx->nsnap)
            return wp_fail(ctx, WP_ERANGE, "snapshot %d of %d", snapshot, ctx->nsnap);
        const void *s = (const char *)ctx->snaps + (size_t)snapshot * ctx->snap_bytes;
        if (ctx->prob.precision == WP_MIXED)
            launch_sum_dot_mixed((const double *)q, (const float *)((char *)q + cells * 8),
                                 (const float *)((char *)q + cells * 12), cells, (const float *)s, cells, cells,
                                 ctx->partials, nb, ctx->red_out, ctx->stream);
        else if (ctx->esz == 8)
            launch_sum_dot<double, double>((const double *)q, cells, (const double *)s, cells, cells, ctx->m,
                                           ctx->partials, nb, ctx->red_out, ctx->stream);
        else
            launch_sum_dot<float, float>((const float *)q, cells, (const float *)s, cells, cells, ctx->m, ctx->partials,
                                         nb, ctx->red_out, ctx->stream);
    } else {
        return wp_fail(ctx, WP_EINVAL, "which must be 0 (J) or 1 (inner product)");
    }
    double v = 0.0;
    int rc2;
    if ((rc2 = wp_host_copy(ctx, &v, ctx->red_out, sizeof v, false)) != WP_OK) return rc2;
    *out = v * dA;
    return wp_check_status(ctx);
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}
