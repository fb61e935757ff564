// Refinement hierarchy on the host side (Davis & LeVeque Sec. 3): regridding
// of a level's children (given boxes or Berger-Rigoutsos clusters of its
// flags), the ghost ring of a fine level from the level below with space-time
// interpolation, the Berger-Oliger recursion and the fine-to-coarse average.
#include <algorithm>
#include <array>
#include <cmath>
#include <vector>

#include "abi_guard.h"
#include "regrid_lists.h"
#include "wp_ctx.h"

using namespace wp;

namespace {

int upload_ints(wp_ctx *ctx, const std::vector<int> &v, int *&dev, long long &n, size_t &cap, const char *what)
{
    n = (long long)v.size();
    if (v.empty()) return WP_OK;
    void *d = dev;
    const int rc = wp_upload(ctx, v.data(), v.size() * sizeof(int), d, cap, what);
    dev = (int *)d;
    return rc;
}

// Byte offset of the float planes (hu, hv) of a mixed-precision canvas: they
// follow the FP64 eta plane.
inline size_t mixed_tail(const Level &lv) { return (size_t)lv.nx * lv.ny * sizeof(double); }

// Fine cells `cells` of level l from level l-1 at time weight alpha between
// the canvas before its last step (cold) and its current one (cnew).

int fill_from_coarse(wp_ctx *ctx, int l, const int *cells, long long n, double alpha, bool use_old, hipStream_t s)
{
    Level &F = ctx->L[l], &C = ctx->L[l - 1];
    const void *cnew = C.q[C.cur];
    const void *cold = use_old ? C.q[C.cur ^ 1] : cnew;
    if (ctx->prob.precision == WP_MIXED) {
        // eta in FP64, then hu and hv in FP32
        launch_ring_fill<double>(cells, n, (double *)F.q[F.cur], F.nx, (const double *)cold, (const double *)cnew,
                                 C.nx, C.ny, F.ratio, alpha, ctx->prob.bc, s, 0, 1);
        launch_ring_fill<float>(cells, n, (float *)((char *)F.q[F.cur] + mixed_tail(F)), F.nx,
                                (const float *)((const char *)cold + mixed_tail(C)),
                                (const float *)((const char *)cnew + mixed_tail(C)), C.nx, C.ny, F.ratio, alpha,
                                ctx->prob.bc, s, 1, 2);
    } else if (ctx->esz == 8)
        launch_ring_fill<double>(cells, n, (double *)F.q[F.cur], F.nx, (const double *)cold, (const double *)cnew,
                                 C.nx, C.ny, F.ratio, alpha, ctx->prob.bc, s);
    else
        launch_ring_fill<float>(cells, n, (float *)F.q[F.cur], F.nx, (const float *)cold, (const float *)cnew, C.nx,
                                C.ny, F.ratio, alpha, ctx->prob.bc, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return wp_fail(ctx, WP_EDEVICE, "coarse-to-fine launch: %s", hipGetErrorString(e));
    return WP_OK;
}

// The ring of level l at time weight alpha in its current canvas; with
// `next`, also the ring at alpha2 in its other canvas (that of the next
// substep, which the current one writes only inside the patches).
int fill_ring(wp_ctx *ctx, int l, double alpha, hipStream_t s, bool next = false, double alpha2 = 0.0)
{
    Level &F = ctx->L[l], &C = ctx->L[l - 1];
    if (F.nring == 0) return WP_OK;
    if (F.nringb == 0) {
        int rc = fill_from_coarse(ctx, l, F.ring_dev, F.nring, alpha, C.prev_valid, s);
        if (rc == WP_OK && next) {
            F.cur ^= 1;
            rc = fill_from_coarse(ctx, l, F.ring_dev, F.nring, alpha2, C.prev_valid, s);
            F.cur ^= 1;
        }
        return rc;
    }
    // by coarse parent: each parent's slopes formed once for all its ring children
    const void *cnew = C.q[C.cur];
    const void *cold = C.prev_valid ? C.q[C.cur ^ 1] : cnew;
    char *f1 = (char *)F.q[F.cur], *f2 = next ? (char *)F.q[F.cur ^ 1] : nullptr;
    if (ctx->prob.precision == WP_MIXED) {
        launch_ring_fill_blocks<double>(F.ringb_dev, F.nringb, (double *)f1, F.nx, (const double *)cold,
                                        (const double *)cnew, C.nx, C.ny, F.ratio, alpha, ctx->prob.bc, s, 0, 1,
                                        (double *)f2, alpha2);
        launch_ring_fill_blocks<float>(F.ringb_dev, F.nringb, (float *)(f1 + mixed_tail(F)), F.nx,
                                       (const float *)((const char *)cold + mixed_tail(C)),
                                       (const float *)((const char *)cnew + mixed_tail(C)), C.nx, C.ny, F.ratio,
                                       alpha, ctx->prob.bc, s, 1, 2, f2 ? (float *)(f2 + mixed_tail(F)) : nullptr,
                                       alpha2);
    } else if (ctx->esz == 8)
        launch_ring_fill_blocks<double>(F.ringb_dev, F.nringb, (double *)f1, F.nx, (const double *)cold,
                                        (const double *)cnew, C.nx, C.ny, F.ratio, alpha, ctx->prob.bc, s, 0, 3,
                                        (double *)f2, alpha2);
    else
        launch_ring_fill_blocks<float>(F.ringb_dev, F.nringb, (float *)f1, F.nx, (const float *)cold,
                                       (const float *)cnew, C.nx, C.ny, F.ratio, alpha, ctx->prob.bc, s, 0, 3,
                                       (float *)f2, alpha2);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return wp_fail(ctx, WP_EDEVICE, "coarse-to-fine launch: %s", hipGetErrorString(e));
    return WP_OK;
}

int average_down(wp_ctx *ctx, int l, hipStream_t s)
{
    Level &F = ctx->L[l], &C = ctx->L[l - 1];
    if (F.ncover == 0) return WP_OK;
    const long long csf = (long long)F.nx * F.ny, csc = (long long)C.nx * C.ny;
    if (ctx->prob.precision == WP_MIXED) {
        launch_average<double>(F.cover_dev, F.ncover, (const double *)F.q[F.cur], F.nx, csf, (double *)C.q[C.cur],
                               C.nx, csc, F.ratio, s, 1);
        launch_average<float>(F.cover_dev, F.ncover, (const float *)((const char *)F.q[F.cur] + mixed_tail(F)), F.nx,
                              csf, (float *)((char *)C.q[C.cur] + mixed_tail(C)), C.nx, csc, F.ratio, s, 2);
    } else if (ctx->esz == 8)
        launch_average<double>(F.cover_dev, F.ncover, (const double *)F.q[F.cur], F.nx, csf, (double *)C.q[C.cur],
                               C.nx, csc, F.ratio, s);
    else
        launch_average<float>(F.cover_dev, F.ncover, (const float *)F.q[F.cur], F.nx, csf, (float *)C.q[C.cur], C.nx,
                              csc, F.ratio, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return wp_fail(ctx, WP_EDEVICE, "average launch: %s", hipGetErrorString(e));
    return WP_OK;
}

// The faces of refluxing between level f's patches and the level f-1 cells
// that none of them covers (see Level and reflux_faces).
int build_faces(wp_ctx *ctx, int f)
{
    Level &F = ctx->L[f], &C = ctx->L[f - 1];
    F.nfaces = F.nfgroups = 0;
    std::vector<int> &flat = ctx->rg_list[0], &groups = ctx->rg_list[1];
    reflux_faces(F.patches, F.ratio, C.nx, C.ny, flat, groups);
    if (flat.empty()) return WP_OK;
    const size_t nf = flat.size() / 4;
    int rc;
    long long n = 0;
    if ((rc = upload_ints(ctx, flat, F.faces_dev, n, F.faces_cap, "reflux faces")) != WP_OK) return rc;
    if ((rc = upload_ints(ctx, groups, F.fgroups_dev, n, F.fgroups_cap, "reflux groups")) != WP_OK) return rc;
    const size_t reg_bytes = sizeof(double) * 3 * nf;
    if (F.freg_cap < reg_bytes || !F.freg_dev) {
        if (F.freg_dev) wp_dfree(ctx, F.freg_dev);
        F.freg_dev = (double *)wp_dalloc(ctx, reg_bytes + reg_bytes / 2);
        F.freg_cap = F.freg_dev ? reg_bytes + reg_bytes / 2 : 0;
        if (!F.freg_dev) return wp_fail(ctx, WP_ENOMEM, "reflux registers");
    }
    F.nfaces = (int)nf;
    F.nfgroups = (int)(groups.size() / 2);
    return WP_OK;
}

// Refluxing steps (see launch_reflux_fine): after each substep of level f
// the fluxes of its faces' fine edges are added to the registers; after the
// last, the level below is corrected.
int reflux_fine(wp_ctx *ctx, int f, double dtf, bool first, hipStream_t s)
{
    Level &F = ctx->L[f];
    const wp_problem &P = ctx->prob;
    if (!ctx->is_acoustics)
        launch_reflux_swe_fine(P.precision, F.faces_dev, F.nfaces, F.q[F.cur ^ 1], F.B, F.nx, F.ny, P.bc, P.g,
                               F.ratio, dtf / F.dx, dtf / F.dy, P.order, P.limiter, P.transverse, first, F.freg_dev,
                               s);
    else if (ctx->esz == 8)
        launch_reflux_fine<double>(F.faces_dev, F.nfaces, (const double *)F.q[F.cur ^ 1], F.mat, F.nx, F.ny, P.bc,
                                   ctx->mtab64, F.ratio, dtf / F.dx, dtf / F.dy, P.order, P.limiter, P.transverse,
                                   first, F.freg_dev, s);
    else
        launch_reflux_fine<float>(F.faces_dev, F.nfaces, (const float *)F.q[F.cur ^ 1], F.mat, F.nx, F.ny, P.bc,
                                  ctx->mtab64, F.ratio, dtf / F.dx, dtf / F.dy, P.order, P.limiter, P.transverse,
                                  first, F.freg_dev, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return wp_fail(ctx, WP_EDEVICE, "reflux launch: %s", hipGetErrorString(e));
    return WP_OK;
}

int reflux_apply(wp_ctx *ctx, int c, double dt, hipStream_t s)
{
    Level &C = ctx->L[c], &F = ctx->L[c + 1];
    const wp_problem &P = ctx->prob;
    if (!ctx->is_acoustics)
        launch_reflux_swe_apply(P.precision, F.fgroups_dev, F.nfgroups, F.faces_dev, F.freg_dev, C.q[C.cur ^ 1],
                                C.q[C.cur], C.B, C.nx, C.ny, P.bc, P.g, F.ratio, dt / C.dx, dt / C.dy, P.order,
                                P.limiter, P.transverse, s);
    else if (ctx->esz == 8)
        launch_reflux_apply<double>(F.fgroups_dev, F.nfgroups, F.faces_dev, F.freg_dev, (const double *)C.q[C.cur ^ 1],
                                    (double *)C.q[C.cur], C.mat, C.nx, C.ny, P.bc, ctx->mtab64, F.ratio, dt / C.dx,
                                    dt / C.dy, P.order, P.limiter, P.transverse, s);
    else
        launch_reflux_apply<float>(F.fgroups_dev, F.nfgroups, F.faces_dev, F.freg_dev, (const float *)C.q[C.cur ^ 1],
                                   (float *)C.q[C.cur], C.mat, C.nx, C.ny, P.bc, ctx->mtab64, F.ratio, dt / C.dx,
                                   dt / C.dy, P.order, P.limiter, P.transverse, s);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return wp_fail(ctx, WP_EDEVICE, "reflux launch: %s", hipGetErrorString(e));
    return WP_OK;
}

// One Berger-Oliger step of level l and, recursively, its finer levels, on
// stream s.  sub: index of this step among the ratio steps of level l within
// one step of level l-1 (time weight sub / ratio for the ghost ring).  With
// launch = false only the host bookkeeping (canvas parity, times) is done:
// the replay of a captured sequence.
int bo_advance(wp_ctx *ctx, int l, double dt, int sub, hipStream_t s, bool launch)
{
    Level &lv = ctx->L[l];
    int rc;
    if ((rc = wp_courant_check(ctx, lv, dt)) != WP_OK) return rc;
    if (lv.patches.empty()) {
        lv.t += dt;
        return WP_OK;
    }
    // the ring at this step's start time; after the first step of a level
    // with children it is already there: the fill after the previous step
    // wrote it for the finer level, from the same canvases of the level
    // below (which does not step meanwhile), and the average of the finer
    // level touches no ring cell (proper nesting)
    const bool has_children = l + 1 < (int)ctx->L.size() && !ctx->L[l + 1].patches.empty();
    // a level without children takes the rings of two substeps in one fill:
    // an even substep's fill also writes the next substep's ring into the
    // other canvas, which this substep's step writes only inside the patches
    const bool paired = !has_children && lv.ratio % 2 == 0;
    if (launch && l > 0 && !(sub > 0 && has_children) && !(paired && sub % 2 == 1) &&
        (rc = fill_ring(ctx, l, (double)sub / (double)lv.ratio, s, paired,
                        (double)(sub + 1) / (double)lv.ratio)) != WP_OK)
        return rc;
    if (launch) {
        if ((rc = wp_step_level(ctx, lv, dt, ctx->equation, s, -1)) != WP_OK) return rc;
    } else {
        lv.cur ^= 1;
    }
    lv.t_prev = lv.t;
    lv.prev_valid = true;
    lv.t += dt;
    if (has_children) {
        const int r = ctx->L[l + 1].ratio;
        // this level's ring at its new time, read by the finer level's
        // interpolation next to the ring
        if (launch && l > 0 && (rc = fill_ring(ctx, l, (double)(sub + 1) / (double)lv.ratio, s)) != WP_OK) return rc;
        // refluxing of a conservative system (the acoustics adjoint, shallow
        // water) at the edges between the finer level's patches and this level
        const bool rf = ctx->reflux && (ctx->equation == 1 || !ctx->is_acoustics) && ctx->L[l + 1].nfaces > 0;
        // a finer level without children of its own averages its last
        // substep's results onto this level in the step itself, where the
        // launch can (acou2d_can_average)
        Level &G = ctx->L[l + 1];
        const bool g_leaf = l + 2 >= (int)ctx->L.size() || ctx->L[l + 2].patches.empty();
        G.averaged = false;
        for (int k = 0; k < r; ++k) {
            G.avg_onto = launch && g_leaf && k == r - 1 ? &lv : nullptr;
            rc = bo_advance(ctx, l + 1, dt / r, k, s, launch);
            G.avg_onto = nullptr;
            if (rc != WP_OK) return rc;
            if (launch && rf && (rc = reflux_fine(ctx, l + 1, dt / r, k == 0, s)) != WP_OK) return rc;
        }
        if (launch && !G.averaged && (rc = average_down(ctx, l + 1, s)) != WP_OK) return rc;
        G.averaged = false;
        if (launch && rf && (rc = reflux_apply(ctx, l, dt, s)) != WP_OK) return rc;
    }
    return WP_OK;
}

// Descriptors of every level for the step sizes of a coarse step dt0, so
// that a capture records launches only.
int prepare_levels(wp_ctx *ctx, double dt0)
{
    double dt = dt0;
    int rc;
    for (size_t l = 0; l < ctx->L.size(); ++l) {
        if (l > 0) dt = dt / ctx->L[l].ratio;
        if (!ctx->L[l].patches.empty() && (rc = wp_prepare_level(ctx, ctx->L[l], dt)) != WP_OK) return rc;
    }
    return WP_OK;
}

std::vector<int> parities(const wp_ctx *ctx)
{
    std::vector<int> p;
    for (const Level &lv : ctx->L) p.push_back(lv.cur);
    return p;
}

// Replace the patches of level f (> 0) with `boxes` (validated).
int install(wp_ctx *ctx, int f, const std::vector<wp_patch> &boxes)
{
    Level &F = ctx->L[f], &C = ctx->L[f - 1];
    int rc;
    // new cells outside every old patch: space interpolation from the level
    // below at its current time (each cell on its own, so in any order)
    std::vector<int> &fresh = ctx->rg_list[0];
    fresh_cells(boxes, F.patches, F.nx, F.ny, fresh);
    if (!fresh.empty()) {
        long long n = 0;
        if ((rc = upload_ints(ctx, fresh, ctx->fresh_dev, n, ctx->fresh_cap, "new cell")) != WP_OK) return rc;
        if ((rc = fill_from_coarse(ctx, f, ctx->fresh_dev, n, 0.0, false, ctx->stream)) != WP_OK) return rc;
    }
    F.patches = boxes;
    if ((rc = wp_upload_tiles(ctx, F)) != WP_OK) return rc;
    {
        // ratios up to 8 fill the ring by coarse parent, larger ones cell by cell
        std::vector<std::array<int, 3>> &runs = ctx->rg_runs;
        ring_runs(F.patches, F.nx, F.ny, runs);
        F.nring = 0;
        for (const auto &u : runs) F.nring += u[2] - u[1];
        std::vector<int> &blocks = ctx->rg_list[0], &cells = ctx->rg_list[1];
        blocks.clear();
        cells.clear();
        if (F.ratio <= 8)
            ring_block_list(runs, F.ratio, C.nx, blocks);
        else
            run_cells(runs, F.nx, cells);
        long long n = 0;
        if ((rc = upload_ints(ctx, cells, F.ring_dev, n, F.ring_cap, "ring")) != WP_OK) return rc;
        if ((rc = upload_ints(ctx, blocks, F.ringb_dev, F.nringb, F.ringb_cap, "ring block")) != WP_OK) return rc;
        F.nringb /= 3;
    }
    cover_cells(F.patches, F.ratio, C.nx, ctx->rg_list[0]);
    if ((rc = upload_ints(ctx, ctx->rg_list[0], F.cover_dev, F.ncover, F.cover_cap, "cover")) != WP_OK) return rc;
    if ((rc = build_faces(ctx, f)) != WP_OK) return rc;
    F.t = C.t;
    F.prev_valid = false;
    F.flags_valid = false;
    // finer levels are emptied: they are regridded from this one next
    for (size_t l = f + 1; l < ctx->L.size(); ++l) {
        Level &G = ctx->L[l];
        if (G.patches.empty()) continue;
        G.patches.clear();
        if ((rc = wp_upload_tiles(ctx, G)) != WP_OK) return rc;
        G.nring = G.nringb = G.ncover = 0;
        G.nfaces = G.nfgroups = 0;
        G.prev_valid = false;
        G.flags_valid = false;
    }
    return WP_OK;
}

}  // namespace

// Ghost ring of `level` from the level below at time t: linear time weight
// between the times of the two canvases of the level below (its current one
// alone when it has not stepped since its state was set).
int wp_fill_coarse_ghosts(wp_ctx *ctx, int level, double t)
{
    const Level &C = ctx->L[level - 1];
    double alpha = 1.0;
    if (C.prev_valid && C.t > C.t_prev) alpha = std::min(std::max((t - C.t_prev) / (C.t - C.t_prev), 0.0), 1.0);
    return fill_ring(ctx, level, alpha, ctx->stream);
}

// Two coarse steps return every canvas to its parity, so their launch
// sequence is captured once as a graph and replayed for each pair of steps
// (re-captured when dt0, the tile tables or the parities change).
extern "C" int wp_advance(wp_ctx *ctx, int nsteps, double dt0)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    if (nsteps < 0) return wp_fail(ctx, WP_EINVAL, "nsteps must be non-negative");
    int rc;
    if ((rc = wp_courant_check(ctx, ctx->L[0], dt0)) != WP_OK) return rc;
    const int pairs = nsteps / 2;
    if (pairs > 0) {
        const std::vector<int> par = parities(ctx);
        if (!ctx->bo_exec || ctx->bo_dt != dt0 || ctx->bo_gen != ctx->topo_gen || ctx->bo_par != par) {
            if ((rc = prepare_levels(ctx, dt0)) != WP_OK) return rc;
            std::vector<Level> saved = ctx->L;   // host bookkeeping is replayed below
            hipStream_t s;
            if ((rc = wp_graph_begin(ctx, s)) != WP_OK) return rc;
            for (int k = 0; k < 2 && rc == WP_OK; ++k) rc = bo_advance(ctx, 0, dt0, 0, s, true);
            const int rc2 = wp_graph_end(ctx, s, ctx->bo_exec);
            for (size_t l = 0; l < ctx->L.size(); ++l) {
                ctx->L[l].cur = saved[l].cur;
                ctx->L[l].t = saved[l].t;
                ctx->L[l].t_prev = saved[l].t_prev;
                ctx->L[l].prev_valid = saved[l].prev_valid;
            }
            if (rc != WP_OK) return rc;
            if (rc2 != WP_OK) return rc2;
            ctx->bo_dt = dt0;
            ctx->bo_gen = ctx->topo_gen;
            ctx->bo_par = par;
        }
        for (int p = 0; p < pairs; ++p) {
            if ((rc = wp_graph_launch(ctx, ctx->bo_exec)) != WP_OK) return rc;
            for (int k = 0; k < 2; ++k)
                if ((rc = bo_advance(ctx, 0, dt0, 0, ctx->stream, false)) != WP_OK) return rc;
        }
    }
    if (nsteps & 1) return bo_advance(ctx, 0, dt0, 0, ctx->stream, true);
    return WP_OK;
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

extern "C" int wp_regrid(wp_ctx *ctx, int level, const wp_patch *patches, int npatches, int buffer)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    if (level < 0 || level + 1 >= (int)ctx->L.size())
        return wp_fail(ctx, WP_EINVAL, "level %d has no finer level", level);
    Level &C = ctx->L[level], &F = ctx->L[level + 1];
    const int r = F.ratio;
    // every cell a finer patch may cover lies in the bounding box of this
    // level's patches: the host images below cover that window only
    int wi0 = C.nx, wj0 = C.ny, wi1 = 0, wj1 = 0;
    for (const wp_patch &p : C.patches) {
        wi0 = std::min(wi0, p.ilo);
        wj0 = std::min(wj0, p.jlo);
        wi1 = std::max(wi1, p.ilo + p.nx);
        wj1 = std::max(wj1, p.jlo + p.ny);
    }
    if (C.patches.empty()) wi0 = wj0 = wi1 = wj1 = 0;
    const int ww = wi1 - wi0, wh = wj1 - wj0;
    std::vector<uint8_t> &allowed = ctx->rg_allowed;
    wp_nesting_mask(C.patches, C.nx, C.ny, wi0, wj0, ww, wh, allowed);
    auto in_window = [&](int i, int j) { return i >= wi0 && i < wi1 && j >= wj0 && j < wj1; };
    std::vector<wp_patch> boxes;
    if (patches) {
        if (npatches < 0) return wp_fail(ctx, WP_EINVAL, "npatches must be non-negative");
        std::vector<uint8_t> used((size_t)ww * wh, 0);
        for (int k = 0; k < npatches; ++k) {
            const wp_patch p = patches[k];
            if (p.nx < 1 || p.ny < 1 || p.ilo < 0 || p.jlo < 0 || p.ilo + p.nx > F.nx || p.jlo + p.ny > F.ny)
                return wp_fail(ctx, WP_EINVAL, "patch %d outside level %d", k, level + 1);
            if (p.ilo % r || p.jlo % r || p.nx % r || p.ny % r)
                return wp_fail(ctx, WP_EINVAL, "patch %d not aligned to the refinement ratio %d", k, r);
            for (int jc = p.jlo / r; jc < (p.jlo + p.ny) / r; ++jc)
                for (int ic = p.ilo / r; ic < (p.ilo + p.nx) / r; ++ic) {
                    if (!in_window(ic, jc))
                        return wp_fail(ctx, WP_EINVAL, "patch %d not properly nested in level %d", k, level);
                    const size_t w = (size_t)(jc - wj0) * ww + (ic - wi0);
                    if (used[w]) return wp_fail(ctx, WP_EINVAL, "patch %d overlaps another", k);
                    if (!allowed[w])
                        return wp_fail(ctx, WP_EINVAL, "patch %d not properly nested in level %d", k, level);
                    used[w] = 1;
                }
            boxes.push_back(p);
        }
    } else {
        if (buffer < 0) return wp_fail(ctx, WP_EINVAL, "buffer must be non-negative");
        if (!C.flags_valid) return wp_fail(ctx, WP_ESTATE, "level %d has no flags (flag it first)", level);
        // the window's rows in one linear copy, then its columns
        std::vector<uint8_t> &rows = ctx->rg_rows, &fl = ctx->rg_flags;
        rows.resize((size_t)C.nx * wh);
        fl.resize((size_t)ww * wh);
        int rcf;
        ctx->host_ms[HT_FLAG_COPY] -= wp_now_ms();
        rcf = wp_host_copy(ctx, rows.data(), C.flags + (size_t)wj0 * C.nx, rows.size(), false);
        ctx->host_ms[HT_FLAG_COPY] += wp_now_ms();
        if (rcf != WP_OK) return rcf;
        ctx->host_ms[HT_CLUSTER] -= wp_now_ms();
        for (int j = 0; j < wh; ++j)
            std::copy_n(&rows[(size_t)j * C.nx + wi0], ww, &fl[(size_t)j * ww]);
        for (size_t k = 0; k < fl.size(); ++k) fl[k] = (fl[k] && allowed[k]) ? 1 : 0;
        // flags outside the window are outside the nesting region, so the
        // window's dilation restricted to it is the whole level's
        std::vector<uint8_t> &dil = ctx->rg_dil;
        wp_dilate(fl, ww, wh, buffer, dil);
        for (size_t k = 0; k < dil.size(); ++k) dil[k] = (dil[k] && allowed[k]) ? 1 : 0;
        if (ww > 0 && wh > 0)
            wp_cluster_boxes(dil.data(), allowed.data(), ww, wh, 0.7, std::max(1, 64 / r), std::max(1, 8 / r), boxes);
        for (wp_patch &p : boxes) p = wp_patch{(p.ilo + wi0) * r, (p.jlo + wj0) * r, p.nx * r, p.ny * r};
        ctx->host_ms[HT_CLUSTER] += wp_now_ms();
    }
    ctx->host_ms[HT_UPLOAD] -= wp_now_ms();
    const int rci = install(ctx, level + 1, boxes);
    ctx->host_ms[HT_UPLOAD] += wp_now_ms();
    return rci;
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

extern "C" int wp_get_patches(const wp_ctx *ctx, int level, wp_patch *out, int cap, int *np)
{
    if (!ctx) return WP_EINVAL;
    if (level < 0 || level >= (int)ctx->L.size()) return wp_fail_get(ctx, WP_EINVAL, "level out of range");
    if (cap > 0 && !out) return wp_fail_get(ctx, WP_EINVAL, "null output with a positive capacity");
    const auto &p = ctx->L[level].patches;
    if (np) *np = (int)p.size();
    for (int k = 0; k < (int)p.size() && k < cap; ++k) out[k] = p[k];
    return WP_OK;
}
