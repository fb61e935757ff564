// Batches of independent single-level 2D acoustics instances: every step of
// every instance in one launch of the patch-update kernel.  The launch reads
// a device array of instance descriptors and one tile table whose entries
// name their instance; each workgroup loads its own instance's material
// tables, so instances may differ in size, medium and time step.
#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "abi_guard.h"
#include "wp_ctx.h"

using namespace wp;

struct wp_batch {
    std::vector<wp_ctx *> inst;
    std::vector<double> dts;
    std::string err;
    hipStream_t stream = nullptr;
    int esz = 8;
    bool full = true;
    int nmat_max = 1;
    int rows = 8;
    void *desc[2] = {nullptr, nullptr};   // forward, adjoint descriptor arrays
    Tile *tiles[2] = {nullptr, nullptr};
    int ntiles[2] = {0, 0};
    int kind[2] = {0, 0};
    // two steps per launch (every instance able to take them): tile tables
    // of the two-step kernel
    int prows = 0;
    Tile *ptiles[2] = {nullptr, nullptr};
    int nptiles[2] = {0, 0};
    int pkind[2] = {0, 0};
    int *status = nullptr;
    hipGraphExec_t exec[2] = {nullptr, nullptr};
    int exec_steps[2] = {0, 0};
    int exec_every[2] = {0, 0};
    int exec_parity[2] = {-1, -1};
    int exec_end[2] = {0, 0};             // canvas parity after the captured sequence
};

static int bfail(wp_batch *b, int code, const char *msg)
{
    if (b) b->err = msg;
    return code;
}

static Level &batch_level(wp_ctx *c, int adjoint) { return adjoint ? c->adj : c->L[0]; }

// Descriptors and the combined tile tables for the forward levels (adjoint =
// 0) or the adjoint levels (adjoint = 1) of every instance.  The tables
// depend on the instances' grids and media only, so they are built once per
// side; the descriptors (step size, snapshot store) are uploaded every time.
static int build_side(wp_batch *b, int adjoint)
{
    const bool tables = !b->tiles[adjoint];
    wp_ctx *c0 = b->inst[0];
    const size_t dsz = b->esz == 8 ? sizeof(AcouInst<double>) : sizeof(AcouInst<float>);
    std::vector<unsigned char> host(dsz * b->inst.size());
    std::vector<Tile> mixed, uni, pmixed, puni;
    for (size_t k = 0; k < b->inst.size(); ++k) {
        wp_ctx *c = b->inst[k];
        Level &lv = batch_level(c, adjoint);
        int rc;
        if ((rc = wp_prepare_level(c, lv, b->dts[k])) != WP_OK) return bfail(b, rc, c->err.c_str());
        memcpy(host.data() + k * dsz, lv.inst_host, dsz);
        if (!tables) continue;
        std::vector<Tile> t = wp_make_tiles(lv.patches, (int)k, b->rows, STRIP, false);
        wp_classify_tiles(c, lv, t, b->rows);
        for (const Tile &x : t) (x.mat < 0 ? mixed : uni).push_back(x);
        if (b->prows) {
            std::vector<Tile> pt = wp_make_tiles(lv.patches, (int)k, b->prows, PAIR_STRIP, false);
            wp_classify_tiles(c, lv, pt, b->prows, 4);
            for (Tile x : pt) {
                x.down = 0;
                (x.mat < 0 ? pmixed : puni).push_back(x);
            }
        }
    }
    // slower mixed-material tiles dispatched first, each group in XCD order
    auto table = [&](std::vector<Tile> &mx, std::vector<Tile> &un, Tile *&dev, int &n, int &kind) {
        wp_xcd_order(mx);
        wp_xcd_order(un);
        std::vector<Tile> all = mx;
        all.insert(all.end(), un.begin(), un.end());
        if (dev) wp_dfree(c0, dev);
        dev = (Tile *)wp_dalloc(c0, sizeof(Tile) * std::max<size_t>(1, all.size()));
        if (!dev) return bfail(b, WP_ENOMEM, "batch tables");
        if (!all.empty() && hipMemcpy(dev, all.data(), sizeof(Tile) * all.size(), hipMemcpyHostToDevice) != hipSuccess)
            return bfail(b, WP_EDEVICE, "batch table upload");
        n = (int)all.size();
        kind = mx.empty() ? 1 : 0;
        return (int)WP_OK;
    };
    int rc;
    if (tables) {
        if ((rc = table(mixed, uni, b->tiles[adjoint], b->ntiles[adjoint], b->kind[adjoint])) != WP_OK) return rc;
        if (b->prows &&
            (rc = table(pmixed, puni, b->ptiles[adjoint], b->nptiles[adjoint], b->pkind[adjoint])) != WP_OK)
            return rc;
    }
    if (!b->desc[adjoint]) b->desc[adjoint] = wp_dalloc(c0, host.size());
    if (!b->desc[adjoint]) return bfail(b, WP_ENOMEM, "batch tables");
    if (hipMemcpy(b->desc[adjoint], host.data(), host.size(), hipMemcpyHostToDevice) != hipSuccess)
        return bfail(b, WP_EDEVICE, "batch table upload");
    if (tables && b->exec[adjoint]) {
        (void)hipGraphExecDestroy(b->exec[adjoint]);
        b->exec[adjoint] = nullptr;
    }
    return WP_OK;
}

static void launch_side(wp_batch *b, int adjoint, int parity, int snap_index, hipStream_t s)
{
    if (b->esz == 8)
        launch_acou2d<double>((const AcouInst<double> *)b->desc[adjoint], b->tiles[adjoint], b->ntiles[adjoint],
                              parity, adjoint, b->nmat_max, b->full, b->rows, b->kind[adjoint], snap_index,
                              b->status, s);
    else
        launch_acou2d<float>((const AcouInst<float> *)b->desc[adjoint], b->tiles[adjoint], b->ntiles[adjoint],
                             parity, adjoint, b->nmat_max, b->full, b->rows, b->kind[adjoint], snap_index, b->status,
                             s);
}

static void launch_side_pair(wp_batch *b, int adjoint, int parity, int snap1, int snap2, hipStream_t s)
{
    if (b->esz == 8)
        launch_acou2d_pair<double>((const AcouInst<double> *)b->desc[adjoint], b->ptiles[adjoint],
                                   b->nptiles[adjoint], parity, adjoint, b->nmat_max, b->prows, b->pkind[adjoint],
                                   snap1, snap2, b->status, s);
    else
        launch_acou2d_pair<float>((const AcouInst<float> *)b->desc[adjoint], b->ptiles[adjoint],
                                  b->nptiles[adjoint], parity, adjoint, b->nmat_max, b->prows, b->pkind[adjoint],
                                  snap1, snap2, b->status, s);
}

static int common_parity(wp_batch *b, int adjoint)
{
    const int p = batch_level(b->inst[0], adjoint).cur;
    for (wp_ctx *c : b->inst)
        if (batch_level(c, adjoint).cur != p) return -1;
    return p;
}

static int check_status(wp_batch *b)
{
    int st = 0;
    if (wp_host_copy(b->inst[0], &st, b->status, sizeof st, false) != WP_OK)
        return bfail(b, WP_EDEVICE, "batch status read");
    if (st) {
        (void)hipMemsetAsync(b->status, 0, sizeof st, b->stream);
        (void)hipStreamSynchronize(b->stream);
        return bfail(b, WP_ENONFINITE, "a batched step produced a non-finite value");
    }
    return WP_OK;
}

extern "C" int wp_batch_create(wp_ctx *const *instances, int n, const double *dts, wp_batch **out)
{
    WP_ABI_TRY
    if (!out) return WP_EINVAL;
    *out = nullptr;
    if (!instances || !dts || n < 1) return WP_EINVAL;
    wp_batch *b = new wp_batch();
    *out = b;
    for (int k = 0; k < n; ++k) {
        wp_ctx *c = instances[k];
        if (!c) return bfail(b, WP_EINVAL, "null instance");
        if (c->prob.kind != WP_ACOUSTICS_2D || c->L.size() != 1)
            return bfail(b, WP_EINVAL, "batches hold single-level 2D acoustics instances");
        if (std::find(b->inst.begin(), b->inst.end(), c) != b->inst.end())
            return bfail(b, WP_EINVAL, "an instance appears twice");
        b->inst.push_back(c);
        b->dts.push_back(dts[k]);
    }
    wp_ctx *c0 = b->inst[0];
    b->esz = c0->esz;
    b->stream = c0->stream;
    const wp_problem &P = c0->prob;
    b->full = P.order == 2 && P.limiter == 1 && P.transverse == 1;
    long long cells = 0;
    for (size_t k = 0; k < b->inst.size(); ++k) {
        wp_ctx *c = b->inst[k];
        if (c->esz != b->esz || c->prob.order != P.order || c->prob.limiter != P.limiter ||
            c->prob.transverse != P.transverse || c->stream != b->stream)
            return bfail(b, WP_EINVAL, "instances of a batch share precision, method options and stream");
        int rc;
        if ((rc = wp_courant_check(c, c->L[0], b->dts[k])) != WP_OK) return bfail(b, rc, c->err.c_str());
        b->nmat_max = std::max(b->nmat_max, c->nmat);
        cells += (long long)c->L[0].nx * c->L[0].ny;
    }
    b->rows = c0->tile_rows > 0 ? c0->tile_rows : (cells <= (1LL << 22) ? 8 : 12);
    // two steps per launch when every instance can take them (the first
    // instance's setting decides the tile height, 0: off)
    bool pairs = c0->pair_rows != 0;
    for (wp_ctx *c : b->inst) pairs = pairs && wp_pair_capable(c, c->L[0]);
    b->prows = !pairs ? 0 : (c0->pair_rows > 0 ? c0->pair_rows : (cells <= (1LL << 19) ? 8 : 12));
    b->status = (int *)wp_dalloc(c0, 256);
    if (!b->status) return bfail(b, WP_ENOMEM, "batch status");
    if (hipMemsetAsync(b->status, 0, 256, b->stream) != hipSuccess) return bfail(b, WP_EDEVICE, "status clear");
    int rc;
    if ((rc = build_side(b, 0)) != WP_OK) return rc;
    if (hipStreamSynchronize(b->stream) != hipSuccess) return bfail(b, WP_EDEVICE, "batch create sync");
    return WP_OK;
    WP_ABI_CATCH(nullptr)
}

extern "C" void wp_batch_destroy(wp_batch *b)
{
    if (!b) return;
    (void)hipStreamSynchronize(b->stream);
    for (int s = 0; s < 2; ++s)
        if (b->exec[s]) (void)hipGraphExecDestroy(b->exec[s]);
    if (!b->inst.empty()) {
        wp_ctx *c0 = b->inst[0];
        for (int s = 0; s < 2; ++s) {
            wp_dfree(c0, b->desc[s]);
            wp_dfree(c0, b->tiles[s]);
            wp_dfree(c0, b->ptiles[s]);
        }
        wp_dfree(c0, b->status);
    }
    delete b;
}

extern "C" const char *wp_batch_last_error(const wp_batch *b) { return b ? b->err.c_str() : "null batch"; }

// nsteps steps of one side as one captured graph (re-captured when the step
// count or the starting parity changes)
static int run_side(wp_batch *b, int adjoint, int nsteps, int snap_every)
{
    const int par = common_parity(b, adjoint);
    if (par < 0) return bfail(b, WP_ESTATE, "instances are on different buffers (step them through the batch)");
    wp_ctx *c0 = b->inst[0];
    int rc;
    // the launches read the descriptors (snapshot store included) at run
    // time, so a sequence is reused while steps, interval and parity match
    if (!b->exec[adjoint] || b->exec_steps[adjoint] != nsteps || b->exec_every[adjoint] != snap_every ||
        b->exec_parity[adjoint] != par) {
        hipStream_t cs;
        if ((rc = wp_graph_begin(c0, cs)) != WP_OK) return bfail(b, rc, c0->err.c_str());
        int p = par;
        auto snap_of = [&](int s) { return snap_every > 0 && s % snap_every == 0 ? s / snap_every : -1; };
        for (int s = 1; s <= nsteps;) {
            // two steps per launch where possible; either way the result
            // lands in the other canvas
            if (b->prows && s + 1 <= nsteps) {
                launch_side_pair(b, adjoint, p, snap_of(s), snap_of(s + 1), cs);
                s += 2;
            } else {
                launch_side(b, adjoint, p, snap_of(s), cs);
                s += 1;
            }
            p ^= 1;
        }
        if ((rc = wp_graph_end(c0, cs, b->exec[adjoint])) != WP_OK) return bfail(b, rc, c0->err.c_str());
        b->exec_steps[adjoint] = nsteps;
        b->exec_every[adjoint] = snap_every;
        b->exec_parity[adjoint] = par;
        b->exec_end[adjoint] = p;
    }
    if ((rc = wp_graph_launch(c0, b->exec[adjoint])) != WP_OK) return bfail(b, rc, c0->err.c_str());
    for (size_t k = 0; k < b->inst.size(); ++k) {
        Level &lv = batch_level(b->inst[k], adjoint);
        lv.cur = b->exec_end[adjoint];
        lv.t += nsteps * b->dts[k];
    }
    return WP_OK;
}

extern "C" int wp_batch_step(wp_batch *b, int nsteps, int adjoint)
{
    WP_ABI_TRY
    if (!b) return WP_EINVAL;
    if (nsteps < 0) return bfail(b, WP_EINVAL, "nsteps must be non-negative");
    if (adjoint && !b->desc[1]) return bfail(b, WP_ESTATE, "no batched adjoint set up (wp_batch_adjoint_run)");
    if (nsteps == 0) return WP_OK;
    return run_side(b, adjoint ? 1 : 0, nsteps, 0);
    WP_ABI_CATCH(b ? &b->err : nullptr)
}

extern "C" int wp_batch_adjoint_run(wp_batch *b, const wp_functional *J, int nsteps, int snap_every)
{
    WP_ABI_TRY
    if (!b || !J) return b ? bfail(b, WP_EINVAL, "null functional array") : WP_EINVAL;
    int rc;
    std::vector<wp_snapshot_spec> sp(b->inst.size());
    for (size_t k = 0; k < b->inst.size(); ++k) {
        sp[k] = wp_snapshot_spec{b->dts[k], nsteps, snap_every};
        if ((rc = wp_adjoint_setup(b->inst[k], &J[k], &sp[k])) != WP_OK) return bfail(b, rc, b->inst[k]->err.c_str());
    }
    if ((rc = build_side(b, 1)) != WP_OK) return rc;
    if ((rc = run_side(b, 1, nsteps, snap_every)) != WP_OK) return rc;
    for (size_t k = 0; k < b->inst.size(); ++k) wp_adjoint_finish(b->inst[k], &sp[k]);
    return check_status(b);
    WP_ABI_CATCH(b ? &b->err : nullptr)
}
