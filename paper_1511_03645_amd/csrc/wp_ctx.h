// Handle layout shared by the host translation units of the library.
#pragma once

#include <string>
#include <array>
#include <vector>

#include "wp_internal.h"

constexpr int RED_BLOCKS = 1024;

// slots of wp_ctx::host_ms (wp_host_times)
enum { HT_FLAG_COPY = 0, HT_CLUSTER, HT_UPLOAD, HT_CAPTURE, HT_NCAPTURE, HT_NUPDATE, HT_H2D, HT_TILES, WP_HOST_TIMES };

// milliseconds since an arbitrary origin (steady clock)
double wp_now_ms();

// One refinement level: a canvas covering the whole domain at the level's
// resolution (double-buffered), the patches that are active on it and the
// tile tables of its launches.
struct Level {
    int nx = 0, ny = 0;
    double dx = 0.0, dy = 0.0;
    int ratio = 1;                       // refinement relative to the level below
    void *q[2] = {nullptr, nullptr};     // state canvases
    int cur = 0;                         // index of the current canvas
    uint8_t *mat = nullptr;              // acoustics material index per cell
    uint8_t *flags = nullptr;            // flag canvas
    bool flags_valid = false;
    std::vector<wp_patch> patches;
    std::vector<wp::Tile> tiles_host;
    wp::Tile *tiles_dev = nullptr;
    int ntiles = 0;
    int tile_rows = 0;                   // rows of the step tiles (compile-time march height if supported)
    int nuni = 0;                        // number of single-material tiles (they follow the mixed ones)
    bool dual = false;                   // some tiles carry a second narrow tile (see Tile)
    // two-step tiles (single-level 2D acoustics; see launch_acou2d_pair):
    // none when the level cannot take two steps per launch
    wp::Tile *ptiles_dev = nullptr;
    int nptiles = 0, npuni = 0, pair_rows = 0;
    wp::Tile *ftiles_dev = nullptr;      // flag / reduction tiles
    int nftiles = 0;
    double t = 0.0;
    void *inst = nullptr;                // device instance descriptor
    double inst_dt = -1.0;
    void *snap_base = nullptr;           // snapshot store written by this level's steps (adjoint)
    void *inst_snap = nullptr;
    alignas(16) unsigned char inst_host[256];
    // the other canvas holds the state at t_prev after a step
    double t_prev = 0.0;
    bool prev_valid = false;
    // refinement: cells of the ghost ring (inside the domain, outside every
    // patch, within two cells of one), filled from the level below before
    // each step; coarse cells covered by the patches (linear indices on the
    // level below), overwritten by the average of their children
    // (nring cells; ring_dev lists them only for ratios above 8, smaller
    // ratios take ringb_dev)
    int *ring_dev = nullptr;
    long long nring = 0;
    int *ringb_dev = nullptr;            // the ring by coarse parent (see launch_ring_fill_blocks)
    long long nringb = 0;
    int *cover_dev = nullptr;
    long long ncover = 0;
    // allocated sizes (bytes) of the tables above: a smaller table is written
    // into the same block
    size_t tiles_cap = 0, ftiles_cap = 0, ptiles_cap = 0, ring_cap = 0, ringb_cap = 0, cover_cap = 0;
    // refluxing (adjoint hierarchy): the edges between this level's patches
    // and level-1 cells that no patch of this level covers, as int4
    // {coarse cell, axis | (coarse cell before the edge) << 1, first fine
    // cell i, j}, sorted by coarse cell; the groups {first face, count} of
    // each coarse cell; one FP64 register of 3 per face
    int *faces_dev = nullptr, *fgroups_dev = nullptr;
    double *freg_dev = nullptr;
    int nfaces = 0, nfgroups = 0;
    size_t faces_cap = 0, fgroups_cap = 0, freg_cap = 0;
    double *B = nullptr;                 // shallow water: bathymetry cell averages of this level (FP64)
    // set for one step: average the step's results onto this level (the
    // level below, see launch_acou2d); averaged: the step did
    Level *avg_onto = nullptr;
    bool averaged = false;
    // false after a tile-table rebuild failed (its tables are empty): steps
    // and flags of the level fail with WP_ESTATE until a rebuild succeeds
    bool tables_ok = true;
};

struct wp_ctx {
    wp_problem prob{};
    wp_grid grid{};
    wp_allocator alloc{};
    bool has_alloc = false;
    hipStream_t stream = nullptr;
    bool kind2d = true, is_acoustics = true;
    int m = 3, esz = 8;
    std::vector<void *> owned;
    std::vector<Level> L;
    Level adj;                           // adjoint grid (level-0 resolution)
    bool adj_ready = false;              // adj fully built (wp_ensure_adjoint_level)
    // acoustics media
    int nmat = 0;
    std::vector<double> rho, K;
    std::vector<uint8_t> mat0;
    double cmax = 0.0;
    void *mtab = nullptr, *ptab = nullptr;
    double *mtab64 = nullptr;            // [nmat][4] Z, c, rho, K in FP64 (flux bookkeeping)
    // shallow water
    void *Bdev = nullptr;                // bathymetry (FP64)
    void *cbar = nullptr;                // sqrt(-g B) in the adjoint precision
    void *swe_inst = nullptr, *swe_adj_inst = nullptr;
    double swe_inst_dt = -1.0, swe_adj_inst_dt = -1.0;
    double last_cfl = 0.0;
    // adjoint snapshots
    void *snaps = nullptr;
    size_t snaps_cap = 0, snap_bytes = 0;
    int nsnap = 0;
    double snap_ds = 0.0, adj_tf = 0.0;
    // device scratch
    int *status = nullptr;
    unsigned long long *count = nullptr;
    double *partials = nullptr, *red_out = nullptr;
    unsigned *cflbits = nullptr;
    uint8_t *ind_dev = nullptr;          // indicator of the cached functional
    wp_functional ind_key{};
    bool ind_valid = false;
    void *phi_dev = nullptr;             // adjoint initial data of the cached functional
    wp_functional phi_key{};
    bool phi_valid = false;
    // host time spent (ms, cumulative; see wp_host_times) and event counts
    double host_ms[WP_HOST_TIMES] = {0};
    // host images of a regrid (flag rows, window flags, nesting mask,
    // buffered flags), kept between regrids
    std::vector<uint8_t> rg_rows, rg_flags, rg_allowed, rg_dil;
    // the lists a regrid builds and uploads (one at a time), kept likewise
    std::vector<int> rg_list[2];
    std::vector<std::array<int, 3>> rg_runs;
    std::string err;
    int equation = 0;                    // system the level hierarchy's steps solve: 0 forward, 1 adjoint
    bool reflux = false;                 // flux correction at coarse-fine edges (adjoint system only)
    int tile_rows = 0;
    int pair_rows = -1;                  // two-step tile height: -1 built-in choice, 0 off
    // captured launch sequences (recorded on an internal stream, replayed on
    // `stream`)
    hipStream_t cap_stream = nullptr;
    // every cached sequence records the tile-table generation it was
    // captured with and is re-captured when a table has been rebuilt since
    hipGraphExec_t graph_exec = nullptr;     // forward steps of level 0
    int graph_steps = 0, graph_parity = -1, graph_flip = 0;   // flip: canvas parity change of one replay
    double graph_dt = 0.0;
    unsigned long long graph_gen = 0;
    hipGraphExec_t bo_exec = nullptr;        // two Berger-Oliger coarse steps of every level
    double bo_dt = 0.0;
    unsigned long long bo_gen = 0;
    std::vector<int> bo_par;
    unsigned long long topo_gen = 1;         // bumped whenever a tile table changes
    hipGraphExec_t ff_exec = nullptr;        // flagged forward run
    double ff_key[6] = {0, 0, 0, 0, 0, 0}, ff_t0 = 0.0;
    int ff_parity = -1, ff_flip = 0;         // flip: canvas parity change of the run
    unsigned long long ff_gen = 0;
    const void *ff_snaps = nullptr;
    double ff_store[2] = {0.0, 0.0};         // snapshot interval and count the window indices came from
    unsigned long long *ev_counts = nullptr;   // flagged cells per flag event (COUNT_SPAN entries each)
    size_t ev_counts_cap = 0;
    unsigned long long *stamps = nullptr;      // workgroup clocks of the timed steps
    size_t stamps_cap = 0;
    unsigned long long *stamp_next = nullptr;  // clock slot for the next 2D acoustics launch
    hipGraphExec_t adj_exec = nullptr;       // adjoint run with snapshot copies
    int adj_steps = 0, adj_every = 0, adj_end = 0;   // adj_end: canvas parity after the run
    double adj_dt = 0.0;
    unsigned long long adj_gen = 0;
    const void *adj_snaps = nullptr;
    // pinned host staging for every transfer between device memory and the
    // caller's (pageable) host memory; allocated on first use, grown up to
    // WP_PIN_CAP, released by wp_destroy
    void *pin = nullptr;
    size_t pin_bytes = 0;
    // new fine cells of a regrid (device list, reused)
    int *fresh_dev = nullptr;
    size_t fresh_cap = 0;
    // Richardson estimate: single-level copies of the problem at this
    // resolution and at half of it (created on first use), and the estimate
    std::vector<wp_ctx *> rich;          // per level: the copies at its resolution and at half of it
    double *richE = nullptr;
    size_t richE_cap = 0;
    uint8_t *rich_valid = nullptr;       // coarse cells kept on a refined level
    size_t rich_valid_cap = 0;
    double *richEf = nullptr;            // the estimate on a refined level's cells (weighted flag)
    size_t richEf_cap = 0;
    size_t snap_esz() const { return prob.precision == WP_FP64 ? 8 : 4; }
};

int wp_fail(wp_ctx *ctx, int code, const char *fmt, ...);
// The getters take a const handle; their argument errors still leave the
// handle's last-error message (a per-handle record, not state).
inline int wp_fail_get(const wp_ctx *ctx, int code, const char *what)
{
    return ctx ? wp_fail(const_cast<wp_ctx *>(ctx), code, "%s", what) : code;
}
// Copies between device memory and host memory through the pinned staging
// buffer, on the handle's stream, complete when they return: `rows` rows of
// `width` bytes, `dpitch` / `spitch` bytes apart on the destination / source.
int wp_host_copy2d(wp_ctx *ctx, void *dst, size_t dpitch, const void *src, size_t spitch, size_t width, size_t rows,
                   bool to_device);
int wp_host_copy(wp_ctx *ctx, void *dst, const void *src, size_t bytes, bool to_device);
// flag counters spread over slots (COUNT_SPAN entries each): clear n, read n
int wp_clear_counts(wp_ctx *ctx, unsigned long long *dev, int n, hipStream_t s);
int wp_read_counts(wp_ctx *ctx, const unsigned long long *dev, int n, int64_t *out);
// Copy a host table to a device block of `cap` bytes, first replacing the
// block by one half as large again as needed when it is too small.
int wp_upload(wp_ctx *ctx, const void *src, size_t bytes, void *&dev, size_t &cap, const char *what);
void *wp_dalloc(wp_ctx *ctx, size_t bytes);
void wp_dfree(wp_ctx *ctx, void *p);
std::vector<wp::Tile> wp_make_tiles(const std::vector<wp_patch> &patches, int inst, int rows, int width, bool xcd_order);
int wp_upload_tiles(wp_ctx *ctx, Level &lv);
int wp_default_rows(const wp_ctx *ctx, const Level &lv);
uint8_t wp_level_mat(const wp_ctx *ctx, const Level &lv, int i, int j);
void wp_classify_tiles(const wp_ctx *ctx, const Level &lv, std::vector<wp::Tile> &tiles, int rows, int halo = 2);
bool wp_pair_capable(const wp_ctx *ctx, const Level &lv);
bool wp_pair_ready(const wp_ctx *ctx, const Level &lv);
int wp_step_pair(wp_ctx *ctx, Level &lv, double dt, int adjoint, hipStream_t s, int snap1, int snap2,
                 const wp::PairFlag *flag = nullptr);
int wp_alloc_level(wp_ctx *ctx, Level &lv);
int wp_check_status(wp_ctx *ctx);
int wp_courant_check(wp_ctx *ctx, const Level &lv, double dt);
int wp_step_level(wp_ctx *ctx, Level &lv, double dt, int adjoint, hipStream_t s, int snap_index);
int wp_prepare_level(wp_ctx *ctx, Level &lv, double dt);
int wp_build_indicator(wp_ctx *ctx, const wp_functional *J, std::vector<uint8_t> &ind);
int wp_ensure_adjoint_level(wp_ctx *ctx);
int wp_adjoint_setup(wp_ctx *ctx, const wp_functional *J, const wp_snapshot_spec *sp);
void wp_adjoint_finish(wp_ctx *ctx, const wp_snapshot_spec *sp);
void wp_xcd_order(std::vector<wp::Tile> &t);
int wp_window(wp_ctx *ctx, double t, double t_s, double t_f, int &n_lo, int &n_hi);
// shallow water (swe_host.hip)
int wp_swe_init(wp_ctx *ctx, const wp_coefficients *coef);
int wp_swe_adj_init(wp_ctx *ctx);
int wp_swe_step(wp_ctx *ctx, Level &lv, double dt, int adjoint, hipStream_t s, int snap_index);
int wp_swe_prepare(wp_ctx *ctx, Level &lv, double dt);
int wp_graph_begin(wp_ctx *ctx, hipStream_t &s);
int wp_graph_end(wp_ctx *ctx, hipStream_t s, hipGraphExec_t &exec);
int wp_graph_launch(wp_ctx *ctx, hipGraphExec_t exec);
// refinement (amr_host.hip, cluster.cpp)
int wp_fill_coarse_ghosts(wp_ctx *ctx, int level, double t);
void wp_nesting_mask(const std::vector<wp_patch> &patches, int nx, int ny, int wi0, int wj0, int ww, int wh,
                     std::vector<uint8_t> &mask);
void wp_dilate(const std::vector<uint8_t> &f, int nx, int ny, int k, std::vector<uint8_t> &out);
void wp_cluster_boxes(const uint8_t *flags, const uint8_t *allowed, int nx, int ny, double efficiency, int maxside,
                      int minside, std::vector<wp_patch> &out);
