/*
 * wp.h -- C ABI of the wave-propagation patch library for AMD MI355X (gfx950).
 *
 * The library implements the data-parallel hot path of adjoint-guided
 * block-structured AMR for linear and shallow-water wave propagation
 * (Davis & LeVeque, "Adjoint methods for guiding adaptive mesh refinement in
 * wave propagation problems", arXiv:1511.03645):
 *   - the high-resolution wave-propagation patch update (Sec. 3): a Riemann
 *     solve at every cell edge into waves and speeds, MC-limited second-order
 *     correction fluxes, transverse propagation in 2D, fluctuation-form update;
 *   - the same update for the time-reversed adjoint (Sec. 2 adjoint equation,
 *     Sec. 4 time reversal), with snapshots kept in device memory;
 *   - the adjoint inner-product flag (Sec. 4; Sec. 5.1.2 time range);
 *   - ghost cells from physical boundaries (Sec. 5.1, 5.2), same-level
 *     neighbours or coarse space-time interpolation (Sec. 3), Berger-Oliger
 *     stepping and Berger-Rigoutsos regridding (Sec. 3).
 *
 * Conventions
 *   - Every call returns an int status: WP_OK (0) or a negative wp_status.
 *     wp_last_error() gives a message for the last failure on a handle.
 *   - Grids: level l has nx_l x ny_l cells covering the whole domain
 *     (nx_0 = grid.nx0, nx_{l+1} = nx_l * ratio[l]); cell (i, j) has centre
 *     (xlo + (i + 1/2) dx_l, ylo + (j + 1/2) dy_l).  Patches are boxes of cells
 *     (ilo, jlo, nx, ny) in their level's index space.
 *   - State arrays exchanged with the caller are component-major, row-major
 *     with x fastest: [m][ny][nx], m = 2 (1D acoustics p, u), 3 (2D acoustics
 *     p, u, v; shallow water eta, hu, hv).  Element type: double for
 *     WP_FP64, float for WP_FP32; WP_MIXED (shallow water only) uses double
 *     for eta and float for hu, hv (eta block first, then hu, hv).
 *   - Host pointers passed in are read before the call returns; the caller
 *     keeps ownership.  Device pointers passed in are borrowed for the call.
 *   - Device memory is owned by the library.  It is obtained from the
 *     caller's wp_allocator if one is given (the Python layer backs it with
 *     the PyTorch caching allocator), else with hipMalloc.
 *   - All device work is enqueued on the HIP stream given at creation (or by
 *     wp_set_stream).  Calls that return data to host memory synchronise that
 *     stream.
 *   - Conditions detected on the device (a Courant number above
 *     problem.cfl_max for shallow water, a non-finite value in a step's
 *     output) are latched in a device status word and reported as WP_ECFL or
 *     WP_ENONFINITE by the next call that synchronises (wp_sync, wp_get_state,
 *     wp_functional_value, ...).  Such a step has already been applied.
 *   - A handle must not be used from two threads at once.
 *   - No C++ exception leaves a call: a host allocation that fails inside a
 *     call returns WP_ENOMEM (with its message in wp_last_error); after such
 *     a failure the handle's state is unspecified apart from wp_last_error
 *     and wp_destroy.
 */
#ifndef WP_H
#define WP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WP_MAX_LEVELS 6

typedef enum {
    WP_OK = 0,
    WP_EINVAL = -1,      /* invalid argument or unsupported combination */
    WP_ENOMEM = -2,      /* device or host allocation failed */
    WP_EDEVICE = -3,     /* a HIP runtime call failed */
    WP_ECFL = -4,        /* Courant number above problem.cfl_max */
    WP_ENONFINITE = -5,  /* NaN or Inf produced */
    WP_ERANGE = -6,      /* time or index outside the stored adjoint snapshots */
    WP_ESTATE = -7       /* call out of order (e.g. flag before adjoint run) */
} wp_status;

typedef enum { WP_ACOUSTICS_1D = 1, WP_ACOUSTICS_2D = 2, WP_SWE_2D = 3 } wp_kind;
typedef enum { WP_BC_EXTRAP = 0, WP_BC_WALL = 1, WP_BC_PERIODIC = 2 } wp_bc;
typedef enum { WP_FP64 = 64, WP_FP32 = 32, WP_MIXED = 16 } wp_precision;
typedef enum { WP_FUNC_INTERVAL = 0, WP_FUNC_BOX = 1, WP_FUNC_DISC = 2 } wp_functional_kind;

/* The PDE and the method options (Sec. 2, 3, 5).
 *   kind       equation family
 *   bc[4]      boundary type at x = xlo, x = xhi, y = ylo, y = yhi.
 *              Extrapolation (zero-order, outflow), wall (mirror, normal
 *              velocity negated), periodic.  The adjoint run uses the same
 *              type on each side (walls for walls, Sec. 5.1/5.2.1; outflow
 *              for outflow, Sec. 5.2.3).
 *   order      1: Godunov fluctuations only; 2: with correction fluxes
 *   limiter    0: none (Lax-Wendroff), 1: MC
 *   transverse 0/1: transverse Riemann propagation in 2D (Sec. 3)
 *   precision  WP_FP64, WP_FP32 (acoustics), WP_MIXED (shallow water: eta and
 *              the well-balanced source term in FP64, the rest in FP32)
 *   cfl_max    largest Courant number accepted
 *   g          gravitational acceleration (shallow water)            */
typedef struct {
    int kind;
    int bc[4];
    int order;
    int limiter;
    int transverse;
    int precision;
    double cfl_max;
    double g;
} wp_problem;

/* Coefficients on the level-0 grid, host arrays [ny0][nx0] (Sec. 5.1/5.2:
 * A(x) = [[0, K], [1/rho, 0]]; Sec. 5.3: bathymetry B, depth h = eta - B).
 * Acoustics media are piecewise constant: at most 16 distinct (rho, K)
 * pairs; a cell of a finer level has the medium of the level-0 cell that
 * contains it.  Shallow-water levels above 0 take their bathymetry from
 * wp_set_bathymetry (by default that of the containing level-0 cell). */
typedef struct {
    const double *rho;
    const double *K;
    const double *B;
} wp_coefficients;

/* Domain and refinement hierarchy (Sec. 3): num_levels levels, ratio[l]
 * (2 .. 16) refining level l to level l+1 in space and in time.  Each level
 * is held as one canvas of the whole domain at its resolution, so the
 * finest level's cell count nx0 ny0 (ratio[0] ... ratio[num_levels-2])^2 is
 * bounded (wp_create fails with WP_EINVAL above 2^32 / (5 x element size)). */
typedef struct {
    double xlo, xhi, ylo, yhi;
    int nx0, ny0;
    int num_levels;
    int ratio[WP_MAX_LEVELS];
} wp_grid;

typedef struct {
    int ilo, jlo, nx, ny;
} wp_patch;

/* Target functional J = int phi^T q(x, t_f) dx (eq. J_general) with
 * phi = I(x) e_component, I the indicator of an interval [x0, x1] (1D), a
 * box [x0,x1]x[y0,y1] or a disc of centre (cx, cy) and radius r, each a
 * closed set sampled at level-0 cell centres (eq. delta_1d, delta_2d,
 * delta_Alaska). */
typedef struct {
    int kind;
    int component;
    double x0, x1, y0, y1, cx, cy, r;
} wp_functional;

/* Adjoint run: nsteps steps of size dt on the level-0 grid; qtilde is
 * stored every snap_every steps, step 0 included (Sec. 4), so snapshot n
 * holds qhat at tau_n = t_f - n * snap_every * dt with t_f = nsteps * dt. */
typedef struct {
    double dt;
    int nsteps;
    int snap_every;
} wp_snapshot_spec;

/* Optional device allocator: alloc(bytes, user) returns device memory
 * (256-byte aligned) or NULL; free(ptr, user) releases it. */
typedef struct {
    void *(*alloc)(size_t bytes, void *user);
    void (*free)(void *ptr, void *user);
    void *user;
} wp_allocator;

typedef struct wp_ctx wp_ctx;

/* Create a solver instance: validates the arguments, uploads the
 * coefficients, allocates one state canvas pair per level and sets level 0
 * to a single patch covering the domain (finer levels start empty).
 * stream: a hipStream_t (NULL: the null stream).  On failure *out is NULL
 * if out, problem, coef or grid is NULL; otherwise it holds a handle whose
 * wp_last_error() says what failed and which the caller releases with
 * wp_destroy.  WP_EINVAL among others for a level-0 grid of fewer than 4
 * cells on a side (nx0; also ny0 in 2D). */
int wp_create(const wp_problem *problem, const wp_coefficients *coef, const wp_grid *grid,
              const wp_allocator *alloc, void *stream, wp_ctx **out);
void wp_destroy(wp_ctx *ctx);
const char *wp_last_error(const wp_ctx *ctx);
const char *wp_status_string(int status);
int wp_set_stream(wp_ctx *ctx, void *stream);

/* Bathymetry cell averages of a refined shallow-water level (host array
 * [ny_l][nx_l], FP64, copied; every value below 0: no dry cells), in place of
 * the default in which each cell takes the value of the level-0 cell
 * containing it.  Cell-integrated values at every level (each coarse value the
 * mean of its children) keep the hierarchy consistent; any values keep a
 * lake at rest (eta = 0, no velocity) exactly at rest, since ghost rings,
 * regrids and averages work on eta = h + B (Sec. 5.3).  WP_EINVAL for level 0
 * (set by wp_create), a level out of range, acoustics or a value >= 0. */
int wp_set_bathymetry(wp_ctx *ctx, int level, const double *B);

/* Number of cells and patches of a level; level l canvas size. */
int wp_level_info(const wp_ctx *ctx, int level, int *nx, int *ny, int *npatches);

/* Copy a state into (set) or out of (get) a level.  patch = -1 addresses the
 * whole level canvas ([m][ny_l][nx_l]); patch = k the k-th patch of the level
 * ([m][ny][nx] of its box).  on_device: src/dst is device memory. */
int wp_set_state(wp_ctx *ctx, int level, int patch, const void *src, int on_device);
int wp_get_state(wp_ctx *ctx, int level, int patch, void *dst, int on_device);

/* Advance every patch of `level` by one step of size dt (Sec. 3 wave
 * propagation).  Ghost cells come from physical boundaries, from same-level
 * patches, and for level > 0 from the level below, interpolated in space
 * and linearly in time between the two coarse times bracketing the level's
 * time (Sec. 3).  Fails with WP_ECFL, without changing the state, if the
 * Courant number known from the coefficients exceeds problem.cfl_max. */
int wp_step_patches(wp_ctx *ctx, int level, double dt);

/* Berger-Oliger time stepping (Sec. 3): nsteps coarse steps of size dt0; each
 * coarse step advances level 0 once, then recursively ratio[l] steps of
 * level l+1 of size dt_l / ratio[l], then averages level l+1 onto the level-l
 * cells it covers.  With one level this is nsteps calls of wp_step_patches. */
int wp_advance(wp_ctx *ctx, int nsteps, double dt0);

/* Select the system that the steps of the level hierarchy solve
 * (wp_step_patches, wp_advance, wp_run_graph): adjoint = 0 the forward
 * system, 1 the adjoint system (Sec. 2 adjoint equation, flux -A^T q, in the
 * reversed time), so that the adjoint can itself be solved with refinement
 * (Sec. 7, the proposed AMR of the adjoint problem).  The states of the levels
 * are kept; the caller sets the adjoint data (e.g. the functional's phi) with
 * wp_set_state.  Ghost rings, interpolation, averaging and regridding are the
 * same for both systems.  2D/1D acoustics only (WP_EINVAL otherwise, and for
 * an adjoint value other than 0 or 1).  While the adjoint system is selected,
 * wp_forward_flagged and wp_flag_richardson fail with WP_ESTATE.  Tile tables
 * are rebuilt on a change, so captured sequences are captured again. */
int wp_set_equation(wp_ctx *ctx, int adjoint);
int wp_get_equation(const wp_ctx *ctx, int *adjoint);

/* Flux correction at coarse-fine edges (refluxing) for the Berger-Oliger
 * steps of wp_advance, for the systems in conservation form (Sec. 3 contrasts
 * the adjoint with the forward acoustics): the 2D acoustics hierarchy while
 * it solves the adjoint system, and the shallow-water hierarchy (eq. swe).
 * An edge carries the flux F = f(Q_left) + A^-dQ + Ftilde, seen from the
 * cell left of / below it, or f(Q_right) - A^+dQ + Ftilde from the other
 * side, Ftilde the limited correction flux with its transverse terms.  The
 * reversed adjoint is in f-wave form with f = -A^T q (x) or -B^T q (y), so
 * both sides agree.  Shallow water: the f-waves split the flux difference
 * less the bathymetry source, and f is the physical flux with the
 * hydrostatic pressure of the sea at rest taken out (1/2 g eta (eta - 2B) in
 * place of 1/2 g h^2); the sides agree in mass, and in every component on a
 * flat bottom, and every flux of a lake at rest is zero.  After the r
 * substeps of a level l+1 and its average onto level l, every level-l cell C
 * that shares an edge with a level-l+1 patch and lies in none is corrected by
 *     Q_C += s dt_l/h_l (F_coarse - sum of the fine fluxes / r^2),
 * s = +1 when C lies left of / below the edge, the fine sum taken over the r
 * fine edges along it and the r substeps, each flux evaluated (in FP64) from
 * the state its step started from and seen from C's side of the edge (for a
 * fine edge, its ghost cell there).  The composite sum of a conserved
 * component then changes only through the domain boundary (p of the adjoint,
 * or the water volume, with walls all round).  wp_step_patches does no
 * correction.  on: 0 or 1; WP_ESTATE for on = 1 while the acoustics forward
 * system is selected (its wave form is not conservative; wp_set_equation(0)
 * turns refluxing off), WP_EINVAL for a 1D problem. */
int wp_set_reflux(wp_ctx *ctx, int on);
int wp_get_reflux(const wp_ctx *ctx, int *on);

/* Time-reversed adjoint (Sec. 2, 4): qtilde(x, 0) = phi from the functional,
 * solved forward in time with flux -A^T qtilde on the level-0 grid, the same
 * boundary types as the forward problem.  Snapshots are kept in device
 * memory; any previous adjoint run is replaced. */
int wp_adjoint_run(wp_ctx *ctx, const wp_functional *J, const wp_snapshot_spec *snaps);
int wp_num_snapshots(const wp_ctx *ctx);
int wp_get_snapshot(wp_ctx *ctx, int n, void *dst, int on_device);

/* Install a snapshot store computed outside wp_adjoint_run, for instance the
 * level-0 composite (after the fine-to-coarse average) of an adjoint solved on
 * a refined hierarchy (wp_set_equation; Sec. 7, the adjoint refined too), in
 * place of the store of the last adjoint run.  src: nsnap snapshots, each
 * [m][ny0][nx0] at the level-0 resolution, in FP64 for WP_FP64 problems and
 * FP32 otherwise (the store's own precision); snapshot n holds the adjoint
 * at adjoint time n * ds, i.e. forward time t_f - n * ds with
 * t_f = (nsnap - 1) * ds, as after wp_adjoint_run.  The data are copied
 * (on_device: src is device memory); the caller keeps src.  WP_EINVAL for a
 * null src, nsnap < 1 or ds <= 0; on any failure no store is left
 * (wp_num_snapshots returns 0). */
int wp_set_snapshots(wp_ctx *ctx, const void *src, int nsnap, double ds, int on_device);

/* Adjoint-guided flag (Sec. 4; Sec. 5.1.2) on every patch of `level` at
 * forward time t: m(x) = max over the snapshots bracketing the window
 * [t, min(t + t_f - t_s, t_f)] of |qhat_n(x)^T q(x, t)|, qhat bilinear from the
 * adjoint grid to the level's cell centres (computed in FP64); a cell is
 * flagged iff m > tol.  Snapshot n holds tau_n = t_f - n * ds; times within
 * 1e-9 ds of a snapshot time count as that time.  flags (optional,
 * [ny_l][nx_l] uint8, 0 outside the level's patches) is device or host
 * memory per on_device; *nflagged (optional) receives the count.
 * WP_ERANGE if the window reaches before the earliest snapshot. */
int wp_flag_adjoint(wp_ctx *ctx, int level, double tol, double t, double t_s, double t_f,
                    uint8_t *flags, int on_device, int64_t *nflagged);

/* The comparison flags that the adjoint-guided flag replaces, on every patch
 * of `level` at its current time, each cell flagged iff its measure exceeds
 * tol (tol >= 0); flags and *nflagged as for wp_flag_adjoint, and wp_regrid
 * with patches == NULL clusters these flags the same way.
 * wp_flag_difference (Sec. 5.2.4, "pressure flagging"): the measure is the
 * largest undivided difference |q_k(nb) - q_k(x)| over the components k and
 * the four face neighbours nb of the cell (two along x for 1D acoustics),
 * compared in FP64 from the stored values.  A neighbour across the domain
 * edge follows the boundary rule: extrapolation gives the cell itself, a
 * wall its mirror with the normal component (1 along x, 2 along y) negated,
 * periodic the wrapped cell.  On a refined level the ghost ring is first
 * filled from the level below at the level's time, so patch-edge cells see
 * interpolated neighbours.  Any kind.
 * wp_flag_surface (Sec. 5.3, "surface flagging"): the measure is the
 * departure |eta| of the sea surface eta = h + B from sea level 0 (every cell
 * is wet).  Shallow water only, WP_EINVAL otherwise. */
int wp_flag_difference(wp_ctx *ctx, int level, double tol, uint8_t *flags, int on_device, int64_t *nflagged);
int wp_flag_surface(wp_ctx *ctx, int level, double tol, uint8_t *flags, int on_device, int64_t *nflagged);

/* Richardson error estimate (the estimator Sec. 1 describes, and that the
 * closing Future Work section proposes to weight by the adjoint) on a level
 * of a 2D acoustics instance with even canvas sizes, from its current state:
 * two steps of dt on the same grid and one step of 2 dt on the 2x coarser
 * grid (each coarse cell takes the medium of its lower-left fine cell,
 * the state its 2 x 2 block mean), and per coarse cell and component
 * E = (coarse result - block mean of the fine result) / (2^(p+1) - 2), p the
 * problem's order: for a method of order p this estimates the error of one
 * step of dt.  Every fine cell is measured with its parent's E: weighted = 0
 * takes max_k |E_k|; weighted = 1 takes max |qhat_n(x)^T E| over the
 * snapshots of the window of wp_flag_adjoint at time t.  A cell is flagged
 * iff the measure exceeds tol.  flags and *nflagged as for wp_flag_adjoint
 * (wp_regrid clusters them); estimate (optional, host, [m][ny/2][nx/2] of
 * the level's canvas, FP64) receives E.  The state and time of the instance are unchanged (the
 * steps run on internal copies of the problem at the level's resolution and
 * at half of it, made on the first call on that level and kept until
 * wp_destroy).
 * On a refined level (level > 0, dt that level's step, sizes those of its
 * canvas) the whole canvas is stepped, and E is kept only on the coarse cells
 * whose 2 x 2 block and every fine cell within 4 of it (the reach of the two
 * fine steps and of the coarse step; clipped to the domain) lie in the
 * level's patches: elsewhere E is 0 and no cell is flagged.  Cells outside
 * the patches are never flagged.  Weighted, each cell's parent E meets the
 * snapshots taken bilinearly at the level's cell centres, as in
 * wp_flag_adjoint on that level.
 * WP_EINVAL for a level out of range or without patches, another kind, odd
 * sizes, dt <= 0 or tol < 0; WP_ECFL as for a step of dt; WP_ESTATE or
 * WP_ERANGE as for wp_flag_adjoint when weighted. */
int wp_flag_richardson(wp_ctx *ctx, int level, double dt, int weighted, double tol, double t, double t_s,
                       double t_f, uint8_t *flags, int on_device, int64_t *nflagged, double *estimate);

/* The flag canvas of `level` ([ny_l][nx_l] uint8, 1 = flagged, 0 outside the
 * level's patches) as the last flag call on that level left it: wp_flag_adjoint,
 * wp_flag_difference, wp_flag_surface, wp_flag_richardson, or the last flag
 * event of wp_forward_flagged (Sec. 4; Sec. 5.1.2).  dst is device or host
 * memory per on_device (a host copy synchronises the stream).  WP_ESTATE if
 * the level has not been flagged since it was created or regridded. */
int wp_get_flags(wp_ctx *ctx, int level, uint8_t *dst, int on_device);

/* The forward run with adjoint-guided flagging (Sec. 4; Sec. 5.1.2) on a
 * single-level instance: nsteps steps of size dt from the current state and
 * time t0, with the flag of wp_flag_adjoint(0, tol, t, t_s, t_f) evaluated at
 * t = t0 + k flag_every dt before each block of flag_every steps
 * (k = 0 .. nsteps/flag_every - 1), all enqueued as one captured sequence.
 * counts (optional, host, nsteps/flag_every entries) receives the number of
 * flagged cells of each event; step_ms (optional, host, same length; 2D
 * acoustics) the duration of the first step launch of each block on the
 * device's constant-rate clock: from its earliest workgroup start to that of
 * the second step (dispatch and completion included), or to its own latest
 * workgroup end when flag_every is 1.  The flag canvas keeps the last event's flags.
 * Either output synchronises the stream.  WP_EINVAL if nsteps is not a multiple of
 * flag_every or the instance has refinement levels; WP_ERANGE if a window
 * reaches before the first snapshot (nothing is enqueued then). */
int wp_forward_flagged(wp_ctx *ctx, double dt, int nsteps, int flag_every, double tol, double t_s, double t_f,
                       int64_t *counts, float *step_ms);

/* Replace the patches of level+1 (Sec. 3 regridding).  patches != NULL: the
 * npatches given boxes (level+1 index space; corners and sides multiples of
 * ratio[level]; disjoint; properly nested: every covered level cell lies in
 * level's patches with all eight neighbours inside the domain also in them,
 * i.e. level's patches shrunk by one cell except along the physical
 * boundary).  patches == NULL: the flags of `level` from the last
 * wp_flag_adjoint, wp_flag_difference, wp_flag_surface or
 * wp_flag_richardson on it, restricted to that nesting region, dilated by `buffer` cells and
 * restricted again, clustered by wp_cluster with
 * efficiency 0.7, sides of at most max(1, 64 / ratio) and at least
 * max(1, 8 / ratio) level cells, then refined by the ratio.  Cells of the new
 * patches keep the old level+1 data where an old patch covered them and are
 * otherwise interpolated in space from level (minmod-limited linear, Sec. 3).
 * Sets level+1's time to level's and empties the levels above level+1 (they
 * are regridded from level+1 next).  WP_EINVAL for a box that breaks the
 * rules above, WP_ESTATE if patches == NULL and `level` has no flags. */
int wp_regrid(wp_ctx *ctx, int level, const wp_patch *patches, int npatches, int buffer);
/* The patches of a level: *npatches receives their number, out (cap
 * entries, caller-owned) the first min(cap, number) of them. */
int wp_get_patches(const wp_ctx *ctx, int level, wp_patch *out, int cap, int *npatches);

/* Berger-Rigoutsos clustering (Sec. 3, after Berger & Rigoutsos 1991) of
 * the flagged cells of an nx x ny image (host memory, [ny][nx] uint8, nonzero
 * = flagged) into boxes, on the host.  allowed (optional, same layout):
 * cells a box may hold; flags outside it are ignored.  Rules, fixed so that
 * the result is unique: shrink a box to the bounding box of its flags (drop
 * it if none); accept it if the flagged fraction is at least `efficiency`,
 * both sides are at most maxside and every cell is allowed; else cut it at
 * the interior zero of the column/row flag counts nearest the centre, else
 * at the largest sign change of their second difference, else in halves of
 * the longer side, each part keeping at least minside cells (1 when the box
 * holds cells that are not allowed), and recurse on the lower/left part
 * first; a box with no admissible cut is accepted.  *npatches receives the
 * number of boxes, out (cap entries, caller-owned) the first min(cap, number).
 * Needs no handle and no device. */
int wp_cluster(const uint8_t *flags, const uint8_t *allowed, int nx, int ny, double efficiency, int maxside,
               int minside, wp_patch *out, int cap, int *npatches);

/* J = sum over level-0 cells of phi^T q dx dy (which = 0), or the inner
 * product integral sum qhat_n^T q dx dy with snapshot n (which = 1; eq. J,
 * constant in t), both accumulated in FP64 with compensated summation. */
int wp_functional_value(wp_ctx *ctx, const wp_functional *J, int which, int snapshot, double *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * compensated FP64 inner-product reduction of wp_functional_value (which = 1,
 * and J when b holds phi) on caller-owned device arrays, needing no handle.
 *   a, b       device arrays [m][cells] (component stride = cells), both
 *              double (precision WP_FP64) or both float (WP_FP32)
 *   out        device memory, one double: dA * sum_k sum_i a_k[i] b_k[i]
 *              (the same block count and summation order as
 *              wp_functional_value, so the two agree)
 *   stream     hipStream_t the two kernels are enqueued on (NULL: the null
 *              stream); nothing is copied to the host and nothing synchronises
 * The per-block partial sums go to a fixed 16 KiB device array of the library
 * (one per GPU, held until the process ends), so the call allocates nothing;
 * calls that overlap on one GPU (two streams, two threads) race on it.
 * WP_EINVAL for a null pointer, another precision, m outside 1..3, or cells
 * outside 1..WP_NOALLOC_MAX_CELLS; WP_EDEVICE if the array's device address
 * cannot be found or a launch fails. */
#define WP_NOALLOC_MAX_CELLS (1LL << 32)
int wp_inner_product_noalloc(const void *a, const void *b, int precision, long long cells, int m, double dA,
                             double *out, void *stream);

/* Current time of a level; largest Courant number of the last step. */
int wp_get_time(const wp_ctx *ctx, int level, double *t);
int wp_set_time(wp_ctx *ctx, int level, double t);

/* Host time the handle has spent, in milliseconds, cumulative since
 * creation or the last reset: ms[0] copying a level's flags to the host for a
 * regrid (including the wait for the work before them), ms[1] clustering and
 * nesting, ms[2] rebuilding and uploading the tables of the new patches,
 * ms[3] capturing launch sequences (and instantiating or updating their
 * graphs); ms[4] the number of captures and ms[5] how many of them updated
 * the existing graph in place instead of instantiating a new one; ms[6] the
 * part of ms[2] spent in host-to-device copies of the tables (staging, copy,
 * wait); ms[7] the time spent rebuilding tile tables (their copies
 * included), most of it within ms[2].  The first min(n, 8) entries are
 * written (the rest of n zeroed); reset = 1 clears the counters afterwards. */
int wp_host_times(wp_ctx *ctx, double *ms, int n, int reset);

/* Wait for all work of the handle and report latched device conditions. */
int wp_sync(wp_ctx *ctx);

/* ------------------------------------------------------------------------
 * Batches: many independent single-level acoustics instances of the same
 * precision advanced together, every step of every instance in one launch.
 * ---------------------------------------------------------------------- */
typedef struct wp_batch wp_batch;

/* Build a batch over n instances (each created with one level and already
 * holding its state).  dts[k]: the fixed step of instance k.  The
 * instances stay owned by the caller and must outlive the batch.  Steps go
 * two per launch (see wp_set_step_pairs) when every instance can take
 * them, at the tile height set on the first instance (0 there: one step
 * per launch); the tile tables are built once, from the instances' grids
 * and media at creation. */
int wp_batch_create(wp_ctx *const *instances, int n, const double *dts, wp_batch **out);
void wp_batch_destroy(wp_batch *b);
/* nsteps steps of every instance, forward (adjoint = 0) or of the adjoint
 * states that wp_batch_adjoint_run set up (adjoint = 1; WP_ESTATE before
 * any). */
int wp_batch_step(wp_batch *b, int nsteps, int adjoint);
/* Adjoint runs of every instance in the batch: J[k], snapshot spec with
 * per-instance dt from the batch; every instance runs spec->nsteps steps. */
int wp_batch_adjoint_run(wp_batch *b, const wp_functional *J, int nsteps, int snap_every);
const char *wp_batch_last_error(const wp_batch *b);

/* Tile shape of the patch-update kernels: rows per tile for the 2D
 * kernels (0: the built-in choice; 0 to 4096, WP_EINVAL otherwise), applied
 * to every level's tile tables at once.  Heights 4, 6, 8, 12 and 16 take a
 * compiled march (on refined levels two narrow tiles may share a wave, and
 * at 4, 8 and 16 the finest level of ratio 4 also averages its last
 * substep onto the level below in the step); other heights take the rolled
 * march.  Exposed for the autotuner. */
int wp_set_tile_rows(wp_ctx *ctx, int rows);
int wp_get_tile_rows(const wp_ctx *ctx, int *rows);

/* Two steps per launch (the wave-propagation update of Sec. 3 applied
 * twice, the intermediate state kept in registers, its ghost cells set by
 * the boundary rules): used by wp_run_graph, wp_adjoint_run and
 * wp_forward_flagged on a single-level 2D acoustics instance with the full
 * method (order 2, MC limiter, transverse terms) and no periodic boundary.
 * rows: -1 the built-in tile height, 0 off (one step per launch), or 4 to
 * 64 rows per tile.  The results equal those of one step per launch up
 * to rounding (bit for bit where both use the same per-cell path).
 * WP_EINVAL for any other rows.  wp_get_step_pairs reports the tile height
 * of level 0 in use, 0 when its steps go one per launch. */
int wp_set_step_pairs(wp_ctx *ctx, int rows);
int wp_get_step_pairs(const wp_ctx *ctx, int *rows);

/* Capture `nsteps` single-level steps of size dt into a HIP graph and replay
 * it `replays` times (the steps of nsteps calls of wp_step_patches on level
 * 0, two per launch where wp_set_step_pairs allows it).  WP_EINVAL unless
 * nsteps >= 1 and replays >= 0; zero replays capture and change nothing. */
int wp_run_graph(wp_ctx *ctx, int nsteps, double dt, int replays);

#ifdef __cplusplus
}
#endif
#endif /* WP_H */
