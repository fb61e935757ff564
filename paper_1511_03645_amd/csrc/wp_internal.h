// Internal declarations shared by the host code and the HIP kernels of the
// wave-propagation library.  Not part of the public C ABI (include/wp.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "wp.h"

namespace wp {

constexpr int MAXMAT = 16;     // distinct (rho, K) pairs per acoustics instance
constexpr int WAVE = 64;       // CDNA wavefront
constexpr int STRIP = WAVE - 4; // output columns per wave in the 2D kernels
constexpr int PAIR_STRIP = WAVE - 8;   // output columns per wave of the two-step kernel

// Height of the mixed-material tiles of a 2D acoustics launch whose
// single-material tiles are `rows` high: their per-cell table lookups make a
// row slower, so they are cut shorter to finish with the rest of the launch.
__host__ __device__ constexpr int acou_mixed_rows(int rows) { return rows >= 8 ? rows / 2 : rows; }

// One unit of work of a patch-update launch: output cells
// [i0, i0 + ni) x [j0, j0 + nj) of instance `inst`.
struct Tile {
    int inst, i0, j0, ni, nj;
    int mat;   // material of every cell the tile reads (halo included), -1 if mixed
    int down;  // 2D acoustics: march the rows downwards (alternates between
               // vertically adjacent tiles, so the halo rows they share are
               // read by both at about the same time)
    // a second tile (nib > 0) in the upper lanes of the wave (one-step 2D
    // acoustics): lanes 0 .. ni + 3 take the first, with its two halo
    // columns either side, lanes ni + 4 .. 63 (i0b, j0b, nib, njb); same
    // instance, material and direction, ni + nib <= TWO_TILE_COLS
    int i0b = 0, j0b = 0, nib = 0, njb = 0;
};
// output columns two tiles of one wave may have together: 64 lanes less a
// two-column halo either side of each
constexpr int TWO_TILE_COLS = WAVE - 8;

// Per-instance description of a 2D (or 1D) acoustics level canvas.  The
// canvas covers the whole domain at the level's resolution with no ghost
// border: ghost cells are resolved by the loaders from the boundary rules
// (or read from the canvas itself when they lie inside the domain).
template <typename T>
struct AcouInst {
    T *q[2];                  // double-buffered state, component stride cs
    const uint8_t *mat;       // material index per cell
    long long cs;             // component stride (elements)
    int nx, ny;
    int bc[4];
    T nux, nuy;               // dt/dx, dt/dy
    const T *mtab;            // [nmat][4]: Z, c, K = Z c, 1/rho = c / Z
    const T *ptab;            // [nmat][nmat][3]: 1/(Z_a+Z_b), kappa1, kappa2
    int nmat;
    int order, limiter, transverse;
    T *snap;                  // snapshot store: on a snapshot step the new state is also written to
    long long snap_stride;    //   snap + snap_index * snap_stride (elements)
};

// Shallow-water instance (single level).  ETA is the storage and arithmetic
// type of the surface elevation eta = h + B and of the well-balanced term
// g hbar d(eta) (double in the FP64 and mixed paths); T is the type of hu,
// hv and of the bulk arithmetic (double for FP64, float for mixed).
template <typename ETA, typename T>
struct SweInst {
    ETA *eta[2];
    T *hu[2];
    T *hv[2];
    const double *B;          // bathymetry cell averages (FP64)
    int nx, ny;
    int bc[4];
    double nux, nuy;          // dt/dx, dt/dy
    double g;
    double cfl_max;
    int order, limiter, transverse;
};

// Linearised shallow-water adjoint (time reversed), state (eta, mu, gamma)
// of type T; cbar = sqrt(g hbar) per cell with hbar = -B.
template <typename T>
struct LsweInst {
    T *q[2];                  // double-buffered, component stride nx*ny
    const T *cbar;
    int nx, ny;
    int bc[4];
    T nux, nuy;
    T g;
    int order, limiter, transverse;
    T *snap;                  // snapshot store (see AcouInst)
    long long snap_stride;
};

// Flag counters: workgroup b adds its count to slot b % COUNT_SLOTS of a
// counter, the slots COUNT_STRIDE entries apart (separate cache lines), so
// that the adds of one launch do not all queue on one address.  A counter
// spans COUNT_SPAN entries and is the sum of its slots.
constexpr int COUNT_SLOTS = 16, COUNT_STRIDE = 16;
constexpr int COUNT_SPAN = COUNT_SLOTS * COUNT_STRIDE;
__device__ __forceinline__ unsigned long long *count_slot(unsigned long long *c)
{
    return c + (blockIdx.x % COUNT_SLOTS) * COUNT_STRIDE;
}

// status word bits latched by kernels
constexpr int ST_NONFINITE = 1;
constexpr int ST_CFL = 2;

// The level below a refined level of ratio 4 (its current canvas: three
// planes of cs elements, rows nx long), which a step can average its results
// onto (see launch_acou2d).
template <typename T>
struct AvgTo {
    T *q;
    int nx;
    long long cs;
};

// dual: some tiles hold a second tile in the wave's upper lanes (forward,
// unrolled heights).  avg (dual, rows 4, 8 or 16, a level of ratio 4 whose
// tiles start on rows and columns of multiples of 4): also write the mean of
// each 4 x 4 block of the results onto the cell of the level below that
// contains it, summed row by row as launch_average sums.
template <typename T>
void launch_acou2d(const AcouInst<T> *insts, const Tile *tiles, int ntiles, int parity, int adjoint,
                   int nmat_max, bool full, int rows, int kind, int snap_index, int *status, hipStream_t s,
                   unsigned long long *stamp = nullptr, bool dual = false, const AvgTo<T> *avg = nullptr);
// whether launch_acou2d can average a step of a level with these settings
inline bool acou2d_can_average(bool dual, bool full, int rows, int ratio)
{
    return dual && full && ratio == 4 && (rows == 4 || rows == 8 || rows == 16);
}
// Two steps per launch on a single-level canvas (tiles PAIR_STRIP wide,
// 4..64 rows high: 8, 10 and 12 unrolled, others rolled; no periodic
// boundary); q^{n+2} lands in
// q[parity ^ 1], and snapshots snap1 / snap2 (-1: none) take q^{n+1} /
// q^{n+2}.
//
// With `flag` (forward only, a single instance whose level is the adjoint
// grid), the launch first takes the adjoint flag of q^n on its tiles'
// cells, as launch_flag does for ratio 1: flags[cell] = max over snapshots
// n_lo..n_hi of |qhat_n . q^n| > tol, and the number flagged added to
// *count.
struct PairFlag {
    const void *snaps;            // snapshot store [n][3][ny][nx], state precision
    long long sstride;            // elements per snapshot
    int n_lo, n_hi;
    double tol;
    uint8_t *flags;               // the level's flag canvas
    unsigned long long *count;
};
template <typename T>
void launch_acou2d_pair(const AcouInst<T> *insts, const Tile *tiles, int ntiles, int parity, int adjoint,
                        int nmat_max, int rows, int kind, int snap1, int snap2, int *status, hipStream_t s,
                        unsigned long long *stamp = nullptr, const PairFlag *flag = nullptr);
template <typename T>
void launch_acou1d(const AcouInst<T> *inst_dev, const AcouInst<T> &inst_host, int parity, int adjoint,
                   int snap_index, int *status, hipStream_t s);

template <typename ETA, typename T>
void launch_swe2d(const SweInst<ETA, T> *inst, const Tile *tiles, int ntiles, int rows, bool full, int parity,
                  int *status, unsigned *cflbits, hipStream_t s);
template <typename T>
void launch_lswe_adj2d(const LsweInst<T> *inst, const Tile *tiles, int ntiles, int rows, int parity, int snap_index,
                       int *status, hipStream_t s);

// Flag: m(x) = max_n |qhat_n(x) . q(x)| over snapshots n_lo..n_hi, bilinear
// from the adjoint grid (refinement `ratio` relative to it).
template <typename TQ, typename TH>
void launch_flag(const TQ *q, long long cs, int nx, int ny, int m, const TH *snaps, long long snap_stride,
                 long long hcs, int NX, int NY, int ratio, int n_lo, int n_hi, double tol, const Tile *tiles,
                 int ntiles, uint8_t *flags, unsigned long long *count, hipStream_t s);
void launch_flag_mixed(const double *eta, const float *hu, const float *hv, long long cs, int nx, int ny,
                       const float *snaps, long long snap_stride, long long hcs, int NX, int NY, int ratio, int n_lo,
                       int n_hi, double tol, const Tile *tiles, int ntiles, uint8_t *flags,
                       unsigned long long *count, hipStream_t s);

// Comparison flags: the undivided difference of every component to its four
// face neighbours (boundary rule across the domain edge, bc[4]), and the
// sea-surface departure |eta| (shallow water).  c2 null: two components.
template <typename TE, typename TU>
void launch_flag_difference(const TE *c0, const TU *c1, const TU *c2, int nx, int ny, const int *bc, double tol,
                            const Tile *tiles, int ntiles, uint8_t *flags, unsigned long long *count, hipStream_t s);
template <typename TE>
void launch_flag_surface(const TE *eta, int nx, double tol, const Tile *tiles, int ntiles, uint8_t *flags,
                         unsigned long long *count, hipStream_t s);

// Richardson estimate: 2 x 2 block means of a canvas, and E = (coarse -
// block mean of fine) / denom per coarse cell (FP64, [m][NY][NX]) with the
// flag of every fine cell of the tiles from its parent's E (snaps null:
// max_k |E_k|; else max over snapshots n_lo..n_hi of |qhat . E|).
template <typename T>
void launch_coarsen2(const T *f, long long fcs, int nx, T *c, long long ccs, int NX, int NY, int m, hipStream_t s);
template <typename T>
void launch_richardson(const T *coarse, long long ccs, const T *fine, long long fcs, int nx, int NX, int NY, int m,
                       double denom, double *E, const void *snaps, long long sstride, long long hcs, int n_lo,
                       int n_hi, double tol, const Tile *tiles, int ntiles, uint8_t *flags,
                       unsigned long long *count, hipStream_t s);

// Compensated FP64 reductions: out[0] = sum_k sum_cells w(cell) a_k b_k where
// a is m component arrays (type TA) and b either an indicator (uint8, times
// unit vector `comp`) or m arrays of type TB (the sum times `scale`).
// partials: 2 * nblocks doubles of scratch.
template <typename TA>
void launch_sum_indicator(const TA *a, long long cs, long long n, int comp, const uint8_t *ind, double *partials,
                          int nblocks, double *out, hipStream_t s);
template <typename TA, typename TB>
void launch_sum_dot(const TA *a, long long acs, const TB *b, long long bcs, long long n, int m, double *partials,
                    int nblocks, double *out, hipStream_t s, double scale = 1.0);
void launch_sum_dot_mixed(const double *eta, const float *hu, const float *hv, long long cs, const float *b,
                          long long bcs, long long n, double *partials, int nblocks, double *out, hipStream_t s);

void launch_fill_u8(uint8_t *p, long long n, uint8_t v, hipStream_t s);

// Refinement transfers: fill fine cells (linear indices into the fine canvas)
// from the coarse level at two times (time weight alpha), and average fine
// children onto covered coarse cells (linear coarse indices).
// k0, nk: the components filled (the pointers address component k0's plane).
template <typename T>
void launch_ring_fill(const int *cells, long long ncells, T *fine, int nxf, const T *cold, const T *cnew, int NX,
                      int NY, int r, double alpha, const int *bc, hipStream_t s, int k0 = 0, int nk = 3);
// The ring fill by coarse parent: blocks[3e] the parent's linear index,
// blocks[3e + 1], blocks[3e + 2] the low and high words of the mask of its
// ring children (child (ii, jj) at bit ii + r jj; r <= 8).
// fine2 (optional): a second canvas filled at time weight alpha2 from the
// same slopes.
template <typename T>
void launch_ring_fill_blocks(const int *blocks, long long nblocks, T *fine, int nxf, const T *cold, const T *cnew,
                             int NX, int NY, int r, double alpha, const int *bc, hipStream_t s, int k0 = 0,
                             int nk = 3, T *fine2 = nullptr, double alpha2 = 0.0);
template <typename T>
void launch_average(const int *cells, long long ncells, const T *fine, int nxf, long long csf, T *coarse, int NX,
                    long long csc, int r, hipStream_t s, int nk = 3);

// Refluxing of the adjoint acoustics hierarchy (conservative f-wave form): add the
// fluxes of the fine edges of every face (r per face, from the canvas the
// fine step started from) to its register (first: start from zero); then
// correct every coarse cell by s dt/h (F_coarse - register / r^2), the
// coarse flux from the canvas the coarse step started from.  faces: int4
// records, groups: int2 {first face, count} per coarse cell.
template <typename T>
void launch_reflux_fine(const int *faces, int nfaces, const T *fine_old, const uint8_t *mat, int nx, int ny,
                        const int *bc, const double *mtab64, int r, double nux, double nuy, int order, int limiter,
                        int transverse, bool first, double *reg, hipStream_t s);
template <typename T>
void launch_reflux_apply(const int *groups, int ngroups, const int *faces, const double *reg, const T *coarse_old,
                         T *coarse_cur, const uint8_t *mat, int nx, int ny, const int *bc, const double *mtab64,
                         int r, double nux, double nuy, int order, int limiter, int transverse, hipStream_t s);
// The same for the shallow-water hierarchy (csrc/reflux_swe.hip): canvases
// of the given precision (WP_FP64, WP_MIXED: eta FP64 and the momenta FP32,
// WP_FP32), the level's bathymetry B in FP64, every flux seen from the
// coarse cell's side of its edge.
void launch_reflux_swe_fine(int precision, const int *faces, int nfaces, const void *fine_old, const double *B,
                            int nx, int ny, const int *bc, double g, int r, double nux, double nuy, int order,
                            int limiter, int transverse, bool first, double *reg, hipStream_t s);
void launch_reflux_swe_apply(int precision, const int *groups, int ngroups, const int *faces, const double *reg,
                             const void *coarse_old, void *coarse_cur, const double *B, int nx, int ny, const int *bc,
                             double g, int r, double nux, double nuy, int order, int limiter, int transverse,
                             hipStream_t s);

}  // namespace wp
