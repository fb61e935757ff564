// Acoustics patch-update kernels for gfx950 (forward wave form and
// time-reversed adjoint f-wave form), Davis & LeVeque Sec. 3 (wave
// propagation), Sec. 5.1/5.2 (acoustics coefficient matrices), Sec. 2/4
// (adjoint equation and time reversal).
//
// 2D kernel layout: one 64-lane wavefront owns a strip of 64 consecutive
// columns (60 outputs plus a two-column halo on each side) and marches up
// the rows of its tile, one row per iteration, keeping every edge quantity in
// registers: each x-edge and y-edge Riemann problem is solved exactly once
// per strip, neighbouring columns are exchanged with DPP wave shifts, and
// the only memory traffic is the state row read, the material byte and the
// state row written.  Ghost cells are resolved in the loader (boundary
// rules, or the canvas itself inside the domain), so no ghost-fill pass is
// needed.
#include "acou_stencil.h"

namespace wp {
namespace {

using namespace march;

// Compile-time march of one wave over a tile of RT rows: iteration `it`
// updates row j0 - 1 + it.  The tile reads RT + 4 rows (two-row halo above
// and below); row r (counted from j0 - 2) is first needed at iteration
// max(0, r - 3) and requested PREFETCH iterations before that, so a few rows
// are always in flight while arithmetic proceeds.  The unrolled march is one
// branch-free block.
//
// A tile flagged `down` is marched from its top row downwards: that is the
// upward march of the problem reflected in y (rows taken in reverse order, v
// negated on load and on store), which the method treats identically.
// AVG: each result row also goes to LDS (avb: [4 rows][3 components][64
// lanes]); when a block of four rows is complete, the first lane of every
// four output lanes sums its 4 x 4 block row by row and writes the mean onto
// the cell of the level below (tiles start on rows and columns of multiples
// of 4, so a block lies in one tile).
template <typename T, bool ADJ, bool UNI, int RT, bool AVG, typename LD>
__device__ __forceinline__ void march_tile(const Media<T, UNI> &md, const Tile &tl, int nx, T nux, T nuy,
                                           unsigned csb, unsigned out_off0, bool out_lane,
                                           __amdgpu_buffer_rsrc_t qw, __amdgpu_buffer_rsrc_t sw, bool snap,
                                           const LD &ld, int &bad, const AvgTo<T> &avg, T *avb, int col)
{
    constexpr int NR = RT + 4;
    constexpr int FIRST = 3 + PREFETCH < NR ? 3 + PREFETCH : NR;   // rows requested before the march
    const int j0 = tl.j0, j1 = tl.j0 + tl.nj;
    const bool down = tl.down != 0;
    const int jb = down ? j0 + RT + 1 : j0 - 2;   // row of rw[0]
    const int js = down ? -1 : 1;                 // row step of the march
    Row<T> rw[NR];
#pragma unroll
    for (int r = 0; r < FIRST; ++r) ld(rw[r], jb + js * r, down);
    __builtin_amdgcn_sched_barrier(SCHED_KEEP_LOADS);
    Carry<T> c;
    march_start<T, ADJ, UNI>(md, rw[0], rw[1], rw[2], c);
    // stores of halo lanes and of rows past a short tile go to this offset,
    // beyond the buffer's range (3 components), where they are dropped; the
    // snapshot store has an empty range when no snapshot is taken
    const unsigned nowhere = 3u * csb;
#pragma unroll
    for (int it = 0; it <= RT; ++it) {
        if (FIRST + it < NR) {
            ld(rw[FIRST + it], jb + js * (FIRST + it), down);
            __builtin_amdgcn_sched_barrier(SCHED_KEEP_LOADS);
        }
        T pn, un, vn;
        row_step<T, ADJ, UNI>(md, true, true, 1, nux, nuy, rw[it + 1], rw[it + 2], rw[it + 3], c, pn, un, vn);
        if (it == 0) continue;   // the first row only starts the y-edge fluxes
        const int j = jb + js * (it + 1);
        if (down) vn = -vn;
        const bool keep = j < j1 && out_lane;
        const unsigned off = keep ? (unsigned)j * (unsigned)nx * (unsigned)sizeof(T) + out_off0 : nowhere;
        bstore(qw, off, 0u, pn);
        bstore(qw, off, csb, un);
        bstore(qw, off, 2u * csb, vn);
        if (snap) {   // wave-uniform
            bstore(sw, off, 0u, pn);
            bstore(sw, off, csb, un);
            bstore(sw, off, 2u * csb, vn);
        }
        bad |= keep & !(isfinite(pn) & isfinite(un) & isfinite(vn));
        if constexpr (AVG) {
            // row t of the tile; a block is complete at its last row in
            // marching order (the same for both tiles of a wave: same
            // direction, rows starting on multiples of 4)
            const int t = j - j0;
            const int lane = threadIdx.x;
            avb[((t & 3) * 3 + 0) * WAVE + lane] = pn;
            avb[((t & 3) * 3 + 1) * WAVE + lane] = un;
            avb[((t & 3) * 3 + 2) * WAVE + lane] = vn;
            if ((t & 3) == (down ? 0 : 3)) {
                __syncthreads();
                const int b0 = t & ~3;   // first row of the block
                const bool lead = out_lane && ((col - tl.i0) & 3) == 0 && b0 < tl.nj;
                if (lead) {
                    const T inv = T(1) / T(16);
                    const long long c = (long long)((j0 + b0) >> 2) * avg.nx + (col >> 2);
                    for (int k = 0; k < 3; ++k) {
                        T sum = T(0);
                        for (int jj = 0; jj < 4; ++jj)
                            for (int ii = 0; ii < 4; ++ii) sum += avb[(jj * 3 + k) * WAVE + lane + ii];
                        avg.q[k * avg.cs + c] = sum * inv;
                    }
                }
                __syncthreads();
            }
        }
    }
}

// One wave marches its tile up the rows.  RT > 0: the compile-time march
// above (full method: second order, MC limiter, transverse terms).  RT = 0
// (runtime height, any options): a rolling window of rows prefetched two
// rows ahead.
template <typename T, bool ADJ, bool UNI, bool FULL, int RT, bool AVG = false>
__device__ __forceinline__ void march(const Media<T, UNI> &md, const Opts &op_rt, const Tile &tl, int lane, int nx,
                                      int ny, int bc2, int bc3, int cx, T sx, unsigned csb, T nux, T nuy,
                                      __amdgpu_buffer_rsrc_t qr, __amdgpu_buffer_rsrc_t qw,
                                      __amdgpu_buffer_rsrc_t mr, __amdgpu_buffer_rsrc_t sw, bool snap, int &bad,
                                      const AvgTo<T> &avg = AvgTo<T>{nullptr, 0, 0}, T *avb = nullptr)
{
    const bool out_lane = lane >= 2 && lane < 2 + tl.ni;
    const unsigned out_off0 = (unsigned)(tl.i0 - 2 + lane) * (unsigned)sizeof(T);
    const Resolver rowres(ny, bc2, bc3);
    // row j into r; `flip` also negates v (the reflected frame of a
    // downward march)
    auto ld = [=](Row<T> &r, int j, bool flip) {
        bool fy;
        const int jy = rowres(j, fy);
        const unsigned idx = (unsigned)(jy * nx + cx);
        const unsigned off = idx * (unsigned)sizeof(T);
        r.p = bload(qr, off, T(0), 0u);
        r.u = sx * bload(qr, off, T(0), csb);
        const T v = bload(qr, off, T(0), 2u * csb);
        r.v = fy != flip ? -v : v;
        r.m = UNI ? 0 : (int)__builtin_amdgcn_raw_buffer_load_b8(mr, idx, 0, 0);
    };
    if constexpr (RT > 0) {
        march_tile<T, ADJ, UNI, RT, AVG>(md, tl, nx, nux, nuy, csb, out_off0, out_lane, qw, sw, snap, ld, bad, avg,
                                         avb, tl.i0 - 2 + lane);
    } else {
        // FULL: second order, MC limiter and transverse terms fixed at compile time
        const bool second = FULL ? true : op_rt.second;
        const bool trans = FULL ? true : op_rt.trans;
        const int lim = FULL ? 1 : op_rt.lim;
        const int j0 = tl.j0, j1 = tl.j0 + tl.nj;
        Carry<T> c;
        Row<T> RA, R0, R1, X0, X1, X2;
        ld(RA, j0 - 2, false);
        ld(R0, j0 - 1, false);
        ld(R1, j0, false);
        ld(X0, j0 + 1, false);
        ld(X1, j0 + 2, false);
        march_start<T, ADJ, UNI>(md, RA, R0, R1, c);
        for (int j = j0 - 1; j < j1; ++j) {
            ld(X2, j + 4, false);   // prefetch; row j+2 (X0) was issued two iterations ago
            T pn, un, vn;
            row_step<T, ADJ, UNI>(md, second, trans, lim, nux, nuy, R0, R1, X0, c, pn, un, vn);
            if (j >= j0 && out_lane) {
                const unsigned off = (unsigned)j * (unsigned)nx * (unsigned)sizeof(T) + out_off0;
                bstore(qw, off, 0u, pn);
                bstore(qw, off, csb, un);
                bstore(qw, off, 2u * csb, vn);
                if (snap) {
                    bstore(sw, off, 0u, pn);
                    bstore(sw, off, csb, un);
                    bstore(sw, off, 2u * csb, vn);
                }
                bad |= !(isfinite(pn) && isfinite(un) && isfinite(vn));
            }
            R0 = R1;
            R1 = X0;
            X0 = X1;
            X1 = X2;
        }
    }
}

// KIND 0: each tile takes the single-material or the mixed path as flagged;
// KIND 1: every tile is single-material (the lean march alone sets the
// register count and so the occupancy).
// stamp (optional): workgroup b writes its start and end on the device's
// constant-rate clock to stamp[2b] and stamp[2b + 1] (one slot each, no
// contention), from which the launch's own duration is read back.
// DUAL (unrolled heights only): a tile may carry a second tile for the lanes
// after its own (its columns and two halo lanes either side).  A cell's
// update reads two lanes either side, so the two tiles, each with its own
// halo lanes, never see each other's outputs; rows, columns and the output
// range become per-lane.
// AVG (with DUAL, heights 4, 8, 16): also the means of the results' 4 x 4
// blocks onto the level below (see march_tile), through LDS after the
// material tables.
template <typename T, bool ADJ, bool FULL, int RT, int KIND, bool DUAL, bool AVG = false>
__global__ __launch_bounds__(WAVE) void acou2d_kernel(const AcouInst<T> *__restrict__ insts,
                                                      const Tile *__restrict__ tiles, int parity,
                                                      int snap_index, int *__restrict__ status,
                                                      unsigned long long *__restrict__ stamp, AvgTo<T> avg)
{
    static_assert(!DUAL || RT > 0, "two tiles per wave need the unrolled march");
    static_assert(!AVG || (RT > 0 && RT % 4 == 0 && acou_mixed_rows(RT) % 4 == 0), "averaging needs rows of 4");
    if (stamp && threadIdx.x == 0) stamp[2 * blockIdx.x] = (unsigned long long)wall_clock64();
    extern __shared__ __align__(16) unsigned char smem[];
    Tile tl = tiles[blockIdx.x];
    const AcouInst<T> *__restrict__ Ip = insts + tl.inst;
    int lane = threadIdx.x;
    if constexpr (DUAL) {
        const int split = tl.ni + 4;   // the first lane of the second tile
        if (tl.nib > 0 && lane >= split) {
            tl.i0 = tl.i0b;
            tl.j0 = tl.j0b;
            tl.ni = tl.nib;
            tl.nj = tl.njb;
            lane -= split;
        }
    }
    MCon<T> *mc = reinterpret_cast<MCon<T> *>(smem);
    T *pt = reinterpret_cast<T *>(smem + sizeof(MCon<T>) * MAXMAT);
    // the averaging rows after the tables (acou_smem's size, 16-aligned)
    T *avb = reinterpret_cast<T *>(
        smem + ((sizeof(MCon<T>) * MAXMAT + sizeof(T) * 3 * (size_t)Ip->nmat * Ip->nmat + 15) & ~(size_t)15));
    build_tables(*Ip, mc, pt, threadIdx.x);
    __syncthreads();

    const int nx = Ip->nx, ny = Ip->ny;
    const int bc0 = Ip->bc[0], bc1 = Ip->bc[1], bc2 = Ip->bc[2], bc3 = Ip->bc[3];
    const unsigned cells = (unsigned)nx * (unsigned)ny;
    const unsigned csb = cells * (unsigned)sizeof(T);
    const __amdgpu_buffer_rsrc_t qr = make_rsrc(Ip->q[parity], 3u * csb);
    const __amdgpu_buffer_rsrc_t qw = make_rsrc(Ip->q[parity ^ 1], 3u * csb);
    const __amdgpu_buffer_rsrc_t mr = make_rsrc(Ip->mat, cells);
    const bool snap = snap_index >= 0;
    const __amdgpu_buffer_rsrc_t sw = make_rsrc(snap ? Ip->snap + (long long)snap_index * Ip->snap_stride : Ip->q[0],
                                                snap ? 3u * csb : 0u);
    const Opts op{Ip->order >= 2, Ip->transverse != 0, Ip->limiter};
    const T nux = Ip->nux, nuy = Ip->nuy;
    const int col = tl.i0 - 2 + lane;
    bool fx;
    const int cx = resolve(col, nx, bc0, bc1, fx);
    const T sx = fx ? T(-1) : T(1);
    int bad = 0;
    if (KIND == 1 || (KIND == 0 && tl.mat >= 0)) {
        // one material: folded constants, wave-uniform, kept in SGPRs
        Media<T, true> md;
        md.u = make_unicon<T, ADJ>(mc[tl.mat], pt[(tl.mat * Ip->nmat + tl.mat) * 3], nux, nuy);
        march<T, ADJ, true, FULL, RT, AVG>(md, op, tl, lane, nx, ny, bc2, bc3, cx, sx, csb, nux, nuy, qr, qw, mr, sw,
                                           snap, bad, avg, avb);
    } else if (KIND != 1) {
        // mixed tiles are acou_mixed_rows(RT) high
        Media<T, false> md{mc, pt, Ip->nmat};
        march<T, ADJ, false, FULL, acou_mixed_rows(RT), AVG>(md, op, tl, lane, nx, ny, bc2, bc3, cx, sx, csb, nux, nuy,
                                                             qr, qw, mr, sw, snap, bad, avg, avb);
    }
    if (__any(bad) && threadIdx.x == 0) atomicOr(status, ST_NONFINITE);
    if (stamp && threadIdx.x == 0) stamp[2 * blockIdx.x + 1] = (unsigned long long)wall_clock64();
}

// 1D: one thread per cell, the five-cell stencil read straight from memory.
template <typename T, bool ADJ>
__global__ __launch_bounds__(256) void acou1d_kernel(const AcouInst<T> *__restrict__ insts, int parity,
                                                     int snap_index, int *__restrict__ status)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const AcouInst<T> &I = *insts;
    MCon<T> *mc = reinterpret_cast<MCon<T> *>(smem);
    T *pt = reinterpret_cast<T *>(smem + sizeof(MCon<T>) * MAXMAT);
    if (threadIdx.x < WAVE) build_tables(I, mc, pt, threadIdx.x);
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= I.nx) return;
    const T *qp = I.q[parity];
    T *qo = I.q[parity ^ 1];
    T p[5], u[5];
    int m[5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
        bool f;
        const int ii = resolve(i - 2 + k, I.nx, I.bc[0], I.bc[1], f);
        p[k] = qp[ii];
        u[k] = (f ? T(-1) : T(1)) * qp[ii + I.cs];
        m[k] = I.mat[ii];
    }
    // edges e = 0..3 between cells (e, e+1) of the stencil: i-3/2 .. i+3/2
    T a1[4], a2[4];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        const T *pp = pt + (m[e] * I.nmat + m[e + 1]) * 3;
        solve<T, ADJ>(p[e], u[e], p[e + 1], u[e + 1], mc[m[e]], mc[m[e + 1]], pp[0], a1[e], a2[e]);
    }
    T Fp[2] = {T(0), T(0)}, Fu[2] = {T(0), T(0)};
    if (I.order >= 2) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {   // h = 0: edge i-1/2 (e = 1), h = 1: edge i+1/2 (e = 2)
            const int e = 1 + h;
            const MCon<T> &L = mc[m[e]], &R = mc[m[e + 1]];
            const T *pp = pt + (m[e] * I.nmat + m[e + 1]) * 3;
            const T t1 = limited(a1[e], pp[1] * a1[e + 1], I.limiter);
            const T t2 = limited(a2[e], pp[2] * a2[e - 1], I.limiter);
            if (!ADJ) {
                Fp[h] = R.hZx * t2 - L.hZx * t1;
                Fu[h] = L.hx * t1 + R.hx * t2;
            } else {
                Fp[h] = R.gx * t2 - L.gx * t1;
                Fu[h] = -(L.gZx * t1 + R.gZx * t2);
            }
        }
    }
    const MCon<T> &C = mc[m[2]];
    const T nu = I.nux;
    T pn, un;
    if (!ADJ) {
        pn = p[2] - nu * (C.K * (a2[1] + a1[2])) - nu * (Fp[1] - Fp[0]);
        un = u[2] - nu * (C.c * (a2[1] - a1[2])) - nu * (Fu[1] - Fu[0]);
    } else {
        pn = p[2] - nu * (a2[1] + a1[2]) - nu * (Fp[1] - Fp[0]);
        un = u[2] - nu * (C.Z * (a1[2] - a2[1])) - nu * (Fu[1] - Fu[0]);
    }
    qo[i] = pn;
    qo[i + I.cs] = un;
    if (snap_index >= 0) {
        T *sn = I.snap + (long long)snap_index * I.snap_stride;
        sn[i] = pn;
        sn[i + I.cs] = un;
    }
    if (!(isfinite(pn) && isfinite(un))) atomicOr(status, ST_NONFINITE);
}

}  // namespace

template <typename T>
static size_t acou_smem(int nmat)
{
    return sizeof(MCon<T>) * MAXMAT + sizeof(T) * 3 * (size_t)nmat * nmat;
}

template <typename T>
void launch_acou2d(const AcouInst<T> *insts, const Tile *tiles, int ntiles, int parity, int adjoint, int nmat_max,
                   bool full, int rows, int kind, int snap_index, int *status, hipStream_t s, unsigned long long *stamp,
                   bool dual, const AvgTo<T> *avg)
{
    if (ntiles <= 0) return;
    const size_t sm = acou_smem<T>(nmat_max);
    const dim3 g(ntiles), b(WAVE);
    const AvgTo<T> none{nullptr, 0, 0};
    if (avg && acou2d_can_average(dual, full, rows, 4) && !adjoint) {
        // the averaging rows after the tables, 16-aligned
        const size_t sma = ((sm + 15) & ~(size_t)15) + sizeof(T) * 12 * WAVE;
#define WP_AVG(RT, KIND)                                                                                       \
    hipLaunchKernelGGL((acou2d_kernel<T, false, true, RT, KIND, true, true>), g, b, sma, s, insts, tiles, parity, \
                       snap_index, status, stamp, *avg)
#define WP_AVG_RT(KIND)                 \
    switch (rows) {                     \
    case 4: WP_AVG(4, KIND); break;     \
    case 8: WP_AVG(8, KIND); break;     \
    default: WP_AVG(16, KIND); break;   \
    }
        if (kind == 1) { WP_AVG_RT(1) } else { WP_AVG_RT(0) }
#undef WP_AVG_RT
#undef WP_AVG
        return;
    }
    if (dual) {
        // forward steps of refined levels with narrow patches, unrolled heights
#define WP_DUAL(RT, KIND)                                                                                     \
    hipLaunchKernelGGL((acou2d_kernel<T, false, true, RT, KIND, true>), g, b, sm, s, insts, tiles, parity, \
                       snap_index, status, stamp, none)
#define WP_DUAL_RT(KIND)                      \
    switch (rows) {                           \
    case 4: WP_DUAL(4, KIND); break;          \
    case 6: WP_DUAL(6, KIND); break;          \
    case 8: WP_DUAL(8, KIND); break;          \
    case 12: WP_DUAL(12, KIND); break;        \
    default: WP_DUAL(16, KIND); break;        \
    }
        if (kind == 1) { WP_DUAL_RT(1) } else { WP_DUAL_RT(0) }
#undef WP_DUAL_RT
#undef WP_DUAL
        return;
    }
#define WP_LAUNCH(ADJ, FULL, RT, KIND)                                                                       \
    hipLaunchKernelGGL((acou2d_kernel<T, ADJ, FULL, RT, KIND, false>), g, b, sm, s, insts, tiles, parity, snap_index, \
                       status, stamp, none)
    // tile heights 4, 6, 8, 12 and 16 have a compile-time march; any other
    // height takes the runtime march
#define WP_BY_RT(ADJ, KIND)                              \
    switch (full ? rows : 0) {                           \
    case 4: WP_LAUNCH(ADJ, true, 4, KIND); break;        \
    case 6: WP_LAUNCH(ADJ, true, 6, KIND); break;        \
    case 8: WP_LAUNCH(ADJ, true, 8, KIND); break;        \
    case 12: WP_LAUNCH(ADJ, true, 12, KIND); break;      \
    case 16: WP_LAUNCH(ADJ, true, 16, KIND); break;      \
    default:                                             \
        if (full) WP_LAUNCH(ADJ, true, 0, 0);            \
        else WP_LAUNCH(ADJ, false, 0, 0);                \
    }
    if (kind == 1) {
        if (adjoint) { WP_BY_RT(true, 1) } else { WP_BY_RT(false, 1) }
    } else {
        if (adjoint) { WP_BY_RT(true, 0) } else { WP_BY_RT(false, 0) }
    }
#undef WP_BY_RT
#undef WP_LAUNCH
}

template <typename T>
void launch_acou1d(const AcouInst<T> *inst_dev, const AcouInst<T> &h, int parity, int adjoint, int snap_index,
                   int *status, hipStream_t s)
{
    const size_t sm = acou_smem<T>(h.nmat);
    const int nb = (h.nx + 255) / 256;
    if (adjoint)
        hipLaunchKernelGGL((acou1d_kernel<T, true>), dim3(nb), dim3(256), sm, s, inst_dev, parity, snap_index, status);
    else
        hipLaunchKernelGGL((acou1d_kernel<T, false>), dim3(nb), dim3(256), sm, s, inst_dev, parity, snap_index, status);
}

template void launch_acou2d<double>(const AcouInst<double> *, const Tile *, int, int, int, int, bool, int, int,
                                    int, int *, hipStream_t, unsigned long long *, bool, const AvgTo<double> *);
template void launch_acou2d<float>(const AcouInst<float> *, const Tile *, int, int, int, int, bool, int, int,
                                   int, int *, hipStream_t, unsigned long long *, bool, const AvgTo<float> *);
template void launch_acou1d<double>(const AcouInst<double> *, const AcouInst<double> &, int, int, int, int *,
                                    hipStream_t);
template void launch_acou1d<float>(const AcouInst<float> *, const AcouInst<float> &, int, int, int, int *,
                                   hipStream_t);

}  // namespace wp
