// Two acoustics time steps per launch on a single-level 2D canvas (Davis &
// LeVeque Sec. 3 wave propagation; Sec. 2/4 for the time-reversed adjoint),
// for gfx950.
//
// One 64-lane wave owns a strip of 64 columns: 56 outputs and a four-column
// halo on each side.  A first march takes the rows j0-4 .. j1+3 of q^n and
// produces q^{n+1} on rows j0-2 .. j1+1 (lanes 2..61 exact); a second march
// follows it four rows behind and turns those rows, straight from
// registers, into q^{n+2} on rows j0 .. j1-1 (lanes 4..59).  q^{n+1} never
// goes to memory unless it is a snapshot step, so a pair of steps reads the
// state once and writes it once.
//
// The second march needs the ghost cells of q^{n+1}.  They follow the
// boundary rule from the first march's interior results: ghost columns by a
// cross-lane permute from the mirrored (wall, u negated) or nearest
// (extrapolation) column, ghost rows by a copy of the mirrored or nearest
// row (wall: v negated), taken as soon as that row exists.  Periodic
// boundaries would need another strip's results and keep the one-step
// kernel.  Every cell of both steps goes through the same row update as the
// one-step kernel.
#include "acou_stencil.h"

namespace wp {
namespace {

using namespace march;

__device__ __forceinline__ double bperm(double v, int addr)
{
    return __hiloint2double(__builtin_amdgcn_ds_bpermute(addr, __double2hiint(v)),
                            __builtin_amdgcn_ds_bpermute(addr, __double2loint(v)));
}
__device__ __forceinline__ float bperm(float v, int addr)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(addr, __float_as_int(v)));
}

// Ghost columns of a first-step row: lane `addr / 4` holds the cell whose
// value the ghost takes; flip: negate u (wall).
struct XFix {
    bool on;     // some lane the second step reads is a ghost column
    int addr;
    bool flip;
};

template <typename T>
__device__ __forceinline__ void fix_columns(Row<T> &r, const XFix &xf)
{
    if (!xf.on) return;
    r.p = bperm(r.p, xf.addr);
    const T u = bperm(r.u, xf.addr);
    r.u = xf.flip ? -u : u;
    r.v = bperm(r.v, xf.addr);
}

template <typename T>
__device__ __forceinline__ Row<T> pick(bool c, const Row<T> &a, const Row<T> &b)
{
    return Row<T>{c ? a.p : b.p, c ? a.u : b.u, c ? a.v : b.v, c ? a.m : b.m};
}

template <typename T>
__device__ __forceinline__ Row<T> reflect_y(const Row<T> &a, bool wall)
{
    return Row<T>{a.p, a.u, wall ? -a.v : a.v, a.m};
}

// The two marches of one tile, unrolled (RT rows at most; j0 is 0 or at
// least 4).
// First-step iteration i updates row j0-3+i from input rows A[i+1..i+3]
// (A[r] is row j0-4+r) into S[i-1] (S[s] is row j0-2+s); second-step
// iteration k = i-4 updates row j0-1+k from S[k+1..k+3].
template <typename T, bool ADJ, bool UNI, int RT, typename LD>
__device__ __forceinline__ void march_pair(const Media<T, UNI> &md, const Tile &tl, int nx, int ny, bool wall_lo,
                                           bool wall_hi, T nux, T nuy, unsigned csb, unsigned out_off0,
                                           bool out_lane, const XFix &xf, __amdgpu_buffer_rsrc_t qw,
                                           __amdgpu_buffer_rsrc_t s1w, __amdgpu_buffer_rsrc_t s2w, bool snap1,
                                           bool snap2, const LD &ld, int &bad)
{
    constexpr int NA = RT + 8;
    constexpr int NS = RT + 4;
    constexpr int FIRST = 3 + PREFETCH < NA ? 3 + PREFETCH : NA;
    const int j0 = tl.j0, j1 = tl.j0 + tl.nj;
    Row<T> A[NA];
    Row<T> S[NS];
#pragma unroll
    for (int r = 0; r < FIRST; ++r) ld(A[r], j0 - 4 + r);
    __builtin_amdgcn_sched_barrier(SCHED_KEEP_LOADS);
    Carry<T> ca, cb;
    march_start<T, ADJ, UNI>(md, A[0], A[1], A[2], ca);
    // stores of halo lanes and of rows outside the tile go to this offset,
    // beyond the buffer's range (3 components), where they are dropped; a
    // snapshot store has an empty range when that step takes no snapshot
    const unsigned nowhere = 3u * csb;
    const unsigned rowb = (unsigned)nx * (unsigned)sizeof(T);
#pragma unroll
    for (int i = 0; i <= RT + 4; ++i) {
        if (FIRST + i < NA) {
            ld(A[FIRST + i], j0 - 4 + FIRST + i);
            __builtin_amdgcn_sched_barrier(SCHED_KEEP_LOADS);
        }
        T pn, un, vn;
        row_step<T, ADJ, UNI>(md, true, true, 1, nux, nuy, A[i + 1], A[i + 2], A[i + 3], ca, pn, un, vn);
        if (i == 0) continue;   // the first row only starts the y-edge fluxes
        const int s = i - 1;
        const int r = j0 - 2 + s;
        if (snap1) {
            // q^{n+1} is a snapshot (a non-finite value in it reaches the
            // second step's checked outputs in any case)
            const bool keep = r >= j0 && r < j1 && out_lane;
            const unsigned off = keep ? (unsigned)r * rowb + out_off0 : nowhere;
            bstore(s1w, off, 0u, pn);
            bstore(s1w, off, csb, un);
            bstore(s1w, off, 2u * csb, vn);
        }
        Row<T> o{pn, un, vn, A[s + 2].m};
        fix_columns(o, xf);
        // ghost rows above the domain (the rows they copy come first); r is
        // wave-uniform, so rows below the top skip this on a scalar branch
        if (s >= 3 && r >= ny) {
            const Row<T> g0 = reflect_y(S[s - 1], wall_hi);              // row ny
            const Row<T> g1 = wall_hi ? reflect_y(S[s - 3], true) : S[s - 2];   // row ny + 1
            o = pick(r == ny, g0, pick(r == ny + 1, g1, o));
        }
        S[s] = o;
        if (s == 3 && j0 == 0) {
            // ghost rows below the domain, once rows 0 and 1 exist
            S[1] = reflect_y(S[2], wall_lo);                             // row -1
            S[0] = wall_lo ? reflect_y(S[3], true) : S[2];               // row -2
        }
        if (i >= 4) {
            const int k = i - 4;
            if (k == 0) march_start<T, ADJ, UNI>(md, S[0], S[1], S[2], cb);
            T qp, qu, qv;
            row_step<T, ADJ, UNI>(md, true, true, 1, nux, nuy, S[k + 1], S[k + 2], S[k + 3], cb, qp, qu, qv);
            if (k == 0) continue;
            const int j = j0 - 1 + k;
            const bool keep = j < j1 && out_lane;
            const unsigned off = keep ? (unsigned)j * rowb + out_off0 : nowhere;
            bstore(qw, off, 0u, qp);
            bstore(qw, off, csb, qu);
            bstore(qw, off, 2u * csb, qv);
            if (snap2) {
                bstore(s2w, off, 0u, qp);
                bstore(s2w, off, csb, qu);
                bstore(s2w, off, 2u * csb, qv);
            }
            bad |= keep & !(isfinite(qp) & isfinite(qu) & isfinite(qv));
        }
    }
}

// The adjoint flag of q^n on the tile's cells (Sec. 4): the measure
// max_n |qhat_n . q| over the window's snapshots, in FP64 with every product
// and sum rounded as written, so that it decides exactly as the flag kernel.
template <typename T>
__device__ void flag_tile(const Tile &tl, int nx, unsigned cells, int col, bool out_lane,
                          __amdgpu_buffer_rsrc_t qr, const PairFlag &fl)
{
#pragma clang fp contract(off)
    const unsigned csb = cells * (unsigned)sizeof(T);
    const __amdgpu_buffer_rsrc_t fw = make_rsrc(fl.flags, cells);
    unsigned local = 0;
    // four rows at a time, so that their loads are in flight together (rows
    // past the tile read and write out of range: loads return 0, stores drop)
    constexpr int G = 4;
    for (int j = tl.j0; j < tl.j0 + tl.nj; j += G) {
        unsigned idx[G], off[G];
        double q0[G], q1[G], q2[G], best[G];
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const bool in = j + g < tl.j0 + tl.nj;
            idx[g] = in ? (unsigned)((j + g) * nx + col) : cells;
            off[g] = idx[g] * (unsigned)sizeof(T);
            q0[g] = (double)bload(qr, off[g], T(0), 0u);
            q1[g] = (double)bload(qr, off[g], T(0), csb);
            q2[g] = (double)bload(qr, off[g], T(0), 2u * csb);
            best[g] = 0.0;
        }
        for (int n = fl.n_lo; n <= fl.n_hi; ++n) {
            const __amdgpu_buffer_rsrc_t sr =
                make_rsrc((const T *)fl.snaps + (long long)n * fl.sstride, 3u * csb);
#pragma unroll
            for (int g = 0; g < G; ++g) {
                double ip = (double)bload(sr, off[g], T(0), 0u) * q0[g];
                ip = ip + (double)bload(sr, off[g], T(0), csb) * q1[g];
                ip = ip + (double)bload(sr, off[g], T(0), 2u * csb) * q2[g];
                best[g] = fmax(best[g], fabs(ip));
            }
        }
#pragma unroll
        for (int g = 0; g < G; ++g) {
            const bool keep = out_lane && idx[g] < cells;
            const unsigned f = best[g] > fl.tol ? 1u : 0u;
            __builtin_amdgcn_raw_buffer_store_b8((unsigned char)f, fw, keep ? idx[g] : cells, 0, 0);
            local += keep ? f : 0u;
        }
    }
    for (int off = 32; off > 0; off >>= 1) local += __shfl_down(local, off);
    if (threadIdx.x == 0 && local) atomicAdd(count_slot(fl.count), (unsigned long long)local);
}

// The same two marches as a rolled loop over the tile's own height (any nj):
// input rows in a rolling window prefetched three rows ahead, the last four
// first-step rows in registers.  Registers are what the window and the two
// carries need, not what an unrolled schedule hoists.
template <typename T, bool ADJ, bool UNI, typename LD>
__device__ __forceinline__ void march_pair_rolled(const Media<T, UNI> &md, const Tile &tl, int nx, int ny,
                                                  bool wall_lo, bool wall_hi, T nux, T nuy, unsigned csb,
                                                  unsigned out_off0, bool out_lane, const XFix &xf,
                                                  __amdgpu_buffer_rsrc_t qw, __amdgpu_buffer_rsrc_t s1w,
                                                  __amdgpu_buffer_rsrc_t s2w, const LD &ld, int &bad)
{
    const int j0 = tl.j0, j1 = tl.j0 + tl.nj;
    Row<T> RA, R0, R1, R2, P0, P1, P2;
    ld(RA, j0 - 4);
    ld(R0, j0 - 3);
    ld(R1, j0 - 2);
    ld(R2, j0 - 1);
    ld(P0, j0);
    ld(P1, j0 + 1);
    Carry<T> ca, cb;
    march_start<T, ADJ, UNI>(md, RA, R0, R1, ca);
    const unsigned nowhere = 3u * csb;
    const unsigned rowb = (unsigned)nx * (unsigned)sizeof(T);
    Row<T> Sm3, Sm2, Sm1;   // first-step rows s-3, s-2, s-1
    for (int i = 0; i <= tl.nj + 4; ++i) {
        ld(P2, j0 + 2 + i);   // input row i + 6, three iterations before its use
        T pn, un, vn;
        row_step<T, ADJ, UNI>(md, true, true, 1, nux, nuy, R0, R1, R2, ca, pn, un, vn);
        const int m0 = R0.m;   // material of the updated row
        R0 = R1;
        R1 = R2;
        R2 = P0;
        P0 = P1;
        P1 = P2;
        if (i == 0) continue;
        const int s = i - 1;
        const int r = j0 - 2 + s;
        {
            const bool keep = r >= j0 && r < j1 && out_lane;
            const unsigned off = keep ? (unsigned)r * rowb + out_off0 : nowhere;
            bstore(s1w, off, 0u, pn);
            bstore(s1w, off, csb, un);
            bstore(s1w, off, 2u * csb, vn);
            bad |= keep & !(isfinite(pn) & isfinite(un) & isfinite(vn));
        }
        Row<T> o{pn, un, vn, m0};
        fix_columns(o, xf);
        if (s >= 3) {
            const Row<T> g0 = reflect_y(Sm1, wall_hi);                    // row ny
            const Row<T> g1 = wall_hi ? reflect_y(Sm3, true) : Sm2;       // row ny + 1
            o = pick(r == ny, g0, pick(r == ny + 1, g1, o));
        }
        if (s == 3 && j0 == 0) {
            // ghost rows below the domain, once rows 0 (Sm1) and 1 (o) exist
            const Row<T> g1 = reflect_y(Sm1, wall_lo);                    // row -1
            const Row<T> g2 = wall_lo ? reflect_y(o, true) : Sm1;         // row -2
            Sm2 = g1;
            Sm3 = g2;
        }
        if (s >= 3) {
            const int k = s - 3;
            if (k == 0) march_start<T, ADJ, UNI>(md, Sm3, Sm2, Sm1, cb);
            T qp, qu, qv;
            row_step<T, ADJ, UNI>(md, true, true, 1, nux, nuy, Sm2, Sm1, o, cb, qp, qu, qv);
            if (k > 0) {
                const int j = j0 - 1 + k;
                const bool keep = j < j1 && out_lane;
                const unsigned off = keep ? (unsigned)j * rowb + out_off0 : nowhere;
                bstore(qw, off, 0u, qp);
                bstore(qw, off, csb, qu);
                bstore(qw, off, 2u * csb, qv);
                bstore(s2w, off, 0u, qp);
                bstore(s2w, off, csb, qu);
                bstore(s2w, off, 2u * csb, qv);
                bad |= keep & !(isfinite(qp) & isfinite(qu) & isfinite(qv));
            }
        }
        Sm3 = Sm2;
        Sm2 = Sm1;
        Sm1 = o;
    }
}

// KIND 0: each tile takes the single-material or the mixed path as flagged;
// KIND 1: every tile is single-material.  RT 0: the rolled march (tiles of
// any height).  stamp: as for the one-step kernel.
// At most 256 registers, so that two waves share a SIMD (the unconstrained
// FP64 march takes a few more and would run one).
// FLAG: take the adjoint flag of q^n on the tile's cells first.
template <typename T, bool ADJ, int RT, int KIND, bool FLAG>
__global__ __launch_bounds__(WAVE) __attribute__((amdgpu_waves_per_eu(2))) void acou2d_pair_kernel(
    const AcouInst<T> *__restrict__ insts, const Tile *__restrict__ tiles, int parity, int snap1, int snap2,
    int *__restrict__ status, unsigned long long *__restrict__ stamp, PairFlag fl)
{
    if (stamp && threadIdx.x == 0) stamp[2 * blockIdx.x] = (unsigned long long)wall_clock64();
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile tl = tiles[blockIdx.x];
    const AcouInst<T> *__restrict__ Ip = insts + tl.inst;
    const int lane = threadIdx.x;
    MCon<T> *mc = reinterpret_cast<MCon<T> *>(smem);
    T *pt = reinterpret_cast<T *>(smem + sizeof(MCon<T>) * MAXMAT);
    build_tables(*Ip, mc, pt, lane);
    __syncthreads();

    const int nx = Ip->nx, ny = Ip->ny;
    const int bc0 = Ip->bc[0], bc1 = Ip->bc[1], bc2 = Ip->bc[2], bc3 = Ip->bc[3];
    const unsigned cells = (unsigned)nx * (unsigned)ny;
    const unsigned csb = cells * (unsigned)sizeof(T);
    const __amdgpu_buffer_rsrc_t qr = make_rsrc(Ip->q[parity], 3u * csb);
    const __amdgpu_buffer_rsrc_t qw = make_rsrc(Ip->q[parity ^ 1], 3u * csb);
    const __amdgpu_buffer_rsrc_t mr = make_rsrc(Ip->mat, cells);
    const __amdgpu_buffer_rsrc_t s1w = make_rsrc(snap1 >= 0 ? Ip->snap + (long long)snap1 * Ip->snap_stride : Ip->q[0],
                                                 snap1 >= 0 ? 3u * csb : 0u);
    const __amdgpu_buffer_rsrc_t s2w = make_rsrc(snap2 >= 0 ? Ip->snap + (long long)snap2 * Ip->snap_stride : Ip->q[0],
                                                 snap2 >= 0 ? 3u * csb : 0u);
    const T nux = Ip->nux, nuy = Ip->nuy;
    const int col = tl.i0 - 4 + lane;
    bool fx;
    const int cx = resolve(col, nx, bc0, bc1, fx);
    const T sx = fx ? T(-1) : T(1);
    // ghost columns among the lanes 2..61 that the second step reads
    XFix xf;
    xf.on = tl.i0 < 2 || tl.i0 + 57 >= nx;
    {
        const bool ghost = col < 0 || col >= nx;
        const int src = min(max(ghost ? cx - (tl.i0 - 4) : lane, 0), WAVE - 1);
        xf.addr = 4 * src;
        xf.flip = ghost && fx;
    }
    const bool out_lane = lane >= 4 && lane < 4 + tl.ni;
    const unsigned out_off0 = (unsigned)col * (unsigned)sizeof(T);
    const Resolver rowres(ny, bc2, bc3);
    auto ld = [=](Row<T> &r, int j) {
        bool fy;
        const int jy = rowres(j, fy);
        const unsigned idx = (unsigned)(jy * nx + cx);
        const unsigned off = idx * (unsigned)sizeof(T);
        r.p = bload(qr, off, T(0), 0u);
        r.u = sx * bload(qr, off, T(0), csb);
        const T v = bload(qr, off, T(0), 2u * csb);
        r.v = fy ? -v : v;
        r.m = KIND == 1 ? 0 : (int)__builtin_amdgcn_raw_buffer_load_b8(mr, idx, 0, 0);
    };
    const bool wall_lo = bc2 == WP_BC_WALL, wall_hi = bc3 == WP_BC_WALL;
    if constexpr (FLAG) flag_tile<T>(tl, nx, cells, col, out_lane, qr, fl);
    int bad = 0;
    if (KIND == 1 || tl.mat >= 0) {
        Media<T, true> md;
        md.u = make_unicon<T, ADJ>(mc[tl.mat], pt[(tl.mat * Ip->nmat + tl.mat) * 3], nux, nuy);
        if constexpr (RT == 0)
            march_pair_rolled<T, ADJ, true>(md, tl, nx, ny, wall_lo, wall_hi, nux, nuy, csb, out_off0, out_lane, xf,
                                            qw, s1w, s2w, ld, bad);
        else
            march_pair<T, ADJ, true, RT>(md, tl, nx, ny, wall_lo, wall_hi, nux, nuy, csb, out_off0, out_lane, xf, qw,
                                         s1w, s2w, snap1 >= 0, snap2 >= 0, ld, bad);
    } else if (KIND != 1) {
        // mixed tiles are acou_mixed_rows(RT) high
        Media<T, false> md{mc, pt, Ip->nmat};
        if constexpr (RT == 0)
            march_pair_rolled<T, ADJ, false>(md, tl, nx, ny, wall_lo, wall_hi, nux, nuy, csb, out_off0, out_lane, xf,
                                             qw, s1w, s2w, ld, bad);
        else
            march_pair<T, ADJ, false, acou_mixed_rows(RT)>(md, tl, nx, ny, wall_lo, wall_hi, nux, nuy, csb, out_off0,
                                                           out_lane, xf, qw, s1w, s2w, snap1 >= 0, snap2 >= 0, ld,
                                                           bad);
    }
    if (__any(bad) && lane == 0) atomicOr(status, ST_NONFINITE);
    if (stamp && lane == 0) stamp[2 * blockIdx.x + 1] = (unsigned long long)wall_clock64();
}

}  // namespace

template <typename T>
void launch_acou2d_pair(const AcouInst<T> *insts, const Tile *tiles, int ntiles, int parity, int adjoint,
                        int nmat_max, int rows, int kind, int snap1, int snap2, int *status, hipStream_t s,
                        unsigned long long *stamp, const PairFlag *flag)
{
    if (ntiles <= 0) return;
    const size_t sm = sizeof(MCon<T>) * MAXMAT + sizeof(T) * 3 * (size_t)nmat_max * nmat_max;
    const dim3 g(ntiles), b(WAVE);
    const PairFlag fl = flag ? *flag : PairFlag{nullptr, 0, 0, -1, 0.0, nullptr, nullptr};
#define WP_LAUNCH(ADJ, RT, KIND, FLAG)                                                                   \
    hipLaunchKernelGGL((acou2d_pair_kernel<T, ADJ, RT, KIND, FLAG>), g, b, sm, s, insts, tiles, parity, \
                       snap1, snap2, status, stamp, fl)
    // heights 8, 10, 12 and 16 have an unrolled march; any other the rolled one
#define WP_BY_RT(ADJ, KIND, FLAG)                   \
    switch (rows) {                                 \
    case 8: WP_LAUNCH(ADJ, 8, KIND, FLAG); break;   \
    case 10: WP_LAUNCH(ADJ, 10, KIND, FLAG); break; \
    case 12: WP_LAUNCH(ADJ, 12, KIND, FLAG); break; \
    case 16: WP_LAUNCH(ADJ, 16, KIND, FLAG); break; \
    default: WP_LAUNCH(ADJ, 0, KIND, FLAG); break;  \
    }
    if (flag && !adjoint) {
        if (kind == 1) { WP_BY_RT(false, 1, true) } else { WP_BY_RT(false, 0, true) }
    } else if (kind == 1) {
        if (adjoint) { WP_BY_RT(true, 1, false) } else { WP_BY_RT(false, 1, false) }
    } else {
        if (adjoint) { WP_BY_RT(true, 0, false) } else { WP_BY_RT(false, 0, false) }
    }
#undef WP_BY_RT
#undef WP_LAUNCH
}

template void launch_acou2d_pair<double>(const AcouInst<double> *, const Tile *, int, int, int, int, int, int, int,
                                         int, int *, hipStream_t, unsigned long long *, const PairFlag *);
template void launch_acou2d_pair<float>(const AcouInst<float> *, const Tile *, int, int, int, int, int, int, int,
                                        int, int *, hipStream_t, unsigned long long *, const PairFlag *);

}  // namespace wp
