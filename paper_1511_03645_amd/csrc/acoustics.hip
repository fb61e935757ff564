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
//
// Media are piecewise constant: every cell carries a material index, and
// per-material and per-material-pair constants sit in LDS.  This removes
// every division from the stencil: 1/(Z_a + Z_b) and the limiter's
// eigenvector projection kappa = (r_upwind . r)/(r . r) come from the pair
// table, so the MC limiter works on wave strengths,
//     alpha * phi(theta) = mc(alpha, kappa * alpha_upwind),
// which equals phi(theta) W with theta = (W_up . W)/(W . W) (the oracle's
// form) up to rounding.
#include "march_common.h"

namespace wp {
namespace {

using namespace march;

// Per-material constants for one launch (depend on dt through nu).
template <typename T>
struct MCon {
    T Z, c, K, ir;       // impedance, sound speed, bulk modulus, 1/rho
    T hx, hZx, hy, hZy;  // forward correction: h = c (1 - nu c) / 2, hZ = h Z
    T gx, gZx, gy, gZy;  // adjoint correction: g = (1 - nu c) / 2, gZ = g Z
    T Khx, Khy;          // forward transverse: nu K / 2
    T Zhx, Zhy;          // adjoint transverse: nu Z / 2
};

template <typename T>
__device__ __forceinline__ void build_tables(const AcouInst<T> &I, MCon<T> *mc, T *pt, int lane)
{
    if (lane < I.nmat) {
        const T Z = I.mtab[lane * 4 + 0], c = I.mtab[lane * 4 + 1];
        const T K = I.mtab[lane * 4 + 2], ir = I.mtab[lane * 4 + 3];
        MCon<T> m;
        m.Z = Z; m.c = c; m.K = K; m.ir = ir;
        const T half = T(0.5);
        m.hx = half * c * (T(1) - I.nux * c);
        m.hy = half * c * (T(1) - I.nuy * c);
        m.hZx = m.hx * Z; m.hZy = m.hy * Z;
        m.gx = half * (T(1) - I.nux * c);
        m.gy = half * (T(1) - I.nuy * c);
        m.gZx = m.gx * Z; m.gZy = m.gy * Z;
        m.Khx = half * I.nux * K; m.Khy = half * I.nuy * K;
        m.Zhx = half * I.nux * Z; m.Zhy = half * I.nuy * Z;
        mc[lane] = m;
    }
    for (int k = lane; k < I.nmat * I.nmat * 3; k += WAVE) pt[k] = I.ptab[k];
}

// alpha * phi_MC(b / alpha): MC limiter applied to a wave strength, with b the
// upwind strength projected on this wave's eigenvector.  limiter 0: no limiting.
template <typename T>
__device__ __forceinline__ T limited(T a, T b, int limiter)
{
    if (limiter == 0) return a;
    const T aa = fabs(a), bb = fabs(b);
    T r = fmin(T(0.5) * (aa + bb), T(2) * fmin(aa, bb));
    r = copysign(r, a);
    return (a * b > T(0)) ? r : T(0);
}

// Normal Riemann solve at an edge between cell L (left/below) and R.
// p: pressure, n: normal velocity.  Forward (wave form): dQ = a1 (-Z_L, 1) +
// a2 (Z_R, 1) at speeds -c_L, +c_R.  Adjoint (f-wave form): the jump of the
// reversed flux (-n/rho, -K p) = a1 (1, Z_L) + a2 (1, -Z_R).
template <typename T, bool ADJ>
__device__ __forceinline__ void solve(T pl, T nl, T pr, T nr, const MCon<T> &L, const MCon<T> &R, T inv, T &a1,
                                      T &a2)
{
    if (!ADJ) {
        const T dp = pr - pl, dn = nr - nl;
        a1 = (R.Z * dn - dp) * inv;
        a2 = (dp + L.Z * dn) * inv;
    } else {
        const T df1 = L.ir * nl - R.ir * nr;
        const T df2 = L.K * pl - R.K * pr;
        a1 = (R.Z * df1 + df2) * inv;
        a2 = (L.Z * df1 - df2) * inv;
    }
}

template <typename T>
struct Row {
    T p, u, v;
    int m;
};

template <typename T, bool UNI>
struct Media;

template <typename T>
struct Media<T, false> {
    const MCon<T> *mc;
    const T *pt;
    int nmat;
    __device__ __forceinline__ const MCon<T> &operator()(int m) const { return mc[m]; }
    __device__ __forceinline__ void pair(int a, int b, T &inv, T &k1, T &k2) const
    {
        const T *p = pt + (a * nmat + b) * 3;
        inv = p[0];
        k1 = p[1];
        k2 = p[2];
    }
    static constexpr bool uniform = false;
};

// A single-material tile.  Every product of material constants, of the
// Riemann normalisation inv = 1/(2Z) and of the step ratios that the update
// applies to a wave strength is folded into one wave-uniform constant, and the
// march carries strengths scaled by 1/inv (A = a / inv); the MC limiter is
// scale-invariant, and its factor 1/2 sits in the constants as well.  With
// (S, S_L) the y-edge fluctuation sums of this and the left column, R the
// x-edge sums of this and the next row, and L_p, M_p the doubled limited
// x- and y-edge strengths:
//   F_p = fp (L_2 - L_1) + tp (S - S_L)      F_u = fu (L_1 + L_2) + tu (S + S_L)
//   G_p = gp (M_2 - M_1) + up (R_1 - R_0)    G_v = gv (M_1 + M_2) + uv (R_0 + R_1)
//   p' = p - p1 (A_2 + A_1r) - p2 (B_2 + B_1) - nux dF_p - nuy dG_p
//   u' = u - u1 (A_2 - A_1r) - nux dF_u,     v' = v - v1 (B_2 - B_1) - nuy dG_v
template <typename T>
struct UniCon {
    T Z, c, K;                   // Riemann solves
    T fp, fu, tp, tu;            // x-edge correction and transverse terms
    T gp, gv, up, uv;            // y-edge correction and transverse terms
    T p1, p2, u1, v1;            // update
};

template <typename T, bool ADJ>
__device__ __forceinline__ UniCon<T> make_unicon(const MCon<T> &m, T inv, T nux, T nuy)
{
    UniCon<T> u;
    const T half = T(0.5), inv2 = inv * inv;
    u.Z = m.Z;
    u.c = m.c;
    u.K = m.K;
    if (!ADJ) {
        u.fp = m.hZx * inv * half;
        u.fu = m.hx * inv * half;
        u.tp = m.K * m.Khy * inv2;
        u.tu = -(m.c * m.Khy * inv2);
        u.gp = m.hZy * inv * half;
        u.gv = m.hy * inv * half;
        u.up = m.K * m.Khx * inv2;
        u.uv = -(m.c * m.Khx * inv2);
        u.p1 = nux * m.K * inv;
        u.p2 = nuy * m.K * inv;
        u.u1 = nux * m.c * inv;
        u.v1 = nuy * m.c * inv;
    } else {
        u.fp = m.gx * inv * half;
        u.fu = -(m.gZx * inv * half);
        u.tp = m.c * m.Zhy * inv2;
        u.tu = m.K * m.Zhy * inv2;
        u.gp = m.gy * inv * half;
        u.gv = -(m.gZy * inv * half);
        u.up = m.c * m.Zhx * inv2;
        u.uv = m.K * m.Zhx * inv2;
        u.p1 = nux * inv;
        u.p2 = nuy * inv;
        u.u1 = -(nux * m.Z * inv);
        u.v1 = -(nuy * m.Z * inv);
    }
    // wave-uniform: keep them in scalar registers
    u.Z = uniform(u.Z); u.c = uniform(u.c); u.K = uniform(u.K);
    u.fp = uniform(u.fp); u.fu = uniform(u.fu); u.tp = uniform(u.tp); u.tu = uniform(u.tu);
    u.gp = uniform(u.gp); u.gv = uniform(u.gv); u.up = uniform(u.up); u.uv = uniform(u.uv);
    u.p1 = uniform(u.p1); u.p2 = uniform(u.p2); u.u1 = uniform(u.u1); u.v1 = uniform(u.v1);
    return u;
}

template <typename T>
struct Media<T, true> {
    UniCon<T> u;
    static constexpr bool uniform = true;
};

// Twice the MC-limited strength, 2 a phi(b / a) = sign(a) max(0, min(|a| + b',
// 4 min(|a|, b'))) with b' = b sign(a) (b' <= 0, opposite signs, gives 0).
// limiter 0: no limiting (2a).
template <typename T>
__device__ __forceinline__ T lim2(T a, T b, int limiter)
{
    if (limiter == 0) return a + a;
    const T aa = fabs(a);
    const T bs = copysign(T(1), a) * b;
    const T r = fmax(fmin(aa + bs, T(4) * fmin(aa, bs)), T(0));
    return copysign(r, a);
}

// Scaled strengths of one edge of a single-material tile (see UniCon):
// forward A1 = Z dn - dp, A2 = Z dn + dp; adjoint A1 = -(c dn + K dp),
// A2 = K dp - c dn, with dp = p_R - p_L, dn = n_R - n_L.
template <typename T, bool ADJ>
__device__ __forceinline__ void solve_uni(T pl, T nl, T pr, T nr, const UniCon<T> &u, T &a1, T &a2)
{
    const T dp = pr - pl, dn = nr - nl;
    if (!ADJ) {
        a1 = u.Z * dn - dp;
        a2 = u.Z * dn + dp;
    } else {
        const T kdp = u.K * dp;
        a1 = -(u.c * dn + kdp);
        a2 = kdp - u.c * dn;
    }
}

struct Opts {
    bool second, trans;
    int lim;
};

// Edge quantities carried from one row of the march to the next.
template <typename T>
struct Carry {
    T a1x0, a2x0;        // x-edge (col-1/2, j) wave strengths
    T b2m;               // y-edge (col, j-1/2) wave 2
    T b1p, b2p;          // y-edge (col, j+1/2) waves 1, 2
    T Gp_prev, Gv_prev;  // correction flux at y-edge (col, j-1/2)
    int mL0;             // material of (col-1, j)
};

// Solves of the edges below and left of row j (R0) that start the march.
template <typename T, bool ADJ, bool UNI>
__device__ __forceinline__ void march_start(const Media<T, UNI> &md, const Row<T> &RA, const Row<T> &R0,
                                            const Row<T> &R1, Carry<T> &c)
{
    if constexpr (UNI) {
        T b1a;
        solve_uni<T, ADJ>(RA.p, RA.v, R0.p, R0.v, md.u, b1a, c.b2m);
        solve_uni<T, ADJ>(R0.p, R0.v, R1.p, R1.v, md.u, c.b1p, c.b2p);
        c.mL0 = 0;
        solve_uni<T, ADJ>(from_left(R0.p), from_left(R0.u), R0.p, R0.u, md.u, c.a1x0, c.a2x0);
        c.Gp_prev = T(0);
        c.Gv_prev = T(0);
        return;
    } else {
    T inv, k1, k2, b1a;
    md.pair(RA.m, R0.m, inv, k1, k2);
    solve<T, ADJ>(RA.p, RA.v, R0.p, R0.v, md(RA.m), md(R0.m), inv, b1a, c.b2m);
    md.pair(R0.m, R1.m, inv, k1, k2);
    solve<T, ADJ>(R0.p, R0.v, R1.p, R1.v, md(R0.m), md(R1.m), inv, c.b1p, c.b2p);
    c.mL0 = UNI ? 0 : from_left(R0.m);
    const T pl = from_left(R0.p), ul = from_left(R0.u);
    md.pair(c.mL0, R0.m, inv, k1, k2);
    solve<T, ADJ>(pl, ul, R0.p, R0.u, md(c.mL0), md(R0.m), inv, c.a1x0, c.a2x0);
    c.Gp_prev = T(0);
    c.Gv_prev = T(0);
    }
}

// New state of cell (col, j) from rows j (R0), j+1 (R1), j+2 (R2) and the
// carried edge quantities, which advance to row j+1.  Per cell: the y-edge
// j+3/2 and x-edge (col-1/2, j+1) Riemann solves (each solved once, the
// neighbours' through DPP lane shifts), limited correction fluxes at the
// x-edge col-1/2 and y-edge j+1/2 with the transverse terms, and the
// fluctuation-form update.
template <typename T, bool ADJ, bool UNI>
__device__ __forceinline__ void row_step(const Media<T, UNI> &md, bool second, bool trans, int lim, T nux, T nuy,
                                         const Row<T> &R0, const Row<T> &R1, const Row<T> &R2, Carry<T> &c, T &pn,
                                         T &un, T &vn)
{
    if constexpr (UNI) {
        const UniCon<T> &u = md.u;
        T b1n, b2n;      // y-edge (col, j+3/2)
        solve_uni<T, ADJ>(R1.p, R1.v, R2.p, R2.v, u, b1n, b2n);
        T a1n, a2n;      // x-edge (col-1/2, j+1)
        solve_uni<T, ADJ>(from_left(R1.p), from_left(R1.u), R1.p, R1.u, u, a1n, a2n);
        const T a1r = from_right(c.a1x0);
        const T a2l = from_left(c.a2x0);
        T Fp = T(0), Fu = T(0), Gp = T(0), Gv = T(0);
        if (second) {
            const T t1 = lim2(c.a1x0, a1r, lim), t2 = lim2(c.a2x0, a2l, lim);
            Fp = u.fp * (t2 - t1);
            Fu = u.fu * (t1 + t2);
            const T s1 = lim2(c.b1p, b1n, lim), s2 = lim2(c.b2p, c.b2m, lim);
            Gp = u.gp * (s2 - s1);
            Gv = u.gv * (s1 + s2);
        }
        if (trans) {
            const T S = c.b2m + c.b1p;
            const T SL = from_left(S);
            Fp += u.tp * (S - SL);
            Fu += u.tu * (S + SL);
            const T R0s = c.a2x0 + a1r, R1s = a2n + from_right(a1n);
            Gp += u.up * (R1s - R0s);
            Gv += u.uv * (R0s + R1s);
        }
        const T Fpr = from_right(Fp), Fur = from_right(Fu);
        pn = R0.p - u.p1 * (c.a2x0 + a1r) - u.p2 * (c.b2m + c.b1p) - nux * (Fpr - Fp) - nuy * (Gp - c.Gp_prev);
        un = R0.u - u.u1 * (c.a2x0 - a1r) - nux * (Fur - Fu);
        vn = R0.v - u.v1 * (c.b2m - c.b1p) - nuy * (Gv - c.Gv_prev);
        c.a1x0 = a1n;
        c.a2x0 = a2n;
        c.b2m = c.b2p;
        c.b1p = b1n;
        c.b2p = b2n;
        c.Gp_prev = Gp;
        c.Gv_prev = Gv;
        return;
    } else {
    T inv, k1, k2;
    T b1n, b2n;      // y-edge (col, j+3/2)
    md.pair(R1.m, R2.m, inv, k1, k2);
    solve<T, ADJ>(R1.p, R1.v, R2.p, R2.v, md(R1.m), md(R2.m), inv, b1n, b2n);
    T a1n, a2n;      // x-edge (col-1/2, j+1)
    const int mL1 = UNI ? 0 : from_left(R1.m);
    {
        const T pl = from_left(R1.p), ul = from_left(R1.u);
        md.pair(mL1, R1.m, inv, k1, k2);
        solve<T, ADJ>(pl, ul, R1.p, R1.u, md(mL1), md(R1.m), inv, a1n, a2n);
    }
    // F at x-edge (col-1/2, j): L = (col-1, j), C = (col, j)
    const T a1r = from_right(c.a1x0);
    const T a2l = from_left(c.a2x0);
    const MCon<T> &L = md(c.mL0);
    const MCon<T> &C = md(R0.m);
    T Fp = T(0), Fu = T(0);
    {
        T invx;
        md.pair(c.mL0, R0.m, invx, k1, k2);
        if (second) {
            const T t1 = limited(c.a1x0, k1 * a1r, lim);
            const T t2 = limited(c.a2x0, k2 * a2l, lim);
            if (!ADJ) {
                Fp = C.hZx * t2 - L.hZx * t1;
                Fu = L.hx * t1 + C.hx * t2;
            } else {
                Fp = C.gx * t2 - L.gx * t1;
                Fu = -(L.gZx * t1 + C.gZx * t2);
            }
        }
        if (trans) {
            // y-edge fluctuations of cells (col, j) and (col-1, j) split at
            // this x-edge: up-going from below plus down-going from above
            const T S = c.b2m + c.b1p;
            const T SL = from_left(S);
            if (!ADJ) {
                const T TR = C.Khy * invx * S, TL = L.Khy * invx * SL;
                Fp += L.K * TR - C.K * TL;
                Fu -= L.c * TR + C.c * TL;
            } else {
                const T TR = C.Zhy * invx * S, TL = L.Zhy * invx * SL;
                Fp += L.c * TR - C.c * TL;
                Fu += L.K * TR + C.K * TL;
            }
        }
    }
    // G at y-edge (col, j+1/2): C = (col, j), A = (col, j+1)
    const MCon<T> &A = md(R1.m);
    T Gp = T(0), Gv = T(0);
    {
        T invy;
        md.pair(R0.m, R1.m, invy, k1, k2);
        if (second) {
            const T s1 = limited(c.b1p, k1 * b1n, lim);
            const T s2 = limited(c.b2p, k2 * c.b2m, lim);
            if (!ADJ) {
                Gp = A.hZy * s2 - C.hZy * s1;
                Gv = C.hy * s1 + A.hy * s2;
            } else {
                Gp = A.gy * s2 - C.gy * s1;
                Gv = -(C.gZy * s1 + A.gZy * s2);
            }
        }
        if (trans) {
            const T a1rn = from_right(a1n);
            const T R0s = c.a2x0 + a1r, R1s = a2n + a1rn;
            if (!ADJ) {
                const T UB = C.Khx * invy * R0s, UA = A.Khx * invy * R1s;
                Gp -= A.K * UB - C.K * UA;
                Gv -= A.c * UB + C.c * UA;
            } else {
                const T UB = C.Zhx * invy * R0s, UA = A.Zhx * invy * R1s;
                Gp += C.c * UA - A.c * UB;
                Gv += A.K * UB + C.K * UA;
            }
        }
    }
    // update cell (col, j)
    const T Fpr = from_right(Fp), Fur = from_right(Fu);
    if (!ADJ) {
        pn = R0.p - nux * (C.K * (c.a2x0 + a1r)) - nuy * (C.K * (c.b2m + c.b1p)) - nux * (Fpr - Fp) -
             nuy * (Gp - c.Gp_prev);
        un = R0.u - nux * (C.c * (c.a2x0 - a1r)) - nux * (Fur - Fu);
        vn = R0.v - nuy * (C.c * (c.b2m - c.b1p)) - nuy * (Gv - c.Gv_prev);
    } else {
        pn = R0.p - nux * (c.a2x0 + a1r) - nuy * (c.b2m + c.b1p) - nux * (Fpr - Fp) - nuy * (Gp - c.Gp_prev);
        un = R0.u - nux * (C.Z * (a1r - c.a2x0)) - nux * (Fur - Fu);
        vn = R0.v - nuy * (C.Z * (c.b1p - c.b2m)) - nuy * (Gv - c.Gv_prev);
    }
    c.mL0 = mL1;
    c.a1x0 = a1n;
    c.a2x0 = a2n;
    c.b2m = c.b2p;
    c.b1p = b1n;
    c.b2p = b2n;
    c.Gp_prev = Gp;
    c.Gv_prev = Gv;
    }
}

// Rows requested ahead of their first use in the compile-time march.
constexpr int PREFETCH = 3;
// sched_barrier mask: ALU instructions and memory writes may be moved across,
// memory reads may not.
constexpr int SCHED_KEEP_LOADS = 0x0001 | 0x0040;

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
template <typename T, bool ADJ, bool UNI, int RT, typename LD>
__device__ __forceinline__ void march_tile(const Media<T, UNI> &md, const Tile &tl, int nx, T nux, T nuy,
                                           unsigned csb, unsigned out_off0, bool out_lane,
                                           __amdgpu_buffer_rsrc_t qw, __amdgpu_buffer_rsrc_t sw, const LD &ld, int &bad)
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
        bstore(sw, off, 0u, pn);
        bstore(sw, off, csb, un);
        bstore(sw, off, 2u * csb, vn);
        bad |= keep & !(isfinite(pn) & isfinite(un) & isfinite(vn));
    }
}

// One wave marches its tile up the rows.  RT > 0: the compile-time march
// above (full method: second order, MC limiter, transverse terms).  RT = 0
// (runtime height, any options): a rolling window of rows prefetched two
// rows ahead.
template <typename T, bool ADJ, bool UNI, bool FULL, int RT>
__device__ __forceinline__ void march(const Media<T, UNI> &md, const Opts &op_rt, const Tile &tl, int lane, int nx,
                                      int ny, int bc2, int bc3, int cx, T sx, unsigned csb, T nux, T nuy,
                                      __amdgpu_buffer_rsrc_t qr, __amdgpu_buffer_rsrc_t qw,
                                      __amdgpu_buffer_rsrc_t mr, __amdgpu_buffer_rsrc_t sw, bool snap, int &bad)
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
        march_tile<T, ADJ, UNI, RT>(md, tl, nx, nux, nuy, csb, out_off0, out_lane, qw, sw, ld, bad);
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
template <typename T, bool ADJ, bool FULL, int RT, int KIND>
__global__ __launch_bounds__(WAVE) void acou2d_kernel(const AcouInst<T> *__restrict__ insts,
                                                      const Tile *__restrict__ tiles, int parity,
                                                      int snap_index, int *__restrict__ status,
                                                      unsigned long long *__restrict__ stamp)
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
        march<T, ADJ, true, FULL, RT>(md, op, tl, lane, nx, ny, bc2, bc3, cx, sx, csb, nux, nuy, qr, qw, mr, sw, snap,
                                      bad);
    } else if (KIND != 1) {
        // mixed tiles are acou_mixed_rows(RT) high
        Media<T, false> md{mc, pt, Ip->nmat};
        march<T, ADJ, false, FULL, acou_mixed_rows(RT)>(md, op, tl, lane, nx, ny, bc2, bc3, cx, sx, csb, nux, nuy, qr,
                                                        qw, mr, sw, snap, bad);
    }
    if (__any(bad) && lane == 0) atomicOr(status, ST_NONFINITE);
    if (stamp && lane == 0) stamp[2 * blockIdx.x + 1] = (unsigned long long)wall_clock64();
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
                   bool full, int rows, int kind, int snap_index, int *status, hipStream_t s, unsigned long long *stamp)
{
    if (ntiles <= 0) return;
    const size_t sm = acou_smem<T>(nmat_max);
    const dim3 g(ntiles), b(WAVE);
#define WP_LAUNCH(ADJ, FULL, RT, KIND)                                                                       \
    hipLaunchKernelGGL((acou2d_kernel<T, ADJ, FULL, RT, KIND>), g, b, sm, s, insts, tiles, parity, snap_index, status, \
                       stamp)
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
                                    int, int *, hipStream_t, unsigned long long *);
template void launch_acou2d<float>(const AcouInst<float> *, const Tile *, int, int, int, int, bool, int, int,
                                   int, int *, hipStream_t, unsigned long long *);
template void launch_acou1d<double>(const AcouInst<double> *, const AcouInst<double> &, int, int, int, int *,
                                    hipStream_t);
template void launch_acou1d<float>(const AcouInst<float> *, const AcouInst<float> &, int, int, int, int *,
                                   hipStream_t);

}  // namespace wp
