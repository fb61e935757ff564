// Acoustics stencil pieces shared by the one-step and the two-step 2D
// kernels (Davis & LeVeque Sec. 3 wave propagation, Sec. 5.1/5.2 acoustics
// coefficient matrices, Sec. 2/4 adjoint and time reversal): per-material
// constants, Riemann solves in wave and f-wave form, the MC limiter on
// wave strengths, and one row of the strip march.
//
// Media are piecewise constant: every cell carries a material index, and
// per-material and per-material-pair constants sit in LDS.  This removes
// every division from the stencil: 1/(Z_a + Z_b) and the limiter's
// eigenvector projection kappa = (r_upwind . r)/(r . r) come from the pair
// table, so the MC limiter works on wave strengths,
//     alpha * phi(theta) = mc(alpha, kappa * alpha_upwind),
// which equals phi(theta) W with theta = (W_up . W)/(W . W) (the oracle's
// form) up to rounding.
#pragma once

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

}  // namespace
}  // namespace wp
