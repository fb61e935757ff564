// Shallow-water patch update (Davis & LeVeque Sec. 5.3, eq. swe) with a
// well-balanced f-wave Roe solver, and the time-reversed linearised
// shallow-water adjoint (Sec. 5.3 linearised system, Sec. 2/4 adjoint and
// time reversal), for gfx950.
//
// Layout (the strip march of the acoustics kernels): one 64-lane wave owns a
// strip of 64 columns (60 outputs and a two-column halo on each side) and
// marches up the rows of its tile.  Every x- and y-edge Riemann problem is
// solved once; quantities of neighbouring columns' edges (upwind waves for
// the limiter, transverse splits, fluctuations, correction fluxes) move
// across lanes by DPP shifts, and those of the y-edges below are carried in
// registers.  Ghost cells are resolved in the loader.
//
// Mixed precision (ETA = double, T = float): eta = h + B is stored and
// updated in FP64 and the well-balanced term g hbar d(eta) is formed in FP64,
// so a lake at rest stays exactly at rest and metre-scale waves are not lost
// against 4000 m of depth; the waves, limiter and transverse terms run in
// FP32.
#include "march_common.h"

namespace wp {
namespace {

using namespace march;

// 1/b from the hardware reciprocal refined by Newton steps, within an ulp
// or two of the quotient (b nonzero and not subnormal: depths, sums of
// square roots and sound speeds, and the limiter's b = 0 is excluded)
__device__ __forceinline__ double recip(double b)
{
    double r = __builtin_amdgcn_rcp(b);
    double e = fma(-b, r, 1.0);
    r = fma(r, e, r);
    e = fma(-b, r, 1.0);
    return fma(r, e, r);
}
__device__ __forceinline__ float recip(float b)
{
    const float r = __builtin_amdgcn_rcpf(b);
    return fmaf(r, fmaf(-b, r, 1.0f), r);
}

// Rows requested ahead of their first use in the compile-time march.
constexpr int PREFETCH = 3;
// sched_barrier mask: ALU instructions and memory writes may be moved across,
// memory reads may not.
constexpr int SCHED_KEEP_LOADS = 0x0001 | 0x0040;

template <typename T>
__device__ __forceinline__ T mc_phi(T theta)
{
    T a = fmin(T(0.5) * (T(1) + theta), T(2));
    a = fmin(a, T(2) * theta);
    return fmax(T(0), a);
}

// limiter factor of wave w against the upwind wave wu (theta = wu.w / w.w)
template <typename T>
__device__ __forceinline__ T lim_factor(const T *w, const T *wu, int limiter)
{
    if (limiter == 0) return T(1);
    const T a = wu[0] * w[0] + wu[1] * w[1] + wu[2] * w[2];
    const T b = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    return b == T(0) ? T(0) : mc_phi(a * recip(b));
}

template <typename T>
__device__ __forceinline__ T sgn(T s) { return s > T(0) ? T(1) : (s < T(0) ? T(-1) : T(0)); }


// Second-order correction flux of an edge with NW waves w[3 p + k] at speeds
// s[p]: per family the upwind wave is that of the lower/left neighbour edge
// (wlo) for s > 0, else of the upper/right one (whi); nu = dt/dx of the
// edge's direction.
template <int NW, typename T>
__device__ __forceinline__ void corr_flux(const T *w, const T *s, const T *wlo, const T *whi, T nu, int lim, T F[3])
{
#pragma unroll
    for (int p = 0; p < NW; ++p) {
        T wu[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) wu[k] = s[p] > T(0) ? wlo[3 * p + k] : whi[3 * p + k];
        const T phi = lim_factor(&w[3 * p], wu, lim);
        const T coef = T(0.5) * sgn(s[p]) * (T(1) - nu * fabs(s[p]));
#pragma unroll
        for (int k = 0; k < 3; ++k) F[k] += coef * (phi * w[3 * p + k]);
    }
}

template <typename T>
__device__ __forceinline__ void sub_scaled(T F[3], T a, const T o[3])
{
#pragma unroll
    for (int k = 0; k < 3; ++k) F[k] -= a * o[k];
}

// ---------------------------------------------------------------------------
// nonlinear shallow water
// ---------------------------------------------------------------------------

// A cell as loaded (momenta already reflected for wall ghosts) ...
template <typename ETA, typename T>
struct SRaw {
    ETA eta;
    double B;
    T hu, hv;
};

// ... and with the quantities derived from it once.
template <typename ETA, typename T>
struct SRow {
    ETA eta, he;   // surface elevation and depth h = eta - B, in the eta precision
    T h, hu, hv, u, v, sq;
};

template <typename ETA, typename T>
__device__ __forceinline__ SRow<ETA, T> derive(const SRaw<ETA, T> &a, int &bad)
{
    SRow<ETA, T> r;
    r.eta = a.eta;
    r.he = a.eta - (ETA)a.B;
    r.h = (T)r.he;
    r.hu = a.hu;
    r.hv = a.hv;
    const T rh = recip(r.h);
    r.u = r.hu * rh;
    r.v = r.hv * rh;
    r.sq = sqrt(r.h);
    bad |= !(r.h > T(0));
    return r;
}

template <typename ETA, typename T>
__device__ __forceinline__ SRow<ETA, T> shift_left(const SRow<ETA, T> &r)
{
    return SRow<ETA, T>{from_left(r.eta), from_left(r.he), from_left(r.h), from_left(r.hu),
                        from_left(r.hv), from_left(r.u), from_left(r.v), from_left(r.sq)};
}

// An edge: f-waves w[3 p + k] at speeds s[p], and the Roe state (u, v, c)
// that splits fluctuations transversally.
template <typename T>
struct SEdge {
    T w[9];
    T s[3];
    T ru, rv, c, hic;   // hic = 1 / (2 c)
};

// Roe f-wave solve at the edge between L and R in direction DIR (0: x,
// 1: y).  The flux difference uses 1/2 g (h_R^2 - h_L^2) + g hbar dB =
// g hbar d(eta), formed in the eta precision, so a lake at rest gives zero
// waves exactly.
template <int DIR, typename ETA, typename T>
__device__ __forceinline__ SEdge<T> roe_edge(const SRow<ETA, T> &L, const SRow<ETA, T> &R, double g)
{
    constexpr int n = DIR == 0 ? 1 : 2, t = DIR == 0 ? 2 : 1;
    const T unl = DIR == 0 ? L.u : L.v, unr = DIR == 0 ? R.u : R.v;
    const T utl = DIR == 0 ? L.v : L.u, utr = DIR == 0 ? R.v : R.u;
    const T qnl = DIR == 0 ? L.hu : L.hv, qnr = DIR == 0 ? R.hu : R.hv;
    const T hbar = T(0.5) * (L.h + R.h);
    const T rs = recip(L.sq + R.sq);
    const T un = (L.sq * unl + R.sq * unr) * rs;
    const T ut = (L.sq * utl + R.sq * utr) * rs;
    // c = sqrt(g hbar) and 1/(2c) from one reciprocal square root
    const T gh = T(g) * hbar;
    const T rq = rsqrt(gh);
    const T c = gh * rq;
    const ETA hbe = ETA(0.5) * (L.he + R.he);
    const T wb = (T)(ETA(g) * hbe * (R.eta - L.eta));
    const T d1 = qnr - qnl;
    const T d2 = (qnr * unr - qnl * unl) + wb;
    const T d3 = qnr * utr - qnl * utl;
    const T s1 = un - c, s3 = un + c;
    const T inv2c = T(0.5) * rq;
    const T b1 = ((un + c) * d1 - d2) * inv2c;
    const T b3 = (d2 - (un - c) * d1) * inv2c;
    const T b2 = d3 - ut * d1;
    SEdge<T> e;
    e.w[0] = b1; e.w[n] = b1 * s1; e.w[t] = b1 * ut;
    e.w[3] = T(0); e.w[3 + n] = T(0); e.w[3 + t] = b2;
    e.w[6] = b3; e.w[6 + n] = b3 * s3; e.w[6 + t] = b3 * ut;
    e.s[0] = s1; e.s[1] = un; e.s[2] = s3;
    e.ru = DIR == 0 ? un : ut;
    e.rv = DIR == 0 ? ut : un;
    e.c = c;
    e.hic = inv2c;
    return e;
}

// Fluctuations of an edge: A-dQ (am, waves with negative speed) and A+dQ
// (ap, positive speed); a zero-speed wave is split evenly.
template <typename T>
__device__ __forceinline__ void flucts(const SEdge<T> &E, T am[3], T ap[3])
{
    T fn[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) fn[p] = E.s[p] < T(0) ? T(1) : (E.s[p] > T(0) ? T(0) : T(0.5));
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        am[k] = fn[0] * E.w[k] + fn[1] * E.w[3 + k] + fn[2] * E.w[6 + k];
        ap[k] = (T(1) - fn[0]) * E.w[k] + (T(1) - fn[1]) * E.w[3 + k] + (T(1) - fn[2]) * E.w[6 + k];
    }
}

// Transverse split of d along direction tdir with the eigen-structure of
// that direction at the Roe state (uh, vh, c; hic = 1/(2c)) of the edge d
// came from: neg
// gets the part carried by negative speeds, pos the part carried by
// non-negative speeds.  The eigenvalues vt - c < vt < vt + c enter through
// 0/1 masks.
template <typename T>
__device__ __forceinline__ void swe_tsplit(int tdir, const T d[3], T uh, T vh, T c, T hic, T neg[3], T pos[3])
{
    const int kt = tdir == 0 ? 1 : 2, ko = tdir == 0 ? 2 : 1;
    const T vt = tdir == 0 ? uh : vh, vo = tdir == 0 ? vh : uh;
    const T inv2c = hic;
    const T g1 = ((vt + c) * d[0] - d[kt]) * inv2c;
    const T g3 = (d[kt] - (vt - c) * d[0]) * inv2c;
    const T g2 = d[ko] - vo * d[0];
    const T l1 = vt - c, l2 = vt, l3 = vt + c;
    const T a1 = l1 * g1, a2 = l2 * g2, a3 = l3 * g3;
    const T c1[3] = {a1, a1 * (vt - c), a1 * vo};   // (mass, tangential-direction, other) parts
    const T c3[3] = {a3, a3 * (vt + c), a3 * vo};
    const T m1 = l1 < T(0) ? T(1) : T(0), m2 = l2 < T(0) ? T(1) : T(0), m3 = l3 < T(0) ? T(1) : T(0);
    neg[0] = m1 * c1[0] + m3 * c3[0];
    neg[kt] = m1 * c1[1] + m3 * c3[1];
    neg[ko] = m1 * c1[2] + m2 * a2 + m3 * c3[2];
    pos[0] = (T(1) - m1) * c1[0] + (T(1) - m3) * c3[0];
    pos[kt] = (T(1) - m1) * c1[1] + (T(1) - m3) * c3[1];
    pos[ko] = (T(1) - m1) * c1[2] + (T(1) - m2) * a2 + (T(1) - m3) * c3[2];
}

template <typename T>
__device__ __forceinline__ T dot3(const T *a, const T *b)
{
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

// Limited correction-flux contribution of wave family p: a = upwind wave .
// own wave, w = own wave, s its speed, nu = dt/dx of the edge's direction.
template <typename T>
__device__ __forceinline__ void corr_add(const T *w, T s, T a, T nu, int lim, T F[3])
{
    T phi = T(1);
    if (lim != 0) {
        const T b = dot3(w, w);
        phi = b == T(0) ? T(0) : mc_phi(a * recip(b));
    }
    const T coef = T(0.5) * sgn(s) * (T(1) - nu * fabs(s));
#pragma unroll
    for (int k = 0; k < 3; ++k) F[k] += coef * (phi * w[k]);
}

template <typename T>
__device__ __forceinline__ T edge_cfl(const T s[3], T nu)
{
    return fmax(fmax(fabs(s[0]) * nu, fabs(s[1]) * nu), fabs(s[2]) * nu);
}

// What the iteration for row j hands to that for row j + 1.  Every edge is
// reduced to what later rows need as soon as it is solved, and everything
// of row j + 1's increment except its G difference is summed ahead.
template <typename T>
struct SCarry {
    T yw[9], ys[3];        // waves and speeds of the y-edge j + 1/2
    T dlo[3];              // per family: waves of y-edges j - 1/2 and j + 1/2 dotted
    T bpP[3];              // B+dQ of the y-edge j + 1/2 (into row j + 1) ...
    T bpl[3], bpr[3];      // ... and its left- and right-going parts
    T apu[3], amu[3];      // up-going parts of the x-fluctuations of row j
    T P[3];                // increment of row j without nuy (G(j + 1/2) - G(j - 1/2))
    T Gp[3];               // correction flux at the y-edge j - 1/2
};

struct SOpts {
    bool second, trans;
    int lim;
};

// Carry for the first iteration (the update of row j0 - 1 is not formed):
// rows Ra = j0 - 2, R0 = j0 - 1, R1 = j0.
template <typename ETA, typename T>
__device__ __forceinline__ void swe_start(const SRow<ETA, T> &Ra, const SRow<ETA, T> &R0, const SRow<ETA, T> &R1,
                                          double g, const SOpts &op, SCarry<T> &c)
{
    const SEdge<T> ym = roe_edge<1>(Ra, R0, g);
    const SEdge<T> yp = roe_edge<1>(R0, R1, g);
#pragma unroll
    for (int p = 0; p < 3; ++p) c.dlo[p] = dot3(&ym.w[3 * p], &yp.w[3 * p]);
#pragma unroll
    for (int k = 0; k < 9; ++k) c.yw[k] = yp.w[k];
#pragma unroll
    for (int p = 0; p < 3; ++p) c.ys[p] = yp.s[p];
    T bm[3];
    flucts(yp, bm, c.bpP);
#pragma unroll
    for (int k = 0; k < 3; ++k) c.bpl[k] = c.bpr[k] = T(0);
    if (op.trans) swe_tsplit(0, c.bpP, yp.ru, yp.rv, yp.c, yp.hic, c.bpl, c.bpr);
    const SEdge<T> xe = roe_edge<0>(shift_left(R0), R0, g);
    T am[3], ap[3], dn[3];
    flucts(xe, am, ap);
#pragma unroll
    for (int k = 0; k < 3; ++k) c.apu[k] = c.amu[k] = T(0);
    if (op.trans) {
        swe_tsplit(1, ap, xe.ru, xe.rv, xe.c, xe.hic, dn, c.apu);
        swe_tsplit(1, am, xe.ru, xe.rv, xe.c, xe.hic, dn, c.amu);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) c.P[k] = c.Gp[k] = T(0);
}

// Iteration for row j: solves the y-edge j + 3/2 and the x-edge of row
// j + 1, forms the correction fluxes G at the y-edge j + 1/2 and F at the
// x-edge of row j + 1, and (upd) the update of row j (R0) into en, qun, qvn.
// cy_in / cx_in: whether the y-edge j + 1/2 / the x-edge of row j + 1 count
// toward the Courant number.
template <typename ETA, typename T>
__device__ __forceinline__ void swe_row(const SRow<ETA, T> &R0, const SRow<ETA, T> &R1, const SRow<ETA, T> &R2,
                                        double g, T nux, T nuy, const SOpts &op, bool upd, bool cy_in, bool cx_in,
                                        SCarry<T> &c, T &cfl, ETA &en, T &qun, T &qvn)
{
    const T hx = T(0.5) * nux, hy = T(0.5) * nuy;
    // y-edge j + 3/2: fluctuations and their splits along x
    const SEdge<T> yn = roe_edge<1>(R1, R2, g);
    T bmN[3], bpN[3], bml[3], bmr[3], bpl[3], bpr[3];
    flucts(yn, bmN, bpN);
#pragma unroll
    for (int k = 0; k < 3; ++k) bml[k] = bmr[k] = bpl[k] = bpr[k] = T(0);
    if (op.trans) {
        swe_tsplit(0, bmN, yn.ru, yn.rv, yn.c, yn.hic, bml, bmr);
        swe_tsplit(0, bpN, yn.ru, yn.rv, yn.c, yn.hic, bpl, bpr);
    }
    T dhi[3];   // per family: waves of y-edges j + 1/2 and j + 3/2 dotted
#pragma unroll
    for (int p = 0; p < 3; ++p) dhi[p] = dot3(&yn.w[3 * p], &c.yw[3 * p]);
    // G at the y-edge (col, j + 1/2): limited waves
    T G[3] = {T(0), T(0), T(0)};
    if (cy_in) cfl = fmax(cfl, edge_cfl(c.ys, nuy));
    if (op.second) {
#pragma unroll
        for (int p = 0; p < 3; ++p) corr_add(&c.yw[3 * p], c.ys[p], c.ys[p] > T(0) ? c.dlo[p] : dhi[p], nuy, op.lim, G);
    }
    // x-edge (col - 1/2, j + 1): fluctuations and their splits along y
    const SEdge<T> xn = roe_edge<0>(shift_left(R1), R1, g);
    T am[3], ap[3], amd[3], amu[3], apd[3], apu[3];
    flucts(xn, am, ap);
#pragma unroll
    for (int k = 0; k < 3; ++k) amd[k] = amu[k] = apd[k] = apu[k] = T(0);
    if (op.trans) {
        swe_tsplit(1, ap, xn.ru, xn.rv, xn.c, xn.hic, apd, apu);
        swe_tsplit(1, am, xn.ru, xn.rv, xn.c, xn.hic, amd, amu);
        // G: the x-fluctuations of (col, j + 1) going down, then those of
        // (col, j) going up; those of the right edges come from the next lane
        T d[3];
        sub_scaled(G, hx, apd);
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] = from_right(amd[k]);
        sub_scaled(G, hx, d);
        sub_scaled(G, hx, c.apu);
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] = from_right(c.amu[k]);
        sub_scaled(G, hx, d);
    }
    if (upd) {
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T inc = c.P[k] + nuy * (G[k] - c.Gp[k]);
            if (k == 0) en = R0.eta - (ETA)inc;
            if (k == 1) qun = R0.hu - inc;
            if (k == 2) qvn = R0.hv - inc;
        }
    }
    // F at the x-edge (col - 1/2, j + 1); the upwind wave's dot product with
    // the left neighbour edge is the left lane's with its right neighbour
    T F[3] = {T(0), T(0), T(0)};
    if (cx_in) cfl = fmax(cfl, edge_cfl(xn.s, nux));
    if (op.second) {
        T dR[3], dL[3];
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            T wr[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) wr[k] = from_right(xn.w[3 * p + k]);
            dR[p] = dot3(wr, &xn.w[3 * p]);
        }
#pragma unroll
        for (int p = 0; p < 3; ++p) dL[p] = from_left(dR[p]);
#pragma unroll
        for (int p = 0; p < 3; ++p) corr_add(&xn.w[3 * p], xn.s[p], xn.s[p] > T(0) ? dL[p] : dR[p], nux, op.lim, F);
    }
    if (op.trans) {
        // the y-fluctuations of row j + 1 going left, then those of the
        // left neighbour going right
        T d[3];
        sub_scaled(F, hy, c.bpl);
        sub_scaled(F, hy, bml);
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] = from_left(c.bpr[k]);
        sub_scaled(F, hy, d);
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] = from_left(bmr[k]);
        sub_scaled(F, hy, d);
    }
    // row j + 1's increment so far: A+dQ + A-dQ, B+dQ + B-dQ, F difference
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T amr = from_right(am[k]), Fr = from_right(F[k]);
        c.P[k] = nux * (ap[k] + amr) + nuy * (c.bpP[k] + bmN[k]) + nux * (Fr - F[k]);
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) c.yw[k] = yn.w[k];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        c.ys[k] = yn.s[k];
        c.dlo[k] = dhi[k];
        c.bpP[k] = bpN[k];
        c.bpl[k] = bpl[k];
        c.bpr[k] = bpr[k];
        c.apu[k] = apu[k];
        c.amu[k] = amu[k];
        c.Gp[k] = G[k];
    }
}

// RT > 0: tiles of at most RT rows, the march fully unrolled with rows
// requested PREFETCH iterations ahead; RT = 0: any height, a rolling window
// of rows prefetched two rows ahead.  FULL: second order, MC limiter and
// transverse terms fixed at compile time, else as the instance says.
template <typename ETA, typename T, int RT, bool FULL>
__global__ __launch_bounds__(WAVE) void swe2d_kernel(const SweInst<ETA, T> *__restrict__ inst,
                                                     const Tile *__restrict__ tiles, int parity,
                                                     int *__restrict__ status, unsigned *__restrict__ cflbits)
{
    const Tile tl = tiles[blockIdx.x];
    const SweInst<ETA, T> &I = *inst;
    const int lane = threadIdx.x;
    const int nx = I.nx, ny = I.ny;
    const unsigned cells = (unsigned)nx * (unsigned)ny;
    constexpr unsigned SE = sizeof(ETA), ST = sizeof(T);
    const __amdgpu_buffer_rsrc_t re = make_rsrc(I.eta[parity], cells * SE);
    const __amdgpu_buffer_rsrc_t ru = make_rsrc(I.hu[parity], cells * ST);
    const __amdgpu_buffer_rsrc_t rv = make_rsrc(I.hv[parity], cells * ST);
    const __amdgpu_buffer_rsrc_t rb = make_rsrc(I.B, cells * 8u);
    const __amdgpu_buffer_rsrc_t we = make_rsrc(I.eta[parity ^ 1], cells * SE);
    const __amdgpu_buffer_rsrc_t wu = make_rsrc(I.hu[parity ^ 1], cells * ST);
    const __amdgpu_buffer_rsrc_t wv = make_rsrc(I.hv[parity ^ 1], cells * ST);
    const double g = I.g;
    const T nux = (T)I.nux, nuy = (T)I.nuy;
    const SOpts op = FULL ? SOpts{true, true, 1} : SOpts{I.order >= 2, I.transverse != 0, I.limiter};
    const int col = tl.i0 - 2 + lane;
    bool fx;
    const int cx = resolve(col, nx, I.bc[0], I.bc[1], fx);
    const T sx = fx ? T(-1) : T(1);
    const Resolver rowres(ny, I.bc[2], I.bc[3]);
    const bool out_lane = lane >= 2 && lane < 2 + tl.ni;
    const bool xedge_lane = lane >= 2 && lane <= 2 + tl.ni;   // x-edges i0 - 1/2 .. i0 + ni - 1/2
    int bad = 0;
    T cfl = T(0);
    auto ld = [&](SRaw<ETA, T> &r, int j) {
        bool fy;
        const int jy = rowres(j, fy);
        const unsigned idx = (unsigned)(jy * nx + cx);
        r.eta = bload(re, idx * SE, ETA(0), 0u);
        r.B = bload(rb, idx * 8u, 0.0, 0u);
        r.hu = sx * bload(ru, idx * ST, T(0), 0u);
        const T qv = bload(rv, idx * ST, T(0), 0u);
        r.hv = fy ? -qv : qv;
    };
    const int j0 = tl.j0, j1 = tl.j0 + tl.nj;
    // stores of halo lanes and of rows past a short tile go beyond the
    // buffers' range, where they are dropped
    const unsigned nowE = cells * SE, nowT = cells * ST;
    auto put = [&](int j, bool valid, ETA en, T qun, T qvn) {
        const bool keep = valid && j < j1 && out_lane;
        const unsigned idx = (unsigned)(j * nx + col);
        bstore(we, keep ? idx * SE : nowE, 0u, en);
        bstore(wu, keep ? idx * ST : nowT, 0u, qun);
        bstore(wv, keep ? idx * ST : nowT, 0u, qvn);
        bad |= keep & !(isfinite((double)en) & isfinite((double)qun) & isfinite((double)qvn));
    };
    SCarry<T> c;
    if constexpr (RT > 0) {
        constexpr int NR = RT + 4;
        constexpr int FIRST = 3 + PREFETCH < NR ? 3 + PREFETCH : NR;
        SRaw<ETA, T> raw[NR];
#pragma unroll
        for (int r = 0; r < FIRST; ++r) ld(raw[r], j0 - 2 + r);
        __builtin_amdgcn_sched_barrier(SCHED_KEEP_LOADS);
        const SRow<ETA, T> Ra = derive(raw[0], bad);
        SRow<ETA, T> R0 = derive(raw[1], bad), R1 = derive(raw[2], bad);
        swe_start(Ra, R0, R1, g, op, c);
#pragma unroll
        for (int it = 0; it <= RT; ++it) {
            if (FIRST + it < NR) {
                ld(raw[FIRST + it], j0 - 2 + FIRST + it);
                __builtin_amdgcn_sched_barrier(SCHED_KEEP_LOADS);
            }
            const int j = j0 - 1 + it;
            const SRow<ETA, T> R2 = derive(raw[it + 3], bad);
            ETA en = ETA(0);
            T qun = T(0), qvn = T(0);
            swe_row(R0, R1, R2, g, nux, nuy, op, it > 0, out_lane && j + 1 <= j1, xedge_lane && j + 1 < j1, c,
                    cfl, en, qun, qvn);
            if (it > 0) put(j, true, en, qun, qvn);
            R0 = R1;
            R1 = R2;
        }
    } else {
        SRaw<ETA, T> X0, X1, X2;
        SRaw<ETA, T> a;
        ld(a, j0 - 2);
        const SRow<ETA, T> Ra = derive(a, bad);
        ld(a, j0 - 1);
        SRow<ETA, T> R0 = derive(a, bad);
        ld(a, j0);
        SRow<ETA, T> R1 = derive(a, bad);
        ld(X0, j0 + 1);
        ld(X1, j0 + 2);
        swe_start(Ra, R0, R1, g, op, c);
        for (int j = j0 - 1; j < j1; ++j) {
            ld(X2, j + 4);   // row j + 2 (X0) was requested two iterations ago
            const SRow<ETA, T> R2 = derive(X0, bad);
            ETA en = ETA(0);
            T qun = T(0), qvn = T(0);
            swe_row(R0, R1, R2, g, nux, nuy, op, true, out_lane, xedge_lane && j + 1 < j1, c, cfl, en, qun, qvn);
            put(j, j >= j0, en, qun, qvn);
            R0 = R1;
            R1 = R2;
            X0 = X1;
            X1 = X2;
        }
    }
    // Courant number and failures: one atomic per wave, skipped when the
    // running maximum is already as large
    for (int off = 32; off > 0; off >>= 1) cfl = fmax(cfl, __shfl_down(cfl, off));
    if (lane == 0) {
        const unsigned cb = __float_as_uint((float)cfl);
        if (cb > __hip_atomic_load(cflbits, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(cflbits, cb);
        if ((double)cfl > I.cfl_max) atomicOr(status, ST_CFL);
    }
    if (__any(bad) && lane == 0) atomicOr(status, ST_NONFINITE);
}

// ---------------------------------------------------------------------------
// linearised shallow-water adjoint, time reversed, f-wave form
// ---------------------------------------------------------------------------

template <typename T>
struct LRow {
    T q[3];   // (eta, mu, gamma) of the time-reversed adjoint
    T c;      // sqrt(g hbar) of the linearisation
};

template <typename T>
__device__ __forceinline__ LRow<T> shift_left(const LRow<T> &r)
{
    return LRow<T>{{from_left(r.q[0]), from_left(r.q[1]), from_left(r.q[2])}, from_left(r.c)};
}

// f-waves of the reversed flux -A^T q = (-c^2 mu_n, -eta, 0): w[0..2] =
// b1 (c_L, 1) at speed -c_L, w[3..5] = b2 (-c_R, 1) at speed +c_R (index n:
// normal momentum).  Wave 1 is the fluctuation into the lower/left cell,
// wave 2 that into the upper/right cell.
template <typename T>
struct LEdge {
    T w[6];
    T s[2];
    T inv;   // 1 / (c_L + c_R)
};

template <int DIR, typename T>
__device__ __forceinline__ LEdge<T> lsw_edge(const LRow<T> &L, const LRow<T> &R)
{
    constexpr int n = DIR == 0 ? 1 : 2, t = DIR == 0 ? 2 : 1;
    const T cl = L.c, cr = R.c;
    const T f1l = -(cl * cl) * L.q[n], f1r = -(cr * cr) * R.q[n];
    const T f2l = -L.q[0], f2r = -R.q[0];
    const T df1 = f1r - f1l, df2 = f2r - f2l;
    const T inv = recip(cl + cr);
    const T b1 = (df1 + cr * df2) * inv;
    const T b2 = (cl * df2 - df1) * inv;
    LEdge<T> e;
    e.w[0] = b1 * cl; e.w[n] = b1; e.w[t] = T(0);
    e.w[3] = -b2 * cr; e.w[3 + n] = b2; e.w[3 + t] = T(0);
    e.s[0] = -cl;
    e.s[1] = cr;
    e.inv = inv;
    return e;
}

// transverse split along tdir of d living in a cell with sound speed cown:
// the part into the lo neighbour (neg, cn = c_lo) or into the hi neighbour
// (cn = c_hi); inv = 1 / (c_lo + cown) or 1 / (cown + c_hi), the edge's own
// reciprocal sum
template <typename T>
__device__ __forceinline__ void lsw_tsplit(int tdir, const T d[3], T cn, T cown, T inv, bool neg, T o[3])
{
    const int n = tdir == 0 ? 1 : 2, t = tdir == 0 ? 2 : 1;
    if (neg) {
        const T gm = (d[0] + cown * d[n]) * inv;
        o[0] = -cn * gm * cn; o[n] = -cn * gm; o[t] = T(0);
    } else {
        const T gp = (cown * d[n] - d[0]) * inv;
        o[0] = -cn * gp * cn; o[n] = cn * gp; o[t] = T(0);
    }
}

template <typename T>
struct LCarry {
    LEdge<T> ym, yp, xe;   // y-edges j -+ 1/2, x-edge (col - 1/2, j)
    T Gp[3];
};

template <typename T>
__device__ __forceinline__ void lswe_row(const LRow<T> &R0, const LRow<T> &R1, const LRow<T> &R2, T nux, T nuy,
                                         const SOpts &op, LCarry<T> &c, T qn[3])
{
    const LEdge<T> yn = lsw_edge<1>(R1, R2);                  // y-edge j + 3/2
    const LEdge<T> xn = lsw_edge<0>(shift_left(R1), R1);      // x-edge (col - 1/2, j + 1)
    const T hx = T(0.5) * nux, hy = T(0.5) * nuy;
    T am[3];   // wave 1 of the x-edge (col + 1/2, j): A-dQ of this cell
#pragma unroll
    for (int k = 0; k < 3; ++k) am[k] = from_right(c.xe.w[k]);
    // F at the x-edge (col - 1/2, j)
    T F[3] = {T(0), T(0), T(0)};
    if (op.second) {
        T wl[6], wr[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            wl[k] = from_left(c.xe.w[k]);
            wr[k] = from_right(c.xe.w[k]);
        }
        corr_flux<2>(c.xe.w, c.xe.s, wl, wr, nux, op.lim, F);
    }
    if (op.trans) {
        const T cL = from_left(R0.c), cR = R0.c, inv = c.xe.inv;
        T d[3], o[3];
        // the y-fluctuations of this cell going left ...
        lsw_tsplit(0, &c.ym.w[3], cL, cR, inv, true, o);
        sub_scaled(F, hy, o);
        lsw_tsplit(0, &c.yp.w[0], cL, cR, inv, true, o);
        sub_scaled(F, hy, o);
        // ... and those of the left neighbour going right
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] = from_left(c.ym.w[3 + k]);
        lsw_tsplit(0, d, cR, cL, inv, false, o);
        sub_scaled(F, hy, o);
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] = from_left(c.yp.w[k]);
        lsw_tsplit(0, d, cR, cL, inv, false, o);
        sub_scaled(F, hy, o);
    }
    // G at the y-edge (col, j + 1/2)
    T G[3] = {T(0), T(0), T(0)};
    if (op.second) corr_flux<2>(c.yp.w, c.yp.s, c.ym.w, yn.w, nuy, op.lim, G);
    if (op.trans) {
        const T cB = R0.c, cA = R1.c, inv = c.yp.inv;
        T d[3], o[3];
        // the x-fluctuations of (col, j + 1) going down ...
        lsw_tsplit(1, &xn.w[3], cB, cA, inv, true, o);
        sub_scaled(G, hx, o);
#pragma unroll
        for (int k = 0; k < 3; ++k) d[k] = from_right(xn.w[k]);
        lsw_tsplit(1, d, cB, cA, inv, true, o);
        sub_scaled(G, hx, o);
        // ... and those of (col, j) going up
        lsw_tsplit(1, &c.xe.w[3], cA, cB, inv, false, o);
        sub_scaled(G, hx, o);
        lsw_tsplit(1, am, cA, cB, inv, false, o);
        sub_scaled(G, hx, o);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T Fr = from_right(F[k]);
        T v = R0.q[k];
        v = v - nux * (c.xe.w[3 + k] + am[k]);
        v = v - nuy * (c.ym.w[3 + k] + c.yp.w[k]);
        v = v - nux * (Fr - F[k]);
        v = v - nuy * (G[k] - c.Gp[k]);
        qn[k] = v;
    }
    c.ym = c.yp;
    c.yp = yn;
    c.xe = xn;
#pragma unroll
    for (int k = 0; k < 3; ++k) c.Gp[k] = G[k];
}

template <typename T, int RT>
__global__ __launch_bounds__(WAVE) void lswe_adj_kernel(const LsweInst<T> *__restrict__ inst,
                                                        const Tile *__restrict__ tiles, int parity, int snap_index,
                                                        int *__restrict__ status)
{
    const Tile tl = tiles[blockIdx.x];
    const LsweInst<T> &I = *inst;
    const int lane = threadIdx.x;
    const int nx = I.nx, ny = I.ny;
    const unsigned cells = (unsigned)nx * (unsigned)ny;
    const unsigned csb = cells * (unsigned)sizeof(T);
    const __amdgpu_buffer_rsrc_t qr = make_rsrc(I.q[parity], 3u * csb);
    const __amdgpu_buffer_rsrc_t cr = make_rsrc(I.cbar, csb);
    const __amdgpu_buffer_rsrc_t qw = make_rsrc(I.q[parity ^ 1], 3u * csb);
    // the snapshot store has an empty range when no snapshot is taken
    const bool snap = snap_index >= 0;
    const __amdgpu_buffer_rsrc_t sw =
        make_rsrc(snap ? (const void *)(I.snap + (long long)snap_index * I.snap_stride) : (const void *)I.q[0],
                  snap ? 3u * csb : 0u);
    const T nux = I.nux, nuy = I.nuy;
    const SOpts op{I.order >= 2, I.transverse != 0, I.limiter};
    const int col = tl.i0 - 2 + lane;
    bool fx;
    const int cx = resolve(col, nx, I.bc[0], I.bc[1], fx);
    const T sx = fx ? T(-1) : T(1);
    const Resolver rowres(ny, I.bc[2], I.bc[3]);
    const bool out_lane = lane >= 2 && lane < 2 + tl.ni;
    auto ld = [&](LRow<T> &r, int j) {
        bool fy;
        const int jy = rowres(j, fy);
        const unsigned off = (unsigned)(jy * nx + cx) * (unsigned)sizeof(T);
        r.q[0] = bload(qr, off, T(0), 0u);
        r.q[1] = sx * bload(qr, off, T(0), csb);
        const T gm = bload(qr, off, T(0), 2u * csb);
        r.q[2] = fy ? -gm : gm;
        r.c = bload(cr, off, T(0), 0u);
    };
    const int j0 = tl.j0, j1 = tl.j0 + tl.nj;
    const unsigned nowhere = 3u * csb;
    int bad = 0;
    auto put = [&](int j, bool valid, const T qn[3]) {
        const bool keep = valid && j < j1 && out_lane;
        const unsigned off = keep ? (unsigned)(j * nx + col) * (unsigned)sizeof(T) : nowhere;
#pragma unroll
        for (int k = 0; k < 3; ++k) bstore(qw, off, (unsigned)k * csb, qn[k]);
        if (snap) {   // wave-uniform
#pragma unroll
            for (int k = 0; k < 3; ++k) bstore(sw, off, (unsigned)k * csb, qn[k]);
        }
        bad |= keep & !(isfinite((double)qn[0]) & isfinite((double)qn[1]) & isfinite((double)qn[2]));
    };
    LCarry<T> c;
#pragma unroll
    for (int k = 0; k < 3; ++k) c.Gp[k] = T(0);
    if constexpr (RT > 0) {
        constexpr int NR = RT + 4;
        constexpr int FIRST = 3 + PREFETCH < NR ? 3 + PREFETCH : NR;
        LRow<T> rw[NR];
#pragma unroll
        for (int r = 0; r < FIRST; ++r) ld(rw[r], j0 - 2 + r);
        __builtin_amdgcn_sched_barrier(SCHED_KEEP_LOADS);
        c.ym = lsw_edge<1>(rw[0], rw[1]);
        c.yp = lsw_edge<1>(rw[1], rw[2]);
        c.xe = lsw_edge<0>(shift_left(rw[1]), rw[1]);
#pragma unroll
        for (int it = 0; it <= RT; ++it) {
            if (FIRST + it < NR) {
                ld(rw[FIRST + it], j0 - 2 + FIRST + it);
                __builtin_amdgcn_sched_barrier(SCHED_KEEP_LOADS);
            }
            T qn[3];
            lswe_row(rw[it + 1], rw[it + 2], rw[it + 3], nux, nuy, op, c, qn);
            if (it > 0) put(j0 - 1 + it, true, qn);
        }
    } else {
        LRow<T> R0, R1, X0, X1, X2, a;
        ld(a, j0 - 2);
        ld(R0, j0 - 1);
        ld(R1, j0);
        ld(X0, j0 + 1);
        ld(X1, j0 + 2);
        c.ym = lsw_edge<1>(a, R0);
        c.yp = lsw_edge<1>(R0, R1);
        c.xe = lsw_edge<0>(shift_left(R0), R0);
        for (int j = j0 - 1; j < j1; ++j) {
            ld(X2, j + 4);
            T qn[3];
            lswe_row(R0, R1, X0, nux, nuy, op, c, qn);
            put(j, j >= j0, qn);
            R0 = R1;
            R1 = X0;
            X0 = X1;
            X1 = X2;
        }
    }
    if (__any(bad) && lane == 0) atomicOr(status, ST_NONFINITE);
}

}  // namespace

// compile-time tile heights; others take the runtime march
#define WP_SWE_BY_RT(F) \
    switch (rows) {     \
    case 4: F(4); break; \
    case 8: F(8); break; \
    case 12: F(12); break; \
    default: F(0); break; \
    }

template <typename ETA, typename T>
void launch_swe2d(const SweInst<ETA, T> *inst, const Tile *tiles, int ntiles, int rows, bool full, int parity,
                  int *status, unsigned *cflbits, hipStream_t s)
{
    if (ntiles <= 0) return;
    if constexpr (sizeof(T) == 8) {
        // FP64: the rolling march (about 250 registers, two waves per SIMD)
        // beats the unrolled one (one wave per SIMD)
        if (full)
            hipLaunchKernelGGL((swe2d_kernel<ETA, T, 0, true>), dim3(ntiles), dim3(WAVE), 0, s, inst, tiles, parity,
                               status, cflbits);
        else
            hipLaunchKernelGGL((swe2d_kernel<ETA, T, 0, false>), dim3(ntiles), dim3(WAVE), 0, s, inst, tiles, parity,
                               status, cflbits);
    } else {
        if (!full) rows = 0;
#define WP_L(R)                                                                                                  \
    hipLaunchKernelGGL((swe2d_kernel<ETA, T, R, (R > 0)>), dim3(ntiles), dim3(WAVE), 0, s, inst, tiles, parity, \
                       status, cflbits)
        WP_SWE_BY_RT(WP_L)
#undef WP_L
    }
}

template <typename T>
void launch_lswe_adj2d(const LsweInst<T> *inst, const Tile *tiles, int ntiles, int rows, int parity, int snap_index,
                       int *status, hipStream_t s)
{
    if (ntiles <= 0) return;
#define WP_L(R)                                                                                                   \
    hipLaunchKernelGGL((lswe_adj_kernel<T, R>), dim3(ntiles), dim3(WAVE), 0, s, inst, tiles, parity, snap_index, \
                       status)
    WP_SWE_BY_RT(WP_L)
#undef WP_L
}

template void launch_swe2d<double, double>(const SweInst<double, double> *, const Tile *, int, int, bool, int,
                                           int *, unsigned *, hipStream_t);
template void launch_swe2d<double, float>(const SweInst<double, float> *, const Tile *, int, int, bool, int, int *,
                                          unsigned *, hipStream_t);
template void launch_lswe_adj2d<double>(const LsweInst<double> *, const Tile *, int, int, int, int, int *,
                                        hipStream_t);
template void launch_lswe_adj2d<float>(const LsweInst<float> *, const Tile *, int, int, int, int, int *,
                                       hipStream_t);

}  // namespace wp
