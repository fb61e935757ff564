// Shallow-water patch update (Davis & LeVeque Sec. 5.3, eq. swe) with a
// well-balanced f-wave Roe solver, and the time-reversed linearised
// shallow-water adjoint (Sec. 5.3 linearised system, Sec. 2/4 adjoint and
// time reversal), for gfx950.
//
// Layout: one 128-thread workgroup per 16 x 8 output tile.  Phase A loads
// the tile and its two-cell halo into LDS (ghosts resolved by the boundary
// rules); phase B solves every x- and y-edge Riemann problem the tile needs
// once, keeping f-waves, speeds and Roe states in LDS; phase C forms the
// limited correction fluxes with the transverse terms, one thread per edge;
// phase D updates one cell per thread.
//
// Mixed precision (ETA = double, T = float): eta = h + B is stored and
// updated in FP64 and the well-balanced term g hbar d(eta) is formed in FP64,
// so a lake at rest stays exactly at rest and metre-scale waves are not lost
// against 4000 m of depth; the waves, limiter and transverse terms run in
// FP32.
#include "wp_internal.h"

namespace wp {
namespace {

constexpr int TX = SWE_TX, TY = SWE_TY;
constexpr int SX = TX + 4, SY = TY + 4;          // state region with halo
constexpr int NS = SX * SY;
constexpr int EXW = TX + 3, EXH = TY + 2;        // x-edges li in [-1, TX+1], lj in [-1, TY]
constexpr int EYW = TX + 2, EYH = TY + 3;        // y-edges li in [-1, TX],   lj in [-1, TY+1]
constexpr int NEX = EXW * EXH, NEY = EYW * EYH;
constexpr int NT = 128;

__device__ __forceinline__ int sidx(int li, int lj) { return (li + 2) + (lj + 2) * SX; }
__device__ __forceinline__ int exid(int li, int lj) { return (li + 1) + (lj + 1) * EXW; }
__device__ __forceinline__ int eyid(int li, int lj) { return (li + 1) + (lj + 1) * EYW; }

__device__ __forceinline__ int resolve(int i, int n, int bclo, int bchi, bool &flip)
{
    i = min(max(i, -2), n + 1);
    flip = false;
    if (i < 0) {
        if (bclo == WP_BC_PERIODIC) return i + n;
        if (bclo == WP_BC_WALL) { flip = true; return -1 - i; }
        return 0;
    }
    if (i >= n) {
        if (bchi == WP_BC_PERIODIC) return i - n;
        if (bchi == WP_BC_WALL) { flip = true; return 2 * n - 1 - i; }
        return n - 1;
    }
    return i;
}

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
    if (b == T(0)) return T(0);
    return mc_phi(a / b);
}

template <typename T>
__device__ __forceinline__ T sgn(T s) { return s > T(0) ? T(1) : (s < T(0) ? T(-1) : T(0)); }

// Transverse split (constant Roe state) of d along direction tdir with the
// eigen-structure of that direction at Roe state (uh, vh, c): returns the
// part with negative speeds (neg = true) or positive speeds.
template <typename T>
__device__ __forceinline__ void swe_tsplit(int tdir, const T d[3], T uh, T vh, T c, bool neg, T out[3])
{
    const int kt = tdir == 0 ? 1 : 2, ko = tdir == 0 ? 2 : 1;
    const T vt = tdir == 0 ? uh : vh, vo = tdir == 0 ? vh : uh;
    const T inv2c = T(0.5) / c;
    const T g1 = ((vt + c) * d[0] - d[kt]) * inv2c;
    const T g3 = (d[kt] - (vt - c) * d[0]) * inv2c;
    const T g2 = d[ko] - vo * d[0];
    const T l1 = vt - c, l2 = vt, l3 = vt + c;
    T o[3] = {T(0), T(0), T(0)};
    if ((l1 < T(0)) == neg && (neg || l1 >= T(0))) {
        o[0] += l1 * g1; o[kt] += l1 * g1 * (vt - c); o[ko] += l1 * g1 * vo;
    }
    if ((l2 < T(0)) == neg && (neg || l2 >= T(0))) {
        o[ko] += l2 * g2;
    }
    if ((l3 < T(0)) == neg && (neg || l3 >= T(0))) {
        o[0] += l3 * g3; o[kt] += l3 * g3 * (vt + c); o[ko] += l3 * g3 * vo;
    }
    out[0] = o[0]; out[1] = o[1]; out[2] = o[2];
}

template <typename ETA, typename T>
struct SweSmem {
    // the tile state is dead once the edges are solved, so the correction
    // fluxes reuse its space
    union {
        struct {
            ETA eta[NS];
            ETA he[NS];      // h = eta - B in the eta precision
            T h[NS], hu[NS], hv[NS], u[NS], v[NS], sq[NS];
        };
        struct {
            T F[3][(TX + 1) * TY];
            T G[3][TX * (TY + 1)];
        };
    };
    T ex[15][NEX];   // x-edges: waves [9], speeds [3], Roe state (u, v, c) [3]
    T ey[15][NEY];
};

template <typename ETA, typename T>
__device__ __forceinline__ void edge_solve(SweSmem<ETA, T> &S, int dir, int il, int ir, double g, T *dst, int e,
                                           int nedge)
{
    const int n = dir == 0 ? 1 : 2, t = dir == 0 ? 2 : 1;
    const T hl = S.h[il], hr = S.h[ir];
    const T sl = S.sq[il], sr = S.sq[ir];
    const T unl = dir == 0 ? S.u[il] : S.v[il], unr = dir == 0 ? S.u[ir] : S.v[ir];
    const T utl = dir == 0 ? S.v[il] : S.u[il], utr = dir == 0 ? S.v[ir] : S.u[ir];
    const T qnl = dir == 0 ? S.hu[il] : S.hv[il], qnr = dir == 0 ? S.hu[ir] : S.hv[ir];
    const T hbar = T(0.5) * (hl + hr);
    const T un = (sl * unl + sr * unr) / (sl + sr);
    const T ut = (sl * utl + sr * utr) / (sl + sr);
    const T c = sqrt(T(g) * hbar);
    // well-balanced term g hbar d(eta) in the eta precision
    const ETA hbe = ETA(0.5) * (S.he[il] + S.he[ir]);
    const T wb = (T)(ETA(g) * hbe * (S.eta[ir] - S.eta[il]));
    const T d1 = qnr - qnl;
    const T d2 = (qnr * unr - qnl * unl) + wb;
    const T d3 = qnr * utr - qnl * utl;
    const T s1 = un - c, s3 = un + c;
    const T inv2c = T(0.5) / c;
    const T b1 = ((un + c) * d1 - d2) * inv2c;
    const T b3 = (d2 - (un - c) * d1) * inv2c;
    const T b2 = d3 - ut * d1;
    T w[9];
    w[0] = b1; w[n] = b1 * s1; w[t] = b1 * ut;
    w[3] = T(0); w[3 + n] = T(0); w[3 + t] = b2;
    w[6] = b3; w[6 + n] = b3 * s3; w[6 + t] = b3 * ut;
    for (int k = 0; k < 9; ++k) dst[k * nedge + e] = w[k];
    dst[9 * nedge + e] = s1;
    dst[10 * nedge + e] = un;
    dst[11 * nedge + e] = s3;
    dst[12 * nedge + e] = dir == 0 ? un : ut;   // Roe u
    dst[13 * nedge + e] = dir == 0 ? ut : un;   // Roe v
    dst[14 * nedge + e] = c;
}

// fluctuations of an edge: waves with negative speed (neg) or positive speed,
// zero-speed waves split evenly
template <typename T>
__device__ __forceinline__ void fluct(const T *E, int e, int nedge, bool neg, T out[3])
{
    out[0] = out[1] = out[2] = T(0);
    for (int p = 0; p < 3; ++p) {
        const T s = E[(9 + p) * nedge + e];
        const T f = s < T(0) ? (neg ? T(1) : T(0)) : (s > T(0) ? (neg ? T(0) : T(1)) : T(0.5));
        for (int k = 0; k < 3; ++k) out[k] += f * E[(p * 3 + k) * nedge + e];
    }
}

template <typename ETA, typename T>
__global__ __launch_bounds__(NT) void swe2d_kernel(const SweInst<ETA, T> *__restrict__ inst,
                                                   const Tile *__restrict__ tiles, int parity,
                                                   int *__restrict__ status, unsigned *__restrict__ cflbits)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    SweSmem<ETA, T> &S = *reinterpret_cast<SweSmem<ETA, T> *>(smem_raw);
    const Tile tl = tiles[blockIdx.x];
    const SweInst<ETA, T> &I = *inst;
    const ETA *__restrict__ eta = I.eta[parity];
    const T *__restrict__ hu = I.hu[parity];
    const T *__restrict__ hv = I.hv[parity];
    const int nx = I.nx, ny = I.ny;
    const int tid = threadIdx.x;
    int bad = 0;
    // phase A: state with halo
    for (int k = tid; k < NS; k += NT) {
        const int li = k % SX - 2, lj = k / SX - 2;
        bool fx, fy;
        const int gi = resolve(tl.i0 + li, nx, I.bc[0], I.bc[1], fx);
        const int gj = resolve(tl.j0 + lj, ny, I.bc[2], I.bc[3], fy);
        const long long g = (long long)gj * nx + gi;
        const ETA e = eta[g];
        const ETA he = e - (ETA)I.B[g];
        const T h = (T)he;
        const T qu = fx ? -hu[g] : hu[g];
        const T qv = fy ? -hv[g] : hv[g];
        S.eta[k] = e;
        S.he[k] = he;
        S.h[k] = h;
        S.hu[k] = qu;
        S.hv[k] = qv;
        S.u[k] = qu / h;
        S.v[k] = qv / h;
        S.sq[k] = sqrt(h);
        bad |= !(h > T(0));
    }
    __syncthreads();
    // the state of this thread's own output cell, kept for the update
    const int own_li = tid % TX, own_lj = tid / TX;
    const ETA own_eta = S.eta[sidx(own_li, own_lj)];
    const T own_hu = S.hu[sidx(own_li, own_lj)], own_hv = S.hv[sidx(own_li, own_lj)];
    // phase B: edge Riemann problems
    for (int e = tid; e < NEX; e += NT) {
        const int li = e % EXW - 1, lj = e / EXW - 1;
        edge_solve(S, 0, sidx(li - 1, lj), sidx(li, lj), I.g, &S.ex[0][0], e, NEX);
    }
    for (int e = tid; e < NEY; e += NT) {
        const int li = e % EYW - 1, lj = e / EYW - 1;
        edge_solve(S, 1, sidx(li, lj - 1), sidx(li, lj), I.g, &S.ey[0][0], e, NEY);
    }
    __syncthreads();   // state no longer read: the fluxes below overwrite it
    // phase C: correction fluxes
    const T nux = (T)I.nux, nuy = (T)I.nuy;
    const bool second = I.order >= 2, trans = I.transverse != 0;
    T cfl = T(0);
    for (int f = tid; f < (TX + 1) * TY; f += NT) {
        const int li = f % (TX + 1), lj = f / (TX + 1);
        const int e = exid(li, lj);
        const T *E = &S.ex[0][0];
        T F[3] = {T(0), T(0), T(0)};
        for (int p = 0; p < 3; ++p) {
            const T s = E[(9 + p) * NEX + e];
            if (li <= tl.ni && lj < tl.nj) cfl = fmax(cfl, fabs(s) * nux);
            if (!second) continue;
            const int eu = s > T(0) ? exid(li - 1, lj) : exid(li + 1, lj);
            T w[3], wu[3];
            for (int k = 0; k < 3; ++k) { w[k] = E[(p * 3 + k) * NEX + e]; wu[k] = E[(p * 3 + k) * NEX + eu]; }
            const T phi = lim_factor(w, wu, I.limiter);
            const T coef = T(0.5) * sgn(s) * (T(1) - nux * fabs(s));
            for (int k = 0; k < 3; ++k) F[k] += coef * (phi * w[k]);
        }
        if (trans) {
            const T *Y = &S.ey[0][0];
            // y-edge fluctuations of cells (li, lj) and (li-1, lj), split along x
            // with each y-edge's Roe state: A- parts from column li, A+ parts from li-1
            const int ys[4] = {eyid(li, lj), eyid(li, lj + 1), eyid(li - 1, lj), eyid(li - 1, lj + 1)};
            const bool up[4] = {true, false, true, false};    // B+dQ at the lower, B-dQ at the upper y-edge
            const bool neg[4] = {true, true, false, false};
            for (int q = 0; q < 4; ++q) {
                T d[3], o[3];
                fluct(Y, ys[q], NEY, !up[q], d);
                swe_tsplit(0, d, Y[12 * NEY + ys[q]], Y[13 * NEY + ys[q]], Y[14 * NEY + ys[q]], neg[q], o);
                for (int k = 0; k < 3; ++k) F[k] -= T(0.5) * nuy * o[k];
            }
        }
        for (int k = 0; k < 3; ++k) S.F[k][f] = F[k];
    }
    for (int f = tid; f < TX * (TY + 1); f += NT) {
        const int li = f % TX, lj = f / TX;
        const int e = eyid(li, lj);
        const T *E = &S.ey[0][0];
        T G[3] = {T(0), T(0), T(0)};
        for (int p = 0; p < 3; ++p) {
            const T s = E[(9 + p) * NEY + e];
            if (li < tl.ni && lj <= tl.nj) cfl = fmax(cfl, fabs(s) * nuy);
            if (!second) continue;
            const int eu = s > T(0) ? eyid(li, lj - 1) : eyid(li, lj + 1);
            T w[3], wu[3];
            for (int k = 0; k < 3; ++k) { w[k] = E[(p * 3 + k) * NEY + e]; wu[k] = E[(p * 3 + k) * NEY + eu]; }
            const T phi = lim_factor(w, wu, I.limiter);
            const T coef = T(0.5) * sgn(s) * (T(1) - nuy * fabs(s));
            for (int k = 0; k < 3; ++k) G[k] += coef * (phi * w[k]);
        }
        if (trans) {
            const T *X = &S.ex[0][0];
            // x-edge fluctuations of cells (li, lj) and (li, lj-1), split along y
            const int xs[4] = {exid(li, lj), exid(li + 1, lj), exid(li, lj - 1), exid(li + 1, lj - 1)};
            const bool plus[4] = {true, false, true, false};   // A+dQ at the left, A-dQ at the right x-edge
            const bool neg[4] = {true, true, false, false};
            for (int q = 0; q < 4; ++q) {
                T d[3], o[3];
                fluct(X, xs[q], NEX, !plus[q], d);
                swe_tsplit(1, d, X[12 * NEX + xs[q]], X[13 * NEX + xs[q]], X[14 * NEX + xs[q]], neg[q], o);
                for (int k = 0; k < 3; ++k) G[k] -= T(0.5) * nux * o[k];
            }
        }
        for (int k = 0; k < 3; ++k) S.G[k][f] = G[k];
    }
    __syncthreads();
    // phase D: update
    ETA *__restrict__ eta_o = I.eta[parity ^ 1];
    T *__restrict__ hu_o = I.hu[parity ^ 1];
    T *__restrict__ hv_o = I.hv[parity ^ 1];
    static_assert(TX * TY == NT, "one output cell per thread");
    {
        const int li = own_li, lj = own_lj;
        T ap[3], am[3], bp[3], bm[3];
        fluct(&S.ex[0][0], exid(li, lj), NEX, false, ap);
        fluct(&S.ex[0][0], exid(li + 1, lj), NEX, true, am);
        fluct(&S.ey[0][0], eyid(li, lj), NEY, false, bp);
        fluct(&S.ey[0][0], eyid(li, lj + 1), NEY, true, bm);
        const int fl = li + lj * (TX + 1), fr = fl + 1;
        const int gb = li + lj * TX, gt = gb + TX;
        T inc[3];
        for (int k = 0; k < 3; ++k)
            inc[k] = nux * (ap[k] + am[k]) + nuy * (bp[k] + bm[k]) + nux * (S.F[k][fr] - S.F[k][fl]) +
                     nuy * (S.G[k][gt] - S.G[k][gb]);
        if (li < tl.ni && lj < tl.nj) {
            const long long g = (long long)(tl.j0 + lj) * nx + (tl.i0 + li);
            const ETA en = own_eta - (ETA)inc[0];
            const T qun = own_hu - inc[1], qvn = own_hv - inc[2];
            eta_o[g] = en;
            hu_o[g] = qun;
            hv_o[g] = qvn;
            bad |= !(isfinite((double)en) && isfinite((double)qun) && isfinite((double)qvn));
        }
    }
    // reductions: Courant number and failures, one atomic per wave
    for (int off = 32; off > 0; off >>= 1) cfl = fmax(cfl, __shfl_down(cfl, off));
    if ((tid & 63) == 0) {
        const float cf = (float)cfl;
        atomicMax(cflbits, __float_as_uint(cf));
        if ((double)cfl > I.cfl_max) atomicOr(status, ST_CFL);
    }
    if (__any(bad) && (tid & 63) == 0) atomicOr(status, ST_NONFINITE);
}

// ---------------------------------------------------------------------------
// linearised shallow-water adjoint, time reversed, f-wave form
// ---------------------------------------------------------------------------
template <typename T>
struct LswSmem {
    T q[3][NS];
    T c[NS];
    T ex[8][NEX];    // waves [6], speeds [2]
    T ey[8][NEY];
    T F[3][(TX + 1) * TY];
    T G[3][TX * (TY + 1)];
};

// reversed flux -A^T q = (-g hbar mu_n, -eta, 0) split into f-waves
// b1 (c_l, 1) at speed -c_l and b2 (-c_r, 1) at speed +c_r (n: normal momentum)
template <typename T>
__device__ __forceinline__ void lsw_edge(LswSmem<T> &S, int dir, int il, int ir, T g, T *dst, int e, int nedge)
{
    const int n = dir == 0 ? 1 : 2, t = dir == 0 ? 2 : 1;
    const T cl = S.c[il], cr = S.c[ir];
    const T f1l = -(cl * cl) * S.q[n][il], f1r = -(cr * cr) * S.q[n][ir];
    const T f2l = -S.q[0][il], f2r = -S.q[0][ir];
    const T df1 = f1r - f1l, df2 = f2r - f2l;
    const T inv = T(1) / (cl + cr);
    const T b1 = (df1 + cr * df2) * inv;
    const T b2 = (cl * df2 - df1) * inv;
    T w[6];
    w[0] = b1 * cl; w[n] = b1; w[t] = T(0);
    w[3] = -b2 * cr; w[3 + n] = b2; w[3 + t] = T(0);
    for (int k = 0; k < 6; ++k) dst[k * nedge + e] = w[k];
    dst[6 * nedge + e] = -cl;
    dst[7 * nedge + e] = cr;
    (void)g;
}

// transverse split of d living in cell `own` along tdir (n = normal momentum of
// tdir): part into the lo neighbour (neg) or into the hi neighbour
template <typename T>
__device__ __forceinline__ void lsw_tsplit(int tdir, const T d[3], T clo, T cown, T chi, bool neg, T o[3])
{
    const int n = tdir == 0 ? 1 : 2, t = tdir == 0 ? 2 : 1;
    if (neg) {
        const T gm = (d[0] + cown * d[n]) / (clo + cown);
        o[0] = -clo * gm * clo; o[n] = -clo * gm; o[t] = T(0);
    } else {
        const T gp = (cown * d[n] - d[0]) / (cown + chi);
        o[0] = -chi * gp * chi; o[n] = chi * gp; o[t] = T(0);
    }
}

template <typename T>
__device__ __forceinline__ void lfluct(const T *E, int e, int nedge, bool neg, T out[3])
{
    const int p = neg ? 0 : 1;
    for (int k = 0; k < 3; ++k) out[k] = E[(p * 3 + k) * nedge + e];
}

template <typename T>
__global__ __launch_bounds__(NT) void lswe_adj_kernel(const LsweInst<T> *__restrict__ inst,
                                                      const Tile *__restrict__ tiles, int parity, int snap_index,
                                                      int *__restrict__ status)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    LswSmem<T> &S = *reinterpret_cast<LswSmem<T> *>(smem_raw);
    const Tile tl = tiles[blockIdx.x];
    const LsweInst<T> &I = *inst;
    const T *__restrict__ q = I.q[parity];
    const int nx = I.nx, ny = I.ny;
    const long long cs = (long long)nx * ny;
    const int tid = threadIdx.x;
    for (int k = tid; k < NS; k += NT) {
        const int li = k % SX - 2, lj = k / SX - 2;
        bool fx, fy;
        const int gi = resolve(tl.i0 + li, nx, I.bc[0], I.bc[1], fx);
        const int gj = resolve(tl.j0 + lj, ny, I.bc[2], I.bc[3], fy);
        const long long g = (long long)gj * nx + gi;
        S.q[0][k] = q[g];
        S.q[1][k] = fx ? -q[g + cs] : q[g + cs];
        S.q[2][k] = fy ? -q[g + 2 * cs] : q[g + 2 * cs];
        S.c[k] = I.cbar[g];
    }
    __syncthreads();
    for (int e = tid; e < NEX; e += NT) {
        const int li = e % EXW - 1, lj = e / EXW - 1;
        lsw_edge(S, 0, sidx(li - 1, lj), sidx(li, lj), I.g, &S.ex[0][0], e, NEX);
    }
    for (int e = tid; e < NEY; e += NT) {
        const int li = e % EYW - 1, lj = e / EYW - 1;
        lsw_edge(S, 1, sidx(li, lj - 1), sidx(li, lj), I.g, &S.ey[0][0], e, NEY);
    }
    __syncthreads();
    const T nux = I.nux, nuy = I.nuy;
    const bool second = I.order >= 2, trans = I.transverse != 0;
    for (int f = tid; f < (TX + 1) * TY; f += NT) {
        const int li = f % (TX + 1), lj = f / (TX + 1);
        const int e = exid(li, lj);
        const T *E = &S.ex[0][0];
        T F[3] = {T(0), T(0), T(0)};
        if (second)
            for (int p = 0; p < 2; ++p) {
                const T s = E[(6 + p) * NEX + e];
                const int eu = s > T(0) ? exid(li - 1, lj) : exid(li + 1, lj);
                T w[3], wu[3];
                for (int k = 0; k < 3; ++k) { w[k] = E[(p * 3 + k) * NEX + e]; wu[k] = E[(p * 3 + k) * NEX + eu]; }
                const T phi = lim_factor(w, wu, I.limiter);
                const T coef = T(0.5) * sgn(s) * (T(1) - nux * fabs(s));
                for (int k = 0; k < 3; ++k) F[k] += coef * (phi * w[k]);
            }
        if (trans) {
            const T *Y = &S.ey[0][0];
            const T cL = S.c[sidx(li - 1, lj)], cR = S.c[sidx(li, lj)];
            T d[3], o[3];
            // A- parts of the y-fluctuations living in (li, lj)
            lfluct(Y, eyid(li, lj), NEY, false, d);
            lsw_tsplit(0, d, cL, cR, T(0), true, o);
            for (int k = 0; k < 3; ++k) F[k] -= T(0.5) * nuy * o[k];
            lfluct(Y, eyid(li, lj + 1), NEY, true, d);
            lsw_tsplit(0, d, cL, cR, T(0), true, o);
            for (int k = 0; k < 3; ++k) F[k] -= T(0.5) * nuy * o[k];
            // A+ parts of those living in (li-1, lj)
            lfluct(Y, eyid(li - 1, lj), NEY, false, d);
            lsw_tsplit(0, d, T(0), cL, cR, false, o);
            for (int k = 0; k < 3; ++k) F[k] -= T(0.5) * nuy * o[k];
            lfluct(Y, eyid(li - 1, lj + 1), NEY, true, d);
            lsw_tsplit(0, d, T(0), cL, cR, false, o);
            for (int k = 0; k < 3; ++k) F[k] -= T(0.5) * nuy * o[k];
        }
        for (int k = 0; k < 3; ++k) S.F[k][f] = F[k];
    }
    for (int f = tid; f < TX * (TY + 1); f += NT) {
        const int li = f % TX, lj = f / TX;
        const int e = eyid(li, lj);
        const T *E = &S.ey[0][0];
        T G[3] = {T(0), T(0), T(0)};
        if (second)
            for (int p = 0; p < 2; ++p) {
                const T s = E[(6 + p) * NEY + e];
                const int eu = s > T(0) ? eyid(li, lj - 1) : eyid(li, lj + 1);
                T w[3], wu[3];
                for (int k = 0; k < 3; ++k) { w[k] = E[(p * 3 + k) * NEY + e]; wu[k] = E[(p * 3 + k) * NEY + eu]; }
                const T phi = lim_factor(w, wu, I.limiter);
                const T coef = T(0.5) * sgn(s) * (T(1) - nuy * fabs(s));
                for (int k = 0; k < 3; ++k) G[k] += coef * (phi * w[k]);
            }
        if (trans) {
            const T *X = &S.ex[0][0];
            const T cB = S.c[sidx(li, lj - 1)], cA = S.c[sidx(li, lj)];
            T d[3], o[3];
            // B- parts of the x-fluctuations living in (li, lj)
            lfluct(X, exid(li, lj), NEX, false, d);
            lsw_tsplit(1, d, cB, cA, T(0), true, o);
            for (int k = 0; k < 3; ++k) G[k] -= T(0.5) * nux * o[k];
            lfluct(X, exid(li + 1, lj), NEX, true, d);
            lsw_tsplit(1, d, cB, cA, T(0), true, o);
            for (int k = 0; k < 3; ++k) G[k] -= T(0.5) * nux * o[k];
            // B+ parts of those living in (li, lj-1)
            lfluct(X, exid(li, lj - 1), NEX, false, d);
            lsw_tsplit(1, d, T(0), cB, cA, false, o);
            for (int k = 0; k < 3; ++k) G[k] -= T(0.5) * nux * o[k];
            lfluct(X, exid(li + 1, lj - 1), NEX, true, d);
            lsw_tsplit(1, d, T(0), cB, cA, false, o);
            for (int k = 0; k < 3; ++k) G[k] -= T(0.5) * nux * o[k];
        }
        for (int k = 0; k < 3; ++k) S.G[k][f] = G[k];
    }
    __syncthreads();
    T *__restrict__ qo = I.q[parity ^ 1];
    T *__restrict__ sn = snap_index >= 0 ? I.snap + (long long)snap_index * I.snap_stride : nullptr;
    int bad = 0;
    for (int c = tid; c < TX * TY; c += NT) {
        const int li = c % TX, lj = c / TX;
        if (li >= tl.ni || lj >= tl.nj) continue;
        T ap[3], am[3], bp[3], bm[3];
        lfluct(&S.ex[0][0], exid(li, lj), NEX, false, ap);
        lfluct(&S.ex[0][0], exid(li + 1, lj), NEX, true, am);
        lfluct(&S.ey[0][0], eyid(li, lj), NEY, false, bp);
        lfluct(&S.ey[0][0], eyid(li, lj + 1), NEY, true, bm);
        const int fl = li + lj * (TX + 1), fr = fl + 1;
        const int gb = li + lj * TX, gt = gb + TX;
        const int si = sidx(li, lj);
        const long long g = (long long)(tl.j0 + lj) * nx + (tl.i0 + li);
        for (int k = 0; k < 3; ++k) {
            T v = S.q[k][si];
            v = v - nux * (ap[k] + am[k]);
            v = v - nuy * (bp[k] + bm[k]);
            v = v - nux * (S.F[k][fr] - S.F[k][fl]);
            v = v - nuy * (S.G[k][gt] - S.G[k][gb]);
            qo[g + k * cs] = v;
            if (sn) sn[g + k * cs] = v;
            bad |= !isfinite((double)v);
        }
    }
    if (__any(bad) && (tid & 63) == 0) atomicOr(status, ST_NONFINITE);
}

}  // namespace

template <typename ETA, typename T>
void launch_swe2d(const SweInst<ETA, T> *inst, const Tile *tiles, int ntiles, int parity, int *status,
                  unsigned *cflbits, hipStream_t s)
{
    if (ntiles <= 0) return;
    hipLaunchKernelGGL((swe2d_kernel<ETA, T>), dim3(ntiles), dim3(NT), sizeof(SweSmem<ETA, T>), s, inst, tiles,
                       parity, status, cflbits);
}

template <typename T>
void launch_lswe_adj2d(const LsweInst<T> *inst, const Tile *tiles, int ntiles, int parity, int snap_index,
                       int *status, hipStream_t s)
{
    if (ntiles <= 0) return;
    hipLaunchKernelGGL((lswe_adj_kernel<T>), dim3(ntiles), dim3(NT), sizeof(LswSmem<T>), s, inst, tiles, parity,
                       snap_index, status);
}

template void launch_swe2d<double, double>(const SweInst<double, double> *, const Tile *, int, int, int *,
                                           unsigned *, hipStream_t);
template void launch_swe2d<double, float>(const SweInst<double, float> *, const Tile *, int, int, int *, unsigned *,
                                          hipStream_t);
template void launch_lswe_adj2d<double>(const LsweInst<double> *, const Tile *, int, int, int, int *, hipStream_t);
template void launch_lswe_adj2d<float>(const LsweInst<float> *, const Tile *, int, int, int, int *, hipStream_t);

}  // namespace wp
