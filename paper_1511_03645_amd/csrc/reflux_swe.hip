// Flux bookkeeping at coarse-fine edges (refluxing) of the shallow-water
// hierarchy (Davis & LeVeque Sec. 3 refinement, Sec. 5.3 and eq. swe).
//
// The well-balanced f-wave solver splits the flux difference less the
// bathymetry source, f(Q_R) - f(Q_L) - psi with psi = (0, -g hbar dB, 0)
// along x, into A^-dQ + A^+dQ.  An edge is seen from the cell on either side
// of it as
//     F = fh(Q_left) + A^-dQ + Ftilde   or   F = fh(Q_right) - A^+dQ + Ftilde,
// Ftilde the limited correction flux with the transverse terms, fh the
// physical flux with the hydrostatic pressure of the sea at rest (eta = 0)
// taken out: 1/2 g eta (eta - 2B) in place of 1/2 g h^2.  The two sides
// agree in the mass component, and in all of them on a flat bottom; for a
// lake at rest every term is zero.  A coarse cell next to a finer patch is
// corrected by
//     Q_C += s dt/h (F_coarse - sum F_fine / r^2),
// every flux seen from the coarse cell's side of the edge (for an edge of the
// finer level, from its ghost cell there), so that the composite mass
// changes only through the domain boundary and a lake at rest stays at rest.
// The fluxes are recomputed per edge in FP64 from the canvas a step started
// from, in the order the update of Sec. 3 forms them.
#include "wp_internal.h"

namespace wp {
namespace {

#pragma clang fp contract(off)

// A shallow-water canvas: eta in E, the momenta in T (mixed precision keeps
// eta in FP64), the level's bathymetry in FP64.
template <typename E, typename T>
struct SweView {
    const E *eta;
    const T *hu, *hv;
    const double *B;
    int nx, ny;
    int bc[4];
    double g;
};

__device__ __forceinline__ int sw_resolve(int i, int n, int bclo, int bchi, bool &flip)
{
    flip = false;
    if (i < 0) {
        if (bclo == WP_BC_WALL) { flip = true; return -1 - i; }
        return bclo == WP_BC_PERIODIC ? i + n : 0;
    }
    if (i >= n) {
        if (bchi == WP_BC_WALL) { flip = true; return 2 * n - 1 - i; }
        return bchi == WP_BC_PERIODIC ? i - n : n - 1;
    }
    return i;
}

// State and bathymetry of cell (i, j), ghost cells outside the domain by the
// boundary rule (a wall mirrors the cell with its normal momentum negated).
template <typename E, typename T>
__device__ __forceinline__ void sw_cell(const SweView<E, T> &V, int i, int j, double q[3], double &B)
{
    bool fi, fj;
    const int ri = sw_resolve(i, V.nx, V.bc[0], V.bc[1], fi);
    const int rj = sw_resolve(j, V.ny, V.bc[2], V.bc[3], fj);
    const long long c = (long long)rj * V.nx + ri;
    q[0] = (double)V.eta[c];
    q[1] = (double)V.hu[c];
    q[2] = (double)V.hv[c];
    if (fi) q[1] = -q[1];
    if (fj) q[2] = -q[2];
    B = V.B[c];
}

// Roe averages at the edge between L and R with normal dir: normal and
// tangential velocities, sound speed sqrt(g hbar), hbar, and the depths.
struct Roe {
    double un, ut, c, hbar, hl, hr;
};

__device__ __forceinline__ Roe roe_avg(int dir, const double *ql, const double *qr, double Bl, double Br, double g)
{
    const int n = dir == 0 ? 1 : 2, t = dir == 0 ? 2 : 1;
    Roe a;
    a.hl = ql[0] - Bl;
    a.hr = qr[0] - Br;
    const double sl = sqrt(a.hl), sr = sqrt(a.hr);
    const double unl = ql[n] / a.hl, unr = qr[n] / a.hr, utl = ql[t] / a.hl, utr = qr[t] / a.hr;
    a.hbar = 0.5 * (a.hl + a.hr);
    a.un = (sl * unl + sr * unr) / (sl + sr);
    a.ut = (sl * utl + sr * utr) / (sl + sr);
    a.c = sqrt(g * a.hbar);
    return a;
}

// The edge between L and R along dir: three f-waves w[p] at speeds s[p]
// (u - c, u, u + c) from the flux jump less the source, and the
// fluctuations (a zero-speed wave split evenly).
struct Edge {
    double w[3][3], s[3], am[3], ap[3];
    Roe roe;
};

template <typename E, typename T>
__device__ __forceinline__ Edge sw_edge(const SweView<E, T> &V, int dir, int i, int j)
{
    // the edge whose right/upper cell is (i, j)
    double ql[3], qr[3], Bl, Br;
    sw_cell(V, dir == 0 ? i - 1 : i, dir == 0 ? j : j - 1, ql, Bl);
    sw_cell(V, i, j, qr, Br);
    const int n = dir == 0 ? 1 : 2, t = dir == 0 ? 2 : 1;
    Edge e;
    const Roe a = roe_avg(dir, ql, qr, Bl, Br, V.g);
    e.roe = a;
    // jumps of mass flux, normal momentum flux (with the source, so g hbar
    // d(eta)) and tangential momentum flux
    const double d1 = qr[n] - ql[n];
    const double d2 = (qr[n] * (qr[n] / a.hr) - ql[n] * (ql[n] / a.hl)) + V.g * a.hbar * (qr[0] - ql[0]);
    const double d3 = qr[n] * (qr[t] / a.hr) - ql[n] * (ql[t] / a.hl);
    const double s1 = a.un - a.c, s3 = a.un + a.c;
    const double b1 = ((a.un + a.c) * d1 - d2) / (2.0 * a.c);
    const double b3 = (d2 - (a.un - a.c) * d1) / (2.0 * a.c);
    const double b2 = d3 - a.ut * d1;
    e.w[0][0] = b1;
    e.w[0][n] = b1 * s1;
    e.w[0][t] = b1 * a.ut;
    e.w[1][0] = 0.0;
    e.w[1][n] = 0.0;
    e.w[1][t] = b2;
    e.w[2][0] = b3;
    e.w[2][n] = b3 * s3;
    e.w[2][t] = b3 * a.ut;
    e.s[0] = s1;
    e.s[1] = a.un;
    e.s[2] = s3;
    for (int k = 0; k < 3; ++k) e.am[k] = e.ap[k] = 0.0;
    for (int p = 0; p < 3; ++p)
        for (int k = 0; k < 3; ++k) {
            if (e.s[p] < 0.0) e.am[k] += e.w[p][k];
            else if (e.s[p] > 0.0) e.ap[k] += e.w[p][k];
            else {
                e.am[k] += 0.5 * e.w[p][k];
                e.ap[k] += 0.5 * e.w[p][k];
            }
        }
    return e;
}

__device__ __forceinline__ double sw_mc(double th)
{
    double a = fmin(0.5 * (1.0 + th), 2.0);
    a = fmin(a, 2.0 * th);
    return fmax(0.0, a);
}

__device__ __forceinline__ double sw_limiter(const double *w, const double *wu, int limiter)
{
    if (limiter == 0) return 1.0;
    double a = 0.0, b = 0.0;
    for (int k = 0; k < 3; ++k) {
        a += wu[k] * w[k];
        b += w[k] * w[k];
    }
    if (b == 0.0) return 0.0;
    return sw_mc(a / b);
}

// Split d along tdir with the eigenvectors of the tdir flux Jacobian at the
// Roe state of the edge d came from (normal 1 - tdir): the parts carried by
// negative (bm) and non-negative (bp) speeds vt - c, vt, vt + c.
__device__ __forceinline__ void sw_tsplit(int tdir, const double *d, const Roe &a, double bm[3], double bp[3])
{
    const double vt = a.ut, vo = a.un, c = a.c;
    const int kt = tdir == 0 ? 1 : 2, ko = tdir == 0 ? 2 : 1;
    const double str[3] = {((vt + c) * d[0] - d[kt]) / (2.0 * c), d[ko] - vo * d[0],
                           (d[kt] - (vt - c) * d[0]) / (2.0 * c)};
    const double lam[3] = {vt - c, vt, vt + c};
    double r[3][3];
    r[0][0] = 1.0;
    r[0][kt] = vt - c;
    r[0][ko] = vo;
    r[1][0] = 0.0;
    r[1][kt] = 0.0;
    r[1][ko] = 1.0;
    r[2][0] = 1.0;
    r[2][kt] = vt + c;
    r[2][ko] = vo;
    for (int k = 0; k < 3; ++k) bm[k] = bp[k] = 0.0;
    for (int p = 0; p < 3; ++p)
        for (int k = 0; k < 3; ++k) {
            const double v = lam[p] * str[p] * r[p][k];
            if (lam[p] < 0.0) bm[k] += v;
            else bp[k] += v;
        }
}

// Numerical flux through the edge of dir whose right/upper cell is (ie, je),
// as the cell on side `right` (true: (ie, je); false: the cell before it)
// sees it.  nu: dt/h along dir; nut: dt/h across it.
template <typename E, typename T>
__device__ void sw_edge_flux(const SweView<E, T> &V, int dir, int ie, int je, bool right, double nu, double nut,
                             int order, int limiter, int transverse, double F[3])
{
    const int di = dir == 0 ? 1 : 0, dj = dir == 0 ? 0 : 1;   // along the normal
    const Edge e = sw_edge(V, dir, ie, je);
    for (int k = 0; k < 3; ++k) F[k] = 0.0;
    if (order >= 2) {
        const Edge el = sw_edge(V, dir, ie - di, je - dj), er = sw_edge(V, dir, ie + di, je + dj);
        for (int p = 0; p < 3; ++p) {
            const double *wu = e.s[p] > 0.0 ? el.w[p] : er.w[p];
            const double phi = sw_limiter(e.w[p], wu, limiter);
            const double as = fabs(e.s[p]);
            const double coef = e.s[p] > 0.0 ? 1.0 : (e.s[p] < 0.0 ? -1.0 : 0.0);
            for (int k = 0; k < 3; ++k) F[k] += 0.5 * coef * (1.0 - nu * as) * (phi * e.w[p][k]);
        }
    }
    if (transverse) {
        // the fluctuations of the transverse edges of the two cells beside
        // this edge, split along dir with their own edge's Roe state; the
        // cell before the edge gives its up-going part, the cell after it its
        // down-going part, in the order the update adds them
        const int tdir = 1 - dir;
        const int ti = dir == 0 ? 0 : 1, tj = dir == 0 ? 1 : 0;   // across the normal
        for (int outer = 0; outer < 2; ++outer) {
            for (int inner = 0; inner < 2; ++inner) {
                const int side = dir == 0 ? outer : inner, c = dir == 0 ? inner : outer;
                const int ci = ie - (c == 0 ? di : 0), cj = je - (c == 0 ? dj : 0);
                // side 0: the transverse edge below / left of the cell (its
                // A^+dQ lives in the cell); side 1: above / right (A^-dQ)
                const Edge et = sw_edge(V, tdir, ci + side * ti, cj + side * tj);
                const double *d = side == 0 ? et.ap : et.am;
                double bm[3], bp[3];
                sw_tsplit(dir, d, et.roe, bm, bp);
                const double *part = c == 0 ? bp : bm;
                for (int k = 0; k < 3; ++k) F[k] -= 0.5 * nut * part[k];
            }
        }
    }
    double q[3], B;
    sw_cell(V, right ? ie : ie - di, right ? je : je - dj, q, B);
    const int n = dir == 0 ? 1 : 2, t = dir == 0 ? 2 : 1;
    const double h = q[0] - B;
    double f[3];
    f[0] = q[n];
    f[n] = q[n] * (q[n] / h) + 0.5 * V.g * q[0] * (q[0] - 2.0 * B);
    f[t] = q[n] * (q[t] / h);
    for (int k = 0; k < 3; ++k) F[k] = right ? (f[k] - e.ap[k]) + F[k] : (f[k] + e.am[k]) + F[k];
}

// The flux of sw_edge_flux formed by the eight lanes base .. base + 7 of a
// wave together, every one of them with the same edge: each solves one edge
// of its stencil (part 0 the edge itself, 1 and 2 its neighbours along the
// normal for the limiter, 3 .. 6 the transverse edges, which they also
// split along dir), and part 0 gathers the rest and forms F in the order of
// sw_edge_flux.  Every lane of the wave calls it (it shuffles); on = false
// for lanes without an edge.  F is set on part 0 only.
template <typename E, typename T>
__device__ void sw_edge_flux8(const SweView<E, T> &V, bool on, int part, int dir, int ie, int je, bool right,
                              double nu, double nut, int order, int limiter, int transverse, double F[3])
{
    const int di = dir == 0 ? 1 : 0, dj = dir == 0 ? 0 : 1;   // along the normal
    const int tdir = 1 - dir;
    const int ti = dir == 0 ? 0 : 1, tj = dir == 0 ? 1 : 0;   // across the normal
    // this lane's edge of the stencil
    int edir = dir, ei = ie, ej = je;
    int side = 0, c = 0;
    if (part == 1) {
        ei = ie - di;
        ej = je - dj;
    } else if (part == 2) {
        ei = ie + di;
        ej = je + dj;
    } else if (part >= 3) {
        const int q = part - 3, outer = q >> 1, inner = q & 1;
        side = dir == 0 ? outer : inner;
        c = dir == 0 ? inner : outer;
        const int ci = ie - (c == 0 ? di : 0), cj = je - (c == 0 ? dj : 0);
        edir = tdir;
        ei = ci + side * ti;
        ej = cj + side * tj;
    }
    const bool need = on && part <= 6 && (part == 0 || (part <= 2 ? order >= 2 : transverse != 0));
    Edge e;
    double pay[9];
    for (int k = 0; k < 9; ++k) pay[k] = 0.0;
    if (need) {
        e = sw_edge(V, edir, ei, ej);
        if (part == 1 || part == 2) {
            for (int p = 0; p < 3; ++p)
                for (int k = 0; k < 3; ++k) pay[3 * p + k] = e.w[p][k];
        } else if (part >= 3) {
            // side 0: the transverse edge below / left of the cell (its
            // A^+dQ lives in the cell); side 1: above / right (A^-dQ); the
            // cell before the edge gives its up-going part, the cell after
            // it its down-going part
            double bm[3], bp[3];
            sw_tsplit(dir, side == 0 ? e.ap : e.am, e.roe, bm, bp);
            for (int k = 0; k < 3; ++k) pay[k] = c == 0 ? bp[k] : bm[k];
        }
    }
    const int base = (threadIdx.x & (WAVE - 1)) & ~7;
    double wl[9], wr[9], tp[4][3];
    for (int k = 0; k < 9; ++k) {
        wl[k] = __shfl(pay[k], base + 1);
        wr[k] = __shfl(pay[k], base + 2);
    }
    for (int q = 0; q < 4; ++q)
        for (int k = 0; k < 3; ++k) tp[q][k] = __shfl(pay[k], base + 3 + q);
    if (!on || part != 0) return;
    for (int k = 0; k < 3; ++k) F[k] = 0.0;
    if (order >= 2) {
        for (int p = 0; p < 3; ++p) {
            const double *wu = e.s[p] > 0.0 ? wl + 3 * p : wr + 3 * p;
            const double phi = sw_limiter(e.w[p], wu, limiter);
            const double as = fabs(e.s[p]);
            const double coef = e.s[p] > 0.0 ? 1.0 : (e.s[p] < 0.0 ? -1.0 : 0.0);
            for (int k = 0; k < 3; ++k) F[k] += 0.5 * coef * (1.0 - nu * as) * (phi * e.w[p][k]);
        }
    }
    if (transverse)
        for (int q = 0; q < 4; ++q)
            for (int k = 0; k < 3; ++k) F[k] -= 0.5 * nut * tp[q][k];
    double qc[3], B;
    sw_cell(V, right ? ie : ie - di, right ? je : je - dj, qc, B);
    const int n = dir == 0 ? 1 : 2, t = dir == 0 ? 2 : 1;
    const double h = qc[0] - B;
    double f[3];
    f[0] = qc[n];
    f[n] = qc[n] * (qc[n] / h) + 0.5 * V.g * qc[0] * (qc[0] - 2.0 * B);
    f[t] = qc[n] * (qc[t] / h);
    for (int k = 0; k < 3; ++k) F[k] = right ? (f[k] - e.ap[k]) + F[k] : (f[k] + e.am[k]) + F[k];
}

// Face records as for the adjoint (x = coarse cell, y = axis | (coarse cell
// before the edge) << 1, z, w = the first of the r fine cells beside the
// edge on the fine side).  Each fine edge takes P lanes (8: its stencil's
// solves on lanes of their own, for r up to 8; 1: one lane), the G = 2^lg
// >= r edges of a face consecutive; the edges are seen from their ghost cells
// on the coarse side, and the face's first lane adds their r fluxes to its
// register in edge order.
template <typename E, typename T, int P>
__global__ __launch_bounds__(256) void reflux_swe_fine_kernel(const int4 *__restrict__ faces, int nfaces,
                                                              SweView<E, T> V, int r, int lg, double nux, double nuy,
                                                              int order, int limiter, int transverse, int first,
                                                              double *__restrict__ reg)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int G = 1 << lg;
    const int part = t % P, slot = t / P;
    const int f = slot >> lg, jj = slot & (G - 1);
    const bool on = f < nfaces && jj < r;
    int axis = 0, ie = 0, je = 0;
    bool coarse_before = false;
    if (on) {
        const int4 e = faces[f];
        axis = e.y & 1;
        coarse_before = (e.y >> 1) & 1;
        const int fi = e.z + (axis == 1 ? jj : 0), fj = e.w + (axis == 0 ? jj : 0);
        ie = coarse_before ? fi : fi + (axis == 0 ? 1 : 0);
        je = coarse_before ? fj : fj + (axis == 1 ? 1 : 0);
    }
    double F[3] = {0.0, 0.0, 0.0};
    const double nu = axis == 0 ? nux : nuy, nut = axis == 0 ? nuy : nux;
    if constexpr (P == 8)
        sw_edge_flux8(V, on, part, axis, ie, je, !coarse_before, nu, nut, order, limiter, transverse, F);
    else if (on)
        sw_edge_flux(V, axis, ie, je, !coarse_before, nu, nut, order, limiter, transverse, F);
    const int base = (threadIdx.x & (WAVE - 1)) & ~(G * P - 1);
    double acc[3] = {0.0, 0.0, 0.0};
    const bool lead = f < nfaces && jj == 0 && part == 0;
    if (!first && lead)
        for (int k = 0; k < 3; ++k) acc[k] = reg[3 * f + k];
    for (int q = 0; q < r; ++q)
        for (int k = 0; k < 3; ++k) acc[k] = acc[k] + __shfl(F[k], base + q * P);
    if (lead)
        for (int k = 0; k < 3; ++k) reg[3 * f + k] = acc[k];
}

// Four faces per coarse cell (a cell has at most one face per side), eight
// lanes per face: the lanes of face k recompute its coarse flux from the
// canvas the coarse step started from, and the cell's first lane adds the
// corrections to the current canvas face by face.
template <typename E, typename T>
__global__ __launch_bounds__(256) void reflux_swe_apply_kernel(const int2 *__restrict__ groups, int ngroups,
                                                               const int4 *__restrict__ faces,
                                                               const double *__restrict__ reg, SweView<E, T> old,
                                                               E *__restrict__ eta, T *__restrict__ hu,
                                                               T *__restrict__ hv, int r, double nux, double nuy,
                                                               double dtdx, double dtdy, int order, int limiter,
                                                               int transverse)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int part = t & 7, g = t >> 5, k4 = (t >> 3) & 3;
    int2 grp = make_int2(0, 0);
    int I = 0, J = 0, C = 0;
    if (g < ngroups) {
        grp = groups[g];
        C = faces[grp.x].x;
        I = C % old.nx;
        J = C / old.nx;
    }
    // the coarse edge of face n of the cell, as the cell sees it
    auto coarse_edge = [&](int n, int &axis, int &ie, int &je, bool &right) {
        const int4 e = faces[n];
        axis = e.y & 1;
        const bool before = (e.y >> 1) & 1;
        ie = before ? I + (axis == 0 ? 1 : 0) : I;
        je = before ? J + (axis == 1 ? 1 : 0) : J;
        right = !before;
    };
    const bool on = g < ngroups && k4 < grp.y;
    int axis = 0, ie = 0, je = 0;
    bool right = false;
    if (on) coarse_edge(grp.x + k4, axis, ie, je, right);
    double F[3] = {0.0, 0.0, 0.0};
    sw_edge_flux8(old, on, part, axis, ie, je, right, axis == 0 ? nux : nuy, axis == 0 ? nuy : nux, order, limiter,
                  transverse, F);
    const int base = (threadIdx.x & (WAVE - 1)) & ~31;
    double Fk[4][3];
    for (int q = 0; q < 4; ++q)
        for (int k = 0; k < 3; ++k) Fk[q][k] = __shfl(F[k], base + 8 * q);
    if (g >= ngroups || k4 != 0 || part != 0) return;
    double q[3] = {(double)eta[C], (double)hu[C], (double)hv[C]};
    const double rr = (double)(r * r);
    for (int n = grp.x; n < grp.x + grp.y; ++n) {
        const int4 e = faces[n];
        const int ax = e.y & 1;
        const double sgn = ((e.y >> 1) & 1) ? 1.0 : -1.0;
        double Fn[3];
        if (n - grp.x < 4) {
            for (int k = 0; k < 3; ++k) Fn[k] = Fk[n - grp.x][k];
        } else {
            int a2, i2, j2;
            bool r2;
            coarse_edge(n, a2, i2, j2, r2);
            sw_edge_flux(old, a2, i2, j2, r2, a2 == 0 ? nux : nuy, a2 == 0 ? nuy : nux, order, limiter, transverse,
                         Fn);
        }
        const double h = ax == 0 ? dtdx : dtdy;
        for (int k = 0; k < 3; ++k) q[k] += sgn * h * (Fn[k] - reg[3 * n + k] / rr);
    }
    eta[C] = (E)q[0];
    hu[C] = (T)q[1];
    hv[C] = (T)q[2];
}

template <typename E, typename T>
SweView<E, T> make_swe_view(const void *q, const double *B, int nx, int ny, const int *bc, double g)
{
    const long long cells = (long long)nx * ny;
    SweView<E, T> V;
    V.eta = (const E *)q;
    V.hu = (const T *)((const char *)q + cells * sizeof(E));
    V.hv = V.hu + cells;
    V.B = B;
    V.nx = nx;
    V.ny = ny;
    for (int k = 0; k < 4; ++k) V.bc[k] = bc[k];
    V.g = g;
    return V;
}

template <typename E, typename T>
void fine_launch(const int *faces, int nfaces, const void *q, const double *B, int nx, int ny, const int *bc,
                 double g, int r, double nux, double nuy, int order, int limiter, int transverse, bool first,
                 double *reg, hipStream_t s)
{
    const SweView<E, T> V = make_swe_view<E, T>(q, B, nx, ny, bc, g);
    int lg = 0;
    while ((1 << lg) < r) ++lg;
    // eight lanes per edge while a face's edges fit in one wave
    if (r <= 8) {
        const long long threads = ((long long)nfaces << lg) * 8;
        hipLaunchKernelGGL((reflux_swe_fine_kernel<E, T, 8>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0,
                           s, (const int4 *)faces, nfaces, V, r, lg, nux, nuy, order, limiter, transverse,
                           first ? 1 : 0, reg);
    } else {
        const long long threads = (long long)nfaces << lg;
        hipLaunchKernelGGL((reflux_swe_fine_kernel<E, T, 1>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0,
                           s, (const int4 *)faces, nfaces, V, r, lg, nux, nuy, order, limiter, transverse,
                           first ? 1 : 0, reg);
    }
}

template <typename E, typename T>
void apply_launch(const int *groups, int ngroups, const int *faces, const double *reg, const void *q_old, void *q_cur,
                  const double *B, int nx, int ny, const int *bc, double g, int r, double nux, double nuy, int order,
                  int limiter, int transverse, hipStream_t s)
{
    const SweView<E, T> V = make_swe_view<E, T>(q_old, B, nx, ny, bc, g);
    const long long cells = (long long)nx * ny;
    E *eta = (E *)q_cur;
    T *hu = (T *)((char *)q_cur + cells * sizeof(E));
    hipLaunchKernelGGL((reflux_swe_apply_kernel<E, T>), dim3((unsigned)((32LL * ngroups + 255) / 256)), dim3(256),
                       0, s,
                       (const int2 *)groups, ngroups, (const int4 *)faces, reg, V, eta, hu, hu + cells, r, nux, nuy,
                       nux, nuy, order, limiter, transverse);
}

}  // namespace

void launch_reflux_swe_fine(int precision, const int *faces, int nfaces, const void *fine_old, const double *B,
                            int nx, int ny, const int *bc, double g, int r, double nux, double nuy, int order,
                            int limiter, int transverse, bool first, double *reg, hipStream_t s)
{
    if (nfaces <= 0) return;
    if (precision == WP_FP64)
        fine_launch<double, double>(faces, nfaces, fine_old, B, nx, ny, bc, g, r, nux, nuy, order, limiter,
                                    transverse, first, reg, s);
    else if (precision == WP_MIXED)
        fine_launch<double, float>(faces, nfaces, fine_old, B, nx, ny, bc, g, r, nux, nuy, order, limiter,
                                   transverse, first, reg, s);
    else
        fine_launch<float, float>(faces, nfaces, fine_old, B, nx, ny, bc, g, r, nux, nuy, order, limiter,
                                  transverse, first, reg, s);
}

void launch_reflux_swe_apply(int precision, const int *groups, int ngroups, const int *faces, const double *reg,
                             const void *coarse_old, void *coarse_cur, const double *B, int nx, int ny, const int *bc,
                             double g, int r, double nux, double nuy, int order, int limiter, int transverse,
                             hipStream_t s)
{
    if (ngroups <= 0) return;
    if (precision == WP_FP64)
        apply_launch<double, double>(groups, ngroups, faces, reg, coarse_old, coarse_cur, B, nx, ny, bc, g, r, nux,
                                     nuy, order, limiter, transverse, s);
    else if (precision == WP_MIXED)
        apply_launch<double, float>(groups, ngroups, faces, reg, coarse_old, coarse_cur, B, nx, ny, bc, g, r, nux,
                                    nuy, order, limiter, transverse, s);
    else
        apply_launch<float, float>(groups, ngroups, faces, reg, coarse_old, coarse_cur, B, nx, ny, bc, g, r, nux,
                                   nuy, order, limiter, transverse, s);
}

}  // namespace wp
