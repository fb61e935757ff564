// Flux bookkeeping at coarse-fine edges (refluxing) of the adjoint hierarchy.
// The time-reversed adjoint is solved in f-wave form, which is in
// conservation form (Sec. 3 contrasts it with the forward problem): every
// edge carries one numerical flux
//     F = f(Q_left) + A^-dQ + Ftilde = f(Q_right) - A^+dQ + Ftilde,
// f(q) = -A^T q = -(u/rho, K p, 0) along x and -B^T q = -(v/rho, 0, K p)
// along y (Sec. 2 adjoint equation), A^-dQ + A^+dQ being the flux difference
// and Ftilde the limited correction flux with the transverse terms.  A coarse
// cell next to a finer patch took the coarse flux through the shared edge,
// while the finer level moved the mean of its own fluxes through it over its
// substeps; the correction
//     Q_C += s dt/h (F_coarse - sum F_fine / r^2)
// (s = +1 when C lies left of / below the edge) makes the two agree, so the
// composite sum of a conserved component changes only through the domain
// boundary.  The fluxes are recomputed here, per edge and in FP64, from the
// canvas a step started from (the stencil of one edge: its normal Riemann
// solve, the two upwind solves of the MC limiter, and the four transverse
// solves of the cells on either side), in the order the update of Sec. 3
// forms them.
#include "wp_internal.h"

namespace wp {
namespace {

#pragma clang fp contract(off)

struct Mat64 {
    double Z, c, rho, K;
};

template <typename T>
struct View {
    const T *q;
    const uint8_t *mat;
    long long cs;
    int nx, ny;
    int bc[4];
    const double *mtab;   // [nmat][4]: Z, c, rho, K
};

__device__ __forceinline__ int resolve_idx(int i, int n, int bclo, int bchi, bool &flip)
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

// State and medium of cell (i, j) of a canvas, ghost cells outside the
// domain by the boundary rule (walls mirror with the normal velocity negated).
template <typename T>
__device__ __forceinline__ void cell(const View<T> &V, int i, int j, double q[3], Mat64 &m)
{
    bool fi, fj;
    const int ri = resolve_idx(i, V.nx, V.bc[0], V.bc[1], fi);
    const int rj = resolve_idx(j, V.ny, V.bc[2], V.bc[3], fj);
    const long long c = (long long)rj * V.nx + ri;
    q[0] = (double)V.q[c];
    q[1] = (double)V.q[V.cs + c];
    q[2] = (double)V.q[2 * V.cs + c];
    if (fi) q[1] = -q[1];
    if (fj) q[2] = -q[2];
    const double *t = V.mtab + 4 * V.mat[c];
    m = Mat64{t[0], t[1], t[2], t[3]};
}

// Normal f-wave solve of the reversed adjoint at the edge between L and R
// along dir (0: x, normal velocity u; 1: y, v): the jump of the flux
// (-n/rho, -K p) = b1 (1, Z_L) + b2 (1, -Z_R), at speeds -c_L and +c_R.
__device__ __forceinline__ void fwave(int dir, const double *ql, const double *qr, const Mat64 &L, const Mat64 &R,
                                      double w[2][3], double s[2])
{
    const int n = dir == 0 ? 1 : 2, t = dir == 0 ? 2 : 1;
    const double f1l = -ql[n] / L.rho, f1r = -qr[n] / R.rho;
    const double f2l = -L.K * ql[0], f2r = -R.K * qr[0];
    const double df1 = f1r - f1l, df2 = f2r - f2l;
    const double b1 = (R.Z * df1 + df2) / (L.Z + R.Z);
    const double b2 = (L.Z * df1 - df2) / (L.Z + R.Z);
    w[0][0] = b1;
    w[0][n] = b1 * L.Z;
    w[0][t] = 0.0;
    w[1][0] = b2;
    w[1][n] = -b2 * R.Z;
    w[1][t] = 0.0;
    s[0] = -L.c;
    s[1] = R.c;
}

// Waves of the edge whose right/upper cell is (i, j) along dir.
template <typename T>
__device__ __forceinline__ void edge_waves(const View<T> &V, int dir, int i, int j, double w[2][3], double s[2])
{
    double ql[3], qr[3];
    Mat64 L, R;
    cell(V, dir == 0 ? i - 1 : i, dir == 0 ? j : j - 1, ql, L);
    cell(V, i, j, qr, R);
    fwave(dir, ql, qr, L, R, w, s);
}

__device__ __forceinline__ double mc_phi(double th)
{
    double a = fmin(0.5 * (1.0 + th), 2.0);
    a = fmin(a, 2.0 * th);
    return fmax(0.0, a);
}

__device__ __forceinline__ double limiter_factor(const double *w, const double *wu, int limiter)
{
    if (limiter == 0) return 1.0;
    double a = 0.0, b = 0.0;
    for (int k = 0; k < 3; ++k) {
        a += wu[k] * w[k];
        b += w[k] * w[k];
    }
    if (b == 0.0) return 0.0;
    return mc_phi(a / b);
}

// Transverse split along tdir of a fluctuation d of the cell with media
// (lo, own, hi) on either side of it along tdir: the parts going down
// (bm, speed -c_lo) and up (bp, speed +c_hi).
__device__ __forceinline__ void tsplit(int tdir, const double *d, const Mat64 &lo, const Mat64 &own, const Mat64 &hi,
                                       double bm[3], double bp[3])
{
    const int n = tdir == 0 ? 1 : 2, t = tdir == 0 ? 2 : 1;
    const double gm = (own.Z * d[0] + d[n]) / (lo.Z + own.Z);
    const double gp = (own.Z * d[0] - d[n]) / (own.Z + hi.Z);
    const double sm = -lo.c, sp = hi.c;
    bm[0] = sm * gm;
    bm[n] = sm * gm * lo.Z;
    bm[t] = 0.0;
    bp[0] = sp * gp;
    bp[n] = -sp * gp * hi.Z;
    bp[t] = 0.0;
}

template <typename T>
__device__ __forceinline__ Mat64 medium(const View<T> &V, int i, int j)
{
    double q[3];
    Mat64 m;
    cell(V, i, j, q, m);
    return m;
}

// Numerical flux through the edge of dir whose right/upper cell is (ie, je),
// as the cell on side `right` (true: (ie, je); false: the cell before it)
// sees it.  nu: dt/h along dir; nut: dt/h across it.
template <typename T>
__device__ void edge_flux(const View<T> &V, int dir, int ie, int je, bool right, double nu, double nut, int order,
                          int limiter, int transverse, double F[3])
{
    const int di = dir == 0 ? 1 : 0, dj = dir == 0 ? 0 : 1;   // along the normal
    double w[2][3], s[2];
    edge_waves(V, dir, ie, je, w, s);
    for (int k = 0; k < 3; ++k) F[k] = 0.0;
    if (order >= 2) {
        double wl[2][3], sl[2], wr[2][3], sr[2];
        edge_waves(V, dir, ie - di, je - dj, wl, sl);
        edge_waves(V, dir, ie + di, je + dj, wr, sr);
        for (int p = 0; p < 2; ++p) {
            const double *wu = s[p] > 0.0 ? wl[p] : wr[p];
            const double phi = limiter_factor(w[p], wu, limiter);
            const double as = fabs(s[p]);
            const double coef = s[p] > 0.0 ? 1.0 : (s[p] < 0.0 ? -1.0 : 0.0);
            for (int k = 0; k < 3; ++k) F[k] += 0.5 * coef * (1.0 - nu * as) * (phi * w[p][k]);
        }
    }
    if (transverse) {
        // fluctuations of the transverse edges of the two cells beside this
        // edge, split along dir; the cell before the edge gives its up-going
        // part, the cell after it its down-going part, in the order the
        // update adds them (row by row, x-edges of a row left to right)
        const int tdir = 1 - dir;
        const int ti = dir == 0 ? 0 : 1, tj = dir == 0 ? 1 : 0;   // across the normal
        for (int outer = 0; outer < 2; ++outer) {
            for (int inner = 0; inner < 2; ++inner) {
                const int side = dir == 0 ? outer : inner, c = dir == 0 ? inner : outer;
                // c = 0: the cell before the edge; c = 1: the cell after it
                const int ci = ie - (c == 0 ? di : 0), cj = je - (c == 0 ? dj : 0);
                // side 0: the transverse edge below / left of the cell (its
                // A^+ part lives in the cell); side 1: above / right (A^-)
                double wt[2][3], st[2];
                edge_waves(V, tdir, ci + side * ti, cj + side * tj, wt, st);
                const double *d = side == 0 ? wt[1] : wt[0];
                const Mat64 lo = medium(V, ci - di, cj - dj), own = medium(V, ci, cj), hi = medium(V, ci + di, cj + dj);
                double bm[3], bp[3];
                tsplit(dir, d, lo, own, hi, bm, bp);
                const double *part = c == 0 ? bp : bm;
                for (int k = 0; k < 3; ++k) F[k] -= 0.5 * nut * part[k];
            }
        }
    }
    double q[3];
    Mat64 m;
    const int ci = right ? ie : ie - di, cj = right ? je : je - dj;
    cell(V, ci, cj, q, m);
    double f[3];
    const int n = dir == 0 ? 1 : 2, t = dir == 0 ? 2 : 1;
    f[0] = -q[n] / m.rho;
    f[n] = -m.K * q[0];
    f[t] = 0.0;
    for (int k = 0; k < 3; ++k) F[k] = right ? (f[k] - w[1][k]) + F[k] : (f[k] + w[0][k]) + F[k];
}

// Face record: x = coarse cell (linear index on the coarse canvas), y = axis
// | (s > 0) << 1, z, w = the first of the r fine cells beside the edge (on
// the fine side); the fine cells run along y (axis 0) or x (axis 1).
// G = 2^lg >= r lanes per face: lane jj of a face's group takes its fine
// edge jj, and the group's first lane adds the r fluxes to the register in
// edge order.
template <typename T>
__global__ __launch_bounds__(256) void reflux_fine_kernel(const int4 *__restrict__ faces, int nfaces, View<T> V,
                                                          int r, int lg, double nux, double nuy, int order,
                                                          int limiter, int transverse, int first,
                                                          double *__restrict__ reg)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int G = 1 << lg;
    const int f = t >> lg, jj = t & (G - 1);
    double F[3] = {0.0, 0.0, 0.0};
    if (f < nfaces && jj < r) {
        const int4 e = faces[f];
        const int axis = e.y & 1;
        const bool coarse_before = (e.y >> 1) & 1;   // the coarse cell lies before the edge
        const int fi = e.z + (axis == 1 ? jj : 0), fj = e.w + (axis == 0 ? jj : 0);
        // the fine cell is after the edge when the coarse cell is before it
        const int ie = coarse_before ? fi : fi + (axis == 0 ? 1 : 0);
        const int je = coarse_before ? fj : fj + (axis == 1 ? 1 : 0);
        edge_flux(V, axis, ie, je, coarse_before, axis == 0 ? nux : nuy, axis == 0 ? nuy : nux, order, limiter,
                  transverse, F);
    }
    const int base = (threadIdx.x & (WAVE - 1)) & ~(G - 1);
    double acc[3] = {0.0, 0.0, 0.0};
    if (!first && f < nfaces && jj == 0)
        for (int k = 0; k < 3; ++k) acc[k] = reg[3 * f + k];
    for (int q = 0; q < r; ++q)
        for (int k = 0; k < 3; ++k) acc[k] = acc[k] + __shfl(F[k], base + q);
    if (f < nfaces && jj == 0)
        for (int k = 0; k < 3; ++k) reg[3 * f + k] = acc[k];
}

// Four lanes per coarse cell (groups: first face, count; faces sorted by
// cell; a cell has at most one face per side): lane k recomputes the coarse
// flux of the cell's face k from the canvas the coarse step started from
// (old), and the first lane adds the corrections to the current canvas face
// by face.
template <typename T>
__global__ __launch_bounds__(256) void reflux_apply_kernel(const int2 *__restrict__ groups, int ngroups,
                                                           const int4 *__restrict__ faces,
                                                           const double *__restrict__ reg, View<T> old,
                                                           T *__restrict__ cur, int r, double nux, double nuy,
                                                           double dtdx, double dtdy, int order, int limiter,
                                                           int transverse)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    const int g = t >> 2, k4 = t & 3;
    int2 grp = make_int2(0, 0);
    int I = 0, J = 0, C = 0;
    if (g < ngroups) {
        grp = groups[g];
        C = faces[grp.x].x;
        I = C % old.nx;
        J = C / old.nx;
    }
    // the coarse flux through face n of the cell, as the cell sees it
    auto coarse_flux = [&](int n, double F[3]) {
        const int4 e = faces[n];
        const int axis = e.y & 1;
        const bool before = (e.y >> 1) & 1;
        // the edge after the coarse cell when it lies before it, else the one before it
        const int ie = before ? I + (axis == 0 ? 1 : 0) : I;
        const int je = before ? J + (axis == 1 ? 1 : 0) : J;
        edge_flux(old, axis, ie, je, !before, axis == 0 ? nux : nuy, axis == 0 ? nuy : nux, order, limiter,
                  transverse, F);
    };
    double F[3] = {0.0, 0.0, 0.0};
    if (g < ngroups && k4 < grp.y) coarse_flux(grp.x + k4, F);
    const int base = (threadIdx.x & (WAVE - 1)) & ~3;
    double Fk[4][3];
    for (int q = 0; q < 4; ++q)
        for (int k = 0; k < 3; ++k) Fk[q][k] = __shfl(F[k], base + q);
    if (g >= ngroups || k4 != 0) return;
    double q[3];
    for (int k = 0; k < 3; ++k) q[k] = (double)cur[k * old.cs + C];
    const double rr = (double)(r * r);
    for (int n = grp.x; n < grp.x + grp.y; ++n) {
        const int4 e = faces[n];
        const int axis = e.y & 1;
        const double sgn = ((e.y >> 1) & 1) ? 1.0 : -1.0;
        double Fn[3];
        if (n - grp.x < 4)
            for (int k = 0; k < 3; ++k) Fn[k] = Fk[n - grp.x][k];
        else
            coarse_flux(n, Fn);
        const double h = axis == 0 ? dtdx : dtdy;
        for (int k = 0; k < 3; ++k) q[k] += sgn * h * (Fn[k] - reg[3 * n + k] / rr);
    }
    for (int k = 0; k < 3; ++k) cur[k * old.cs + C] = (T)q[k];
}

template <typename T>
View<T> make_view(const T *q, const uint8_t *mat, int nx, int ny, const int *bc, const double *mtab)
{
    View<T> V;
    V.q = q;
    V.mat = mat;
    V.cs = (long long)nx * ny;
    V.nx = nx;
    V.ny = ny;
    for (int k = 0; k < 4; ++k) V.bc[k] = bc[k];
    V.mtab = mtab;
    return V;
}

}  // namespace

template <typename T>
void launch_reflux_fine(const int *faces, int nfaces, const T *fine_old, const uint8_t *mat, int nx, int ny,
                        const int *bc, const double *mtab64, int r, double nux, double nuy, int order, int limiter,
                        int transverse, bool first, double *reg, hipStream_t s)
{
    if (nfaces <= 0) return;
    const View<T> V = make_view(fine_old, mat, nx, ny, bc, mtab64);
    int lg = 0;
    while ((1 << lg) < r) ++lg;
    const long long threads = (long long)nfaces << lg;
    hipLaunchKernelGGL((reflux_fine_kernel<T>), dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s,
                       (const int4 *)faces, nfaces, V, r, lg, nux, nuy, order, limiter, transverse, first ? 1 : 0,
                       reg);
}

template <typename T>
void launch_reflux_apply(const int *groups, int ngroups, const int *faces, const double *reg, const T *coarse_old,
                         T *coarse_cur, const uint8_t *mat, int nx, int ny, const int *bc, const double *mtab64,
                         int r, double nux, double nuy, int order, int limiter, int transverse, hipStream_t s)
{
    if (ngroups <= 0) return;
    const View<T> V = make_view(coarse_old, mat, nx, ny, bc, mtab64);
    hipLaunchKernelGGL((reflux_apply_kernel<T>), dim3((unsigned)((4LL * ngroups + 255) / 256)), dim3(256), 0, s,
                       (const int2 *)groups,
                       ngroups, (const int4 *)faces, reg, V, coarse_cur, r, nux, nuy, nux, nuy, order, limiter,
                       transverse);
}

template void launch_reflux_fine<double>(const int *, int, const double *, const uint8_t *, int, int, const int *,
                                         const double *, int, double, double, int, int, int, bool, double *,
                                         hipStream_t);
template void launch_reflux_fine<float>(const int *, int, const float *, const uint8_t *, int, int, const int *,
                                        const double *, int, double, double, int, int, int, bool, double *,
                                        hipStream_t);
template void launch_reflux_apply<double>(const int *, int, const int *, const double *, const double *, double *,
                                          const uint8_t *, int, int, const int *, const double *, int, double,
                                          double, int, int, int, hipStream_t);
template void launch_reflux_apply<float>(const int *, int, const int *, const double *, const float *, float *,
                                         const uint8_t *, int, int, const int *, const double *, int, double, double,
                                         int, int, int, hipStream_t);

}  // namespace wp
