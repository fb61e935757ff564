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
#include "wp_internal.h"

namespace wp {
namespace {

__device__ __forceinline__ int dpp_from_left(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false);   // wave_shr:1
}
__device__ __forceinline__ int dpp_from_right(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false);   // wave_shl:1
}
__device__ __forceinline__ double from_left(double v)
{
    return __hiloint2double(dpp_from_left(__double2hiint(v)), dpp_from_left(__double2loint(v)));
}
__device__ __forceinline__ double from_right(double v)
{
    return __hiloint2double(dpp_from_right(__double2hiint(v)), dpp_from_right(__double2loint(v)));
}
__device__ __forceinline__ float from_left(float v) { return __int_as_float(dpp_from_left(__float_as_int(v))); }
__device__ __forceinline__ float from_right(float v) { return __int_as_float(dpp_from_right(__float_as_int(v))); }
__device__ __forceinline__ int from_left(int v) { return dpp_from_left(v); }
__device__ __forceinline__ int from_right(int v) { return dpp_from_right(v); }

// Ghost index resolution for one direction; i is first clamped to the
// two-cell ghost band.  flip: the normal velocity changes sign (wall).
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

template <typename T, bool ADJ>
__global__ __launch_bounds__(WAVE) void acou2d_kernel(const AcouInst<T> *__restrict__ insts,
                                                      const Tile *__restrict__ tiles, int parity,
                                                      int *__restrict__ status)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile tl = tiles[blockIdx.x];
    const AcouInst<T> I = insts[tl.inst];
    const int lane = threadIdx.x;
    MCon<T> *mc = reinterpret_cast<MCon<T> *>(smem);
    T *pt = reinterpret_cast<T *>(smem + sizeof(MCon<T>) * MAXMAT);
    build_tables(I, mc, pt, lane);
    __syncthreads();

    const T *__restrict__ qp = I.q[parity];
    T *__restrict__ qo = I.q[parity ^ 1];
    const long long cs = I.cs;
    const int nmat = I.nmat;
    const T nux = I.nux, nuy = I.nuy;
    const bool second = I.order >= 2;
    const bool trans = I.transverse != 0;
    const int lim = I.limiter;

    const int col = tl.i0 - 2 + lane;
    bool fx;
    const int cx = resolve(col, I.nx, I.bc[0], I.bc[1], fx);
    const T sx = fx ? T(-1) : T(1);
    const bool out_lane = lane >= 2 && lane < 2 + tl.ni;

    auto load = [&](int j, T &p, T &u, T &v, int &m) {
        bool fy;
        const int jy = resolve(j, I.ny, I.bc[2], I.bc[3], fy);
        const long long idx = (long long)jy * I.nx + cx;
        p = qp[idx];
        u = sx * qp[idx + cs];
        v = (fy ? T(-1) : T(1)) * qp[idx + 2 * cs];
        m = I.mat[idx];
    };
    auto pair = [&](int a, int b) -> const T * { return pt + (a * nmat + b) * 3; };

    const int j0 = tl.j0;
    // rows j0-2 .. j0: prologue for the first (discarded) iteration j = j0-1
    T pA, uA, vA, p0, u0, v0, p1, u1, v1;
    int mA, m0, m1;
    load(j0 - 2, pA, uA, vA, mA);
    load(j0 - 1, p0, u0, v0, m0);
    load(j0, p1, u1, v1, m1);

    // y-edge (j0-3/2): strengths (only a2 is used later)
    T b1m, b2m, b1p, b2p;
    {
        const T *pp = pair(mA, m0);
        solve<T, ADJ>(pA, vA, p0, v0, mc[mA], mc[m0], pp[0], b1m, b2m);
        const T *pq = pair(m0, m1);
        solve<T, ADJ>(p0, v0, p1, v1, mc[m0], mc[m1], pq[0], b1p, b2p);
    }
    // x-edge (col-1/2) on row j0-1
    T a1x0, a2x0;
    int mL0 = from_left(m0);
    {
        const T pl = from_left(p0), ul = from_left(u0);
        const T *pp = pair(mL0, m0);
        solve<T, ADJ>(pl, ul, p0, u0, mc[mL0], mc[m0], pp[0], a1x0, a2x0);
    }
    T Gp_prev = T(0), Gv_prev = T(0);
    int bad = 0;

    for (int j = j0 - 1; j < j0 + tl.nj; ++j) {
        // 1. new row j+2
        T p2, u2, v2;
        int m2;
        load(j + 2, p2, u2, v2, m2);
        // 2. y-edge (j+3/2) between rows j+1 and j+2
        T b1n, b2n;
        {
            const T *pp = pair(m1, m2);
            solve<T, ADJ>(p1, v1, p2, v2, mc[m1], mc[m2], pp[0], b1n, b2n);
        }
        // 3. x-edge (col-1/2) on row j+1
        T a1n, a2n;
        const int mL1 = from_left(m1);
        {
            const T pl = from_left(p1), ul = from_left(u1);
            const T *pp = pair(mL1, m1);
            solve<T, ADJ>(pl, ul, p1, u1, mc[mL1], mc[m1], pp[0], a1n, a2n);
        }
        // 4a. flux correction F at x-edge (col-1/2, j): L = (col-1, j), R = (col, j)
        const T a1r = from_right(a1x0);   // a1 at edge col+1/2 (upwind of wave 1)
        const T a2l = from_left(a2x0);    // a2 at edge col-3/2 (upwind of wave 2)
        const MCon<T> &L = mc[mL0];
        const MCon<T> &C = mc[m0];
        T Fp = T(0), Fu = T(0);
        {
            const T *pp = pair(mL0, m0);
            const T invx = pp[0];
            if (second) {
                const T t1 = limited(a1x0, pp[1] * a1r, lim);
                const T t2 = limited(a2x0, pp[2] * a2l, lim);
                if (!ADJ) {
                    Fp = C.hZx * t2 - L.hZx * t1;
                    Fu = L.hx * t1 + C.hx * t2;
                } else {
                    Fp = C.gx * t2 - L.gx * t1;
                    Fu = -(L.gZx * t1 + C.gZx * t2);
                }
            }
            if (trans) {
                // transverse: y-edge fluctuations of cells (col, j) and (col-1, j),
                // split at this x-edge (up-going from below plus down-going from above)
                const T S = b2m + b1p;
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
        // 4b. flux correction G at y-edge (col, j+1/2): B = (col, j), A = (col, j+1)
        const MCon<T> &A = mc[m1];
        T Gp = T(0), Gv = T(0);
        {
            const T *pp = pair(m0, m1);
            const T invy = pp[0];
            if (second) {
                const T s1 = limited(b1p, pp[1] * b1n, lim);
                const T s2 = limited(b2p, pp[2] * b2m, lim);
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
                const T R0 = a2x0 + a1r, R1 = a2n + a1rn;
                if (!ADJ) {
                    const T UB = C.Khx * invy * R0, UA = A.Khx * invy * R1;
                    Gp -= A.K * UB - C.K * UA;
                    Gv -= A.c * UB + C.c * UA;
                } else {
                    const T UB = C.Zhx * invy * R0, UA = A.Zhx * invy * R1;
                    Gp += C.c * UA - A.c * UB;
                    Gv += A.K * UB + C.K * UA;
                }
            }
        }
        // 4c. update cell (col, j)
        const T Fpr = from_right(Fp), Fur = from_right(Fu);
        T pn, un, vn;
        if (!ADJ) {
            pn = p0 - nux * (C.K * (a2x0 + a1r)) - nuy * (C.K * (b2m + b1p)) - nux * (Fpr - Fp) - nuy * (Gp - Gp_prev);
            un = u0 - nux * (C.c * (a2x0 - a1r)) - nux * (Fur - Fu);
            vn = v0 - nuy * (C.c * (b2m - b1p)) - nuy * (Gv - Gv_prev);
        } else {
            pn = p0 - nux * (a2x0 + a1r) - nuy * (b2m + b1p) - nux * (Fpr - Fp) - nuy * (Gp - Gp_prev);
            un = u0 - nux * (C.Z * (a1r - a2x0)) - nux * (Fur - Fu);
            vn = v0 - nuy * (C.Z * (b1p - b2m)) - nuy * (Gv - Gv_prev);
        }
        if (j >= j0 && out_lane) {
            const long long idx = (long long)j * I.nx + col;
            qo[idx] = pn;
            qo[idx + cs] = un;
            qo[idx + 2 * cs] = vn;
            bad |= !(isfinite(pn) && isfinite(un) && isfinite(vn));
        }
        // 5. rotate
        p0 = p1; u0 = u1; v0 = v1; m0 = m1;
        p1 = p2; u1 = u2; v1 = v2; m1 = m2;
        mL0 = mL1;
        a1x0 = a1n; a2x0 = a2n;
        b2m = b2p;
        b1p = b1n; b2p = b2n;
        Gp_prev = Gp; Gv_prev = Gv;
        (void)b1m;
    }
    if (__any(bad) && lane == 0) atomicOr(status, ST_NONFINITE);
}

// 1D: one thread per cell, the five-cell stencil read straight from memory.
template <typename T, bool ADJ>
__global__ __launch_bounds__(256) void acou1d_kernel(const AcouInst<T> *__restrict__ insts, int parity,
                                                     int *__restrict__ status)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const AcouInst<T> I = insts[0];
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
    for (int k = 0; k < 5; ++k) {
        bool f;
        const int ii = resolve(i - 2 + k, I.nx, I.bc[0], I.bc[1], f);
        p[k] = qp[ii];
        u[k] = (f ? T(-1) : T(1)) * qp[ii + I.cs];
        m[k] = I.mat[ii];
    }
    // edges e = 0..3 between cells (e, e+1) of the stencil: i-3/2 .. i+3/2
    T a1[4], a2[4];
    for (int e = 0; e < 4; ++e) {
        const T *pp = pt + (m[e] * I.nmat + m[e + 1]) * 3;
        solve<T, ADJ>(p[e], u[e], p[e + 1], u[e + 1], mc[m[e]], mc[m[e + 1]], pp[0], a1[e], a2[e]);
    }
    T Fp[2] = {T(0), T(0)}, Fu[2] = {T(0), T(0)};
    if (I.order >= 2) {
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
                   int *status, hipStream_t s)
{
    if (ntiles <= 0) return;
    const size_t sm = acou_smem<T>(nmat_max);
    if (adjoint)
        hipLaunchKernelGGL((acou2d_kernel<T, true>), dim3(ntiles), dim3(WAVE), sm, s, insts, tiles, parity, status);
    else
        hipLaunchKernelGGL((acou2d_kernel<T, false>), dim3(ntiles), dim3(WAVE), sm, s, insts, tiles, parity, status);
}

template <typename T>
void launch_acou1d(const AcouInst<T> *inst_dev, const AcouInst<T> &h, int parity, int adjoint, int *status,
                   hipStream_t s)
{
    const size_t sm = acou_smem<T>(h.nmat);
    const int nb = (h.nx + 255) / 256;
    if (adjoint)
        hipLaunchKernelGGL((acou1d_kernel<T, true>), dim3(nb), dim3(256), sm, s, inst_dev, parity, status);
    else
        hipLaunchKernelGGL((acou1d_kernel<T, false>), dim3(nb), dim3(256), sm, s, inst_dev, parity, status);
}

template void launch_acou2d<double>(const AcouInst<double> *, const Tile *, int, int, int, int, int *, hipStream_t);
template void launch_acou2d<float>(const AcouInst<float> *, const Tile *, int, int, int, int, int *, hipStream_t);
template void launch_acou1d<double>(const AcouInst<double> *, const AcouInst<double> &, int, int, int *,
                                    hipStream_t);
template void launch_acou1d<float>(const AcouInst<float> *, const AcouInst<float> &, int, int, int *, hipStream_t);

}  // namespace wp
