// Adjoint inner-product flag kernel (Davis & LeVeque Sec. 4 and Sec. 5.1.2),
// the two comparison flags of Sec. 5.2.4 and 5.3 (undivided differences,
// sea-surface departure), the Richardson error estimate and its flag (Sec. 1
// and Future Work), and compensated FP64 reductions for the functional J
// (eq. J_general) and the inner-product integral (eq. q_equality / eq. J).
#include <algorithm>

#include "march_common.h"
#include "richardson_level.h"

namespace wp {
namespace {

// FP64 products and sums in the flag measure are rounded exactly as written
// (no contraction), so flags do not depend on instruction selection.
#pragma clang fp contract(off)

// Index and weight of the adjoint-grid cell centres bracketing fine cell i
// when the fine grid refines the adjoint grid by `ratio`; exact for
// power-of-two ratios, clamped at the domain edge.
__device__ __forceinline__ void bracket(int i, int ratio, int N, int &i0, double &w)
{
    if (ratio == 1) {
        i0 = i;
        w = 0.0;
        return;
    }
    const int num = 2 * i + 1 - ratio;
    int f = num >= 0 ? num / (2 * ratio) : -((-num + 2 * ratio - 1) / (2 * ratio));
    f = min(max(f, 0), max(N - 2, 0));
    double ww = (double)(num - 2 * ratio * f) / (double)(2 * ratio);
    w = fmin(fmax(ww, 0.0), 1.0);
    if (N == 1) w = 0.0;
    i0 = f;
}

template <typename TH>
__device__ __forceinline__ double interp(const TH *s, int NX, int NY, int ratio, int i0, double wx, int j0, double wy)
{
    if (ratio == 1) return (double)s[(long long)j0 * NX + i0];
    const int i1 = min(i0 + 1, NX - 1), j1 = min(j0 + 1, NY - 1);
    const double q00 = s[(long long)j0 * NX + i0], q10 = s[(long long)j0 * NX + i1];
    const double q01 = s[(long long)j1 * NX + i0], q11 = s[(long long)j1 * NX + i1];
    const double a = (1.0 - wx) * (1.0 - wy) * q00 + wx * (1.0 - wy) * q10;
    const double b = (1.0 - wx) * wy * q01 + wx * wy * q11;
    return a + b;
}

// One workgroup of 4 waves per flag tile (at most 64 columns x 16 rows):
// lane x takes column i0 + x, wave y rows j0 + y, j0 + y + 4, ...  SAME: the
// level is the adjoint grid itself (no interpolation).
template <typename TQ, typename TH, bool SAME>
__global__ __launch_bounds__(256) void flag_kernel(const TQ *__restrict__ q, long long cs, int nx, int m,
                                                   const TH *__restrict__ snaps, long long sstride, long long hcs,
                                                   int NX, int NY, int ratio, int n_lo, int n_hi, double tol,
                                                   const Tile *__restrict__ tiles, uint8_t *__restrict__ flags,
                                                   unsigned long long *__restrict__ count)
{
    const Tile tl = tiles[blockIdx.x];
    const int x = threadIdx.x & 63, y = threadIdx.x >> 6;
    unsigned long long local = 0;
    if (x < tl.ni) {
        const int i = tl.i0 + x;
        int i0 = i;
        double wx = 0.0;
        if (!SAME) bracket(i, ratio, NX, i0, wx);
        for (int j = tl.j0 + y; j < tl.j0 + tl.nj; j += 4) {
            const long long idx = (long long)j * nx + i;
            int j0 = j;
            double wy = 0.0;
            if (!SAME) bracket(j, ratio, NY, j0, wy);
            double qv[3];
            for (int c = 0; c < m; ++c) qv[c] = (double)q[idx + c * cs];
            double best = 0.0;
            for (int n = n_lo; n <= n_hi; ++n) {
                const TH *sn = snaps + (long long)n * sstride;
                double ip, h;
                h = SAME ? (double)sn[idx] : interp(sn, NX, NY, ratio, i0, wx, j0, wy);
                ip = h * qv[0];
                for (int c = 1; c < m; ++c) {
                    h = SAME ? (double)sn[idx + c * hcs] : interp(sn + c * hcs, NX, NY, ratio, i0, wx, j0, wy);
                    ip = ip + h * qv[c];
                }
                best = fmax(best, fabs(ip));
            }
            const uint8_t f = best > tol ? 1 : 0;
            flags[idx] = f;
            local += f;
        }
    }
    // wave-level sum then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) local += __shfl_down(local, off);
    if ((threadIdx.x & 63) == 0 && local) atomicAdd(count_slot(count), local);
}

__global__ __launch_bounds__(256) void flag_mixed_kernel(const double *__restrict__ eta, const float *__restrict__ hu,
                                                         const float *__restrict__ hv, int nx,
                                                         const float *__restrict__ snaps, long long sstride,
                                                         long long hcs, int NX, int NY, int ratio, int n_lo, int n_hi,
                                                         double tol, const Tile *__restrict__ tiles,
                                                         uint8_t *__restrict__ flags,
                                                         unsigned long long *__restrict__ count)
{
    const Tile tl = tiles[blockIdx.x];
    const int ncell = tl.ni * tl.nj;
    unsigned long long local = 0;
    for (int k = threadIdx.x; k < ncell; k += blockDim.x) {
        const int i = tl.i0 + k % tl.ni, j = tl.j0 + k / tl.ni;
        const long long idx = (long long)j * nx + i;
        const double a = eta[idx], b = hu[idx], c = hv[idx];
        int i0 = i, j0 = j;
        double wx = 0.0, wy = 0.0;
        bracket(i, ratio, NX, i0, wx);
        bracket(j, ratio, NY, j0, wy);
        double best = 0.0;
        for (int n = n_lo; n <= n_hi; ++n) {
            const float *sn = snaps + (long long)n * sstride;
            double ip = interp(sn, NX, NY, ratio, i0, wx, j0, wy) * a;
            ip = ip + interp(sn + hcs, NX, NY, ratio, i0, wx, j0, wy) * b;
            ip = ip + interp(sn + 2 * hcs, NX, NY, ratio, i0, wx, j0, wy) * c;
            best = fmax(best, fabs(ip));
        }
        const uint8_t f = best > tol ? 1 : 0;
        flags[idx] = f;
        local += f;
    }
    for (int off = 32; off > 0; off >>= 1) local += __shfl_down(local, off);
    if ((threadIdx.x & 63) == 0 && local) atomicAdd(count_slot(count), local);
}

// Undivided-difference flag, the comparison criterion of Sec. 5.2.4 ("pressure
// flagging"): d(x) = max over the components k and the four face neighbours
// nb of |q_k(nb) - q_k(x)|; a neighbour across the physical boundary is the
// cell the boundary rule maps it to (extrapolation: the cell itself; wall:
// its mirror with the normal component, 1 along x and 2 along y, negated;
// periodic: the wrapped cell).  Flagged iff d > tol.  Component 0 is of type
// TE, components 1 and 2 of type TU (c2 null for 1D acoustics, which has no
// y-neighbours).  Tiles and threads as flag_kernel.
template <typename TE, typename TU>
__global__ __launch_bounds__(256) void diff_flag_kernel(const TE *__restrict__ c0, const TU *__restrict__ c1,
                                                        const TU *__restrict__ c2, int nx, int ny, int bc0, int bc1,
                                                        int bc2, int bc3, double tol, const Tile *__restrict__ tiles,
                                                        uint8_t *__restrict__ flags,
                                                        unsigned long long *__restrict__ count)
{
    const Tile tl = tiles[blockIdx.x];
    const int x = threadIdx.x & 63, y = threadIdx.x >> 6;
    unsigned long long local = 0;
    if (x < tl.ni) {
        const int i = tl.i0 + x;
        bool fl, fr;
        const int il = march::resolve(i - 1, nx, bc0, bc1, fl);
        const int ir = march::resolve(i + 1, nx, bc0, bc1, fr);
        for (int j = tl.j0 + y; j < tl.j0 + tl.nj; j += 4) {
            const long long row = (long long)j * nx, idx = row + i;
            double d = 0.0;
            auto diff = [&](double nb, double c) { d = fmax(d, fabs(nb - c)); };
            {
                const double c = c0[idx];
                diff(c0[row + il], c);
                diff(c0[row + ir], c);
            }
            {
                const double c = c1[idx];
                const double l = c1[row + il], r = c1[row + ir];
                diff(fl ? -l : l, c);
                diff(fr ? -r : r, c);
            }
            if (c2) {
                const double c = c2[idx];
                diff(c2[row + il], c);
                diff(c2[row + ir], c);
            }
            if (ny > 1) {
                bool fd, fu;
                const long long rd = (long long)march::resolve(j - 1, ny, bc2, bc3, fd) * nx + i;
                const long long ru = (long long)march::resolve(j + 1, ny, bc2, bc3, fu) * nx + i;
                diff(c0[rd], c0[idx]);
                diff(c0[ru], c0[idx]);
                diff(c1[rd], c1[idx]);
                diff(c1[ru], c1[idx]);
                if (c2) {
                    const double c = c2[idx];
                    const double dn = c2[rd], up = c2[ru];
                    diff(fd ? -dn : dn, c);
                    diff(fu ? -up : up, c);
                }
            }
            const uint8_t f = d > tol ? 1 : 0;
            flags[idx] = f;
            local += f;
        }
    }
    for (int off = 32; off > 0; off >>= 1) local += __shfl_down(local, off);
    if ((threadIdx.x & 63) == 0 && local) atomicAdd(count_slot(count), local);
}

// Surface flag, the comparison criterion of Sec. 5.3 ("surface flagging"):
// the sea surface eta = h + B departs from sea level (0) by more than tol.
// Every cell of the path is wet (bathymetry below sea level is required).
template <typename TE>
__global__ __launch_bounds__(256) void surface_flag_kernel(const TE *__restrict__ eta, int nx, double tol,
                                                           const Tile *__restrict__ tiles,
                                                           uint8_t *__restrict__ flags,
                                                           unsigned long long *__restrict__ count)
{
    const Tile tl = tiles[blockIdx.x];
    const int x = threadIdx.x & 63, y = threadIdx.x >> 6;
    unsigned long long local = 0;
    if (x < tl.ni) {
        for (int j = tl.j0 + y; j < tl.j0 + tl.nj; j += 4) {
            const long long idx = (long long)j * nx + tl.i0 + x;
            const uint8_t f = fabs((double)eta[idx]) > tol ? 1 : 0;
            flags[idx] = f;
            local += f;
        }
    }
    for (int off = 32; off > 0; off >>= 1) local += __shfl_down(local, off);
    if ((threadIdx.x & 63) == 0 && local) atomicAdd(count_slot(count), local);
}

// Richardson error estimate (the estimator named in Sec. 1 and in the
// closing Future Work): the 2 x 2 block mean of a fine canvas, summed as
// ((lower-left + lower-right) + (upper-left + upper-right)) / 4 in FP64.
template <typename T>
__global__ __launch_bounds__(256) void coarsen2_kernel(const T *__restrict__ f, long long fcs, int nx,
                                                       T *__restrict__ c, long long ccs, int NX, int NY, int m)
{
    const long long n = (long long)NX * NY;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
        const int I = (int)(k % NX), J = (int)(k / NX);
        const long long a = (long long)(2 * J) * nx + 2 * I;
        for (int q = 0; q < m; ++q) {
            const T *fq = f + q * fcs;
            const double s = ((double)fq[a] + (double)fq[a + 1]) + ((double)fq[a + nx] + (double)fq[a + nx + 1]);
            c[q * ccs + k] = (T)(s * 0.25);
        }
    }
}

// E = (coarse step of 2 dt - block mean of two fine steps) / denom, FP64,
// per coarse cell and component ([m][NY][NX]).
template <typename T>
__global__ __launch_bounds__(256) void richardson_estimate_kernel(const T *__restrict__ coarse, long long ccs,
                                                                  const T *__restrict__ fine, long long fcs, int nx,
                                                                  int NX, int NY, int m, double denom,
                                                                  double *__restrict__ E)
{
    const long long n = (long long)NX * NY;
    for (long long k = blockIdx.x * (long long)blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x) {
        const int I = (int)(k % NX), J = (int)(k / NX);
        const long long a = (long long)(2 * J) * nx + 2 * I;
        for (int q = 0; q < m; ++q) {
            const T *fq = fine + q * fcs;
            const double s = ((double)fq[a] + (double)fq[a + 1]) + ((double)fq[a + nx] + (double)fq[a + nx + 1]);
            E[q * n + k] = ((double)coarse[q * ccs + k] - s * 0.25) / denom;
        }
    }
}

// Flag of a fine cell from its parent's estimate: max_k |E_k| (snaps null),
// or max over snapshots n_lo..n_hi of |qhat_n(x) . E(parent)| with qhat on
// the fine grid (the adjoint grid).  Tiles and threads as flag_kernel.
template <typename TH>
__global__ __launch_bounds__(256) void richardson_flag_kernel(const double *__restrict__ E, int NX, int NY, int m,
                                                              int nx, const TH *__restrict__ snaps, long long sstride,
                                                              long long hcs, int n_lo, int n_hi, double tol,
                                                              const Tile *__restrict__ tiles,
                                                              uint8_t *__restrict__ flags,
                                                              unsigned long long *__restrict__ count)
{
    const Tile tl = tiles[blockIdx.x];
    const int x = threadIdx.x & 63, y = threadIdx.x >> 6;
    const long long nc = (long long)NX * NY;
    unsigned long long local = 0;
    if (x < tl.ni) {
        const int i = tl.i0 + x;
        for (int j = tl.j0 + y; j < tl.j0 + tl.nj; j += 4) {
            const long long idx = (long long)j * nx + i, par = (long long)(j / 2) * NX + i / 2;
            double e[3] = {0.0, 0.0, 0.0};
            for (int c = 0; c < m; ++c) e[c] = E[c * nc + par];
            double best = 0.0;
            if (!snaps) {
                for (int c = 0; c < m; ++c) best = fmax(best, fabs(e[c]));
            } else {
                for (int n = n_lo; n <= n_hi; ++n) {
                    const TH *sn = snaps + (long long)n * sstride;
                    double ip = (double)sn[idx] * e[0];
                    for (int c = 1; c < m; ++c) ip = ip + (double)sn[idx + c * hcs] * e[c];
                    best = fmax(best, fabs(ip));
                }
            }
            const uint8_t f = best > tol ? 1 : 0;
            flags[idx] = f;
            local += f;
        }
    }
    for (int off = 32; off > 0; off >>= 1) local += __shfl_down(local, off);
    if ((threadIdx.x & 63) == 0 && local) atomicAdd(count_slot(count), local);
}

// ---------------------------------------------------------------------------
// compensated reductions
// ---------------------------------------------------------------------------
struct KSum {
    double s, c;
};

__device__ __forceinline__ void kadd(KSum &a, double x)
{
    const double t = a.s + x;
    if (fabs(a.s) >= fabs(x))
        a.c += (a.s - t) + x;
    else
        a.c += (x - t) + a.s;
    a.s = t;
}

__device__ __forceinline__ void kmerge(KSum &a, const KSum &b)
{
    kadd(a, b.s);
    a.c += b.c;
}

template <int NT>
__device__ __forceinline__ KSum block_reduce(KSum v)
{
    __shared__ double ss[NT], sc[NT];
    ss[threadIdx.x] = v.s;
    sc[threadIdx.x] = v.c;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            KSum a{ss[threadIdx.x], sc[threadIdx.x]};
            KSum b{ss[threadIdx.x + w], sc[threadIdx.x + w]};
            kmerge(a, b);
            ss[threadIdx.x] = a.s;
            sc[threadIdx.x] = a.c;
        }
        __syncthreads();
    }
    return KSum{ss[0], sc[0]};
}

template <typename TA>
__global__ __launch_bounds__(256) void sum_indicator_kernel(const TA *__restrict__ a, long long cs, long long n,
                                                            int comp, const uint8_t *__restrict__ ind,
                                                            double *__restrict__ partials)
{
    KSum acc{0.0, 0.0};
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        if (ind[i]) kadd(acc, (double)a[comp * cs + i]);
    KSum r = block_reduce<256>(acc);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = r.s;
        partials[2 * blockIdx.x + 1] = r.c;
    }
}

template <typename TA, typename TB>
__global__ __launch_bounds__(256) void sum_dot_kernel(const TA *__restrict__ a, long long acs,
                                                      const TB *__restrict__ b, long long bcs, long long n, int m,
                                                      double *__restrict__ partials)
{
    KSum acc{0.0, 0.0};
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256)
        for (int c = 0; c < m; ++c) kadd(acc, (double)a[c * acs + i] * (double)b[c * bcs + i]);
    KSum r = block_reduce<256>(acc);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = r.s;
        partials[2 * blockIdx.x + 1] = r.c;
    }
}

__global__ __launch_bounds__(256) void sum_dot_mixed_kernel(const double *__restrict__ eta,
                                                            const float *__restrict__ hu,
                                                            const float *__restrict__ hv, long long cs,
                                                            const float *__restrict__ b, long long bcs, long long n,
                                                            double *__restrict__ partials)
{
    KSum acc{0.0, 0.0};
    for (long long i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        kadd(acc, eta[i] * (double)b[i]);
        kadd(acc, (double)hu[i] * (double)b[bcs + i]);
        kadd(acc, (double)hv[i] * (double)b[2 * bcs + i]);
    }
    KSum r = block_reduce<256>(acc);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = r.s;
        partials[2 * blockIdx.x + 1] = r.c;
    }
}

__global__ __launch_bounds__(256) void finish_kernel(const double *__restrict__ partials, int nb,
                                                     double *__restrict__ out, double scale)
{
    KSum acc{0.0, 0.0};
    for (int i = threadIdx.x; i < nb; i += 256) kmerge(acc, KSum{partials[2 * i], partials[2 * i + 1]});
    KSum r = block_reduce<256>(acc);
    if (threadIdx.x == 0) out[0] = (r.s + r.c) * scale;
}

__global__ void fill_u8_kernel(uint8_t *p, long long n, uint8_t v)
{
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

template <typename TQ, typename TH>
void launch_flag(const TQ *q, long long cs, int nx, int ny, int m, const TH *snaps, long long snap_stride,
                 long long hcs, int NX, int NY, int ratio, int n_lo, int n_hi, double tol, const Tile *tiles,
                 int ntiles, uint8_t *flags, unsigned long long *count, hipStream_t s)
{
    (void)ny;
    if (ntiles <= 0) return;
    if (ratio == 1)
        hipLaunchKernelGGL((flag_kernel<TQ, TH, true>), dim3(ntiles), dim3(256), 0, s, q, cs, nx, m, snaps,
                           snap_stride, hcs, NX, NY, ratio, n_lo, n_hi, tol, tiles, flags, count);
    else
        hipLaunchKernelGGL((flag_kernel<TQ, TH, false>), dim3(ntiles), dim3(256), 0, s, q, cs, nx, m, snaps,
                           snap_stride, hcs, NX, NY, ratio, n_lo, n_hi, tol, tiles, flags, count);
}

void launch_flag_mixed(const double *eta, const float *hu, const float *hv, long long cs, int nx, int ny,
                       const float *snaps, long long snap_stride, long long hcs, int NX, int NY, int ratio, int n_lo,
                       int n_hi, double tol, const Tile *tiles, int ntiles, uint8_t *flags,
                       unsigned long long *count, hipStream_t s)
{
    (void)cs;
    (void)ny;
    if (ntiles <= 0) return;
    hipLaunchKernelGGL(flag_mixed_kernel, dim3(ntiles), dim3(256), 0, s, eta, hu, hv, nx, snaps, snap_stride, hcs, NX,
                       NY, ratio, n_lo, n_hi, tol, tiles, flags, count);
}

template <typename TA>
void launch_sum_indicator(const TA *a, long long cs, long long n, int comp, const uint8_t *ind, double *partials,
                          int nblocks, double *out, hipStream_t s)
{
    hipLaunchKernelGGL((sum_indicator_kernel<TA>), dim3(nblocks), dim3(256), 0, s, a, cs, n, comp, ind, partials);
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(256), 0, s, partials, nblocks, out, 1.0);
}

template <typename TA, typename TB>
void launch_sum_dot(const TA *a, long long acs, const TB *b, long long bcs, long long n, int m, double *partials,
                    int nblocks, double *out, hipStream_t s, double scale)
{
    hipLaunchKernelGGL((sum_dot_kernel<TA, TB>), dim3(nblocks), dim3(256), 0, s, a, acs, b, bcs, n, m, partials);
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(256), 0, s, partials, nblocks, out, scale);
}

void launch_sum_dot_mixed(const double *eta, const float *hu, const float *hv, long long cs, const float *b,
                          long long bcs, long long n, double *partials, int nblocks, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(sum_dot_mixed_kernel, dim3(nblocks), dim3(256), 0, s, eta, hu, hv, cs, b, bcs, n, partials);
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(256), 0, s, partials, nblocks, out, 1.0);
}

template <typename TE, typename TU>
void launch_flag_difference(const TE *c0, const TU *c1, const TU *c2, int nx, int ny, const int *bc, double tol,
                            const Tile *tiles, int ntiles, uint8_t *flags, unsigned long long *count, hipStream_t s)
{
    if (ntiles <= 0) return;
    hipLaunchKernelGGL((diff_flag_kernel<TE, TU>), dim3(ntiles), dim3(256), 0, s, c0, c1, c2, nx, ny, bc[0], bc[1],
                       bc[2], bc[3], tol, tiles, flags, count);
}

template <typename TE>
void launch_flag_surface(const TE *eta, int nx, double tol, const Tile *tiles, int ntiles, uint8_t *flags,
                         unsigned long long *count, hipStream_t s)
{
    if (ntiles <= 0) return;
    hipLaunchKernelGGL((surface_flag_kernel<TE>), dim3(ntiles), dim3(256), 0, s, eta, nx, tol, tiles, flags, count);
}

template <typename T>
void launch_coarsen2(const T *f, long long fcs, int nx, T *c, long long ccs, int NX, int NY, int m, hipStream_t s)
{
    const long long n = (long long)NX * NY;
    if (n <= 0) return;
    const int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL((coarsen2_kernel<T>), dim3(blocks), dim3(256), 0, s, f, fcs, nx, c, ccs, NX, NY, m);
}

template <typename T>
void launch_richardson(const T *coarse, long long ccs, const T *fine, long long fcs, int nx, int NX, int NY, int m,
                       double denom, double *E, const void *snaps, long long sstride, long long hcs, int n_lo,
                       int n_hi, double tol, const Tile *tiles, int ntiles, uint8_t *flags,
                       unsigned long long *count, hipStream_t s)
{
    const long long n = (long long)NX * NY;
    if (n > 0) {
        const int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
        hipLaunchKernelGGL((richardson_estimate_kernel<T>), dim3(blocks), dim3(256), 0, s, coarse, ccs, fine, fcs, nx,
                           NX, NY, m, denom, E);
    }
    if (ntiles <= 0) return;
    hipLaunchKernelGGL((richardson_flag_kernel<T>), dim3(ntiles), dim3(256), 0, s, E, NX, NY, m, nx,
                       (const T *)snaps, sstride, hcs, n_lo, n_hi, tol, tiles, flags, count);
}

__global__ void mask_estimate_kernel(double *__restrict__ E, const uint8_t *__restrict__ valid, long long n, int m)
{
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x)
        if (!valid[c])
            for (int k = 0; k < m; ++k) E[(long long)k * n + c] = 0.0;
}

template <typename T>
void launch_richardson_masked(const T *coarse, long long ccs, const T *fine, long long fcs, int nx, int NX, int NY,
                              int m, double denom, double *E, const uint8_t *valid, double tol, const Tile *tiles,
                              int ntiles, uint8_t *flags, unsigned long long *count, hipStream_t s)
{
    const long long n = (long long)NX * NY;
    if (n > 0) {
        const int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
        hipLaunchKernelGGL((richardson_estimate_kernel<T>), dim3(blocks), dim3(256), 0, s, coarse, ccs, fine, fcs, nx,
                           NX, NY, m, denom, E);
        hipLaunchKernelGGL(mask_estimate_kernel, dim3(blocks), dim3(256), 0, s, E, valid, n, m);
    }
    if (ntiles <= 0) return;
    hipLaunchKernelGGL((richardson_flag_kernel<T>), dim3(ntiles), dim3(256), 0, s, E, NX, NY, m, nx, (const T *)nullptr,
                       0LL, 0LL, 0, -1, tol, tiles, flags, count);
}

__global__ void expand_estimate_kernel(const double *__restrict__ E, int NX, int NY, int m, double *__restrict__ Ef,
                                       int nx, int ny)
{
    const long long n = (long long)nx * ny, nc = (long long)NX * NY;
    for (long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x; c < n; c += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(c % nx), j = (int)(c / nx);
        const long long par = (long long)(j / 2) * NX + i / 2;
        for (int k = 0; k < m; ++k) Ef[(long long)k * n + c] = E[(long long)k * nc + par];
    }
}

void launch_expand_estimate(const double *E, int NX, int NY, int m, double *Ef, int nx, int ny, hipStream_t s)
{
    const long long n = (long long)nx * ny;
    if (n <= 0) return;
    const int blocks = (int)std::min<long long>((n + 255) / 256, 8192);
    hipLaunchKernelGGL(expand_estimate_kernel, dim3(blocks), dim3(256), 0, s, E, NX, NY, m, Ef, nx, ny);
}

void launch_fill_u8(uint8_t *p, long long n, uint8_t v, hipStream_t s)
{
    if (n <= 0) return;
    const long long nb = std::min<long long>((n + 255) / 256, 4096);
    hipLaunchKernelGGL(fill_u8_kernel, dim3((unsigned)nb), dim3(256), 0, s, p, n, v);
}

template void launch_flag<double, double>(const double *, long long, int, int, int, const double *, long long,
                                          long long, int, int, int, int, int, double, const Tile *, int, uint8_t *,
                                          unsigned long long *, hipStream_t);
template void launch_flag<float, float>(const float *, long long, int, int, int, const float *, long long, long long,
                                        int, int, int, int, int, double, const Tile *, int, uint8_t *,
                                        unsigned long long *, hipStream_t);
template void launch_sum_indicator<double>(const double *, long long, long long, int, const uint8_t *, double *, int,
                                           double *, hipStream_t);
template void launch_sum_indicator<float>(const float *, long long, long long, int, const uint8_t *, double *, int,
                                          double *, hipStream_t);
template void launch_sum_dot<double, double>(const double *, long long, const double *, long long, long long, int,
                                             double *, int, double *, hipStream_t, double);
template void launch_sum_dot<float, float>(const float *, long long, const float *, long long, long long, int,
                                           double *, int, double *, hipStream_t, double);

template void launch_flag_difference<double, double>(const double *, const double *, const double *, int, int,
                                                     const int *, double, const Tile *, int, uint8_t *,
                                                     unsigned long long *, hipStream_t);
template void launch_flag_difference<float, float>(const float *, const float *, const float *, int, int, const int *,
                                                   double, const Tile *, int, uint8_t *, unsigned long long *,
                                                   hipStream_t);
template void launch_flag_difference<double, float>(const double *, const float *, const float *, int, int,
                                                    const int *, double, const Tile *, int, uint8_t *,
                                                    unsigned long long *, hipStream_t);
template void launch_flag_surface<double>(const double *, int, double, const Tile *, int, uint8_t *,
                                          unsigned long long *, hipStream_t);
template void launch_flag_surface<float>(const float *, int, double, const Tile *, int, uint8_t *,
                                         unsigned long long *, hipStream_t);

template void launch_coarsen2<double>(const double *, long long, int, double *, long long, int, int, int, hipStream_t);
template void launch_coarsen2<float>(const float *, long long, int, float *, long long, int, int, int, hipStream_t);
template void launch_richardson<double>(const double *, long long, const double *, long long, int, int, int, int,
                                        double, double *, const void *, long long, long long, int, int, double,
                                        const Tile *, int, uint8_t *, unsigned long long *, hipStream_t);
template void launch_richardson<float>(const float *, long long, const float *, long long, int, int, int, int, double,
                                       double *, const void *, long long, long long, int, int, double, const Tile *,
                                       int, uint8_t *, unsigned long long *, hipStream_t);

template void launch_richardson_masked<double>(const double *, long long, const double *, long long, int, int, int,
                                               int, double, double *, const uint8_t *, double, const Tile *, int,
                                               uint8_t *, unsigned long long *, hipStream_t);
template void launch_richardson_masked<float>(const float *, long long, const float *, long long, int, int, int, int,
                                              double, double *, const uint8_t *, double, const Tile *, int, uint8_t *,
                                              unsigned long long *, hipStream_t);

template void launch_flag<double, float>(const double *, long long, int, int, int, const float *, long long,
                                         long long, int, int, int, int, int, double, const Tile *, int, uint8_t *,
                                         unsigned long long *, hipStream_t);

}  // namespace wp
