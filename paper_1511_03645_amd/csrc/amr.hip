// Coarse/fine transfer kernels of the block-structured refinement (Davis &
// LeVeque Sec. 3): ghost cells of a fine level filled from the level below,
// interpolated in space (minmod-limited linear slopes per direction, the
// physical boundary by the boundary rule) and in time (linear between the two
// coarse times), and fine-to-coarse averaging of covered coarse cells.
#include <climits>

#include "wp_internal.h"

namespace wp {
namespace {

#pragma clang fp contract(off)

__device__ __forceinline__ int resolve1(int i, int n, int bclo, int bchi, bool &flip)
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
__device__ __forceinline__ T minmod(T a, T b)
{
    if (a * b <= T(0)) return T(0);
    return copysign(fmin(fabs(a), fabs(b)), a);
}

// Value of plane k of a coarse canvas at (i, j), ghost cells outside the
// domain by the boundary rule; kc is the state component (1 and 2 are the
// velocities or momenta, negated across x and y walls).
template <typename T>
__device__ __forceinline__ T cval(const T *C, int k, int kc, int i, int j, int NX, int NY, const int *bc,
                                  long long cs)
{
    bool fi, fj;
    const int ri = resolve1(i, NX, bc[0], bc[1], fi);
    const int rj = resolve1(j, NY, bc[2], bc[3], fj);
    T v = C[k * cs + (long long)rj * NX + ri];
    if ((fi && kc == 1) || (fj && kc == 2)) v = -v;
    return v;
}

template <typename T>
__device__ __forceinline__ T space(const T *C, int k, int kc, int ic, int jc, T xi, T eta, int NX, int NY,
                                   const int *bc, long long cs)
{
    const T c0 = C[k * cs + (long long)jc * NX + ic];
    const T sx = minmod(cval(C, k, kc, ic + 1, jc, NX, NY, bc, cs) - c0,
                        c0 - cval(C, k, kc, ic - 1, jc, NX, NY, bc, cs));
    const T sy = minmod(cval(C, k, kc, ic, jc + 1, NX, NY, bc, cs) - c0,
                        c0 - cval(C, k, kc, ic, jc - 1, NX, NY, bc, cs));
    return (c0 + xi * sx) + eta * sy;
}

// Components k0 .. k0 + nk - 1 of the state (the canvases point at component
// k0's plane, planes cs apart): all three in one type, or one launch per
// type where the state mixes them (shallow water with eta in FP64).
template <typename T>
__global__ __launch_bounds__(256) void ring_fill_kernel(const int *__restrict__ cells, long long ncells,
                                                        T *__restrict__ fine, int nxf, const T *__restrict__ cold,
                                                        const T *__restrict__ cnew, int NX, int NY, int r, T alpha,
                                                        int bc0, int bc1, int bc2, int bc3, int k0, int nk)
{
    const int bc[4] = {bc0, bc1, bc2, bc3};
    const long long csf = (long long)nxf * (NY * r);
    const long long csc = (long long)NX * NY;
    for (long long n = blockIdx.x * 256LL + threadIdx.x; n < ncells; n += (long long)gridDim.x * 256) {
        const int lin = cells[n];
        const int I = lin % nxf, J = lin / nxf;
        const int ic = I / r, jc = J / r;
        const T xi = (T((I % r)) + T(0.5)) / T(r) - T(0.5);
        const T eta = (T((J % r)) + T(0.5)) / T(r) - T(0.5);
        for (int k = 0; k < nk; ++k) {
            const T a = space(cold, k, k0 + k, ic, jc, xi, eta, NX, NY, bc, csc);
            const T b = space(cnew, k, k0 + k, ic, jc, xi, eta, NX, NY, bc, csc);
            fine[k * csf + lin] = (T(1) - alpha) * a + alpha * b;
        }
    }
}

// The same fill organised by coarse parent: entry e is (linear index of a
// coarse cell, 64-bit mask of its r x r children in the ring, child (ii, jj)
// at bit ii + r jj).  The parent's slopes at both times are formed once and
// every ring child is written from them, with the arithmetic of
// ring_fill_kernel.  fine2 (optional): a second canvas that takes the ring at
// time weight alpha2 from the same slopes (the ring of the next substep, whose
// input canvas the current substep writes only inside the patches).
template <typename T>
__global__ __launch_bounds__(256) void ring_block_kernel(const int *__restrict__ blocks, long long nblocks,
                                                         T *__restrict__ fine, int nxf, const T *__restrict__ cold,
                                                         const T *__restrict__ cnew, int NX, int NY, int r, T alpha,
                                                         int bc0, int bc1, int bc2, int bc3, int k0, int nk,
                                                         T *__restrict__ fine2, T alpha2)
{
    const int bc[4] = {bc0, bc1, bc2, bc3};
    const long long csf = (long long)nxf * (NY * r);
    const long long csc = (long long)NX * NY;
    const bool pow2 = (r & (r - 1)) == 0;
    const int lr = __builtin_ctz((unsigned)r);
    const T inv_r = T(1) / T(r);
    // one thread per (component, parent), component-major: neighbouring
    // lanes take neighbouring parents of one component plane, so their
    // children's stores fall close together
    for (long long w = blockIdx.x * 256LL + threadIdx.x; w < nk * nblocks; w += (long long)gridDim.x * 256) {
        const int k = (int)(w / nblocks), kc = k0 + k;
        const long long n = w - (long long)k * nblocks;
        const int lin = blocks[3 * n];
        const unsigned long long mask =
            (unsigned long long)(unsigned)blocks[3 * n + 1] | ((unsigned long long)(unsigned)blocks[3 * n + 2] << 32);
        const int ic = lin % NX, jc = lin / NX;
        {
            T c0[2], sx[2], sy[2];
            for (int t = 0; t < 2; ++t) {
                const T *C = t == 0 ? cold : cnew;
                c0[t] = C[k * csc + (long long)jc * NX + ic];
                sx[t] = minmod(cval(C, k, kc, ic + 1, jc, NX, NY, bc, csc) - c0[t],
                               c0[t] - cval(C, k, kc, ic - 1, jc, NX, NY, bc, csc));
                sy[t] = minmod(cval(C, k, kc, ic, jc + 1, NX, NY, bc, csc) - c0[t],
                               c0[t] - cval(C, k, kc, ic, jc - 1, NX, NY, bc, csc));
            }
          for (int o = 0; o < (fine2 ? 2 : 1); ++o) {
            T *__restrict__ out = o ? fine2 : fine;
            const T al = o ? alpha2 : alpha;
            auto child = [&](int ii, int jj) {
                // a power-of-two ratio divides exactly as its reciprocal multiplies
                const T xi = (pow2 ? (T(ii) + T(0.5)) * inv_r : (T(ii) + T(0.5)) / T(r)) - T(0.5);
                const T eta = (pow2 ? (T(jj) + T(0.5)) * inv_r : (T(jj) + T(0.5)) / T(r)) - T(0.5);
                const T a = (c0[0] + xi * sx[0]) + eta * sy[0];
                const T v = (c0[1] + xi * sx[1]) + eta * sy[1];
                return (T(1) - al) * a + al * v;
            };
            if (r == 4) {
                // a full row of four children (along a patch's lower or upper
                // edge) goes out as one contiguous 4-element store (aligned:
                // the fine row length and the component stride are multiples
                // of 4 elements, the canvas 256-byte aligned)
                for (int jj = 0; jj < 4; ++jj) {
                    const unsigned rm = (unsigned)(mask >> (4 * jj)) & 0xfu;
                    if (!rm) continue;
                    T *dst = out + k * csf + (long long)(jc * 4 + jj) * nxf + (long long)ic * 4;
                    if (rm == 0xfu) {
                        typedef T T4 __attribute__((ext_vector_type(4)));
                        T4 q;
                        q.x = child(0, jj);
                        q.y = child(1, jj);
                        q.z = child(2, jj);
                        q.w = child(3, jj);
                        *reinterpret_cast<T4 *>(dst) = q;
                    } else {
                        for (int ii = 0; ii < 4; ++ii)
                            if (rm >> ii & 1u) dst[ii] = child(ii, jj);
                    }
                }
            } else {
                for (unsigned long long m = mask; m; m &= m - 1) {
                    const int b = __builtin_ctzll(m);
                    const int ii = pow2 ? (b & (r - 1)) : b % r, jj = pow2 ? (b >> lr) : b / r;
                    out[k * csf + (long long)(jc * r + jj) * nxf + (ic * r + ii)] = child(ii, jj);
                }
            }
          }
        }
    }
}

// ring_block_kernel for ratio 4, with the same arithmetic: the component is
// blockIdx.y (no index division), parents away from the physical boundary
// load their five-point stencils directly, and the child offsets are
// compile-time constants, which keeps the kernel short and its register
// count low.
template <typename T>
__global__ __launch_bounds__(256) void ring_block4_kernel(const int *__restrict__ blocks, int nblocks,
                                                          T *__restrict__ fine, int nxf, const T *__restrict__ cold,
                                                          const T *__restrict__ cnew, int NX, int NY, T alpha,
                                                          int bc0, int bc1, int bc2, int bc3, int k0,
                                                          T *__restrict__ fine2, T alpha2)
{
    const int n = blockIdx.x * 256 + threadIdx.x;
    if (n >= nblocks) return;
    const int k = blockIdx.y, kc = k0 + k;
    const long long csf = (long long)nxf * (NY * 4);
    const long long csc = (long long)NX * NY;
    const int lin = blocks[3 * n];
    const unsigned mask = (unsigned)blocks[3 * n + 1];
    const int jc = lin / NX, ic = lin - jc * NX;
    T c0[2], sx[2], sy[2];
    if (ic > 0 && ic < NX - 1 && jc > 0 && jc < NY - 1) {
        for (int t = 0; t < 2; ++t) {
            const T *C = (t == 0 ? cold : cnew) + k * csc + (long long)jc * NX + ic;
            c0[t] = C[0];
            sx[t] = minmod(C[1] - c0[t], c0[t] - C[-1]);
            sy[t] = minmod(C[NX] - c0[t], c0[t] - C[-NX]);
        }
    } else {
        const int bc[4] = {bc0, bc1, bc2, bc3};
        for (int t = 0; t < 2; ++t) {
            const T *C = t == 0 ? cold : cnew;
            c0[t] = C[k * csc + (long long)jc * NX + ic];
            sx[t] = minmod(cval(C, k, kc, ic + 1, jc, NX, NY, bc, csc) - c0[t],
                           c0[t] - cval(C, k, kc, ic - 1, jc, NX, NY, bc, csc));
            sy[t] = minmod(cval(C, k, kc, ic, jc + 1, NX, NY, bc, csc) - c0[t],
                           c0[t] - cval(C, k, kc, ic, jc - 1, NX, NY, bc, csc));
        }
    }
    typedef T T4 __attribute__((ext_vector_type(4)));
    typedef T T2 __attribute__((ext_vector_type(2)));
    for (int o = 0; o < (fine2 ? 2 : 1); ++o) {
        T *__restrict__ out = o ? fine2 : fine;
        const T al = o ? alpha2 : alpha;
        auto child = [&](int ii, int jj) {
            const T xi = (T(ii) + T(0.5)) * T(0.25) - T(0.5);
            const T eta = (T(jj) + T(0.5)) * T(0.25) - T(0.5);
            const T a = (c0[0] + xi * sx[0]) + eta * sy[0];
            const T v = (c0[1] + xi * sx[1]) + eta * sy[1];
            return (T(1) - al) * a + al * v;
        };
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) {
            const unsigned rm = mask >> (4 * jj) & 0xfu;
            if (!rm) continue;
            // aligned: the fine row length and the component stride are
            // multiples of 4 elements, the canvas 256-byte aligned
            T *dst = out + k * csf + (long long)(jc * 4 + jj) * nxf + (long long)ic * 4;
            if (rm == 0xfu) {
                // a full row of four children (a patch's lower or upper edge)
                *reinterpret_cast<T4 *>(dst) = T4{child(0, jj), child(1, jj), child(2, jj), child(3, jj)};
            } else if (rm == 0x3u) {
                // the two children beside a patch's left edge
                *reinterpret_cast<T2 *>(dst) = T2{child(0, jj), child(1, jj)};
            } else if (rm == 0xcu) {
                // ... or beside its right edge
                *reinterpret_cast<T2 *>(dst + 2) = T2{child(2, jj), child(3, jj)};
            } else {
#pragma unroll
                for (int ii = 0; ii < 4; ++ii)
                    if (rm >> ii & 1u) dst[ii] = child(ii, jj);
            }
        }
    }
}

template <typename T>
__global__ __launch_bounds__(256) void average_kernel(const int *__restrict__ cells, long long ncells,
                                                      const T *__restrict__ fine, int nxf, long long csf,
                                                      T *__restrict__ coarse, int NX, long long csc, int r, int nk)
{
    // the mean as the sum over r^2: a power-of-two ratio's reciprocal
    // multiplies exactly as it divides
    const bool pow2 = (r & (r - 1)) == 0;
    const T inv = T(1) / T(r * r);
    // one thread per (component, coarse cell), component-major
    for (long long w = blockIdx.x * 256LL + threadIdx.x; w < nk * ncells; w += (long long)gridDim.x * 256) {
        const int k = (int)(w / ncells);
        const long long n = w - (long long)k * ncells;
        const int lin = cells[n];
        const int ic = lin % NX, jc = lin / NX;
        T s = T(0);
        if (r == 4) {
            // each row of four children in one aligned vector load, summed
            // in the same order
            typedef T T4 __attribute__((ext_vector_type(4)));
            for (int jj = 0; jj < 4; ++jj) {
                const T4 q = *reinterpret_cast<const T4 *>(fine + k * csf + (long long)(4 * jc + jj) * nxf + 4 * ic);
                s += q.x;
                s += q.y;
                s += q.z;
                s += q.w;
            }
        } else {
            for (int jj = 0; jj < r; ++jj)
                for (int ii = 0; ii < r; ++ii) s += fine[k * csf + (long long)(r * jc + jj) * nxf + (r * ic + ii)];
        }
        coarse[k * csc + lin] = pow2 ? s * inv : s / T(r * r);
    }
}

unsigned grid_for(long long n)
{
    long long b = (n + 255) / 256;
    return (unsigned)std::min<long long>(std::max<long long>(b, 1), 8192);
}

}  // namespace

template <typename T>
void launch_ring_fill(const int *cells, long long ncells, T *fine, int nxf, const T *cold, const T *cnew, int NX,
                      int NY, int r, double alpha, const int *bc, hipStream_t s, int k0, int nk)
{
    if (ncells <= 0) return;
    hipLaunchKernelGGL((ring_fill_kernel<T>), dim3(grid_for(ncells)), dim3(256), 0, s, cells, ncells, fine, nxf, cold,
                       cnew, NX, NY, r, (T)alpha, bc[0], bc[1], bc[2], bc[3], k0, nk);
}

template <typename T>
void launch_ring_fill_blocks(const int *blocks, long long nblocks, T *fine, int nxf, const T *cold, const T *cnew,
                             int NX, int NY, int r, double alpha, const int *bc, hipStream_t s, int k0, int nk,
                             T *fine2, double alpha2)
{
    if (nblocks <= 0) return;
    if (r == 4 && nblocks <= INT_MAX - 255) {
        hipLaunchKernelGGL((ring_block4_kernel<T>), dim3((unsigned)((nblocks + 255) / 256), (unsigned)nk), dim3(256), 0,
                           s, blocks, (int)nblocks, fine, nxf, cold, cnew, NX, NY, (T)alpha, bc[0], bc[1], bc[2],
                           bc[3], k0, fine2, (T)alpha2);
        return;
    }
    hipLaunchKernelGGL((ring_block_kernel<T>), dim3(grid_for(nk * nblocks)), dim3(256), 0, s, blocks, nblocks, fine,
                       nxf, cold, cnew, NX, NY, r, (T)alpha, bc[0], bc[1], bc[2], bc[3], k0, nk, fine2, (T)alpha2);
}

template <typename T>
void launch_average(const int *cells, long long ncells, const T *fine, int nxf, long long csf, T *coarse, int NX,
                    long long csc, int r, hipStream_t s, int nk)
{
    if (ncells <= 0) return;
    hipLaunchKernelGGL((average_kernel<T>), dim3(grid_for((long long)nk * ncells)), dim3(256), 0, s, cells, ncells,
                       fine, nxf, csf, coarse, NX, csc, r, nk);
}

template void launch_ring_fill<double>(const int *, long long, double *, int, const double *, const double *, int,
                                       int, int, double, const int *, hipStream_t, int, int);
template void launch_ring_fill<float>(const int *, long long, float *, int, const float *, const float *, int, int,
                                      int, double, const int *, hipStream_t, int, int);
template void launch_ring_fill_blocks<double>(const int *, long long, double *, int, const double *, const double *,
                                              int, int, int, double, const int *, hipStream_t, int, int, double *,
                                              double);
template void launch_ring_fill_blocks<float>(const int *, long long, float *, int, const float *, const float *, int,
                                             int, int, double, const int *, hipStream_t, int, int, float *, double);
template void launch_average<double>(const int *, long long, const double *, int, long long, double *, int,
                                     long long, int, hipStream_t, int);
template void launch_average<float>(const int *, long long, const float *, int, long long, float *, int, long long,
                                    int, hipStream_t, int);

}  // namespace wp
