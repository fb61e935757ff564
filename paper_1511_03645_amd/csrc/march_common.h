// Device helpers shared by the strip-march kernels (2D acoustics and
// shallow water): lane shifts, wave-uniform values, ghost-index resolution
// and raw buffer access.
#pragma once

#include "wp_internal.h"

namespace wp {
namespace march {

// Lane shifts by one across the whole wave.  The lane without a source (0
// for a shift from the left, 63 from the right) reads 0; those are halo
// columns whose results are never stored, and no stored column depends on
// them.
__device__ __forceinline__ int dpp_from_left(int v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true);   // wave_shr:1
}
__device__ __forceinline__ int dpp_from_right(int v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true);   // wave_shl:1
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

__device__ __forceinline__ double uniform(double v)
{
    return __hiloint2double(__builtin_amdgcn_readfirstlane(__double2hiint(v)),
                            __builtin_amdgcn_readfirstlane(__double2loint(v)));
}
__device__ __forceinline__ float uniform(float v)
{
    return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// The same resolution as an affine map per side, i -> a i + b below 0 and
// above n - 1 (periodic: a = 1; wall: a = -1; extrapolation: a = 0), so that
// a wave-uniform index resolves with selects instead of branches.
struct Resolver {
    int n, alo, blo, ahi, bhi;
    bool flo, fhi;
    __device__ __forceinline__ Resolver(int n_, int bclo, int bchi) : n(n_)
    {
        alo = bclo == WP_BC_PERIODIC ? 1 : (bclo == WP_BC_WALL ? -1 : 0);
        blo = bclo == WP_BC_PERIODIC ? n : (bclo == WP_BC_WALL ? -1 : 0);
        ahi = bchi == WP_BC_PERIODIC ? 1 : (bchi == WP_BC_WALL ? -1 : 0);
        bhi = bchi == WP_BC_PERIODIC ? -n : (bchi == WP_BC_WALL ? 2 * n - 1 : n - 1);
        flo = bclo == WP_BC_WALL;
        fhi = bchi == WP_BC_WALL;
    }
    __device__ __forceinline__ int operator()(int i, bool &flip) const
    {
        i = min(max(i, -2), n + 1);
        const bool below = i < 0, above = i >= n;
        flip = (below & flo) | (above & fhi);
        const int a = below ? alo : (above ? ahi : 1);
        const int b = below ? blo : (above ? bhi : 0);
        return a * i + b;
    }
};

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

// Raw buffer access with 32-bit byte offsets (out-of-range reads return 0,
// out-of-range writes are dropped).
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr int BUF_FLAGS = 0x00020000;   // gfx9-family buffer resource word 3

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *base, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, BUF_FLAGS);
}
__device__ __forceinline__ double bload(__amdgpu_buffer_rsrc_t r, unsigned off, double, unsigned soff)
{
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, soff, 0));
}
__device__ __forceinline__ float bload(__amdgpu_buffer_rsrc_t r, unsigned off, float, unsigned soff)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, soff, 0));
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff, double v)
{
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, soff, 0);
}
__device__ __forceinline__ void bstore(__amdgpu_buffer_rsrc_t r, unsigned off, unsigned soff, float v)
{
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, soff, 0);
}

}  // namespace march
}  // namespace wp
