// The inner-product reduction for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops, harnesses that forbid
// hipMalloc): the per-block partial sums live in a fixed device array of the
// library instead of a handle's scratch block.
#include <algorithm>
#include <mutex>

#include "wp_ctx.h"

using namespace wp;

namespace {

constexpr int NOALLOC_BLOCKS = RED_BLOCKS;
constexpr int MAX_DEVICES = 64;

// (sum, correction) of each block of one reduction: 16 KiB per device,
// shared by every call on that device and kept until the process ends
static __device__ __align__(256) double scratch[2 * NOALLOC_BLOCKS];

std::mutex scratch_mu;
double *scratch_addr[MAX_DEVICES] = {};

// Device address of `scratch` on the current device, looked up once per
// device (host code must never pass the array's own name to a kernel: that
// is a host-side stand-in, not a device address).
int scratch_on_current_device(double **out)
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        (void)hipGetLastError();
        return WP_EDEVICE;
    }
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return WP_EDEVICE;
        }
        scratch_addr[dev] = (double *)p;
    }
    *out = scratch_addr[dev];
    return WP_OK;
}

}  // namespace

extern "C" int wp_inner_product_noalloc(const void *a, const void *b, int precision, long long cells, int m, double dA,
                                        double *out, void *stream)
{
    if (!a || !b || !out) return WP_EINVAL;
    if (precision != WP_FP64 && precision != WP_FP32) return WP_EINVAL;
    if (m < 1 || m > 3 || cells < 1 || cells > WP_NOALLOC_MAX_CELLS) return WP_EINVAL;
    double *partials = nullptr;
    int rc;
    if ((rc = scratch_on_current_device(&partials)) != WP_OK) return rc;
    // the block count of wp_functional_value, so that both sum in the same order
    const int nb = (int)std::min<long long>(NOALLOC_BLOCKS, (cells + 255) / 256);
    hipStream_t s = (hipStream_t)stream;
    if (precision == WP_FP64)
        launch_sum_dot<double, double>((const double *)a, cells, (const double *)b, cells, cells, m, partials, nb, out,
                                       s, dA);
    else
        launch_sum_dot<float, float>((const float *)a, cells, (const float *)b, cells, cells, m, partials, nb, out, s,
                                     dA);
    if (hipGetLastError() != hipSuccess) return WP_EDEVICE;
    return WP_OK;
}
