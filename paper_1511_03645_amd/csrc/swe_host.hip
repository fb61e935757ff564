// Host side of the shallow-water path: bathymetry, descriptors, launches.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "abi_guard.h"
#include "wp_ctx.h"

using namespace wp;

int wp_swe_init(wp_ctx *ctx, const wp_coefficients *coef)
{
    const Level &l0 = ctx->L[0];
    const size_t cells = (size_t)l0.nx * l0.ny;
    double cmax = 0.0;
    for (size_t k = 0; k < cells; ++k) {
        const double B = coef->B[k];
        if (!std::isfinite(B) || !(B < 0.0))
            return wp_fail(ctx, WP_EINVAL, "bathymetry must be below sea level everywhere (no dry cells), cell %zu", k);
        cmax = std::max(cmax, std::sqrt(ctx->prob.g * -B));
    }
    ctx->cmax = cmax;   // linearised speeds about the ocean at rest (adjoint)
    ctx->Bdev = wp_dalloc(ctx, cells * sizeof(double));
    ctx->cbar = wp_dalloc(ctx, cells * ctx->snap_esz());
    if (!ctx->Bdev || !ctx->cbar) return wp_fail(ctx, WP_ENOMEM, "bathymetry");
    if (hipMemcpy(ctx->Bdev, coef->B, cells * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
        return wp_fail(ctx, WP_EDEVICE, "bathymetry upload");
    std::vector<double> c(cells);
    for (size_t k = 0; k < cells; ++k) c[k] = std::sqrt(ctx->prob.g * -coef->B[k]);
    hipError_t e;
    if (ctx->snap_esz() == 8) {
        e = hipMemcpy(ctx->cbar, c.data(), cells * 8, hipMemcpyHostToDevice);
    } else {
        std::vector<float> cf(c.begin(), c.end());
        e = hipMemcpy(ctx->cbar, cf.data(), cells * 4, hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return wp_fail(ctx, WP_EDEVICE, "wave speed upload");
    ctx->L[0].B = (double *)ctx->Bdev;
    // finer levels: each cell takes the value of the level-0 cell containing
    // it until wp_set_bathymetry gives the level's own cell averages
    for (size_t l = 1; l < ctx->L.size(); ++l) {
        Level &lv = ctx->L[l];
        const int r = lv.nx / l0.nx;
        std::vector<double> Bl((size_t)lv.nx * lv.ny);
        for (int j = 0; j < lv.ny; ++j)
            for (int i = 0; i < lv.nx; ++i) Bl[(size_t)j * lv.nx + i] = coef->B[(size_t)(j / r) * l0.nx + i / r];
        lv.B = (double *)wp_dalloc(ctx, Bl.size() * sizeof(double));
        if (!lv.B) return wp_fail(ctx, WP_ENOMEM, "bathymetry of level %zu", l);
        int rc;
        if ((rc = wp_host_copy(ctx, lv.B, Bl.data(), Bl.size() * sizeof(double), true)) != WP_OK) return rc;
    }
    return WP_OK;
}

extern "C" int wp_set_bathymetry(wp_ctx *ctx, int level, const double *B)
{
    WP_ABI_TRY
    if (!ctx) return WP_EINVAL;
    if (ctx->is_acoustics) return wp_fail(ctx, WP_EINVAL, "bathymetry is for shallow water");
    if (level < 1 || level >= (int)ctx->L.size())
        return wp_fail(ctx, WP_EINVAL, "level %d: refined levels 1..%d only", level, (int)ctx->L.size() - 1);
    if (!B) return wp_fail(ctx, WP_EINVAL, "null bathymetry");
    Level &lv = ctx->L[level];
    const size_t cells = (size_t)lv.nx * lv.ny;
    for (size_t k = 0; k < cells; ++k)
        if (!std::isfinite(B[k]) || !(B[k] < 0.0))
            return wp_fail(ctx, WP_EINVAL, "bathymetry must be below sea level everywhere (no dry cells), cell %zu", k);
    return wp_host_copy(ctx, lv.B, B, cells * sizeof(double), true);
    WP_ABI_CATCH(ctx ? &ctx->err : nullptr)
}

int wp_swe_adj_init(wp_ctx *ctx)
{
    (void)ctx;
    return WP_OK;
}

template <typename ETA, typename T>
static int prep_fwd(wp_ctx *ctx, Level &lv, double dt)
{
    SweInst<ETA, T> I;
    memset(&I, 0, sizeof I);
    const size_t cells = (size_t)lv.nx * lv.ny;
    for (int b = 0; b < 2; ++b) {
        char *base = (char *)lv.q[b];
        I.eta[b] = (ETA *)base;
        I.hu[b] = (T *)(base + cells * sizeof(ETA));
        I.hv[b] = (T *)(base + cells * (sizeof(ETA) + sizeof(T)));
    }
    I.B = lv.B;
    I.nx = lv.nx;
    I.ny = lv.ny;
    for (int k = 0; k < 4; ++k) I.bc[k] = ctx->prob.bc[k];
    I.nux = dt / lv.dx;
    I.nuy = dt / lv.dy;
    I.g = ctx->prob.g;
    I.cfl_max = ctx->prob.cfl_max;
    I.order = ctx->prob.order;
    I.limiter = ctx->prob.limiter;
    I.transverse = ctx->prob.transverse;
    if (!lv.inst) lv.inst = wp_dalloc(ctx, 256);
    if (!lv.inst) return wp_fail(ctx, WP_ENOMEM, "instance");
    static_assert(sizeof(I) <= 256, "descriptor size");
    if (hipMemcpy(lv.inst, &I, sizeof I, hipMemcpyHostToDevice) != hipSuccess)
        return wp_fail(ctx, WP_EDEVICE, "instance upload");
    memcpy(lv.inst_host, &I, sizeof I);
    return WP_OK;
}

template <typename T>
static int prep_adj(wp_ctx *ctx, Level &lv, double dt)
{
    LsweInst<T> I;
    memset(&I, 0, sizeof I);
    I.q[0] = (T *)lv.q[0];
    I.q[1] = (T *)lv.q[1];
    I.cbar = (const T *)ctx->cbar;
    I.nx = lv.nx;
    I.ny = lv.ny;
    for (int k = 0; k < 4; ++k) I.bc[k] = ctx->prob.bc[k];
    I.nux = (T)(dt / lv.dx);
    I.nuy = (T)(dt / lv.dy);
    I.g = (T)ctx->prob.g;
    I.order = ctx->prob.order;
    I.limiter = ctx->prob.limiter;
    I.transverse = ctx->prob.transverse;
    I.snap = (T *)lv.snap_base;
    I.snap_stride = (long long)lv.nx * lv.ny * 3;
    if (!lv.inst) lv.inst = wp_dalloc(ctx, 256);
    if (!lv.inst) return wp_fail(ctx, WP_ENOMEM, "instance");
    static_assert(sizeof(I) <= 256, "descriptor size");
    if (hipMemcpy(lv.inst, &I, sizeof I, hipMemcpyHostToDevice) != hipSuccess)
        return wp_fail(ctx, WP_EDEVICE, "instance upload");
    memcpy(lv.inst_host, &I, sizeof I);
    return WP_OK;
}

int wp_swe_prepare(wp_ctx *ctx, Level &lv, double dt)
{
    if (lv.inst && lv.inst_dt == dt && lv.inst_snap == lv.snap_base) return WP_OK;
    const bool adj = &lv == &ctx->adj;
    const bool f64 = ctx->prob.precision == WP_FP64;
    int rc;
    if (adj) rc = f64 ? prep_adj<double>(ctx, lv, dt) : prep_adj<float>(ctx, lv, dt);
    else rc = f64 ? prep_fwd<double, double>(ctx, lv, dt) : prep_fwd<double, float>(ctx, lv, dt);
    if (rc != WP_OK) return rc;
    lv.inst_dt = dt;
    lv.inst_snap = lv.snap_base;
    return WP_OK;
}

int wp_swe_step(wp_ctx *ctx, Level &lv, double dt, int adjoint, hipStream_t s, int snap_index)
{
    int rc;
    if ((rc = wp_swe_prepare(ctx, lv, dt)) != WP_OK) return rc;
    const bool f64 = ctx->prob.precision == WP_FP64;
    // second order, MC limiter and transverse terms: the compile-time march
    const bool full = ctx->prob.order == 2 && ctx->prob.limiter == 1 && ctx->prob.transverse == 1;
    if (adjoint) {
        if (f64)
            launch_lswe_adj2d<double>((const LsweInst<double> *)lv.inst, lv.tiles_dev, lv.ntiles, lv.tile_rows, lv.cur, snap_index,
                                      ctx->status, s);
        else
            launch_lswe_adj2d<float>((const LsweInst<float> *)lv.inst, lv.tiles_dev, lv.ntiles, lv.tile_rows, lv.cur, snap_index,
                                     ctx->status, s);
    } else {
        if (f64)
            launch_swe2d<double, double>((const SweInst<double, double> *)lv.inst, lv.tiles_dev, lv.ntiles, lv.tile_rows, full,
                                         lv.cur, ctx->status, ctx->cflbits, s);
        else
            launch_swe2d<double, float>((const SweInst<double, float> *)lv.inst, lv.tiles_dev, lv.ntiles, lv.tile_rows, full,
                                        lv.cur, ctx->status, ctx->cflbits, s);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return wp_fail(ctx, WP_EDEVICE, "shallow-water launch: %s", hipGetErrorString(e));
    lv.cur ^= 1;
    return WP_OK;
}
