// Entry points whose implementation is pending in this build.
#include "wp_ctx.h"

int wp_fill_coarse_ghosts(wp_ctx *ctx, int, double) { return wp_fail(ctx, WP_EINVAL, "refinement not built"); }
extern "C" int wp_advance(wp_ctx *ctx, int nsteps, double dt0)
{
    if (!ctx) return WP_EINVAL;
    if (ctx->L.size() > 1) return wp_fail(ctx, WP_EINVAL, "refinement not built");
    for (int s = 0; s < nsteps; ++s) {
        int rc = wp_step_patches(ctx, 0, dt0);
        if (rc != WP_OK) return rc;
    }
    return WP_OK;
}
extern "C" int wp_regrid(wp_ctx *ctx, int, const wp_patch *, int, int) { return wp_fail(ctx, WP_EINVAL, "refinement not built"); }
extern "C" int wp_get_patches(const wp_ctx *ctx, int level, wp_patch *out, int cap, int *np)
{
    if (!ctx || level < 0 || level >= (int)ctx->L.size()) return WP_EINVAL;
    const auto &p = ctx->L[level].patches;
    if (np) *np = (int)p.size();
    for (int k = 0; k < (int)p.size() && k < cap; ++k) out[k] = p[k];
    return WP_OK;
}
