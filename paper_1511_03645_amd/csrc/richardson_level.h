// The Richardson estimate on a refined level: the estimate and flag launches
// of launch_richardson with a mask between them that clears the estimate of
// the coarse cells whose stencils reach outside the level's patches.
#pragma once

#include "wp_internal.h"

namespace wp {

// valid: NX * NY bytes, 1 where the coarse cell's estimate is kept.
// Unweighted measure only (the snapshots are at level-0 resolution).
template <typename T>
void launch_richardson_masked(const T *coarse, long long ccs, const T *fine, long long fcs, int nx, int NX, int NY,
                              int m, double denom, double *E, const uint8_t *valid, double tol, const Tile *tiles,
                              int ntiles, uint8_t *flags, unsigned long long *count, hipStream_t s);

// Ef [m][ny][nx] (the level's canvas) = E of each cell's 2 x 2 parent, so
// that the adjoint flag of launch_flag weights the estimate.
void launch_expand_estimate(const double *E, int NX, int NY, int m, double *Ef, int nx, int ny, hipStream_t s);

}  // namespace wp
