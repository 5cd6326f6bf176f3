// Per-tile aggregates of the dynamical stage, shared by every step kernel.
// Internal.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pd_device.hpp"
#include "pd_internal.hpp"

namespace pd {

// Tile aggregates from a wave's view of the tile's log-weights (an LDS array
// of n values): lane l folds values l, l+64, l+128, ... in that order, then a
// fixed butterfly combines the lanes.  Both step variants use exactly this
// order, so the launch configuration never changes a rounding.
__device__ __forceinline__ void tile_aggregate(const InstDev& I, int tile, const double* sell,
                                               int n, uint64_t hops_lane)
{
    const int lane = threadIdx.x & 63;
    double mx = -INFINITY;
    for (int i = lane; i < n; i += 64) mx = fmax(mx, sell[i]);
    mx = wave_reduce(mx, OpMax());
    double pc[14];   // exp's Taylor coefficients as uniform operands
#pragma unroll
    for (int q = 0; q < 14; ++q) pc[q] = I.exp_poly[q];
    double sm = 0.0;
    for (int i = lane; i < n; i += 64) sm += exp_nonpos(sell[i] - mx, I.ln2_hi, I.ln2_lo, pc);
    sm = wave_reduce(sm, OpSum());
    const uint64_t th = wave_reduce(hops_lane, OpSum());
    if (lane == 0) {
        gptr(I.tile_max)[tile] = mx;
        gptr(I.tile_sum)[tile] = sm;
        gptr(I.tile_hops)[tile] = th;
    }
}

}  // namespace pd
