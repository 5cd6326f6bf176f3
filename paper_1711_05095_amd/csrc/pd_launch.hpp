// Host-side launchers of the kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "pd_internal.hpp"

namespace pd {
hipError_t launch_init(const InstDev* insts, int n_inst, const TileDesc* tiles, int ntiles,
                       hipStream_t st);
hipError_t launch_step(int W, const InstDev* insts, const TileDesc* tiles, int tile_base,
                       int ntiles, int src, int use_anc, hipStream_t st);
hipError_t launch_resample(const InstDev* insts, const TileDesc* tiles, int ntiles,
                           hipStream_t st);
hipError_t launch_zero_ksum(const InstDev* insts, int n_inst, hipStream_t st);
hipError_t launch_ksum(const InstDev* insts, const TileDesc* tiles, int ntiles, int cur,
                       int use_anc, hipStream_t st);
hipError_t launch_gather(int W, const InstDev* insts, const TileDesc* tiles, int tile_base,
                         int ntiles, int src, hipStream_t st);
}  // namespace pd
