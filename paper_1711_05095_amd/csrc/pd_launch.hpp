// Host-side launchers of the kernels (internal).
#pragma once
#include <hip/hip_runtime.h>

#include "pd_internal.hpp"

namespace pd {

// One launch of the dynamical stage: the tiles [base, base + count) of the
// step order, all with W words per state.
struct StepLaunch {
    int W;                 // words per state (variant 5: the bucket 2, 4 or 8 of the largest)
    int variant;           // 0: one clone per lane; 1..3: persistent queued waves; 4:
                           // compacting, a block per tile; 5: compacting, one persistent
                           // launch over every plain tile (mixed W)
    bool guided;           // guided instances (always one clone per lane)
    int base, count;       // tiles
    int blocks;            // grid of the persistent variant
    int refill;            // finished lanes that trigger a refill (variant 1)
    uint32_t* counter;     // work counter of the persistent variant
};

hipError_t launch_init(const InstDev* insts, int n_inst, const TileDesc* tiles, int ntiles,
                       hipStream_t st);
hipError_t launch_step(const StepLaunch& s, const InstDev* insts, const TileDesc* tiles, int src,
                       int use_anc, hipStream_t st);
// Tiles from which the guided stage is split in two launches (a budgeted one,
// then the clones it handed on, densely).  Below it each SIMD holds fewer than
// four of the launch's waves, so the lanes that a wave's Poisson tail leaves
// idle cost few issue slots that another wave could have used, and a second
// launch only adds its own time (measured at 391 to 2528 tiles, L = 50 and
// 100: the split costs 3% at 586 and 782 tiles and saves 3% at 1172 and 2528).
constexpr int kSplitTiles = 4 * 256;
// Guided launches of fewer tiles than the chip has CUs run blocks of one wave
// (a quarter tile each), so that their waves spread over four times as many CUs.
constexpr int kQuarterTiles = 256;

hipError_t launch_step_guided(int W, int count, const InstDev* insts, const TileDesc* tiles,
                              int base, int src, int use_anc, hipStream_t st);
hipError_t step_occupancy(int W, int variant, int* blocks_per_cu);
constexpr int kMaxHistBins = 4096;   // bins of pd_histogram (LDS counters per block)
hipError_t launch_histogram(const InstDev* insts, int inst, int64_t Nc, int cur,
                            const double* values, int ancestral, double lo, double width,
                            int nbins, uint64_t* counts, hipStream_t st);
hipError_t launch_density_mode(int W, const InstDev* insts, int inst, int64_t Nc, int cur, int n,
                               double* out, hipStream_t st);
hipError_t launch_mean(const InstDev* insts, int inst, int64_t Nc, int cur, const double* values,
                       int ancestral, hipStream_t st);
hipError_t launch_hop_counts(const InstDev* insts, int n, uint64_t* out, hipStream_t st);
hipError_t launch_descendants(const InstDev* insts, int inst, int64_t Nc, int cur,
                              uint32_t* counts, hipStream_t st);
hipError_t launch_prefix(const InstDev* insts, int n_inst, hipStream_t st);
hipError_t launch_resample(const InstDev* insts, const TileDesc* tiles, int ntiles, int tpb,
                           hipStream_t st);
hipError_t launch_select_iid(const InstDev* insts, const TileDesc* tiles, int ntiles,
                             hipStream_t st);
hipError_t launch_iota_origin(const InstDev* insts, int inst, int64_t Nc, int cur, hipStream_t st);
hipError_t launch_zero_ksum(const InstDev* insts, int n_inst, hipStream_t st);
hipError_t launch_ksum(const InstDev* insts, const TileDesc* tiles, int ntiles, int cur,
                       int use_anc, hipStream_t st);
hipError_t launch_carry_burn(const InstDev* insts, const TileDesc* tiles, int ntiles, int src,
                             int use_anc, hipStream_t st);
hipError_t launch_gather(int W, const InstDev* insts, const TileDesc* tiles, int tile_base,
                         int ntiles, int src, hipStream_t st);
}  // namespace pd
