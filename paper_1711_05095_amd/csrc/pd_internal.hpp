// Device-side data structures shared by the kernels and the host runtime of
// the library.  Internal: not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pd {

constexpr int kTile = 256;          // clones per tile = threads per block
constexpr int kMaxWords = 8;        // 64-site words per state
constexpr int kMaxSites = 512;      // L <= kMaxSites
constexpr int kLogRows = 128;       // rows of the logarithm table
constexpr int kLogCols = 3;         // c, -ln c (multiple of 2^-42), remainder
constexpr int kLogPoly = 6;         // log1p coefficients 1/7, -1/6, ..., -1/2

enum : uint32_t { TAG_INIT = 1, TAG_DYN = 2, TAG_RESAMPLE = 3, TAG_IID = 4, TAG_GUIDE = 5 };
constexpr int kGuideEntries = 8192; // 13-site bond neighbourhoods
enum : int32_t { MODE_MODIFIED = 0, MODE_DIRECT = 1, MODE_GUIDED = 2 };
enum : int32_t { SEL_EQ = 0, SEL_IID = 1 };

// Mutable per-instance state that lives in device memory, so that captured
// graphs advance it on every replay.
struct InstCtl {
    int64_t beta;          // intervals whose dynamical stage has run
    uint32_t ncont;        // clones the guided stage's first launch handed on (zeroed by k_prefix)
    uint32_t ev_budget;    // events per clone of the guided stage's first launch (0: no limit)
    double lmax;           // max_i ln Ups_i of the current interval
    double lbeta;          // ln mean Ups of the current interval
    double psi_sum, psi_comp;    // Neumaier sum of lbeta over all intervals
    double psib_sum, psib_comp;  // ... over intervals beyond burn_in
    uint64_t hops;         // hops performed so far
    uint64_t ksum;         // scratch: sum of K over the population (estimates)
    double d_eq;           // offset d of the [eq] points of interval beta (set by k_prefix)
    uint64_t ksnap_sum;    // scratch: sum of the burn-in snapshots of K (estimates)
    uint64_t iters;        // guided stage: proposals of the current interval (zeroed by k_prefix)
    uint64_t draws;        // guided stage: random draws over the run (proposals and closing draws)
    uint32_t s_carried;    // guided: rate[src] holds S of the population (set by k_prefix;
                           // cleared wherever the population or the table changes otherwise)
    uint32_t pad_;
};

// Per-instance descriptor (written by the host at creation, read-only after).
struct InstDev {
    int32_t L, N, W, mode;
    int32_t selection, ntiles, log_cycles, pad0;
    uint32_t key0, key1, tag_hi, pad1;
    double s, es, c, dt;
    int64_t Nc, burn_in;
    uint64_t* state[2];    // [W][Nc] words, two buffers
    uint64_t* K[2];        // [Nc] accumulated hops, two buffers
    uint32_t* Kb;          // [Nc] hops of the last interval
    double* A;             // [Nc] integral of r dt over the last interval
    double* ell;           // [Nc] ln Ups of the last interval
    int32_t* anc;          // [Nc] ancestor map of the last cloning stage
    int32_t* origin[2];    // [Nc] carried origin slots, two buffers (null: not tracked)
    uint64_t* ksnap[2];    // [Nc] carried K of the ancestor at the end of interval burn_in,
                           // two buffers (null: burn_in = 0)
    double* ykey;          // [Nc] interval ends in spacing units ([iid] only)
    double* tile_max;      // [ntiles]
    double* tile_sum;      // [ntiles] sum of exp(ell - tile_max)
    uint64_t* tile_hops;   // [ntiles]
    double* tile_off;      // [ntiles + 1] exclusive prefix of the tile sums, scale lmax
    double inv_scale;      // 1 / (rate of one allowed hop): e^{s} (modified) or 1
    const double* inv_count;// [kMaxSites + 1] 1 / r for r = 0..kMaxSites (shared)
    double* log;           // [log_cycles][2] (lbeta, mean K^beta)
    const uint32_t* guide; // [8192] guide table e^g 2^16 over bond neighbourhoods
    uint64_t guide_max;    // largest table entry (acceptance bound)
    double guide_scale;    // 2^16 / (e^{-s} guide_max): 1 / (proposal rate of one allowed bond)
    uint32_t* iters;       // [Nc] guided: proposals of the last interval, by slot
    uint64_t* rate[2];     // [Nc] guided: S (sum of the table over the allowed hops) of each
                           // clone at the end of its interval, two buffers like K (else null)
    const double* log_tab; // [kLogRows][kLogCols] table of the device logarithm
    const uint8_t* sel_tab;// [2048] byte table of select_bit_lut (shared)
    double ln2_hi, ln2_lo; // ln 2 = ln2_hi (a multiple of 2^-42) + ln2_lo
    double log_poly[kLogPoly]; // 1/7, -1/6, ..., -1/2: Taylor coefficients of log1p (uniform
                           // operands, so the polynomial's fma take them from SGPRs)
    double exp_poly[14];   // 1/13!, 1/12!, ..., 1/1!, 1: Taylor coefficients of exp (uniform)
    InstCtl* ctl;
    uint32_t* next_tile;   // work counters of the persistent step launches
    // clones the guided stage's first launch left unfinished, in the order it
    // handed them on (guided instances only, else null)
    uint64_t* cont_u64;    // [W + 2][Nc]: state words, carried K, S
    double* cont_f64;      // [4][Nc]: tau, integral of r dt, integral of S dt, jump product
    uint32_t* cont_u32;    // [4][Nc]: slot, proposal index, hops, jump exponent
};

constexpr int kMaxGroups = 16;     // step launches per cycle (one per word count)

struct TileDesc {
    int32_t inst;          // instance index
    int32_t tile;          // tile index within the instance
    int32_t first;         // first clone slot
    int32_t count;         // clones in the tile (<= kTile)
};

}  // namespace pd
