// HIP kernels of the cloning algorithm for gfx950 (MI355X).
//
// One cycle of the algorithm (arXiv:1711.05095, Sec. 2.3) is three launches
// (plus one per extra word count in a mixed batch):
//
//   k_step / k_step_q  the dynamical stage (Sec. 4, first paragraph): every
//              clone's occupancy bit-packed in registers, continuous-time
//              (BKL) hops for one interval Delta t driven by Philox4x32-10.
//              A clone's state is pulled through the ancestor map of the
//              previous cloning stage as it is loaded, so the copy of the
//              surviving clones (Sec. 6.1) is fused into this load.  Each tile
//              of 256 clones leaves (max ln Ups, sum exp(ln Ups - max), hops).
//              k_step runs one clone per lane; k_step_q runs persistent waves
//              that take tiles from a counter and keep every lane busy with a
//              queue of the tile's clones (the next one prefetched).
//   k_prefix   per instance: ln of the population mean of Upsilon (eq.
//              psihat) and the psi sums, and the prefix offsets of the tiles.
//   k_resample the cloning stage (Sec. 4.1, eq. alpha-Ups): an FP64 scan of
//              the weights over each tile on top of its prefix offset, the
//              interval ends y_k in units of the point spacing, and for every
//              old clone k the range of new slots j whose point j + d falls in
//              its interval; k writes itself as the ancestor of those slots.
//
// The guided dynamical stage (Sec. 2.2) is in pd_guided.hip.
//
// No kernel communicates across workgroups through memory within a launch
// except through the work counter of k_step_q; everything else is ordered by
// the launch boundaries.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pd_device.hpp"
#include "pd_internal.hpp"
#include "pd_launch.hpp"
#include "pd_tile.hpp"

namespace pd {

// ---------------------------------------------------------------------------
// Initial condition: a uniform N-subset of the L sites per clone (selection
// sampling, site i taken iff u * (L - i) / 2^64 < N - taken with u the 64-bit
// number of words 2i, 2i+1 of the INIT stream of the slot).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kTile) void k_init(const InstDev* __restrict__ insts,
                                                const TileDesc* __restrict__ tiles)
{
    const TileDesc td = tiles[blockIdx.x];
    const InstDev& I = insts[td.inst];
    if ((int)threadIdx.x >= td.count) return;
    const int64_t j = td.first + threadIdx.x;
    const int L = I.L;
    int taken = 0;
    uint64_t word = 0;
    uint4 x = make_uint4(0, 0, 0, 0);
    for (int i = 0; i < L; ++i) {
        if ((i & 1) == 0) x = philox10((uint32_t)(i >> 1), (uint32_t)j, 0u, TAG_INIT | I.tag_hi,
                                       I.key0, I.key1);
        const uint32_t a = (i & 1) ? x.z : x.x;
        const uint32_t b = (i & 1) ? x.w : x.y;
        // floor(((a << 32) | b) * m / 2^64) with m = L - i <= 512
        const uint32_t hi = mulhi64_small(a, b, (uint32_t)(L - i));
        if (hi < (uint32_t)(I.N - taken)) {
            word |= 1ull << (i & 63);
            ++taken;
        }
        if ((i & 63) == 63 || i == L - 1) {
            I.state[0][(int64_t)(i >> 6) * I.Nc + j] = word;
            word = 0;
        }
    }
    I.K[0][j] = 0;
}

__global__ void k_reset_ctl(const InstDev* __restrict__ insts, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kMaxGroups) insts[0].next_tile[i] = 0;
    if (i >= n) return;
    InstCtl* c = insts[i].ctl;
    c->beta = 0;
    c->ncont = 0;
    c->ev_budget = 0;
    c->lmax = 0.0;
    c->lbeta = 0.0;
    c->psi_sum = c->psi_comp = 0.0;
    c->psib_sum = c->psib_comp = 0.0;
    c->hops = 0;
    c->ksum = 0;
    c->ksnap_sum = 0;
    c->iters = 0;
    c->draws = 0;
    c->s_carried = 0;
}

// Neumaier compensated addition.
__device__ __forceinline__ void neumaier_add(double& sum, double& comp, double x)
{
    const double t = sum + x;
    if (fabs(sum) >= fabs(x)) comp += (sum - t) + x;
    else comp += (x - t) + sum;
    sum = t;
}

// ---------------------------------------------------------------------------
// One clone through one interval.  The state is in registers; the event loop
// is the hot loop of the whole method.
// ---------------------------------------------------------------------------
struct StepConst {
    const double* invr;    // LDS: 1 / r, or inv_scale / r (SCALED), for r = 0..kMaxSites
    const double* logt;    // LDS: logarithm table
    const uint8_t* sel;    // LDS: byte table of select_bit_lut
    double inv_scale;      // 1 / rate of one allowed hop
    double dt, ln2_hi, ln2_lo;
    double poly[kLogPoly]; // log1p coefficients (uniform)
    uint32_t beta, c3, key0, key1;
    int L, lb;
};

// Draws and performs events until the interval ends.  Returns true when the
// clone reached the end of the interval; A gets the final sojourn.  SCALED:
// the table holds inv_scale / r, the product the unscaled form forms per
// event (so both give the same rounding).
template <int W, bool SCALED = false>
__device__ __forceinline__ bool one_event(const StepConst& C, uint32_t slot, uint64_t (&x)[W],
                                          uint64_t (&m)[W], int& r, double& tau, double& A,
                                          uint32_t& k, uint32_t& kb)
{
    if (r == 0) return true;
    const uint4 y = philox10(k, slot, C.beta, C.c3, C.key0, C.key1);
    ++k;
    const double E = -log_unit(unit_scaled(y.x, y.y), C.logt, C.ln2_hi, C.ln2_lo, C.poly, 53);
    // waiting time E / R with R = (rate of one hop) * r
    const double w = E * (SCALED ? C.invr[r] : C.inv_scale * C.invr[r]);
    if (tau + w >= C.dt || k >= 0x80000000u) {
        // k < 2^31 always: the host admits at most 2^24 expected hops per
        // interval; the bound only guarantees that the loop ends
        A = fma((double)r, C.dt - tau, A);
        return true;
    }
    A = fma((double)r, w, A);
    tau = tau + w;
    const uint32_t q = mulhi64_small(y.z, y.w, (uint32_t)r);
    hop<W>(x, select_bit_lut<W>(m, q, C.sel), C.L);
    bond_mask<W>(x, C.lb, m);
    r = popcount_words<W>(m);
    ++kb;
    return false;
}

// one_event with the draw's random numbers formed beforehand (y, E): an
// event's Philox block and logarithm depend only on (event index, slot,
// interval), so when MORE, those of the next event are formed beside this
// event's hop, their chains of dependent instructions side by side.  Not
// after the closing draw, nor (MORE = false) after the last event of a round.
__device__ __forceinline__ void draw_event(const StepConst& C, uint32_t slot, uint32_t k,
                                           uint4& y, double& E)
{
    y = philox10(k, slot, C.beta, C.c3, C.key0, C.key1);
    E = -log_unit(unit_scaled(y.x, y.y), C.logt, C.ln2_hi, C.ln2_lo, C.poly, 53);
}

template <int W, bool MORE>
__device__ __forceinline__ bool event_ahead(const StepConst& C, uint32_t slot, uint64_t (&x)[W],
                                            uint64_t (&m)[W], int& r, double& tau, double& A,
                                            uint32_t& k, uint32_t& kb, uint4& y, double& E)
{
    if (r == 0) return true;
    ++k;
    const double w = E * C.invr[r];   // the table holds inv_scale / r
    if (tau + w >= C.dt || k >= 0x80000000u) {
        A = fma((double)r, C.dt - tau, A);
        return true;
    }
    A = fma((double)r, w, A);
    tau = tau + w;
    const uint32_t q = mulhi64_small(y.z, y.w, (uint32_t)r);
    if (MORE) draw_event(C, slot, k, y, E);
    hop<W>(x, select_bit_lut<W>(m, q, C.sel), C.L);
    bond_mask<W>(x, C.lb, m);
    r = popcount_words<W>(m);
    ++kb;
    return false;
}

// The logarithm table and 1 / r (scaled by the instance's inv_scale when
// `scaled`: one instance per block).
__device__ __forceinline__ void load_tables(const InstDev& I, double* s_log, double* s_invr,
                                            int tid, int nthr, int rmax, bool scaled)
{
    for (int i = tid; i < kLogRows * kLogCols; i += nthr) s_log[i] = gptr(I.log_tab)[i];
    const double sc = I.inv_scale;
    for (int i = tid; i <= rmax; i += nthr)
        s_invr[i] = scaled ? sc * gptr(I.inv_count)[i] : gptr(I.inv_count)[i];
}

// ---------------------------------------------------------------------------
// Dynamical stage, one clone per lane: block = one tile of 256 clones.
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(kTile) void k_step(const InstDev* __restrict__ insts,
                                                const TileDesc* __restrict__ tiles, int tile_base,
                                                int src, int use_anc)
{
    __shared__ double s_invr[kMaxSites + 1];
    __shared__ double s_log[kLogRows * kLogCols];
    __shared__ double s_ell[kTile];
    __shared__ uint64_t s_u[kTile];
    __shared__ __align__(8) uint8_t s_sel[2048];

    const TileDesc td = tiles[tile_base + blockIdx.x];
    const InstDev& I = insts[td.inst];
    const int L = I.L;
    load_tables(I, s_log, s_invr, threadIdx.x, kTile, kMaxSites, true);
    load_select_table(s_sel, I.sel_tab, threadIdx.x, kTile);
    __syncthreads();

    StepConst C;
    C.invr = s_invr; C.logt = s_log; C.sel = s_sel; C.inv_scale = I.inv_scale;
    C.dt = I.dt; C.ln2_hi = I.ln2_hi; C.ln2_lo = I.ln2_lo;
#pragma unroll
    for (int k = 0; k < kLogPoly; ++k) C.poly[k] = I.log_poly[k];
    C.beta = (uint32_t)(I.ctl->beta + 1); C.c3 = TAG_DYN | I.tag_hi;
    C.key0 = I.key0; C.key1 = I.key1; C.L = L; C.lb = (L - 1) & 63;

    const int tid = threadIdx.x;
    const bool valid = tid < td.count;
    const int64_t j = td.first + tid;
    const int64_t Nc = I.Nc;

    uint32_t kb = 0;
    double ell = -INFINITY;
    if (valid) {
        const int64_t from = use_anc ? (int64_t)gptr(I.anc)[j] : j;
        uint64_t x[W], m[W];
#pragma unroll
        for (int w = 0; w < W; ++w) x[w] = gptr(I.state[src])[w * Nc + from];
        const uint64_t Kfrom = gptr(I.K[src])[from];
        bond_mask<W>(x, C.lb, m);
        int r = popcount_words<W>(m);
        double tau = 0.0, A = 0.0;
        uint32_t k = 0;
        while (!one_event<W, true>(C, (uint32_t)j, x, m, r, tau, A, k, kb)) {}
        ell = (I.mode == MODE_MODIFIED) ? -I.c * A : -I.s * (double)kb;
        const int dst = src ^ 1;
#pragma unroll
        for (int w = 0; w < W; ++w) gptr(I.state[dst])[w * Nc + j] = x[w];
        gptr(I.K[dst])[j] = Kfrom + kb;
        gptr(I.Kb)[j] = kb;
        gptr(I.A)[j] = A;
        gptr(I.ell)[j] = ell;
        if (I.origin[0]) gptr(I.origin[dst])[j] = gptr(I.origin[src])[from];
    }
    s_ell[tid] = ell;
    s_u[tid] = kb;
    __syncthreads();
    if (tid < 64) {
        uint64_t h = 0;
        for (int i = tid; i < td.count; i += 64) h += s_u[i];
        tile_aggregate(I, td.tile, s_ell, td.count, h);
    }
}

// ---------------------------------------------------------------------------
// Dynamical stage with compaction: block = one tile of 256 clones.  A wave
// runs until its slowest lane is done, and the number of events per clone
// is Poisson, so a third of the lane slots idle at the end of an interval.
// Here the tile runs in rounds of a bounded number of events; after each
// round the unfinished clones (their registers: state, time, integral, event
// counters, carried K and tile index) are packed through LDS into the lowest
// lanes of the block, so emptied waves wait at the barrier and leave the
// SIMDs to other waves.  A clone's random numbers are keyed by its slot and
// event index and its outputs are written by slot, so the results are those
// of k_step bit for bit.
// ---------------------------------------------------------------------------
template <int W>
struct Pack {
    uint64_t x[W][kTile];
    uint64_t K[kTile];
    double tau[kTile], A[kTile];
    uint32_t k[kTile], kb[kTile], t[kTile];
};

// The LDS arrays of one compacting tile run (the tables are filled by the
// caller: the logarithm and selection tables once, 1 / r per instance).
template <int W>
struct TileLds {
    double* invr;          // [64 W + 1]: inv_scale / r
    double* log;           // logarithm table
    uint8_t* sel;          // selection byte table
    double* ell;           // [kTile]
    uint32_t* kb;          // [kTile]
    int* wc;               // [kTile / 64]
    Pack<W>* P;
};

// One tile of 256 clones through the interval, in rounds with compaction (the
// body of k_step_c, also run tile after tile by k_step_cp).  Every thread of
// the block calls it; it ends with every thread past its last barrier.
template <int W>
__device__ __forceinline__ void run_tile_c(const InstDev& I, const TileDesc& td,
                                           const TileLds<W>& S, int src, int use_anc,
                                           int first16)
{
    const int L = I.L;
    StepConst C;
    C.invr = S.invr; C.logt = S.log; C.sel = S.sel; C.inv_scale = I.inv_scale;
    C.dt = I.dt; C.ln2_hi = I.ln2_hi; C.ln2_lo = I.ln2_lo;
#pragma unroll
    for (int k = 0; k < kLogPoly; ++k) C.poly[k] = I.log_poly[k];
    C.beta = (uint32_t)(I.ctl->beta + 1); C.c3 = TAG_DYN | I.tag_hi;
    C.key0 = I.key0; C.key1 = I.key1; C.L = L; C.lb = (L - 1) & 63;

    double* const s_ell = S.ell;
    uint32_t* const s_kb = S.kb;
    int* const s_wc = S.wc;
    Pack<W>& P = *S.P;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t Nc = I.Nc;
    const int dst = src ^ 1;
    const bool directw = I.mode != MODE_MODIFIED;

    bool active = tid < td.count;
    uint32_t t = (uint32_t)tid;
    uint64_t x[W], m[W], Kfrom = 0;
    int r = 0;
    double tau = 0.0, A = 0.0;
    uint32_t k = 0, kb = 0;
    if (active) {
        const int64_t j = td.first + tid;
        const int64_t from = use_anc ? (int64_t)gptr(I.anc)[j] : j;
#pragma unroll
        for (int w = 0; w < W; ++w) x[w] = gptr(I.state[src])[w * Nc + from];
        Kfrom = gptr(I.K[src])[from];
        if (I.origin[0]) gptr(I.origin[dst])[j] = gptr(I.origin[src])[from];
        bond_mask<W>(x, C.lb, m);
        r = popcount_words<W>(m);
    } else {
#pragma unroll
        for (int w = 0; w < W; ++w) x[w] = m[w] = 0;
        s_ell[tid] = -INFINITY;
        s_kb[tid] = 0;
    }
    // expected events per clone: (rate of one hop) x (mean allowed bonds) x dt, + 1;
    // the first round runs first16/16 of it, later rounds 0.15 of that
    const double rbar = L > 1 ? 2.0 * I.N * (double)(L - I.N) / (double)(L - 1) : 0.0;
    const double ev = (rbar * C.dt / C.inv_scale + 1.0) * (double)first16 * (1.0 / 16.0);
    int budget = max(1, (int)fmin(ev + 1.0, 1.0e6));
    const int later = max(2, (int)fmin(0.15 * ev + 1.0, 1.0e6));
    __syncthreads();

    bool fin = false;   // finished in this round, outputs not yet written
    for (;;) {
        {
            const uint32_t slot = (uint32_t)(td.first + t);
            uint4 y{0u, 0u, 0u, 0u};
            double E = 0.0;
            if (active && r > 0) draw_event(C, slot, k, y, E);
            int it = 0;
            for (; active && it + 1 < budget; ++it) {
                if (event_ahead<W, true>(C, slot, x, m, r, tau, A, k, kb, y, E)) {
                    active = false;
                    fin = true;
                }
            }
            // the round's last event forms no draw after it
            if (active && it < budget &&
                event_ahead<W, false>(C, slot, x, m, r, tau, A, k, kb, y, E)) {
                active = false;
                fin = true;
            }
        }
        // the clones that finished in this round write their outputs once,
        // after the event loop (their registers are left as they finished)
        if (fin) {
            const int64_t j = td.first + t;
            const double ell = directw ? -I.s * (double)kb : -I.c * A;
#pragma unroll
            for (int w = 0; w < W; ++w) gptr(I.state[dst])[w * Nc + j] = x[w];
            gptr(I.K[dst])[j] = Kfrom + kb;
            gptr(I.Kb)[j] = kb;
            gptr(I.A)[j] = A;
            gptr(I.ell)[j] = ell;
            s_ell[t] = ell;
            s_kb[t] = kb;
            fin = false;
        }
        // rank of each unfinished clone among the block's unfinished clones
        const uint64_t bal = __ballot(active);
        if (lane == 0) s_wc[wave] = __popcll(bal);
        __syncthreads();
        int before = 0, total = 0;
#pragma unroll
        for (int v = 0; v < kTile / 64; ++v) {
            before += v < wave ? s_wc[v] : 0;
            total += s_wc[v];
        }
        if (total == 0) break;
        if (active) {
            const int p = before + __popcll(bal & ((1ull << lane) - 1ull));
#pragma unroll
            for (int w = 0; w < W; ++w) P.x[w][p] = x[w];
            P.K[p] = Kfrom; P.tau[p] = tau; P.A[p] = A;
            P.k[p] = k; P.kb[p] = kb; P.t[p] = t;
        }
        __syncthreads();
        active = tid < total;
        if (active) {
#pragma unroll
            for (int w = 0; w < W; ++w) x[w] = P.x[w][tid];
            Kfrom = P.K[tid]; tau = P.tau[tid]; A = P.A[tid];
            k = P.k[tid]; kb = P.kb[tid]; t = P.t[tid];
            bond_mask<W>(x, C.lb, m);
            r = popcount_words<W>(m);
        }
        __syncthreads();
        // once the unfinished clones fit in one wave no pack can empty another:
        // that wave runs them to the end in one round
        budget = total <= 64 ? 0x7FFFFFFF : later;
    }
    if (tid < 64) {
        uint64_t h = 0;
        for (int i = tid; i < td.count; i += 64) h += s_kb[i];
        tile_aggregate(I, td.tile, s_ell, td.count, h);
    }
}

template <int W>
__global__ __launch_bounds__(kTile) void k_step_c(const InstDev* __restrict__ insts,
                                                  const TileDesc* __restrict__ tiles,
                                                  int tile_base, int src, int use_anc,
                                                  int first16)
{
    __shared__ double s_invr[64 * W + 1];     // r <= L <= 64 W
    __shared__ double s_log[kLogRows * kLogCols];
    __shared__ double s_ell[kTile];
    __shared__ uint32_t s_kb[kTile];
    __shared__ int s_wc[kTile / 64];
    __shared__ __align__(8) uint8_t s_sel[2048];
    __shared__ Pack<W> P;

    const TileDesc td = tiles[tile_base + blockIdx.x];
    const InstDev& I = insts[td.inst];
    load_tables(I, s_log, s_invr, threadIdx.x, kTile, 64 * W, true);
    load_select_table(s_sel, I.sel_tab, threadIdx.x, kTile);
    const TileLds<W> S{s_invr, s_log, s_sel, s_ell, s_kb, s_wc, &P};
    run_tile_c<W>(I, td, S, src, use_anc, first16);   // its first barrier orders the tables
}

// ---------------------------------------------------------------------------
// Dynamical stage, compacting, in one persistent launch for all plain tiles of
// a context, word counts W <= WMAX mixed (the batched form): each block takes
// tiles from the launch's work counter in the step order (largest word count
// and expected work first) and runs each as k_step_c does, dispatching on the
// tile's W (uniform over the block).  The logarithm and selection tables are
// loaded once per block, 1 / r when the instance changes.  Results are those of
// k_step_c bit for bit: random numbers are keyed by slot, outputs written by
// slot, each tile aggregated in the same order.
// ---------------------------------------------------------------------------
// run_tile_c for the tile's word count w (W <= w <= WMAX), the packing buffer
// taken as a Pack<w>.
template <int W, int WMAX>
__device__ __forceinline__ void step_tile_w(int w, const InstDev& I, const TileDesc& td,
                                            double* s_invr, double* s_log, uint8_t* s_sel,
                                            double* s_ell, uint32_t* s_kb, int* s_wc,
                                            unsigned char* s_pack, int src, int use_anc,
                                            int first16)
{
    if (w == W) {
        const TileLds<W> S{s_invr, s_log, s_sel, s_ell, s_kb, s_wc, (Pack<W>*)s_pack};
        run_tile_c<W>(I, td, S, src, use_anc, first16);
        return;
    }
    if constexpr (W < WMAX)
        step_tile_w<W + 1, WMAX>(w, I, td, s_invr, s_log, s_sel, s_ell, s_kb, s_wc, s_pack, src,
                                 use_anc, first16);
}

template <int WMAX>
__global__ __launch_bounds__(kTile) void k_step_cp(const InstDev* __restrict__ insts,
                                                   const TileDesc* __restrict__ tiles,
                                                   int tile_base, int tile_count,
                                                   uint32_t* __restrict__ counter, int src,
                                                   int use_anc, int first16)
{
    __shared__ double s_invr[64 * WMAX + 1];
    __shared__ double s_log[kLogRows * kLogCols];
    __shared__ double s_ell[kTile];
    __shared__ uint32_t s_kb[kTile];
    __shared__ int s_wc[kTile / 64];
    __shared__ __align__(8) uint8_t s_sel[2048];
    __shared__ __align__(16) unsigned char s_pack[sizeof(Pack<WMAX>)];
    __shared__ int s_next;

    for (int i = threadIdx.x; i < kLogRows * kLogCols; i += kTile) s_log[i] = gptr(insts[0].log_tab)[i];
    load_select_table(s_sel, insts[0].sel_tab, threadIdx.x, kTile);
    int inst = -1;
    for (;;) {
        if (threadIdx.x == 0) s_next = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int n = s_next;
        __syncthreads();   // every thread has read s_next before it is written again
        if (n >= tile_count) break;
        const TileDesc td = tiles[tile_base + n];
        const InstDev& I = insts[td.inst];
        if (td.inst != inst) {
            // the previous tile's last barrier is behind every thread: the old
            // 1 / r is no longer read
            inst = td.inst;
            const double sc = I.inv_scale;
            for (int r = threadIdx.x; r <= 64 * I.W; r += kTile)
                s_invr[r] = sc * gptr(I.inv_count)[r];
        }
        // run_tile_c's first barrier orders the tables and the packing buffer
        step_tile_w<1, WMAX>(I.W, I, td, s_invr, s_log, s_sel, s_ell, s_kb, s_wc, s_pack, src,
                             use_anc, first16);
    }
}

// ---------------------------------------------------------------------------
// Dynamical stage, persistent queued waves.  Each wave takes tiles from the
// launch's counter; within a tile every lane runs one clone at a time and,
// once `refill` lanes have finished theirs, all finished lanes take the next
// clones of the tile (each lane's next clone is already loaded).
// ---------------------------------------------------------------------------
constexpr int kQWaves = 4;

template <int W, int OCC>
__global__ __launch_bounds__(64 * kQWaves) __attribute__((amdgpu_waves_per_eu(OCC))) void k_step_q(const InstDev* __restrict__ insts,
                                                         const TileDesc* __restrict__ tiles,
                                                         int tile_base, int tile_count,
                                                         uint32_t* __restrict__ counter,
                                                         int src, int use_anc, int refill)
{
    __shared__ double s_log[kLogRows * kLogCols];
    __shared__ double s_invr[kMaxSites + 1];
    __shared__ double s_ell[kQWaves][kTile];
    __shared__ int32_t s_from[kQWaves][kTile];
    __shared__ __align__(8) uint8_t s_sel[2048];

    const int wave = threadIdx.x >> 6;
    const int lane = threadIdx.x & 63;
    load_tables(insts[0], s_log, s_invr, threadIdx.x, 64 * kQWaves, kMaxSites, false);
    load_select_table(s_sel, insts[0].sel_tab, threadIdx.x, 64 * kQWaves);
    __syncthreads();

    double* sell = s_ell[wave];
    int32_t* sfrom = s_from[wave];

    for (;;) {
        uint32_t t = 0;
        if (lane == 0) t = atomicAdd(counter, 1u);
        t = __builtin_amdgcn_readfirstlane(t);
        if ((int)t >= tile_count) break;
        const TileDesc td = tiles[tile_base + t];
        const InstDev& I = insts[td.inst];
        const int L = I.L;
        const int n = td.count;
        const int64_t Nc = I.Nc;
        for (int i = lane; i < n; i += 64)
            sfrom[i] = use_anc ? gptr(I.anc)[td.first + i] : (int32_t)(td.first + i);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

        StepConst C;
        C.invr = s_invr; C.logt = s_log; C.sel = s_sel; C.inv_scale = I.inv_scale;
        C.dt = I.dt; C.ln2_hi = I.ln2_hi; C.ln2_lo = I.ln2_lo;
#pragma unroll
        for (int k = 0; k < kLogPoly; ++k) C.poly[k] = I.log_poly[k];
        C.beta = (uint32_t)(I.ctl->beta + 1); C.c3 = TAG_DYN | I.tag_hi;
        C.key0 = I.key0; C.key1 = I.key1; C.L = L; C.lb = (L - 1) & 63;
        const auto st_src = gptr(I.state[src]);
        const auto st_dst = gptr(I.state[src ^ 1]);
        const auto K_src = gptr(I.K[src]);
        const auto K_dst = gptr(I.K[src ^ 1]);
        const auto Kb_out = gptr(I.Kb);
        const auto A_out = gptr(I.A);
        const auto ell_out = gptr(I.ell);
        const bool modified = (I.mode == MODE_MODIFIED);
        const double cw = modified ? -I.c : -I.s;

        // lane state: current clone (slot cur) and the prefetched next (slot nxt)
        int cur = lane < n ? lane : -1;
        int nxt = lane + 64 < n ? lane + 64 : -1;
        int next_free = min(128, n);
        uint64_t x[W], m[W], px[W];
        uint64_t Kf = 0, pK = 0;
        if (cur >= 0) {
            const int64_t f = sfrom[cur];
#pragma unroll
            for (int w = 0; w < W; ++w) x[w] = st_src[w * Nc + f];
            Kf = K_src[f];
        } else {
#pragma unroll
            for (int w = 0; w < W; ++w) x[w] = 0;
        }
        if (nxt >= 0) {
            const int64_t f = sfrom[nxt];
#pragma unroll
            for (int w = 0; w < W; ++w) px[w] = st_src[w * Nc + f];
            pK = K_src[f];
        } else {
#pragma unroll
            for (int w = 0; w < W; ++w) px[w] = 0;
        }
        bond_mask<W>(x, C.lb, m);
        int r = popcount_words<W>(m);
        double tau = 0.0, A = 0.0;
        uint32_t k = 0, kb = 0, hops = 0;
        bool active = cur >= 0;
        bool waiting = false;
        // outputs of a finished clone, stored at the next refill (after the
        // prefetched clone has been moved in, so that the wait for the
        // prefetch never includes these stores)
        uint64_t ox[W];
        uint64_t oK = 0;
        uint32_t okb = 0, oslot = 0;
        double oA = 0.0, oell = 0.0;
#pragma unroll
        for (int w = 0; w < W; ++w) ox[w] = 0;

        for (;;) {
            if (active) {
                const uint32_t j = (uint32_t)(td.first + cur);
                if (one_event<W>(C, j, x, m, r, tau, A, k, kb)) {
                    oell = modified ? cw * A : cw * (double)kb;
                    sell[cur] = oell;
#pragma unroll
                    for (int w = 0; w < W; ++w) ox[w] = x[w];
                    oK = Kf + kb;
                    okb = kb;
                    oA = A;
                    oslot = j;
                    hops += kb;
                    active = false;
                    waiting = true;
                }
            }
            const uint64_t wmask = __ballot(waiting);
            const uint64_t amask = __ballot(active);
            if (amask == 0 && wmask == 0) break;
            if (__popcll(wmask) >= refill || amask == 0) {
                if (waiting) {
                    waiting = false;
                    cur = nxt;
                    if (cur >= 0) {
#pragma unroll
                        for (int w = 0; w < W; ++w) x[w] = px[w];
                        Kf = pK;
                        bond_mask<W>(x, C.lb, m);
                        r = popcount_words<W>(m);
                        tau = 0.0;
                        A = 0.0;
                        k = 0;
                        kb = 0;
                        active = true;
                    }
#pragma unroll
                    for (int w = 0; w < W; ++w) st_dst[w * Nc + oslot] = ox[w];
                    K_dst[oslot] = oK;
                    Kb_out[oslot] = okb;
                    A_out[oslot] = oA;
                    ell_out[oslot] = oell;
                    if (cur >= 0) {
                        const int rank = __builtin_amdgcn_mbcnt_hi(
                            (uint32_t)(wmask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)wmask, 0));
                        nxt = next_free + rank < n ? next_free + rank : -1;
                        if (nxt >= 0) {
                            const int64_t f = sfrom[nxt];
#pragma unroll
                            for (int w = 0; w < W; ++w) px[w] = st_src[w * Nc + f];
                            pK = K_src[f];
                        }
                    }
                }
                next_free = min(n, next_free + (int)__popcll(wmask));
            }
        }

        // tile aggregates from the wave's copy of the log-weights
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        tile_aggregate(I, td.tile, sell, n, hops);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
}

// ---------------------------------------------------------------------------
// Interval statistics, one block per instance: lmax, ln mean Upsilon, the psi
// sums, and the tile offsets tile_off[0..n] (exclusive prefix sums of the
// tile weights in the scale exp(. - lmax)), made non-decreasing by a running
// maximum so that rounding can never reorder interval ends; tile_off[n] is
// the total weight T.  Completes the interval: beta += 1.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double tile_weight(const InstDev& I, int b, double M)
{
    return I.tile_sum[b] * exp(I.tile_max[b] - M);
}

// Offset d of the [eq] points of interval beta: 52 bits of the RESAMPLE
// stream plus one half, times 2^-52, strictly inside (0, 1).
__device__ __forceinline__ double eq_offset(const InstDev& I, uint32_t beta)
{
    const uint4 y = philox10(0u, 0u, beta, TAG_RESAMPLE | I.tag_hi, I.key0, I.key1);
    const double hi = (double)y.x * 1048576.0;   // y.x * 2^20
    const double lo = (double)(y.y >> 12) + 0.5;
    return (hi + lo) * 0x1p-52;
}

// The interval's closing work, on one thread: the total, ln of the mean
// weight and the psi sums, the per-interval log, beta, and the [eq] offset of
// the next cloning stage.
__device__ __forceinline__ void prefix_finish(const InstDev& I, uint32_t beta, double M, double T,
                                              uint64_t hops)
{
    I.tile_off[I.ntiles] = T;
    InstCtl* c = I.ctl;
    const double lbeta = M + log(T / (double)I.Nc);
    c->lmax = M;
    c->lbeta = lbeta;
    neumaier_add(c->psi_sum, c->psi_comp, lbeta);
    if ((int64_t)beta > I.burn_in) neumaier_add(c->psib_sum, c->psib_comp, lbeta);
    c->hops += hops;
    if ((int64_t)beta <= (int64_t)I.log_cycles) {
        I.log[2 * (beta - 1)] = lbeta;
        I.log[2 * (beta - 1) + 1] = (double)hops / (double)I.Nc;
    }
    c->beta = beta;
    c->d_eq = eq_offset(I, beta);
    // the guided stage's next first launch: 1.1 times this interval's mean
    // proposals per clone (taken, not taken and the closing draw), the rest in
    // its second launch
    c->ncont = 0;
    const double per_clone = c->iters ? (double)c->iters / (double)I.Nc
                                      : (double)hops / (double)I.Nc + 1.0;
    c->draws += c->iters;
    c->iters = 0;
    // the guided stage has just written S of every clone it stepped
    if (I.mode == MODE_GUIDED) c->s_carried = 1;
    c->ev_budget = (uint32_t)fmin(1.1 * per_clone + 2.0, 1073741824.0);
}

// Tiles per thread that k_prefix keeps in registers (instances of up to
// kTile * kPrefixRegs tiles); larger instances re-read their tile arrays.
constexpr int kPrefixRegs = 16;

__global__ __launch_bounds__(kTile) void k_prefix(const InstDev* __restrict__ insts)
{
    __shared__ double s_d[kTile / 64];
    __shared__ uint64_t s_u[kTile / 64];
    __shared__ double s_x[kTile];
    const InstDev& I = insts[blockIdx.x];
    const int n = I.ntiles;
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid < kMaxGroups) I.next_tile[tid] = 0;
    const uint32_t beta = (uint32_t)(I.ctl->beta + 1);

    // thread tid owns tiles [b0, b1)
    const int ch = (n + kTile - 1) / kTile;
    const int b0 = min(tid * ch, n), b1 = min(b0 + ch, n);
    double T;
    if (ch <= kPrefixRegs) {
        // every tile value is loaded once, up front, and kept in registers;
        // the arithmetic is the same as below, in the same order
        double tm[kPrefixRegs], ts[kPrefixRegs];
        double m = -INFINITY;
        uint64_t h = 0;
#pragma unroll
        for (int q = 0; q < kPrefixRegs; ++q) {
            if (b0 + q < b1) {
                tm[q] = I.tile_max[b0 + q];
                ts[q] = I.tile_sum[b0 + q];
                h += I.tile_hops[b0 + q];
                m = fmax(m, tm[q]);
            }
        }
        const double M = block_reduce(m, OpMax(), s_d);
        const uint64_t hops = block_reduce(h, OpSum(), s_u);
        double loc = 0.0;
#pragma unroll
        for (int q = 0; q < kPrefixRegs; ++q) {
            if (b0 + q < b1) {
                ts[q] = ts[q] * exp(tm[q] - M);   // the tile's weight
                loc += ts[q];
            }
        }
        double total;
        const double incl = block_scan_incl(loc, OpSum(), s_d, total);
        s_x[tid] = incl;
        __syncthreads();
        const double base = (tid == 0) ? 0.0 : s_x[tid - 1];
        double lp = 0.0, run = -INFINITY;
#pragma unroll
        for (int q = 0; q < kPrefixRegs; ++q) {
            if (b0 + q < b1) {
                run = fmax(run, base + lp);
                tm[q] = run;   // the tile's offset before the fix-up below
                lp += ts[q];
            }
        }
        double all_max;
        const double pm = block_scan_incl(run, OpMax(), s_d, all_max);
        __syncthreads();
        s_x[tid] = pm;
        __syncthreads();
        const double before = (tid == 0) ? -INFINITY : s_x[tid - 1];
#pragma unroll
        for (int q = 0; q < kPrefixRegs; ++q)
            if (b0 + q < b1) I.tile_off[b0 + q] = fmax(tm[q], before);
        T = fmax(total, all_max);
        if (tid == 0) prefix_finish(I, beta, M, T, hops);
        return;
    }

    double m = -INFINITY;
    uint64_t h = 0;
    for (int b = tid; b < n; b += kTile) {
        m = fmax(m, I.tile_max[b]);
        h += I.tile_hops[b];
    }
    const double M = block_reduce(m, OpMax(), s_d);
    const uint64_t hops = block_reduce(h, OpSum(), s_u);

    double loc = 0.0;
    for (int b = b0; b < b1; ++b) loc += tile_weight(I, b, M);
    double total;
    const double incl = block_scan_incl(loc, OpSum(), s_d, total);
    s_x[tid] = incl;
    __syncthreads();
    const double base = (tid == 0) ? 0.0 : s_x[tid - 1];

    double lp = 0.0, run = -INFINITY;
    for (int b = b0; b < b1; ++b) {
        run = fmax(run, base + lp);
        I.tile_off[b] = run;
        lp += tile_weight(I, b, M);
    }
    double all_max;
    const double pm = block_scan_incl(run, OpMax(), s_d, all_max);
    __syncthreads();
    s_x[tid] = pm;
    __syncthreads();
    const double before = (tid == 0) ? -INFINITY : s_x[tid - 1];
    for (int b = b0; b < b1; ++b) I.tile_off[b] = fmax(I.tile_off[b], before);
    T = fmax(total, all_max);
    if (tid == 0) prefix_finish(I, beta, M, T, hops);
}

// ---------------------------------------------------------------------------
// Cloning stage ([eq]).
// ---------------------------------------------------------------------------

// #{ j in [0, Nc) : j + d < y }, exactly: y - j is exact whenever it lies in
// [0, 1), so the test fl(y - j) > d decides j + d < y without error.  The
// count is kept as a double (integers below 2^31 are exact) until it is
// returned.
__device__ __forceinline__ int count_points_below(double y, double d, double Ncd)
{
    double m = fmin(fmax(ceil(y - d), 0.0), Ncd);
    while (m > 0.0 && !((y - (m - 1.0)) > d)) m -= 1.0;
    while (m < Ncd && ((y - m) > d)) m += 1.0;
    return (int)m;
}

// One wave per tile of 256 clones: lane l holds clones 4l .. 4l+3 of the tile,
// sums their weights in order, and a wave scan of the lane totals carries the
// sum across lanes, so the tile needs no block barrier.  A wave takes TPW
// consecutive tiles of the step order and loads all of them before it works on
// the first, so their memory latencies overlap (the tiling the autotuner
// chooses; the per-tile arithmetic and so every result is the same for any
// TPW).  The interval ends are y_k = C_k (Nc / T) with one quotient per tile,
// so the end of a tile and the start of the next are the same number.
// Slots of one clone's offspring range that its own lane writes in the
// cloning stage; the rest the wave writes together.
constexpr int kShortRun = 8;

template <int TPW>
__global__ __launch_bounds__(kTile) void k_resample(const InstDev* __restrict__ insts,
                                                    const TileDesc* __restrict__ tiles,
                                                    int ntiles)
{
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (kTile / 64) +
                                                          (threadIdx.x >> 6)));
    const int t0 = wave * TPW;
    if (t0 >= ntiles) return;   // uniform over the wave; no barrier follows

    TileDesc td[TPW];
    double e[TPW][4];
#pragma unroll
    for (int t = 0; t < TPW; ++t) td[t] = tiles[min(t0 + t, ntiles - 1)];
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        const InstDev& I = insts[td[t].inst];
        const int first = 4 * lane;
        const auto ell = gptr(I.ell) + td[t].first + first;
        if (first + 3 < td[t].count) {
            typedef double f64x2 __attribute__((ext_vector_type(2)));
            const f64x2 a = *(const __attribute__((address_space(1))) f64x2*)(ell);
            const f64x2 b = *(const __attribute__((address_space(1))) f64x2*)(ell + 2);
            e[t][0] = a.x; e[t][1] = a.y; e[t][2] = b.x; e[t][3] = b.y;
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) e[t][i] = (first + i < td[t].count) ? ell[i] : -INFINITY;
        }
    }

#pragma unroll
    for (int t = 0; t < TPW; ++t) {
        if (t0 + t >= ntiles) break;
        const InstDev& I = insts[td[t].inst];
        const int count = td[t].count;
        const int k0 = td[t].first + 4 * lane;   // first of the lane's clones
        const int Nc = (int)I.Nc;
        const double Ncd = (double)Nc;
        const double M = I.ctl->lmax;
        const int b = td[t].tile;
        const double off0 = I.tile_off[b];
        const double off1 = I.tile_off[b + 1];
        const double sN = Ncd / I.tile_off[I.ntiles];   // Nc / T
        const double d = I.ctl->d_eq;   // k_prefix drew it for this interval
        double pc[14];
#pragma unroll
        for (int q = 0; q < 14; ++q) pc[q] = I.exp_poly[q];

        // weights and their running sum over the lane's four clones
        double c[4];
        double run = 0.0;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double w = exp_nonpos(e[t][i] - M, I.ln2_hi, I.ln2_lo, pc);
            run += (4 * lane + i < count) ? w : 0.0;
            c[i] = run;
        }
        // (every lane takes part in each shuffle; the lane-0 case is a select
        // after it, never a condition around it)
        const double incl = wave_scan_dpp(run, OpSum(), 0.0);
        const double up = __shfl_up(incl, 1, 64);
        const double base = lane ? up : 0.0;
        const double top = base + c[3];
        // non-decreasing over the tile: a lane starts no lower than the end of
        // every lane before it (the scan's rounding order differs from the
        // lanes' own)
        const double pmax = wave_scan_dpp(top, OpMax(), -INFINITY);
        const double pup = __shfl_up(pmax, 1, 64);
        const double floor_ = lane ? pup : -INFINITY;
        int hi[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const double v = fmax(base + c[i], floor_);
            const bool last = (4 * lane + i == count - 1);
            const double Ck = last ? off1 : fmin(off0 + v, off1);
            const double y = Ck * sN;
            hi[i] = (k0 + i == Nc - 1) ? Nc : count_points_below(y, d, Ncd);
            if (I.ykey && 4 * lane + i < count) gptr(I.ykey)[k0 + i] = y;
        }
        if (I.selection == SEL_EQ) {
            const int prev = __shfl_up(hi[3], 1, 64);
            int lo = lane ? prev : count_points_below(off0 * sN, d, Ncd);
            const auto anc = gptr(I.anc);
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                // a lane writes up to kShortRun slots of each of its clones; the
                // rest of a longer range (one clone pulled into many slots, as
                // strongly concentrated weights give) the whole wave writes, 64
                // slots a pass, so no lane runs a range alone
                const bool mine = 4 * lane + i < count;
                const int end = mine ? hi[i] : lo;
                const int cut = min(end, lo + kShortRun);
                for (int jj = lo; jj < cut; ++jj) anc[jj] = k0 + i;
                uint64_t longs = __ballot(cut < end);
                while (longs) {
                    const int src = __builtin_ctzll(longs);
                    longs &= longs - 1;
                    const int a = __builtin_amdgcn_readlane(cut, src);
                    const int z = __builtin_amdgcn_readlane(end, src);
                    const int v = __builtin_amdgcn_readlane(k0 + i, src);
                    for (int jj = a + lane; jj < z; jj += 64) anc[jj] = v;
                }
                lo = hi[i];
            }
        }
    }
}

// [iid] selection (Sec. 4.1): new slot j draws its own point, uniform on the
// cumulative line, Nc v_j in units of the point spacing with v_j in (0, 1)
// from 53 bits of the IID stream of (slot j, interval beta), and is pulled
// from the clone whose interval holds it: a_j = #{k : y_k <= Nc v_j}, found by
// binary search over the interval ends y_k that k_resample wrote.
__global__ __launch_bounds__(kTile) void k_select_iid(const InstDev* __restrict__ insts,
                                                      const TileDesc* __restrict__ tiles)
{
    const TileDesc td = tiles[blockIdx.x];
    const InstDev& I = insts[td.inst];
    if (I.selection != SEL_IID || (int)threadIdx.x >= td.count) return;
    const int64_t j = td.first + threadIdx.x;
    const int64_t Nc = I.Nc;
    const uint32_t beta = (uint32_t)I.ctl->beta;
    const uint4 y = philox10(0u, (uint32_t)j, beta, TAG_IID | I.tag_hi, I.key0, I.key1);
    const double hi = (double)y.x * 2097152.0;          // y.x * 2^21
    const double lo = (double)(y.y >> 11) + 0.5;
    const double pt = ((hi + lo) * 0x1p-53) * (double)Nc;
    const auto yk = gptr(I.ykey);
    int64_t a = 0, b = Nc;   // answer in [a, b]
    while (a < b) {
        const int64_t mid = a + (b - a) / 2;
        if (yk[mid] <= pt) a = mid + 1; else b = mid;
    }
    gptr(I.anc)[j] = (int32_t)(a < Nc ? a : Nc - 1);
}

// Sums of K and of its burn-in snapshot over the current population (through
// the ancestor map if any).
__global__ __launch_bounds__(kTile) void k_ksum(const InstDev* __restrict__ insts,
                                                const TileDesc* __restrict__ tiles, int cur,
                                                int use_anc)
{
    __shared__ uint64_t s_u[kTile / 64];
    const TileDesc td = tiles[blockIdx.x];
    const InstDev& I = insts[td.inst];
    const int tid = threadIdx.x;
    uint64_t v = 0, q = 0;
    if (tid < td.count) {
        const int64_t j = td.first + tid;
        const int64_t from = use_anc ? (int64_t)I.anc[j] : j;
        v = I.K[cur][from];
        if (I.ksnap[0]) q = I.ksnap[cur][from];
    }
    const uint64_t s = block_reduce(v, OpSum(), s_u);
    if (tid == 0) atomicAdd((unsigned long long*)&I.ctl->ksum, (unsigned long long)s);
    if (I.ksnap[0]) {
        __syncthreads();   // s_u is reused
        const uint64_t sq = block_reduce(q, OpSum(), s_u);
        if (tid == 0) atomicAdd((unsigned long long*)&I.ctl->ksnap_sum, (unsigned long long)sq);
    }
}

__global__ void k_zero_ksum(const InstDev* __restrict__ insts, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        insts[i].ctl->ksum = 0;
        insts[i].ctl->ksnap_sum = 0;
    }
}

// The burn-in snapshot of the carried K, for the interval about to be stepped
// (beta = the completed intervals + 1; launched before the dynamical stage):
// in interval burn_in + 1 every new clone j records the K it inherits (its
// ancestor's K at the end of interval burn_in); in later intervals it
// inherits its ancestor's record, as K itself is inherited.  K minus the
// record is then the hops of the intervals beyond burn_in along the clone's
// ancestral line (the transient-excluded activity, Sec. 5.1).
__global__ __launch_bounds__(kTile) void k_carry_burn(const InstDev* __restrict__ insts,
                                                      const TileDesc* __restrict__ tiles,
                                                      int src, int use_anc)
{
    const TileDesc td = tiles[blockIdx.x];
    const InstDev& I = insts[td.inst];
    if (!I.ksnap[0] || (int)threadIdx.x >= td.count) return;
    const int64_t beta = I.ctl->beta + 1;
    if (beta <= I.burn_in) return;
    const int64_t j = td.first + threadIdx.x;
    const int64_t from = use_anc ? (int64_t)gptr(I.anc)[j] : j;
    gptr(I.ksnap[src ^ 1])[j] = beta == I.burn_in + 1 ? gptr(I.K[src])[from]
                                                       : gptr(I.ksnap[src])[from];
}

// Materialise the population: dst[j] = src[anc[j]] for the state, K and the
// carried origins, burn-in snapshots and guided rates.
template <int W>
__global__ __launch_bounds__(kTile) void k_gather(const InstDev* __restrict__ insts,
                                                  const TileDesc* __restrict__ tiles,
                                                  int tile_base, int src)
{
    const TileDesc td = tiles[tile_base + blockIdx.x];
    const InstDev& I = insts[td.inst];
    if ((int)threadIdx.x >= td.count) return;
    const int64_t j = td.first + threadIdx.x;
    const int64_t from = I.anc[j];
    const int64_t Nc = I.Nc;
#pragma unroll
    for (int w = 0; w < W; ++w) I.state[src ^ 1][w * Nc + j] = I.state[src][w * Nc + from];
    I.K[src ^ 1][j] = I.K[src][from];
    if (I.origin[0]) I.origin[src ^ 1][j] = I.origin[src][from];
    if (I.ksnap[0]) I.ksnap[src ^ 1][j] = I.ksnap[src][from];
    if (I.rate[0]) I.rate[src ^ 1][j] = I.rate[src][from];
}

// origin[cur][j] = j for every clone of instance `inst`.
__global__ void k_iota_origin(const InstDev* __restrict__ insts, int inst, int cur)
{
    const InstDev& I = insts[inst];
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < I.Nc) I.origin[cur][j] = (int32_t)j;
}

hipError_t launch_iota_origin(const InstDev* insts, int inst, int64_t Nc, int cur, hipStream_t st)
{
    hipLaunchKernelGGL(k_iota_origin, dim3((unsigned)((Nc + 255) / 256)), dim3(256), 0, st, insts,
                       inst, cur);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
hipError_t launch_init(const InstDev* insts, int n_inst, const TileDesc* tiles, int ntiles,
                       hipStream_t st)
{
    const int nr = n_inst > kMaxGroups ? n_inst : kMaxGroups;
    hipLaunchKernelGGL(k_reset_ctl, dim3((nr + 63) / 64), dim3(64), 0, st, insts, n_inst);
    hipLaunchKernelGGL(k_init, dim3(ntiles), dim3(kTile), 0, st, insts, tiles);
    return hipGetLastError();
}

#define PD_W_SWITCH(W, CASE)                                                                  \
    switch (W) {                                                                              \
        CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)                       \
        default: return hipErrorInvalidValue;                                                 \
    }

hipError_t launch_step(const StepLaunch& s, const InstDev* insts, const TileDesc* tiles, int src,
                       int use_anc, hipStream_t st)
{
    if (s.count <= 0) return hipSuccess;
    if (s.guided) {
        return launch_step_guided(s.W, s.count, insts, tiles, s.base, src, use_anc, st);
    } else if (s.variant == 0) {
#define PD_CASE(w)                                                                            \
    case w:                                                                                   \
        hipLaunchKernelGGL(k_step<w>, dim3(s.count), dim3(kTile), 0, st, insts, tiles,        \
                           s.base, src, use_anc);                                             \
        break;
        PD_W_SWITCH(s.W, PD_CASE)
#undef PD_CASE
    } else if (s.variant == 4) {
#define PD_CASE(w)                                                                            \
    case w:                                                                                   \
        hipLaunchKernelGGL(k_step_c<w>, dim3(s.count), dim3(kTile), 0, st, insts, tiles,      \
                           s.base, src, use_anc, s.refill);                                   \
        break;
        PD_W_SWITCH(s.W, PD_CASE)
#undef PD_CASE
    } else if (s.variant == 5) {
        // one persistent launch over every plain tile; s.W is the bucket (2, 4, 8)
        switch (s.W) {
            case 2: hipLaunchKernelGGL(k_step_cp<2>, dim3(s.blocks), dim3(kTile), 0, st, insts,
                                       tiles, s.base, s.count, s.counter, src, use_anc, s.refill);
                    break;
            case 4: hipLaunchKernelGGL(k_step_cp<4>, dim3(s.blocks), dim3(kTile), 0, st, insts,
                                       tiles, s.base, s.count, s.counter, src, use_anc, s.refill);
                    break;
            case 8: hipLaunchKernelGGL(k_step_cp<8>, dim3(s.blocks), dim3(kTile), 0, st, insts,
                                       tiles, s.base, s.count, s.counter, src, use_anc, s.refill);
                    break;
            default: return hipErrorInvalidValue;
        }
    } else if (s.variant == 1) {
#define PD_CASE(w)                                                                            \
    case w:                                                                                   \
        hipLaunchKernelGGL((k_step_q<w, 4>), dim3(s.blocks), dim3(64 * kQWaves), 0, st, insts, \
                           tiles, s.base, s.count, s.counter, src, use_anc, s.refill);        \
        break;
        PD_W_SWITCH(s.W, PD_CASE)
#undef PD_CASE
    } else if (s.variant == 2) {
#define PD_CASE(w)                                                                            \
    case w:                                                                                   \
        hipLaunchKernelGGL((k_step_q<w, 6>), dim3(s.blocks), dim3(64 * kQWaves), 0, st, insts, \
                           tiles, s.base, s.count, s.counter, src, use_anc, s.refill);        \
        break;
        PD_W_SWITCH(s.W, PD_CASE)
#undef PD_CASE
    } else {
#define PD_CASE(w)                                                                            \
    case w:                                                                                   \
        hipLaunchKernelGGL((k_step_q<w, 8>), dim3(s.blocks), dim3(64 * kQWaves), 0, st, insts, \
                           tiles, s.base, s.count, s.counter, src, use_anc, s.refill);        \
        break;
        PD_W_SWITCH(s.W, PD_CASE)
#undef PD_CASE
    }
    return hipGetLastError();
}

hipError_t step_occupancy(int W, int variant, int* blocks_per_cu)
{
    *blocks_per_cu = 0;
    if (variant == 0) {
#define PD_CASE(w)                                                                            \
    case w:                                                                                   \
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_step<w>, kTile, 0);
        PD_W_SWITCH(W, PD_CASE)
#undef PD_CASE
    }
    if (variant == 4) {
#define PD_CASE(w)                                                                            \
    case w:                                                                                   \
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_step_c<w>, kTile, 0);
        PD_W_SWITCH(W, PD_CASE)
#undef PD_CASE
    }
    if (variant == 5) {
        switch (W) {
            case 2: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_step_cp<2>, kTile, 0);
            case 4: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_step_cp<4>, kTile, 0);
            case 8: return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_step_cp<8>, kTile, 0);
            default: return hipErrorInvalidValue;
        }
    }
#define PD_CASE(w)                                                                            \
    case w:                                                                                   \
        if (variant == 1)                                                                     \
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu,               \
                                                                k_step_q<w, 4>, 64 * kQWaves, 0); \
        if (variant == 2)                                                                     \
            return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu,               \
                                                                k_step_q<w, 6>, 64 * kQWaves, 0); \
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k_step_q<w, 8>,   \
                                                            64 * kQWaves, 0);
    PD_W_SWITCH(W, PD_CASE)
#undef PD_CASE
}

hipError_t launch_prefix(const InstDev* insts, int n_inst, hipStream_t st)
{
    hipLaunchKernelGGL(k_prefix, dim3(n_inst), dim3(kTile), 0, st, insts);
    return hipGetLastError();
}

hipError_t launch_resample(const InstDev* insts, const TileDesc* tiles, int ntiles, int tpb,
                           hipStream_t st)
{
    const int waves = (ntiles + tpb - 1) / tpb;
    const int blocks = (waves + kTile / 64 - 1) / (kTile / 64);
    switch (tpb) {
        case 1: hipLaunchKernelGGL(k_resample<1>, dim3(blocks), dim3(kTile), 0, st, insts, tiles, ntiles); break;
        case 2: hipLaunchKernelGGL(k_resample<2>, dim3(blocks), dim3(kTile), 0, st, insts, tiles, ntiles); break;
        case 4: hipLaunchKernelGGL(k_resample<4>, dim3(blocks), dim3(kTile), 0, st, insts, tiles, ntiles); break;
        case 8: hipLaunchKernelGGL(k_resample<8>, dim3(blocks), dim3(kTile), 0, st, insts, tiles, ntiles); break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_select_iid(const InstDev* insts, const TileDesc* tiles, int ntiles,
                             hipStream_t st)
{
    hipLaunchKernelGGL(k_select_iid, dim3(ntiles), dim3(kTile), 0, st, insts, tiles);
    return hipGetLastError();
}

hipError_t launch_zero_ksum(const InstDev* insts, int n_inst, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_ksum, dim3((n_inst + 63) / 64), dim3(64), 0, st, insts, n_inst);
    return hipGetLastError();
}

hipError_t launch_ksum(const InstDev* insts, const TileDesc* tiles, int ntiles, int cur,
                       int use_anc, hipStream_t st)
{
    hipLaunchKernelGGL(k_ksum, dim3(ntiles), dim3(kTile), 0, st, insts, tiles, cur, use_anc);
    return hipGetLastError();
}

hipError_t launch_carry_burn(const InstDev* insts, const TileDesc* tiles, int ntiles, int src,
                             int use_anc, hipStream_t st)
{
    hipLaunchKernelGGL(k_carry_burn, dim3(ntiles), dim3(kTile), 0, st, insts, tiles, src, use_anc);
    return hipGetLastError();
}

hipError_t launch_gather(int W, const InstDev* insts, const TileDesc* tiles, int tile_base,
                         int ntiles, int src, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
#define PD_CASE(w)                                                                            \
    case w:                                                                                   \
        hipLaunchKernelGGL(k_gather<w>, dim3(ntiles), dim3(kTile), 0, st, insts, tiles,       \
                           tile_base, src);                                                   \
        break;
    PD_W_SWITCH(W, PD_CASE)
#undef PD_CASE
    return hipGetLastError();
}

}  // namespace pd
