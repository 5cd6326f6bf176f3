// HIP kernels of the cloning algorithm for gfx950 (MI355X).
//
// One cycle of the algorithm (arXiv:1711.05095, Sec. 2.3) is two launches:
//
//   k_step     the dynamical stage (Sec. 4, first paragraph): one clone per
//              lane, its occupancy bit-packed in registers, continuous-time
//              (BKL) hops for one interval Delta t driven by Philox4x32-10.
//              A clone's state is pulled through the ancestor map of the
//              previous cloning stage as it is loaded, so the copy of the
//              surviving clones (Sec. 6.1) is fused into this load.  Each
//              block reduces its tile's log-weights to (max, sum of exp); the
//              last block of an instance forms the population mean of
//              Upsilon (eq. psihat), the tile prefix offsets and the total.
//   k_resample the cloning stage (Sec. 4.1, eq. alpha-Ups): an FP64 scan of
//              the weights over each tile on top of its prefix offset, the
//              interval ends y_k in units of the point spacing, and for every
//              old clone k the range of new slots j whose point j + d falls in
//              its interval; k writes itself as the ancestor of those slots.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pd_device.hpp"
#include "pd_internal.hpp"
#include "pd_launch.hpp"

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
    if (i >= n) return;
    InstCtl* c = insts[i].ctl;
    c->beta = 0;
    c->tiles_done = 0;
    c->tiles_done2 = 0;
    c->lmax = 0.0;
    c->lbeta = 0.0;
    c->psi_sum = c->psi_comp = 0.0;
    c->psib_sum = c->psib_comp = 0.0;
    c->hops = 0;
    c->ksum = 0;
}

// Neumaier compensated addition.
__device__ __forceinline__ void neumaier_add(double& sum, double& comp, double x)
{
    const double t = sum + x;
    if (fabs(sum) >= fabs(x)) comp += (sum - t) + x;
    else comp += (x - t) + sum;
    sum = t;
}

// The last block of an instance's step launch: population statistics of the
// interval from the per-tile (max, sum exp, hops).  Block-wide.  Produces
// lmax, ln mean Upsilon, and the tile offsets tile_off[0..n] (exclusive
// prefix sums of the tile weights in the scale exp(. - lmax)), made
// non-decreasing by a running maximum so that rounding can never reorder
// interval ends; tile_off[n] is the total weight T.
__device__ __forceinline__ double tile_weight(const InstDev& I, int b, double M)
{
    return I.tile_sum[b] * exp(I.tile_max[b] - M);
}

__device__ void finish_interval(const InstDev& I, uint32_t beta)
{
    __shared__ double s_d[kTile / 64];
    __shared__ uint64_t s_u[kTile / 64];
    __shared__ double s_x[kTile];
    const int n = I.ntiles;
    const int tid = threadIdx.x;

    double m = -INFINITY;
    uint64_t h = 0;
    for (int b = tid; b < n; b += kTile) {
        m = fmax(m, I.tile_max[b]);
        h += I.tile_hops[b];
    }
    const double M = block_reduce(m, OpMax(), s_d);
    const uint64_t hops = block_reduce(h, OpSum(), s_u);

    // thread tid owns tiles [b0, b1)
    const int ch = (n + kTile - 1) / kTile;
    const int b0 = min(tid * ch, n), b1 = min(b0 + ch, n);
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
    const double T = fmax(total, all_max);

    if (tid == 0) {
        I.tile_off[n] = T;
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
        c->tiles_done = 0;
    }
}

// ---------------------------------------------------------------------------
// Dynamical stage.
// ---------------------------------------------------------------------------
template <int W>
__global__ __launch_bounds__(kTile) void k_step(const InstDev* __restrict__ insts,
                                                const TileDesc* __restrict__ tiles, int tile_base,
                                                int src, int use_anc)
{
    __shared__ double s_inv[kMaxSites + 1];
    __shared__ double s_d[kTile / 64];
    __shared__ uint64_t s_u[kTile / 64];
    __shared__ int s_last;

    const TileDesc td = tiles[tile_base + blockIdx.x];
    const InstDev& I = insts[td.inst];
    const int L = I.L;
    for (int i = threadIdx.x; i <= L; i += kTile) s_inv[i] = I.inv_rate[i];
    __syncthreads();

    const uint32_t beta = (uint32_t)(I.ctl->beta + 1);
    const int tid = threadIdx.x;
    const bool valid = tid < td.count;
    const int64_t j = td.first + tid;
    const int64_t Nc = I.Nc;

    uint32_t kb = 0;
    double A = 0.0, ell = -INFINITY;
    if (valid) {
        const int64_t from = use_anc ? (int64_t)I.anc[j] : j;
        uint64_t x[W];
#pragma unroll
        for (int w = 0; w < W; ++w) x[w] = I.state[src][w * Nc + from];
        const uint64_t Kfrom = I.K[src][from];

        const int lb = (L - 1) & 63;
        const double dt = I.dt;
        const uint32_t c3 = TAG_DYN | I.tag_hi;
        uint64_t m[W];
        bond_mask<W>(x, lb, m);
        int r = popcount_words<W>(m);
        double tau = 0.0;
        uint32_t k = 0;
        // k < 2^31: the host admits only parameters with at most 2^24 expected
        // hops per interval, so this bound never binds; it only guarantees an end
        while (r > 0 && k < 0x80000000u) {
            const uint4 y = philox10(k, (uint32_t)j, beta, c3, I.key0, I.key1);
            ++k;
            const double E = -log(unit_open0(y.x, y.y));
            const double w = E * s_inv[r];
            if (tau + w >= dt) {
                A = fma((double)r, dt - tau, A);
                break;
            }
            A = fma((double)r, w, A);
            tau = tau + w;
            const uint32_t q = mulhi64_small(y.z, y.w, (uint32_t)r);
            const int b = select_bit<W>(m, q);
            hop<W>(x, b, L);
            bond_mask<W>(x, lb, m);
            r = popcount_words<W>(m);
            ++kb;
        }
        ell = (I.mode == MODE_MODIFIED) ? -I.c * A : -I.s * (double)kb;

        const int dst = src ^ 1;
#pragma unroll
        for (int w = 0; w < W; ++w) I.state[dst][w * Nc + j] = x[w];
        I.K[dst][j] = Kfrom + kb;
        I.Kb[j] = kb;
        I.A[j] = A;
        I.ell[j] = ell;
    }

    // tile aggregates
    const double tmax = block_reduce(ell, OpMax(), s_d);
    const double e = valid ? exp(ell - tmax) : 0.0;
    const double tsum = block_reduce(e, OpSum(), s_d);
    const uint64_t thops = block_reduce((uint64_t)kb, OpSum(), s_u);
    if (tid == 0) {
        I.tile_max[td.tile] = tmax;
        I.tile_sum[td.tile] = tsum;
        I.tile_hops[td.tile] = thops;
        __threadfence();
        const uint32_t done = atomicAdd(&I.ctl->tiles_done, 1u);
        s_last = (done == (uint32_t)(I.ntiles - 1));
    }
    __syncthreads();
    if (s_last) {
        __threadfence();
        finish_interval(I, beta);
    }
}

// ---------------------------------------------------------------------------
// Cloning stage ([eq]).
// ---------------------------------------------------------------------------

// #{ j in [0, Nc) : j + d < y }, exactly: y - j is exact whenever it lies in
// [0, 1), so the test fl(y - j) > d decides j + d < y without error.
__device__ __forceinline__ int64_t count_points_below(double y, double d, int64_t Nc)
{
    double c = ceil(y - d);
    int64_t m = (c <= 0.0) ? 0 : (c >= (double)Nc ? Nc : (int64_t)c);
    while (m > 0 && !((y - (double)(m - 1)) > d)) --m;
    while (m < Nc && ((y - (double)m) > d)) ++m;
    return m;
}

__device__ __forceinline__ double eq_offset(const InstDev& I, uint32_t beta)
{
    const uint4 y = philox10(0u, 0u, beta, TAG_RESAMPLE | I.tag_hi, I.key0, I.key1);
    const double hi = (double)y.x * 1048576.0;   // y.x * 2^20
    const double lo = (double)(y.y >> 12) + 0.5;
    return (hi + lo) * 0x1p-52;
}

__global__ __launch_bounds__(kTile) void k_resample(const InstDev* __restrict__ insts,
                                                    const TileDesc* __restrict__ tiles)
{
    __shared__ double s_d[kTile / 64];
    __shared__ int64_t s_hi[kTile];
    __shared__ int s_last;

    const TileDesc td = tiles[blockIdx.x];
    const InstDev& I = insts[td.inst];
    const int tid = threadIdx.x;
    const bool valid = tid < td.count;
    const int64_t k = td.first + tid;
    const int64_t Nc = I.Nc;
    const double Ncd = (double)Nc;
    const uint32_t beta = (uint32_t)(I.ctl->beta + 1);
    const double M = I.ctl->lmax;
    const int b = td.tile;
    const double off0 = I.tile_off[b];
    const double off1 = I.tile_off[b + 1];
    const double T = I.tile_off[I.ntiles];
    const double d = eq_offset(I, beta);

    const double w = valid ? exp(I.ell[k] - M) : 0.0;
    double tot;
    double incl = block_scan_incl(w, OpSum(), s_d, tot);
    incl = block_scan_incl(incl, OpMax(), s_d, tot);  // non-decreasing in k
    const bool last = (tid == td.count - 1);
    const double Ck = last ? off1 : fmin(off0 + incl, off1);
    int64_t hi = count_points_below((Ck * Ncd) / T, d, Nc);
    if (k == Nc - 1) hi = Nc;
    s_hi[tid] = hi;
    __syncthreads();
    if (valid) {
        const int64_t lo = (tid == 0) ? count_points_below((off0 * Ncd) / T, d, Nc) : s_hi[tid - 1];
        for (int64_t jj = lo; jj < hi; ++jj) I.anc[jj] = (int32_t)k;
        if (I.ykey) I.ykey[k] = (Ck * Ncd) / T;
    }
    __syncthreads();
    if (tid == 0) {
        __threadfence();
        const uint32_t done = atomicAdd(&I.ctl->tiles_done2, 1u);
        s_last = (done == (uint32_t)(I.ntiles - 1));
    }
    __syncthreads();
    if (s_last && tid == 0) {
        I.ctl->beta += 1;
        I.ctl->tiles_done2 = 0;
    }
}

// Sum of K over the current population (through the ancestor map if any).
__global__ __launch_bounds__(kTile) void k_ksum(const InstDev* __restrict__ insts,
                                                const TileDesc* __restrict__ tiles, int cur,
                                                int use_anc)
{
    __shared__ uint64_t s_u[kTile / 64];
    const TileDesc td = tiles[blockIdx.x];
    const InstDev& I = insts[td.inst];
    const int tid = threadIdx.x;
    uint64_t v = 0;
    if (tid < td.count) {
        const int64_t j = td.first + tid;
        const int64_t from = use_anc ? (int64_t)I.anc[j] : j;
        v = I.K[cur][from];
    }
    const uint64_t s = block_reduce(v, OpSum(), s_u);
    if (tid == 0) atomicAdd((unsigned long long*)&I.ctl->ksum, (unsigned long long)s);
}

// Materialise the population: dst[j] = src[anc[j]] for state and K.
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
}

// ---------------------------------------------------------------------------
// Host-side launchers.
// ---------------------------------------------------------------------------
hipError_t launch_init(const InstDev* insts, int n_inst, const TileDesc* tiles, int ntiles,
                       hipStream_t st)
{
    hipLaunchKernelGGL(k_reset_ctl, dim3((n_inst + 63) / 64), dim3(64), 0, st, insts, n_inst);
    hipLaunchKernelGGL(k_init, dim3(ntiles), dim3(kTile), 0, st, insts, tiles);
    return hipGetLastError();
}

__global__ void k_zero_ksum(const InstDev* __restrict__ insts, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) insts[i].ctl->ksum = 0;
}

hipError_t launch_zero_ksum(const InstDev* insts, int n_inst, hipStream_t st)
{
    hipLaunchKernelGGL(k_zero_ksum, dim3((n_inst + 63) / 64), dim3(64), 0, st, insts, n_inst);
    return hipGetLastError();
}

hipError_t launch_step(int W, const InstDev* insts, const TileDesc* tiles, int tile_base,
                       int ntiles, int src, int use_anc, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    switch (W) {
#define PD_CASE(w)                                                                            \
    case w:                                                                                   \
        hipLaunchKernelGGL(k_step<w>, dim3(ntiles), dim3(kTile), 0, st, insts, tiles,         \
                           tile_base, src, use_anc);                                          \
        break;
        PD_CASE(1) PD_CASE(2) PD_CASE(3) PD_CASE(4) PD_CASE(5) PD_CASE(6) PD_CASE(7) PD_CASE(8)
#undef PD_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_resample(const InstDev* insts, const TileDesc* tiles, int ntiles, hipStream_t st)
{
    hipLaunchKernelGGL(k_resample, dim3(ntiles), dim3(kTile), 0, st, insts, tiles);
    return hipGetLastError();
}

hipError_t launch_ksum(const InstDev* insts, const TileDesc* tiles, int ntiles, int cur,
                       int use_anc, hipStream_t st)
{
    hipLaunchKernelGGL(k_ksum, dim3(ntiles), dim3(kTile), 0, st, insts, tiles, cur, use_anc);
    return hipGetLastError();
}

hipError_t launch_gather(int W, const InstDev* insts, const TileDesc* tiles, int tile_base,
                         int ntiles, int src, hipStream_t st)
{
    if (ntiles <= 0) return hipSuccess;
    switch (W) {
#define PD_CASE(w)                                                                            \
    case w:                                                                                   \
        hipLaunchKernelGGL(k_gather<w>, dim3(ntiles), dim3(kTile), 0, st, insts, tiles,       \
                           tile_base, src);                                                   \
        break;
        PD_CASE(1) PD_CASE(2) PD_CASE(3) PD_CASE(4) PD_CASE(5) PD_CASE(6) PD_CASE(7) PD_CASE(8)
#undef PD_CASE
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace pd
