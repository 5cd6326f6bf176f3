// Guided dynamical stage for gfx950 (arXiv:1711.05095, Sec. 2.2): the
// continuous-time SSEP with every allowed hop's rate multiplied by a guide
// factor from a table over the bond's 13-site neighbourhood, and the exact
// compensating weight that keeps psi-hat unbiased.  One clone per lane in two
// launches (a budgeted one, then the unfinished clones densely), and the tile
// aggregates of the plain step kernels (pd_tile.hpp) in a third.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "pd_device.hpp"
#include "pd_internal.hpp"
#include "pd_launch.hpp"
#include "pd_tile.hpp"

namespace pd {

// ---------------------------------------------------------------------------
// Dynamical stage with a guide (eqs. modpdef, upsdef of Sec. 2.2), one clone
// per lane.  The guide is the table eg[u] over 13-site bond neighbourhoods
// (site b-6 in bit 0; the bond's sites in bits 6 and 7): the hop across an
// allowed bond b has rate e^{-s} eg[u_b] 2^-16.  S = sum of eg over allowed
// bonds is kept exactly in integers, so the escape rate is e^{-s} S 2^-16,
// and the compensating factor is
// ln Ups = -sum_jumps ln(eg 2^-16) - int (r - e^{-s} S 2^-16) dt.
// The jumps come by thinning: proposals at rate e^{-s} eg_max 2^-16 per
// allowed bond (a bound of every controlled rate, so the waiting time is E
// times a per-r table, no division), each across a uniform allowed bond,
// taken with probability eg / eg_max.  Every pass of the loop is one proposal
// and draws one Philox block, so no lane waits on another lane's retries.
// Random numbers of a clone in interval beta: proposal k (counted over the
// interval from 0) takes block (k, slot, beta, GUIDE): the waiting time from
// words 0, 1, the 64-bit bond word bw from words 2, 3, the bond q =
// floor(bw r / 2^64) among the allowed ones, and the acceptance word
// (bw r) mod 2^64, taken iff floor(word eg_max / 2^64) < eg.
// The whole table sits in LDS: its entries of neighbourhoods whose bond is no
// hop are 0, so a sum over neighbourhoods needs no test of the bond.
// sum_jumps ln eg is formed as the logarithm of the running product of the eg,
// kept in [0.5, 1) by frexp with the binary exponents summed separately.
// ---------------------------------------------------------------------------

// i mod L in [0, L) for i >= -L * 8.
__device__ __forceinline__ int ring_mod(int i, int L)
{
    while (i < 0) i += L;
    return i;
}

// ring_bits for a window no longer than the ring (n <= L, n <= 32): at most
// two pieces, the second one from site 0, formed without a loop.
template <int W>
__device__ __forceinline__ uint32_t ring_bits_short(const uint64_t (&x)[W], int L, int p, int n)
{
    const int take = min(n, L - p);                 // >= 1
    const int rest = n - take;                      // sites wrapped to 0 .. rest-1
    const uint32_t wrapped = (uint32_t)x[0] & ((1u << rest) - 1u);
    return lin_bits<W>(x, p, take) | (rest ? wrapped << take : 0u);
}

__device__ __forceinline__ bool bond_allowed(uint32_t u) { return ((u >> 6) ^ (u >> 7)) & 1u; }


template <int W>
__device__ __forceinline__ uint64_t guided_total(const uint64_t (&x)[W], const uint64_t (&m)[W],
                                                 int L, const uint32_t* eg)
{
    uint64_t S = 0;
#pragma unroll
    for (int w = 0; w < W; ++w) {
        uint64_t bits = m[w];
        while (bits) {
            const int b = w * 64 + __builtin_ctzll(bits);
            bits &= bits - 1;
            S += eg[ring_bits<W>(x, L, ring_mod(b - 6, L), 13)];
        }
    }
    return S;
}

// The guided stage runs in two launches of this kernel (one when the launch is
// small, see kSplitTiles).  CONT = false: one clone per lane, at most
// ev_budget events (about 1.1 times the mean of the previous interval); a
// clone not done by then is handed on, registers and slot, to the second
// launch.  CONT = true: block b of an instance's tiles takes the handed-on
// clones 256 b .. 256 b + 255 (in hand-on order) and runs each to the end of
// the interval, so a wave of the first launch never waits for the Poisson
// tail of its 64 clones.  Random numbers are keyed by slot and by the event
// and proposal indices the clone carries, so the split changes no result.
template <int W, bool CONT>
__global__ __launch_bounds__(kTile) void k_step_g(const InstDev* __restrict__ insts,
                                                  const TileDesc* __restrict__ tiles,
                                                  int tile_base, int src, int use_anc,
                                                  int budgeted)
{
    __shared__ __align__(16) uint32_t s_eg[kGuideEntries];
    __shared__ double s_log[kLogRows * kLogCols];
    __shared__ double s_invg[64 * W + 1];   // guide_scale / r: 1 / (proposal rate), r <= 64 W
    __shared__ __align__(8) uint8_t s_sel[2048];

    // a block runs a whole tile, or (blocks of one wave, for launches smaller
    // than the chip, so that the waves spread over more CUs) a quarter of one
    const bool quarter = blockDim.x == 64u;          // uniform: no division
    const int nb = quarter ? 64 : kTile;
    const int sub = quarter ? (int)(blockIdx.x & 3u) : 0;
    const TileDesc td = tiles[tile_base + (int)(quarter ? blockIdx.x >> 2 : blockIdx.x)];
    const InstDev& I = insts[td.inst];
    const int L = I.L;
    const int64_t Nc = I.Nc;
    const uint32_t ncont = CONT ? I.ctl->ncont : 0u;
    // first handed-on clone of the block
    const uint32_t e0 = (uint32_t)td.tile * kTile + (uint32_t)(sub * nb);
    if (CONT && e0 >= ncont) return;                  // uniform over the block
    for (int i = threadIdx.x; i < kLogRows * kLogCols; i += nb) s_log[i] = gptr(I.log_tab)[i];
    for (int i = threadIdx.x; i <= 64 * W; i += nb)
        s_invg[i] = I.guide_scale * gptr(I.inv_count)[i];
    load_select_table(s_sel, I.sel_tab, threadIdx.x, nb);
    // 16-byte pieces (the host checks the table's alignment)
    for (int i = threadIdx.x; i < kGuideEntries / 4; i += nb)
        reinterpret_cast<uint4*>(s_eg)[i] = reinterpret_cast<const uint4*>(I.guide)[i];
    __syncthreads();

    const int tid = sub * nb + (int)threadIdx.x;       // the clone's place in its tile
    const uint32_t q = (uint32_t)td.tile * kTile + (uint32_t)tid;   // handed-on clone (CONT)
    if (CONT ? q >= ncont : tid >= td.count) return;  // no barrier follows
    const uint32_t beta = (uint32_t)(I.ctl->beta + 1);
    const uint32_t c3 = TAG_GUIDE | I.tag_hi;
    const double es = I.es, dt = I.dt;
    const uint64_t egmax = I.guide_max;
    // 14 entries of at most egmax each fit 32 bits (true for any guide whose
    // largest entry is below 2^32 / 14)
    const bool narrow = egmax <= 0xFFFFFFFFull / 14u;
    double poly[kLogPoly];   // log1p coefficients as uniform operands
#pragma unroll
    for (int w = 0; w < kLogPoly; ++w) poly[w] = I.log_poly[w];
    const int dst = src ^ 1;
    const int lb = (L - 1) & 63;

    int64_t j;
    uint64_t x[W], m[W], Kfrom, S;
    uint32_t k, kb;
    double tau, A, AS, P;
    int pexp;
    if (CONT) {
        j = gptr(I.cont_u32)[q];
#pragma unroll
        for (int w = 0; w < W; ++w) x[w] = gptr(I.cont_u64)[w * Nc + q];
        Kfrom = gptr(I.cont_u64)[W * Nc + q];
        S = gptr(I.cont_u64)[(W + 1) * Nc + q];
        tau = gptr(I.cont_f64)[q];
        A = gptr(I.cont_f64)[Nc + q];
        AS = gptr(I.cont_f64)[2 * Nc + q];
        P = gptr(I.cont_f64)[3 * Nc + q];
        k = gptr(I.cont_u32)[Nc + q];
        kb = gptr(I.cont_u32)[2 * Nc + q];
        pexp = (int)gptr(I.cont_u32)[3 * Nc + q];
        bond_mask<W>(x, lb, m);
    } else {
        j = td.first + tid;
        const int64_t from = use_anc ? (int64_t)gptr(I.anc)[j] : j;
#pragma unroll
        for (int w = 0; w < W; ++w) x[w] = gptr(I.state[src])[w * Nc + from];
        Kfrom = gptr(I.K[src])[from];
        if (I.origin[0]) gptr(I.origin[dst])[j] = gptr(I.origin[src])[from];
        bond_mask<W>(x, lb, m);
        // S as the clone's ancestor ended the last interval (the same integer
        // the sum over the allowed hops gives), unless the population or the
        // table has changed since
        S = I.ctl->s_carried ? gptr(I.rate[src])[from] : guided_total<W>(x, m, L, s_eg);
        tau = 0.0; A = 0.0; AS = 0.0; P = 1.0;
        k = 0; kb = 0; pexp = 0;
    }
    int r = popcount_words<W>(m);
    const uint32_t eb = (CONT || !budgeted) ? 0u : I.ctl->ev_budget;
    const uint32_t kend = eb ? eb : 0xFFFFFFFFu;   // the first launch stops at event kend
    bool done = true;
    // A draw's random numbers depend only on (draw index, slot, interval), not
    // on the state: those of draw k + 1 are formed while draw k is decided, so
    // their chain of dependent instructions runs beside the bond choice.  They
    // are formed only where another draw follows (not after the closing one).
    uint4 y{0u, 0u, 0u, 0u};
    double E = 0.0;
    if (r > 0 && (CONT || k < kend)) {
        y = philox10(k, (uint32_t)j, beta, c3, I.key0, I.key1);
        E = -log_unit(unit_scaled(y.x, y.y), s_log, I.ln2_hi, I.ln2_lo, poly, 53);
    }
    while (r > 0 && k < (1u << 30)) {
        if (!CONT && k >= kend) {
            done = false;
            break;
        }
        ++k;
        // waiting time of the next proposal: E / (e^{-s} eg_max 2^-16 r)
        const double w = E * s_invg[r];
        if (tau + w >= dt) {
            A = fma((double)r, dt - tau, A);
            AS = fma((double)S, dt - tau, AS);
            break;
        }
        A = fma((double)r, w, A);
        AS = fma((double)S, w, AS);
        tau = tau + w;
        const uint32_t yz = y.z, yw = y.w;
        y = philox10(k, (uint32_t)j, beta, c3, I.key0, I.key1);
        E = -log_unit(unit_scaled(y.x, y.y), s_log, I.ln2_hi, I.ln2_lo, poly, 53);
        // bw r = q 2^64 + a with bw = (y.z << 32) | y.w: the bond and the acceptance word
        const uint64_t plo = (uint64_t)yw * (uint32_t)r;
        const uint64_t phi = (uint64_t)yz * (uint32_t)r + (plo >> 32);
        const int b = select_bit_lut<W>(m, (uint32_t)(phi >> 32), s_sel);
        uint32_t e, win0 = 0;          // L >= 26: the 26 sites from b-12
        // the neighbourhood of b is bits 6..18 of the window from b-12, which
        // the update after a hop reuses
        if (L >= 26) {
            win0 = ring_bits_short<W>(x, L, b >= 12 ? b - 12 : b - 12 + L, 26);
            e = s_eg[(win0 >> 6) & 0x1FFFu];
        } else {
            e = s_eg[ring_bits<W>(x, L, ring_mod(b - 6, L), 13)];
        }
        // taken iff floor(a eg_max / 2^64) < e, a = (phi << 32) | (plo mod 2^32)
        if (mulhi64_small((uint32_t)phi, (uint32_t)plo, (uint32_t)egmax) >= e) continue;
        P *= (double)e;
        pexp += __builtin_amdgcn_frexp_exp(P);
        P = __builtin_amdgcn_frexp_mant(P);
        if (L >= 26) {
            // the 14 bonds whose neighbourhood holds site b or b+1 are
            // bits o..o+12 of the 26 sites from b-12, o = 0..13
            const uint32_t win1 = win0 ^ (3u << 12);
            // branch-free: all 14 neighbourhoods are read before and after;
            // those whose bond is no hop read 0 (`narrow` is the same for
            // every lane of the launch)
            uint64_t add = 0, sub = 0;
            if (narrow) {
                uint32_t add32 = 0, sub32 = 0;
#pragma unroll
                for (int o = 0; o < 14; ++o) {
                    sub32 += s_eg[(win0 >> o) & 0x1FFFu];
                    add32 += s_eg[(win1 >> o) & 0x1FFFu];
                }
                add = add32;
                sub = sub32;
            } else {
#pragma unroll
                for (int o = 0; o < 14; ++o) {
                    sub += s_eg[(win0 >> o) & 0x1FFFu];
                    add += s_eg[(win1 >> o) & 0x1FFFu];
                }
            }
            hop<W>(x, b, L);
            bond_mask<W>(x, lb, m);
            S = S + add - sub;
        } else {
            hop<W>(x, b, L);
            bond_mask<W>(x, lb, m);
            S = guided_total<W>(x, m, L, s_eg);
        }
        r = popcount_words<W>(m);
        ++kb;
    }
    if (!done) {
        // one atomic per wave (the counter is shared by every block of the
        // instance): the wave's handing-on lanes take consecutive entries
        const int lane = tid & 63;
        const uint64_t hm = __ballot(1);
        const int lead = __ffsll((unsigned long long)hm) - 1;
        const uint32_t rank = (uint32_t)__popcll(hm & ((1ull << lane) - 1ull));
        uint32_t base = 0;
        if (lane == lead) base = atomicAdd(&I.ctl->ncont, (uint32_t)__popcll(hm));
        const uint32_t h = (uint32_t)__shfl((int)base, lead, 64) + rank;
#pragma unroll
        for (int w = 0; w < W; ++w) gptr(I.cont_u64)[w * Nc + h] = x[w];
        gptr(I.cont_u64)[W * Nc + h] = Kfrom;
        gptr(I.cont_u64)[(W + 1) * Nc + h] = S;
        gptr(I.cont_f64)[h] = tau;
        gptr(I.cont_f64)[Nc + h] = A;
        gptr(I.cont_f64)[2 * Nc + h] = AS;
        gptr(I.cont_f64)[3 * Nc + h] = P;
        gptr(I.cont_u32)[h] = (uint32_t)j;
        gptr(I.cont_u32)[Nc + h] = k;
        gptr(I.cont_u32)[2 * Nc + h] = kb;
        gptr(I.cont_u32)[3 * Nc + h] = (uint32_t)pexp;
        return;
    }
    // sum_jumps ln(eg 2^-16) = ln P + (pexp - 16 kb) ln 2
    const double G = log_unit(P, s_log, I.ln2_hi, I.ln2_lo, poly, 0) +
                     (double)(pexp - 16 * (int)kb) * (I.ln2_hi + I.ln2_lo);
    const double ell = -G - (A - (es * 0x1p-16) * AS);
#pragma unroll
    for (int w = 0; w < W; ++w) gptr(I.state[dst])[w * Nc + j] = x[w];
    gptr(I.K[dst])[j] = Kfrom + kb;
    gptr(I.Kb)[j] = kb;
    gptr(I.A)[j] = A;
    gptr(I.ell)[j] = ell;
    gptr(I.iters)[j] = k;
    gptr(I.rate[dst])[j] = S;
}

// Tile aggregates from the outputs written by slot, one wave per tile (the
// order of tile_aggregate, as in every step kernel).
__global__ __launch_bounds__(kTile) void k_tile_stats(const InstDev* __restrict__ insts,
                                                      const TileDesc* __restrict__ tiles,
                                                      int tile_base, int count)
{
    const int t = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * (kTile / 64) +
                                                       (threadIdx.x >> 6)));
    if (t >= count) return;   // uniform over the wave; no barrier follows
    const TileDesc td = tiles[tile_base + t];
    const InstDev& I = insts[td.inst];
    uint64_t h = 0, it = 0;
    for (int i = threadIdx.x & 63; i < td.count; i += 64) {
        h += gptr(I.Kb)[td.first + i];
        it += gptr(I.iters)[td.first + i];
    }
    tile_aggregate(I, td.tile, I.ell + td.first, td.count, h);
    // proposals of the tile, for the next interval's event budget (k_prefix)
    it = wave_reduce(it, OpSum());
    if ((threadIdx.x & 63) == 0)
        atomicAdd((unsigned long long*)&I.ctl->iters, (unsigned long long)it);
}

hipError_t launch_tile_stats(const InstDev* insts, const TileDesc* tiles, int base, int count,
                             hipStream_t st)
{
    const int blocks = (count + kTile / 64 - 1) / (kTile / 64);
    hipLaunchKernelGGL(k_tile_stats, dim3(blocks), dim3(kTile), 0, st, insts, tiles, base, count);
    return hipGetLastError();
}

hipError_t launch_step_guided(int W, int count, const InstDev* insts, const TileDesc* tiles,
                              int base, int src, int use_anc, hipStream_t st)
{
    const int split = count >= kSplitTiles;
    // fewer tiles than CUs: one-wave blocks, a quarter tile each
    const int nsub = count < kQuarterTiles ? 4 : 1;
    switch (W) {
#define PD_CASE(w)                                                                            \
    case w:                                                                                   \
        hipLaunchKernelGGL((k_step_g<w, false>), dim3(count * nsub), dim3(kTile / nsub), 0,  \
                           st, insts, tiles, base, src, use_anc, split);                     \
        if (split)                                                                            \
            hipLaunchKernelGGL((k_step_g<w, true>), dim3(count * nsub), dim3(kTile / nsub),  \
                               0, st, insts, tiles, base, src, use_anc, 1);                  \
        break;
        PD_CASE(1) PD_CASE(2) PD_CASE(3) PD_CASE(4) PD_CASE(5) PD_CASE(6) PD_CASE(7)
        PD_CASE(8)
#undef PD_CASE
        default: return hipErrorInvalidValue;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_tile_stats(insts, tiles, base, count, st);
}

}  // namespace pd
