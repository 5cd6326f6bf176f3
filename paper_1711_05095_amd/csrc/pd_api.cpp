// Host runtime of the library: the C ABI declared in include/pd.h.
//
// The runtime validates parameters, carves the caller's workspace into the
// per-instance arrays, orders the tiles of all instances by estimated cost
// (largest first) for the dynamical stage, and queues the kernels.  Which of
// the two state buffers holds the population, and whether it is still to be
// read through the ancestor map, is tracked here on the host: it changes
// deterministically with every call, so a captured graph of an even number of
// cycles can be replayed with fixed kernel arguments.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/pd.h"
#include "pd_internal.hpp"
#include "pd_launch.hpp"

using namespace pd;

namespace {

thread_local std::string g_create_error;

constexpr size_t kAlign = 256;
constexpr double kMaxEventsPerInterval = 16777216.0;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int words_of(int L) { return (L + 63) / 64; }

int64_t cycles_of(const pd_params& p) { return llround(p.t_obs / p.dt); }

pd_tuning default_tuning()
{
    pd_tuning t;
    t.step_variant = 4;
    t.refill = 13;
    t.graph_cycles = 16;
    t.scan_tiles = 1;
    return t;
}

// Byte table of the device's bond selection: entry b * 8 + q is the position
// of the q-th set bit (ascending) of the byte b for q < popcount(b), else 0.
std::vector<uint8_t> select_table()
{
    std::vector<uint8_t> t(2048, 0);
    for (int b = 0; b < 256; ++b)
        for (int i = 0, q = 0; i < 8; ++i)
            if ((b >> i) & 1) t[b * 8 + q++] = (uint8_t)i;
    return t;
}

// Table of the device logarithm (rows of [c, -ln c (multiple of 2^-42),
// remainder]: row i covers m in [0.75 + 0.75 i/128, 0.75 + 0.75 (i+1)/128)
// and c ~ 1/centre, exactly 1 on the row that holds 1) and the split of ln 2,
// computed in extended precision.
std::vector<double> log_table(double* ln2_hi, double* ln2_lo)
{
    const long double two42 = 4398046511104.0L;
    const long double l2 = logl(2.0L);
    const long double l2h = nearbyintl(l2 * two42) / two42;
    *ln2_hi = (double)l2h;
    *ln2_lo = (double)(l2 - l2h);
    std::vector<double> t(kLogCols * kLogRows, 0.0);
    const long double width = 0.75L / kLogRows;
    for (int i = 0; i < kLogRows; ++i) {
        const long double lo = 0.75L + (long double)i * width;
        const long double centre = lo + width / 2;
        // the row that holds m = 1 uses c = 1 so that r = m - 1 exactly
        const bool one = lo <= 1.0L && 1.0L < lo + width;
        const double c = one ? 1.0 : (double)(1.0L / centre);
        const long double nlc = -logl((long double)c);
        const long double hi = nearbyintl(nlc * two42) / two42;
        t[kLogCols * i] = c;
        t[kLogCols * i + 1] = (double)hi;
        t[kLogCols * i + 2] = (double)(nlc - hi);
    }
    return t;
}

std::string validate(const pd_params& p)
{
    if (p.L < 2 || p.L > PD_MAX_L) return "L must be in [2, 512]";
    if (p.N < 0 || p.N > p.L) return "N must be in [0, L]";
    if (!std::isfinite(p.s) || std::fabs(p.s) > 700.0) return "s must be finite with |s| <= 700";
    if (p.Nc < 1 || p.Nc > INT32_MAX) return "Nc must be in [1, 2^31 - 1]";
    if (!(p.t_obs > 0.0) || !std::isfinite(p.t_obs)) return "t_obs must be positive and finite";
    if (!(p.dt > 0.0) || !std::isfinite(p.dt)) return "dt must be positive and finite";
    const double Md = p.t_obs / p.dt;
    if (!(Md < 4.0e9)) return "t_obs / dt must be below 2^32";
    const int64_t M = cycles_of(p);
    if (M < 1) return "t_obs / dt must round to at least 1";
    if (std::fabs((double)M * p.dt - p.t_obs) > 1e-9 * p.t_obs)
        return "t_obs must be an integer multiple of dt";
    {
        // expected hops of one clone in one interval, at most e^{-s} L dt
        const double rate = (p.weight_mode == PD_W_DIRECT ? 1.0 : std::exp(-p.s)) * (double)p.L;
        if (!(rate * p.dt <= kMaxEventsPerInterval))
            return "expected hops per clone per interval (e^{-s} L dt) must be <= 2^24";
    }
    if (p.selection != PD_SEL_EQ && p.selection != PD_SEL_IID) return "unknown selection";
    if (p.weight_mode < PD_W_MODIFIED || p.weight_mode > PD_W_GUIDED) return "unknown weight mode";
    if (p.instance >= (1u << 24)) return "instance must be below 2^24";
    if (p.log_cycles < 0) return "log_cycles must be >= 0";
    if (p.burn_in < 0) return "burn_in must be >= 0";
    if (p.track_origin != 0 && p.track_origin != 1) return "track_origin must be 0 or 1";
    if (p.reserved != 0) return "reserved must be 0";
    return "";
}

struct Layout {
    size_t state[2], K[2], Kb, A, ell, anc, origin[2], ksnap[2], ykey, tmax, tsum, thops, toff,
        log, ctl;
    size_t cu64, cf64, cu32;   // guided continuation records (0: not guided)
    size_t iters;              // guided: proposals per clone of the last interval
    size_t rate[2];            // guided: S of each clone at the end of its interval
    size_t end;
    int ntiles;
};

// Byte offsets of one instance's arrays, starting at `base`.
Layout layout_of(const pd_params& p, size_t base)
{
    Layout o;
    const size_t Nc = (size_t)p.Nc;
    const int W = words_of(p.L);
    o.ntiles = (int)((Nc + kTile - 1) / kTile);
    size_t at = align_up(base);
    auto take = [&](size_t bytes) { size_t r = at; at = align_up(at + bytes); return r; };
    o.state[0] = take(8 * Nc * W);
    o.state[1] = take(8 * Nc * W);
    o.K[0] = take(8 * Nc);
    o.K[1] = take(8 * Nc);
    o.Kb = take(4 * Nc);
    o.A = take(8 * Nc);
    o.ell = take(8 * Nc);
    o.anc = take(4 * Nc);
    o.origin[0] = p.track_origin ? take(4 * Nc) : 0;
    o.origin[1] = p.track_origin ? take(4 * Nc) : 0;
    o.ksnap[0] = p.burn_in > 0 ? take(8 * Nc) : 0;
    o.ksnap[1] = p.burn_in > 0 ? take(8 * Nc) : 0;
    o.ykey = (p.selection == PD_SEL_IID) ? take(8 * Nc) : 0;
    // records of clones the guided stage's first launch hands on to its second
    const bool guided = p.weight_mode == PD_W_GUIDED;
    o.cu64 = guided ? take(8 * Nc * (W + 2)) : 0;
    o.cf64 = guided ? take(8 * Nc * 4) : 0;
    o.cu32 = guided ? take(4 * Nc * 4) : 0;
    o.iters = guided ? take(4 * Nc) : 0;
    o.rate[0] = guided ? take(8 * Nc) : 0;
    o.rate[1] = guided ? take(8 * Nc) : 0;
    o.tmax = take(8 * (size_t)o.ntiles);
    o.tsum = take(8 * (size_t)o.ntiles);
    o.thops = take(8 * (size_t)o.ntiles);
    o.toff = take(8 * ((size_t)o.ntiles + 1));
    o.log = take(16 * (size_t)std::max(p.log_cycles, 1));
    o.ctl = take(sizeof(InstCtl));
    o.end = at;
    return o;
}

struct Plan {
    size_t insts_off, tiles_off, log_off, sel_off, invc_off, counters_off, guide_off, total;
    std::vector<Layout> lay;
    int ntiles;
};

Plan plan_of(const pd_params* p, int n)
{
    Plan pl;
    pl.insts_off = 0;
    size_t at = align_up(sizeof(InstDev) * (size_t)n);
    int nt = 0;
    for (int i = 0; i < n; ++i) nt += (int)((p[i].Nc + kTile - 1) / kTile);
    pl.ntiles = nt;
    pl.tiles_off = at;
    at = align_up(at + sizeof(TileDesc) * (size_t)nt);
    pl.log_off = at;
    at = align_up(at + sizeof(double) * kLogCols * kLogRows);
    pl.sel_off = at;
    at = align_up(at + 2048);
    pl.invc_off = at;
    at = align_up(at + sizeof(double) * (kMaxSites + 1));
    pl.counters_off = at;
    at = align_up(at + sizeof(uint32_t) * kMaxGroups);
    // the library's own copy of the guide table (guided instances only)
    bool guided = false;
    for (int i = 0; i < n; ++i) guided = guided || p[i].weight_mode == PD_W_GUIDED;
    pl.guide_off = guided ? at : 0;
    if (guided) at = align_up(at + sizeof(uint32_t) * kGuideEntries);
    for (int i = 0; i < n; ++i) {
        pl.lay.push_back(layout_of(p[i], at));
        at = pl.lay.back().end;
    }
    pl.total = at;
    return pl;
}

}  // namespace

struct pd_ctx {
    hipStream_t stream = nullptr;
    int n = 0;
    std::vector<pd_params> params;
    std::vector<InstDev> dev;        // host copies of the descriptors
    Plan plan;
    char* ws = nullptr;
    InstDev* d_insts = nullptr;
    TileDesc* d_tiles = nullptr;
    std::vector<TileDesc> tiles;     // host copy, step order
    std::vector<StepLaunch> steps;   // tile groups, one per word count (and the gathers)
    std::vector<StepLaunch> launches;// the dynamical stage's launches under the tuning
    pd_tuning tuning;
    bool any_iid = false;
    bool any_guided = false;
    bool guide_set = false;
    bool any_origin = false;
    bool any_burn = false;           // an instance carries burn-in snapshots of K
    int cur = 0;                     // buffer holding the population
    bool perm = false;               // population = state[cur][anc[j]]
    bool stepped = false;            // a dynamical stage awaits its cloning stage
    bool anc_valid = false;          // anc holds the last cloning stage's map
    int64_t beta = 0;                // completed cycles (host mirror)
    int graph_cycles = 16;
    hipGraphExec_t graph[2] = {nullptr, nullptr};
    // stage timing (pd_time_stages): events around the launches of pd_step and
    // pd_resample, never inside a captured graph
    bool timing = false;
    bool capturing = false;
    std::vector<hipEvent_t> ev_step;     // triples: before the step kernels, before k_prefix, after
    std::vector<hipEvent_t> ev_res;      // pairs: before and after the cloning stage
    std::string err;
};

#define PD_HIP(call)                                                                    \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);               \
            return PD_EDEVICE;                                                          \
        }                                                                               \
    } while (0)

namespace {

pd_status fail(pd_ctx* ctx, pd_status st, const std::string& msg)
{
    if (ctx) ctx->err = msg; else g_create_error = msg;
    return st;
}

// Records a timing event on the context stream (pd_time_stages).
pd_status record_event(pd_ctx* ctx, std::vector<hipEvent_t>& into)
{
    hipEvent_t e = nullptr;
    PD_HIP(hipEventCreate(&e));
    into.push_back(e);
    PD_HIP(hipEventRecord(e, ctx->stream));
    return PD_OK;
}

#define PD_TIME(into)                                                                   \
    do {                                                                                \
        if (ctx->timing && !ctx->capturing) {                                           \
            pd_status s_ = record_event(ctx, into);                                     \
            if (s_ != PD_OK) return s_;                                                 \
        }                                                                               \
    } while (0)

// Cloning stage of every instance.
pd_status enqueue_resample(pd_ctx* ctx)
{
    PD_TIME(ctx->ev_res);
    PD_HIP(launch_resample(ctx->d_insts, ctx->d_tiles, (int)ctx->tiles.size(),
                           std::max(1, ctx->tuning.scan_tiles), ctx->stream));
    if (ctx->any_iid)
        PD_HIP(launch_select_iid(ctx->d_insts, ctx->d_tiles, (int)ctx->tiles.size(), ctx->stream));
    PD_TIME(ctx->ev_res);
    return PD_OK;
}

// Dynamical stage of every instance and the interval statistics.
pd_status enqueue_step(pd_ctx* ctx, int use_anc, int src)
{
    if (ctx->any_burn)
        PD_HIP(launch_carry_burn(ctx->d_insts, ctx->d_tiles, (int)ctx->tiles.size(), src, use_anc,
                                 ctx->stream));
    PD_TIME(ctx->ev_step);
    for (const auto& g : ctx->launches)
        PD_HIP(launch_step(g, ctx->d_insts, ctx->d_tiles, src, use_anc, ctx->stream));
    PD_TIME(ctx->ev_step);
    PD_HIP(launch_prefix(ctx->d_insts, ctx->n, ctx->stream));
    PD_TIME(ctx->ev_step);
    return PD_OK;
}

pd_status enqueue_cycle(pd_ctx* ctx, int use_anc, int src)
{
    pd_status st = enqueue_step(ctx, use_anc, src);
    if (st != PD_OK) return st;
    return enqueue_resample(ctx);
}

// Applies a tuning: kernel variant and grid of every step launch.
pd_status apply_tuning(pd_ctx* ctx, const pd_tuning& t)
{
    if (t.step_variant < 0 || t.step_variant > 5 || t.refill < 1 || t.refill > 64 ||
        t.graph_cycles < 0 || (t.graph_cycles & 1) ||
        !(t.scan_tiles == 0 || t.scan_tiles == 1 || t.scan_tiles == 2 || t.scan_tiles == 4 ||
          t.scan_tiles == 8))
        return fail(ctx, PD_EINVAL, "invalid tuning");
    int dev = 0, cus = 0;
    PD_HIP(hipGetDevice(&dev));
    PD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    for (auto& g : ctx->steps) {
        // the guided stage has no variants; the queued variants do not carry origins;
        // under variant 5 the groups keep variant 4 (the merged launch is built below)
        g.variant = g.guided ? 0
                  : (ctx->any_origin && t.step_variant >= 1 && t.step_variant <= 3) ? 0
                  : t.step_variant == 5 ? 4
                  : t.step_variant;
        g.refill = t.refill;
        int per_cu = 0;
        PD_HIP(step_occupancy(g.W, g.variant, &per_cu));
        const int want = (g.count + 3) / 4;          // four waves per block, a tile each
        g.blocks = std::max(1, std::min(want, std::max(1, per_cu) * std::max(1, cus)));
    }
    // the launches: variant 5 merges the plain groups (the first ones in the step
    // order) into one persistent launch, the guided groups keep theirs
    ctx->launches.clear();
    if (t.step_variant == 5) {
        StepLaunch m{};
        int wmax = 0, count = 0;
        for (const auto& g : ctx->steps)
            if (!g.guided) { wmax = std::max(wmax, g.W); count += g.count; }
        if (count > 0) {
            m.W = wmax <= 2 ? 2 : wmax <= 4 ? 4 : 8;
            m.variant = 5;
            m.guided = false;
            m.base = 0;
            m.count = count;
            m.refill = t.refill;
            m.counter = ctx->steps[0].counter;
            int per_cu = 0;
            PD_HIP(step_occupancy(m.W, 5, &per_cu));
            m.blocks = std::max(1, std::min(count, std::max(1, per_cu) * std::max(1, cus)));
            ctx->launches.push_back(m);
        }
        for (const auto& g : ctx->steps)
            if (g.guided) ctx->launches.push_back(g);
    } else {
        ctx->launches = ctx->steps;
    }
    if (t.graph_cycles != ctx->tuning.graph_cycles)
        for (auto& gx : ctx->graph)
            if (gx) { (void)hipGraphExecDestroy(gx); gx = nullptr; }
    // captured graphs hold the launch configuration: recapture on change
    if (t.step_variant != ctx->tuning.step_variant || t.refill != ctx->tuning.refill ||
        t.scan_tiles != ctx->tuning.scan_tiles)
        for (auto& gx : ctx->graph)
            if (gx) { (void)hipGraphExecDestroy(gx); gx = nullptr; }
    ctx->tuning = t;
    ctx->graph_cycles = t.graph_cycles;
    return PD_OK;
}

pd_status check_inst(pd_ctx* ctx, int32_t inst)
{
    if (!ctx) return PD_EINVAL;
    if (inst < 0 || inst >= ctx->n) return fail(ctx, PD_EINVAL, "instance index out of range");
    return PD_OK;
}

// The guided stage of instance i forms S from the state at its next step: the
// carried rates no longer match the population or the table.
pd_status drop_carried_rates(pd_ctx* ctx, int i)
{
    static const uint32_t zero = 0;
    if (ctx->params[i].weight_mode != PD_W_GUIDED) return PD_OK;
    PD_HIP(hipMemcpyAsync(&ctx->dev[i].ctl->s_carried, &zero, sizeof zero, hipMemcpyHostToDevice,
                          ctx->stream));
    return PD_OK;
}

// Makes state[cur] hold the population in slot order.
pd_status materialise(pd_ctx* ctx)
{
    if (!ctx->perm) return PD_OK;
    for (const auto& g : ctx->steps)
        PD_HIP(launch_gather(g.W, ctx->d_insts, ctx->d_tiles, g.base, g.count, ctx->cur,
                             ctx->stream));
    ctx->cur ^= 1;
    ctx->perm = false;
    return PD_OK;
}

}  // namespace

extern "C" {

pd_status pd_workspace_bytes(const pd_params* params, int32_t n, size_t* bytes)
{
    if (!params || n < 1 || !bytes) return fail(nullptr, PD_EINVAL, "null argument or n < 1");
    for (int i = 0; i < n; ++i) {
        std::string m = validate(params[i]);
        if (!m.empty()) return fail(nullptr, PD_EINVAL, "instance " + std::to_string(i) + ": " + m);
    }
    *bytes = plan_of(params, n).total;
    return PD_OK;
}

pd_status pd_create(const pd_params* params, int32_t n, void* d_workspace, size_t bytes,
                    void* hip_stream, pd_ctx** out)
{
    if (!params || n < 1 || !out || !d_workspace)
        return fail(nullptr, PD_EINVAL, "null argument or n < 1");
    *out = nullptr;
    for (int i = 0; i < n; ++i) {
        std::string m = validate(params[i]);
        if (!m.empty()) return fail(nullptr, PD_EINVAL, "instance " + std::to_string(i) + ": " + m);
    }
    if ((uintptr_t)d_workspace % kAlign != 0)
        return fail(nullptr, PD_EINVAL, "workspace must be 256-byte aligned");
    Plan pl = plan_of(params, n);
    if (bytes < pl.total) return fail(nullptr, PD_ENOMEM, "workspace too small");

    pd_ctx* ctx = new pd_ctx();
    ctx->stream = (hipStream_t)hip_stream;
    ctx->n = n;
    ctx->params.assign(params, params + n);
    ctx->plan = pl;
    ctx->ws = (char*)d_workspace;
    ctx->d_insts = (InstDev*)(ctx->ws + pl.insts_off);
    ctx->d_tiles = (TileDesc*)(ctx->ws + pl.tiles_off);

    // descriptors and rate tables
    double ln2_hi = 0.0, ln2_lo = 0.0;
    const std::vector<double> logt = log_table(&ln2_hi, &ln2_lo);
    const std::vector<uint8_t> selt = select_table();
    for (int i = 0; i < n; ++i) {
        const pd_params& p = params[i];
        const Layout& o = pl.lay[i];
        InstDev d;
        std::memset(&d, 0, sizeof d);
        d.L = p.L; d.N = p.N; d.W = words_of(p.L); d.mode = p.weight_mode;
        for (int k = 0; k < kLogPoly; ++k) d.log_poly[k] = ((k & 1) ? -1.0 : 1.0) / (double)(7 - k);
        for (int k = 0; k < 14; ++k) {
            long double f = 1.0L;
            for (int q = 2; q <= 13 - k; ++q) f *= (long double)q;
            d.exp_poly[k] = (double)(1.0L / f);
        }
        d.selection = p.selection; d.ntiles = o.ntiles; d.log_cycles = p.log_cycles;
        d.key0 = (uint32_t)p.seed; d.key1 = (uint32_t)(p.seed >> 32);
        d.tag_hi = p.instance << 8;
        d.s = p.s;
        d.es = std::exp(-p.s);
        d.c = -std::expm1(-p.s);
        d.dt = p.dt;
        d.Nc = p.Nc;
        d.burn_in = p.burn_in;
        char* b = ctx->ws;
        d.state[0] = (uint64_t*)(b + o.state[0]);
        d.state[1] = (uint64_t*)(b + o.state[1]);
        d.K[0] = (uint64_t*)(b + o.K[0]);
        d.K[1] = (uint64_t*)(b + o.K[1]);
        d.Kb = (uint32_t*)(b + o.Kb);
        d.A = (double*)(b + o.A);
        d.ell = (double*)(b + o.ell);
        d.anc = (int32_t*)(b + o.anc);
        d.origin[0] = o.origin[0] ? (int32_t*)(b + o.origin[0]) : nullptr;
        d.origin[1] = o.origin[1] ? (int32_t*)(b + o.origin[1]) : nullptr;
        if (p.track_origin) ctx->any_origin = true;
        d.ksnap[0] = o.ksnap[0] ? (uint64_t*)(b + o.ksnap[0]) : nullptr;
        d.ksnap[1] = o.ksnap[1] ? (uint64_t*)(b + o.ksnap[1]) : nullptr;
        if (p.burn_in > 0) ctx->any_burn = true;
        d.ykey = o.ykey ? (double*)(b + o.ykey) : nullptr;
        d.tile_max = (double*)(b + o.tmax);
        d.tile_sum = (double*)(b + o.tsum);
        d.tile_hops = (uint64_t*)(b + o.thops);
        d.tile_off = (double*)(b + o.toff);
        d.inv_scale = (p.weight_mode == PD_W_MODIFIED) ? 1.0 / d.es : 1.0;
        d.inv_count = (const double*)(b + pl.invc_off);
        d.log = (double*)(b + o.log);
        d.guide = nullptr;
        d.ctl = (InstCtl*)(b + o.ctl);
        d.log_tab = (const double*)(b + pl.log_off);
        d.sel_tab = (const uint8_t*)(b + pl.sel_off);
        d.ln2_hi = ln2_hi;
        d.ln2_lo = ln2_lo;
        d.next_tile = (uint32_t*)(b + pl.counters_off);
        d.cont_u64 = o.cu64 ? (uint64_t*)(b + o.cu64) : nullptr;
        d.cont_f64 = o.cf64 ? (double*)(b + o.cf64) : nullptr;
        d.cont_u32 = o.cu32 ? (uint32_t*)(b + o.cu32) : nullptr;
        d.iters = o.iters ? (uint32_t*)(b + o.iters) : nullptr;
        d.rate[0] = o.rate[0] ? (uint64_t*)(b + o.rate[0]) : nullptr;
        d.rate[1] = o.rate[1] ? (uint64_t*)(b + o.rate[1]) : nullptr;
        ctx->dev.push_back(d);
        if (p.selection == PD_SEL_IID) ctx->any_iid = true;
        if (p.weight_mode == PD_W_GUIDED) ctx->any_guided = true;
    }

    // tiles: grouped by word count, largest expected work first within a group
    struct Cand { TileDesc t; int W; bool guided; double cost; };
    std::vector<Cand> cand;
    for (int i = 0; i < n; ++i) {
        const pd_params& p = params[i];
        const double rbar = p.L > 1 ? 2.0 * p.N * (double)(p.L - p.N) / (double)(p.L - 1) : 0.0;
        const double rate = (p.weight_mode == PD_W_MODIFIED ? std::exp(-p.s) : 1.0) * rbar;
        const int nt = pl.lay[i].ntiles;
        for (int t = 0; t < nt; ++t) {
            TileDesc td;
            td.inst = i;
            td.tile = t;
            td.first = t * kTile;
            td.count = (int)std::min<int64_t>(kTile, p.Nc - (int64_t)t * kTile);
            cand.push_back({td, words_of(p.L), p.weight_mode == PD_W_GUIDED,
                            td.count * (rate * p.dt + 1.0)});
        }
    }
    // plain tiles first (variant 5 runs them as one launch from tile 0), the
    // larger word counts first, the larger expected work first within a word count
    std::stable_sort(cand.begin(), cand.end(), [](const Cand& a, const Cand& b) {
        if (a.guided != b.guided) return !a.guided;
        if (a.W != b.W) return a.W > b.W;
        return a.cost > b.cost;
    });
    for (size_t k = 0; k < cand.size(); ++k) {
        ctx->tiles.push_back(cand[k].t);
        if (ctx->steps.empty() || ctx->steps.back().W != cand[k].W ||
            ctx->steps.back().guided != cand[k].guided) {
            if ((int)ctx->steps.size() == kMaxGroups) {
                delete ctx;
                return fail(nullptr, PD_EUNSUPPORTED, "too many distinct word counts");
            }
            StepLaunch sl;
            sl.W = cand[k].W;
            sl.guided = cand[k].guided;
            sl.variant = 0;
            sl.base = (int)k;
            sl.count = 0;
            sl.blocks = 1;
            sl.refill = 8;
            sl.counter = (uint32_t*)(ctx->ws + pl.counters_off) + ctx->steps.size();
            ctx->steps.push_back(sl);
        }
        ctx->steps.back().count++;
    }

    auto bail = [&](pd_status st) { g_create_error = ctx->err; delete ctx; return st; };
#define PD_HIP_CREATE(call)                                                             \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ctx->err = std::string(#call) + ": " + hipGetErrorString(e_);               \
            return bail(PD_EDEVICE);                                                    \
        }                                                                               \
    } while (0)
    PD_HIP_CREATE(hipMemcpyAsync(ctx->d_insts, ctx->dev.data(), sizeof(InstDev) * (size_t)n,
                                 hipMemcpyHostToDevice, ctx->stream));
    PD_HIP_CREATE(hipMemcpyAsync(ctx->d_tiles, ctx->tiles.data(),
                                 sizeof(TileDesc) * ctx->tiles.size(), hipMemcpyHostToDevice,
                                 ctx->stream));
    std::vector<double> invc(kMaxSites + 1, 0.0);
    for (int r = 1; r <= kMaxSites; ++r) invc[r] = 1.0 / (double)r;
    PD_HIP_CREATE(hipMemcpyAsync(ctx->ws + pl.invc_off, invc.data(), sizeof(double) * invc.size(),
                                 hipMemcpyHostToDevice, ctx->stream));
    PD_HIP_CREATE(hipMemcpyAsync(ctx->ws + pl.log_off, logt.data(), sizeof(double) * logt.size(),
                                 hipMemcpyHostToDevice, ctx->stream));
    PD_HIP_CREATE(hipMemcpyAsync(ctx->ws + pl.sel_off, selt.data(), selt.size(),
                                 hipMemcpyHostToDevice, ctx->stream));
    PD_HIP_CREATE(launch_init(ctx->d_insts, n, ctx->d_tiles, (int)ctx->tiles.size(), ctx->stream));
    {
        pd_tuning t = default_tuning();
        ctx->tuning = t;
        ctx->tuning.step_variant = -1;   // force the first application
        if (apply_tuning(ctx, t) != PD_OK) return bail(PD_EDEVICE);
    }
    // the host vectors above are pageable: wait before they go out of scope
    PD_HIP_CREATE(hipStreamSynchronize(ctx->stream));
#undef PD_HIP_CREATE
    *out = ctx;
    return PD_OK;
}

pd_status pd_destroy(pd_ctx* ctx)
{
    if (!ctx) return PD_EINVAL;
    for (auto& g : ctx->graph)
        if (g) (void)hipGraphExecDestroy(g);
    if (!ctx->ev_step.empty() || !ctx->ev_res.empty()) {
        (void)hipStreamSynchronize(ctx->stream);
        for (hipEvent_t e : ctx->ev_step) (void)hipEventDestroy(e);
        for (hipEvent_t e : ctx->ev_res) (void)hipEventDestroy(e);
    }
    delete ctx;
    return PD_OK;
}

pd_status pd_step(pd_ctx* ctx)
{
    if (!ctx) return PD_EINVAL;
    if (ctx->stepped) return fail(ctx, PD_ESTATE, "pd_step called twice without pd_resample");
    if (ctx->any_guided && !ctx->guide_set)
        return fail(ctx, PD_ESTATE, "guided instances need pd_set_guide first");
    {
        pd_status st = enqueue_step(ctx, ctx->perm ? 1 : 0, ctx->cur);
        if (st != PD_OK) return st;
    }
    ctx->cur ^= 1;
    ctx->perm = false;
    ctx->stepped = true;
    ctx->anc_valid = false;
    return PD_OK;
}

pd_status pd_resample(pd_ctx* ctx)
{
    if (!ctx) return PD_EINVAL;
    if (!ctx->stepped) return fail(ctx, PD_ESTATE, "pd_resample needs a pd_step first");
    {
        pd_status st = enqueue_resample(ctx);
        if (st != PD_OK) return st;
    }
    ctx->perm = true;
    ctx->stepped = false;
    ctx->anc_valid = true;
    ctx->beta += 1;
    return PD_OK;
}

// Captures (without running) the graph of graph_cycles cycles that starts
// from state buffer `which` with the population read through the ancestor
// map; pd_run replays it.
pd_status capture_graph(pd_ctx* ctx, int which)
{
    hipGraphExec_t& ex = ctx->graph[which];
    if (ex) return PD_OK;
    const int G = ctx->graph_cycles;
    hipGraph_t g = nullptr;
    PD_HIP(hipStreamBeginCapture(ctx->stream, hipStreamCaptureModeThreadLocal));
    pd_status st = PD_OK;
    ctx->capturing = true;
    for (int c = 0; c < G && st == PD_OK; ++c) st = enqueue_cycle(ctx, 1, which ^ (c & 1));
    ctx->capturing = false;
    hipError_t e = hipStreamEndCapture(ctx->stream, &g);
    if (st != PD_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    PD_HIP(e);
    hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    PD_HIP(ei);
    // the executable's upload to the device is paid here, not by its first replay
    PD_HIP(hipGraphUpload(ex, ctx->stream));
    return PD_OK;
}

pd_status pd_run(pd_ctx* ctx, int64_t cycles)
{
    if (!ctx || cycles < 0) return PD_EINVAL;
    if (ctx->stepped) return fail(ctx, PD_ESTATE, "a pd_step awaits its pd_resample");
    if (ctx->any_guided && !ctx->guide_set)
        return fail(ctx, PD_ESTATE, "guided instances need pd_set_guide first");
    if (cycles == 0) {
        // nothing runs: the graphs that later calls replay are captured now
        if (ctx->stream != nullptr && ctx->graph_cycles > 0)
            for (int which = 0; which < 2; ++which) {
                pd_status st = capture_graph(ctx, which);
                if (st != PD_OK) return st;
            }
        return PD_OK;
    }
    int64_t left = cycles;
    if (left > 0 && !ctx->perm) {
        pd_status st = enqueue_cycle(ctx, 0, ctx->cur);
        if (st != PD_OK) return st;
        ctx->cur ^= 1;
        ctx->perm = true;
        --left;
    }
    const int G = ctx->graph_cycles;
    if (ctx->stream != nullptr && G > 0 && left >= G) {
        pd_status st = capture_graph(ctx, ctx->cur);
        if (st != PD_OK) return st;
        hipGraphExec_t ex = ctx->graph[ctx->cur];
        while (left >= G) {
            PD_HIP(hipGraphLaunch(ex, ctx->stream));
            left -= G;   // G is even: the population returns to buffer cur
        }
    }
    while (left > 0) {
        pd_status st = enqueue_cycle(ctx, 1, ctx->cur);
        if (st != PD_OK) return st;
        ctx->cur ^= 1;
        --left;
    }
    ctx->perm = ctx->perm || cycles > 0;
    ctx->anc_valid = cycles > 0 ? true : ctx->anc_valid;
    ctx->beta += cycles;
    return PD_OK;
}

pd_status pd_estimates_get(pd_ctx* ctx, int32_t inst, pd_estimates* out)
{
    pd_status st = check_inst(ctx, inst);
    if (st != PD_OK) return st;
    if (!out) return fail(ctx, PD_EINVAL, "null output");
    const InstDev& d = ctx->dev[inst];
    const pd_params& p = ctx->params[inst];
    PD_HIP(launch_zero_ksum(ctx->d_insts, ctx->n, ctx->stream));
    PD_HIP(launch_ksum(ctx->d_insts, ctx->d_tiles, (int)ctx->tiles.size(), ctx->cur,
                       ctx->perm ? 1 : 0, ctx->stream));
    InstCtl c;
    PD_HIP(hipMemcpyAsync(&c, d.ctl, sizeof c, hipMemcpyDeviceToHost, ctx->stream));
    PD_HIP(hipStreamSynchronize(ctx->stream));
    const double t = (double)c.beta * p.dt;
    out->cycles = c.beta;
    out->t = t;
    out->hops = c.hops;
    out->psi = c.beta > 0 ? (c.psi_sum + c.psi_comp) / t : 0.0;
    out->psi_burn = c.beta > p.burn_in
                        ? (c.psib_sum + c.psib_comp) / ((double)(c.beta - p.burn_in) * p.dt) : 0.0;
    out->k_hat = c.beta > 0 ? (double)c.ksum / ((double)p.Nc * (double)p.L * t) : 0.0;
    // hops of the intervals beyond burn_in along the ancestral lines: K minus its
    // snapshot at the end of interval burn_in (every clone's K when burn_in = 0)
    out->k_hat_burn = c.beta > p.burn_in
                          ? (double)(c.ksum - c.ksnap_sum) /
                                ((double)p.Nc * (double)p.L * (double)(c.beta - p.burn_in) * p.dt)
                          : 0.0;
    out->draws = c.draws;
    return PD_OK;
}

pd_status pd_scgf(pd_ctx* ctx, double* psi, double* k_hat, int64_t* cycles_done)
{
    pd_estimates e;
    pd_status st = pd_estimates_get(ctx, 0, &e);
    if (st != PD_OK) return st;
    if (psi) *psi = e.psi;
    if (k_hat) *k_hat = e.k_hat;
    if (cycles_done) *cycles_done = e.cycles;
    return PD_OK;
}

pd_status pd_population_bytes(const pd_params* params, size_t* bytes)
{
    if (!params || !bytes) return PD_EINVAL;
    std::string m = validate(*params);
    if (!m.empty()) return fail(nullptr, PD_EINVAL, m);
    *bytes = 8 * (size_t)params->Nc * (size_t)(words_of(params->L) + 1);
    return PD_OK;
}

pd_status pd_get_population(pd_ctx* ctx, int32_t inst, void* host, size_t bytes)
{
    pd_status st = check_inst(ctx, inst);
    if (st != PD_OK) return st;
    const pd_params& p = ctx->params[inst];
    const size_t Nc = (size_t)p.Nc, W = (size_t)words_of(p.L);
    if (!host || bytes < 8 * Nc * (W + 1)) return fail(ctx, PD_ENOMEM, "host buffer too small");
    st = materialise(ctx);
    if (st != PD_OK) return st;
    const InstDev& d = ctx->dev[inst];
    PD_HIP(hipMemcpyAsync(host, d.state[ctx->cur], 8 * Nc * W, hipMemcpyDeviceToHost, ctx->stream));
    PD_HIP(hipMemcpyAsync((char*)host + 8 * Nc * W, d.K[ctx->cur], 8 * Nc, hipMemcpyDeviceToHost,
                          ctx->stream));
    PD_HIP(hipStreamSynchronize(ctx->stream));
    return PD_OK;
}

// A host image of Nc states ([W][Nc] words): "" if every state has N particles on sites 0..L-1.
static std::string check_states(const pd_params& p, const void* words)
{
    const size_t Nc = (size_t)p.Nc, W = (size_t)words_of(p.L);
    for (size_t j = 0; j < Nc; ++j) {
        int cnt = 0;
        for (size_t w = 0; w < W; ++w) {
            uint64_t v;
            std::memcpy(&v, (const char*)words + 8 * (w * Nc + j), 8);
            const int hi_bits = p.L - 64 * (int)w;
            if (hi_bits < 64 && (v >> hi_bits) != 0) return "state has a bit set at or beyond site L";
            cnt += __builtin_popcountll(v);
        }
        if (cnt != p.N) return "state does not hold N particles";
    }
    return "";
}

pd_status pd_set_population(pd_ctx* ctx, int32_t inst, const void* host, size_t bytes)
{
    pd_status st = check_inst(ctx, inst);
    if (st != PD_OK) return st;
    const pd_params& p = ctx->params[inst];
    const size_t Nc = (size_t)p.Nc, W = (size_t)words_of(p.L);
    if (!host || bytes < 8 * Nc * (W + 1)) return fail(ctx, PD_ENOMEM, "host buffer too small");
    std::string m = check_states(p, host);
    if (!m.empty()) return fail(ctx, PD_EINVAL, m);
    st = materialise(ctx);   // keep the other instances' populations in slot order
    if (st != PD_OK) return st;
    const InstDev& d = ctx->dev[inst];
    PD_HIP(hipMemcpyAsync(d.state[ctx->cur], host, 8 * Nc * W, hipMemcpyHostToDevice, ctx->stream));
    PD_HIP(hipMemcpyAsync(d.K[ctx->cur], (const char*)host + 8 * Nc * W, 8 * Nc,
                          hipMemcpyHostToDevice, ctx->stream));
    // hops beyond burn_in count from here for the new clones
    if (d.ksnap[0])
        PD_HIP(hipMemcpyAsync(d.ksnap[ctx->cur], (const char*)host + 8 * Nc * W, 8 * Nc,
                              hipMemcpyHostToDevice, ctx->stream));
    st = drop_carried_rates(ctx, inst);
    if (st != PD_OK) return st;
    PD_HIP(hipStreamSynchronize(ctx->stream));
    ctx->stepped = false;
    ctx->anc_valid = false;
    return PD_OK;
}

pd_status pd_get_step_outputs(pd_ctx* ctx, int32_t inst, uint32_t* Kb, double* A, double* ell)
{
    pd_status st = check_inst(ctx, inst);
    if (st != PD_OK) return st;
    const InstDev& d = ctx->dev[inst];
    const size_t Nc = (size_t)ctx->params[inst].Nc;
    if (Kb) PD_HIP(hipMemcpyAsync(Kb, d.Kb, 4 * Nc, hipMemcpyDeviceToHost, ctx->stream));
    if (A) PD_HIP(hipMemcpyAsync(A, d.A, 8 * Nc, hipMemcpyDeviceToHost, ctx->stream));
    if (ell) PD_HIP(hipMemcpyAsync(ell, d.ell, 8 * Nc, hipMemcpyDeviceToHost, ctx->stream));
    PD_HIP(hipStreamSynchronize(ctx->stream));
    return PD_OK;
}

pd_status pd_get_ancestors(pd_ctx* ctx, int32_t inst, int32_t* anc)
{
    pd_status st = check_inst(ctx, inst);
    if (st != PD_OK) return st;
    if (!ctx->anc_valid) return fail(ctx, PD_ESTATE, "no cloning stage since the last step");
    if (!anc) return fail(ctx, PD_EINVAL, "null output");
    const InstDev& d = ctx->dev[inst];
    PD_HIP(hipMemcpyAsync(anc, d.anc, 4 * (size_t)ctx->params[inst].Nc, hipMemcpyDeviceToHost,
                          ctx->stream));
    PD_HIP(hipStreamSynchronize(ctx->stream));
    return PD_OK;
}

pd_status pd_get_log(pd_ctx* ctx, int32_t inst, double* lbeta, double* mean_kb, int32_t n_rows)
{
    pd_status st = check_inst(ctx, inst);
    if (st != PD_OK) return st;
    const pd_params& p = ctx->params[inst];
    if (n_rows < 0 || n_rows > p.log_cycles) return fail(ctx, PD_EINVAL, "n_rows exceeds log_cycles");
    if (n_rows == 0) return PD_OK;
    std::vector<double> buf(2 * (size_t)n_rows);
    PD_HIP(hipMemcpyAsync(buf.data(), ctx->dev[inst].log, buf.size() * 8, hipMemcpyDeviceToHost,
                          ctx->stream));
    PD_HIP(hipStreamSynchronize(ctx->stream));
    for (int r = 0; r < n_rows; ++r) {
        if (lbeta) lbeta[r] = buf[2 * r];
        if (mean_kb) mean_kb[r] = buf[2 * r + 1];
    }
    return PD_OK;
}

// Checkpoint: magic, n, host beta, then per instance: InstCtl, population image.
static const uint64_t kMagic = 0x31315044434c4e31ull;

pd_status pd_save_bytes(pd_ctx* ctx, size_t* bytes)
{
    if (!ctx || !bytes) return PD_EINVAL;
    size_t b = 3 * 8;
    for (const auto& p : ctx->params) {
        b += sizeof(InstCtl) + 8 * (size_t)p.Nc * (size_t)(words_of(p.L) + 1);
        if (p.track_origin) b += (4 * (size_t)p.Nc + 7) / 8 * 8;
        if (p.burn_in > 0) b += 8 * (size_t)p.Nc;
    }
    *bytes = b;
    return PD_OK;
}

pd_status pd_save(pd_ctx* ctx, void* host, size_t bytes)
{
    size_t need = 0;
    pd_status st = pd_save_bytes(ctx, &need);
    if (st != PD_OK) return st;
    if (ctx->stepped) return fail(ctx, PD_ESTATE, "save between pd_step and pd_resample");
    if (!host || bytes < need) return fail(ctx, PD_ENOMEM, "host buffer too small");
    st = materialise(ctx);
    if (st != PD_OK) return st;
    uint64_t* h = (uint64_t*)host;
    h[0] = kMagic;
    h[1] = (uint64_t)ctx->n;
    h[2] = (uint64_t)ctx->beta;
    char* at = (char*)host + 24;
    for (int i = 0; i < ctx->n; ++i) {
        const InstDev& d = ctx->dev[i];
        const size_t Nc = (size_t)ctx->params[i].Nc, W = (size_t)words_of(ctx->params[i].L);
        PD_HIP(hipMemcpyAsync(at, d.ctl, sizeof(InstCtl), hipMemcpyDeviceToHost, ctx->stream));
        at += sizeof(InstCtl);
        PD_HIP(hipMemcpyAsync(at, d.state[ctx->cur], 8 * Nc * W, hipMemcpyDeviceToHost, ctx->stream));
        at += 8 * Nc * W;
        PD_HIP(hipMemcpyAsync(at, d.K[ctx->cur], 8 * Nc, hipMemcpyDeviceToHost, ctx->stream));
        at += 8 * Nc;
        if (d.origin[0]) {
            PD_HIP(hipMemcpyAsync(at, d.origin[ctx->cur], 4 * Nc, hipMemcpyDeviceToHost,
                                  ctx->stream));
            at += (4 * Nc + 7) / 8 * 8;
        }
        if (d.ksnap[0]) {
            PD_HIP(hipMemcpyAsync(at, d.ksnap[ctx->cur], 8 * Nc, hipMemcpyDeviceToHost,
                                  ctx->stream));
            at += 8 * Nc;
        }
    }
    PD_HIP(hipStreamSynchronize(ctx->stream));
    return PD_OK;
}

pd_status pd_load(pd_ctx* ctx, const void* host, size_t bytes)
{
    size_t need = 0;
    pd_status st = pd_save_bytes(ctx, &need);
    if (st != PD_OK) return st;
    if (!host || bytes < need) return fail(ctx, PD_ENOMEM, "checkpoint too small");
    uint64_t h[3];
    std::memcpy(h, host, sizeof h);
    if (h[0] != kMagic || h[1] != (uint64_t)ctx->n || h[2] > (uint64_t)INT64_MAX)
        return fail(ctx, PD_EINVAL, "not a checkpoint of this configuration");
    // Everything is checked before anything is uploaded, so a rejected checkpoint leaves the
    // context as it was.  Origins index the caller's values in pd_mean/pd_histogram and ncont
    // counts records of the guided stage, so neither is taken on trust; a checkpoint is taken
    // after a cloning stage, where ncont is 0.
    std::vector<InstCtl> ctl(ctx->n);
    const char* at = (const char*)host + 24;
    for (int i = 0; i < ctx->n; ++i) {
        const pd_params& p = ctx->params[i];
        const size_t Nc = (size_t)p.Nc, W = (size_t)words_of(p.L);
        std::memcpy(&ctl[i], at, sizeof(InstCtl));
        ctl[i].ncont = 0;
        ctl[i].s_carried = 0;   // the guided rates are not part of a checkpoint
        if (ctl[i].beta < 0) return fail(ctx, PD_EINVAL, "checkpoint has a negative interval count");
        at += sizeof(InstCtl);
        std::string m = check_states(p, at);
        if (!m.empty()) return fail(ctx, PD_EINVAL, "instance " + std::to_string(i) + ": " + m);
        at += 8 * Nc * (W + 1);
        if (ctx->dev[i].origin[0]) {
            for (size_t j = 0; j < Nc; ++j) {
                int32_t o;
                std::memcpy(&o, at + 4 * j, 4);
                if (o < 0 || (size_t)o >= Nc)
                    return fail(ctx, PD_EINVAL, "checkpoint has an origin outside [0, Nc)");
            }
            at += (4 * Nc + 7) / 8 * 8;
        }
        if (ctx->dev[i].ksnap[0]) at += 8 * Nc;
    }
    at = (const char*)host + 24;
    for (int i = 0; i < ctx->n; ++i) {
        const InstDev& d = ctx->dev[i];
        const size_t Nc = (size_t)ctx->params[i].Nc, W = (size_t)words_of(ctx->params[i].L);
        PD_HIP(hipMemcpyAsync(d.ctl, &ctl[i], sizeof(InstCtl), hipMemcpyHostToDevice, ctx->stream));
        at += sizeof(InstCtl);
        PD_HIP(hipMemcpyAsync(d.state[ctx->cur], at, 8 * Nc * W, hipMemcpyHostToDevice, ctx->stream));
        at += 8 * Nc * W;
        PD_HIP(hipMemcpyAsync(d.K[ctx->cur], at, 8 * Nc, hipMemcpyHostToDevice, ctx->stream));
        at += 8 * Nc;
        if (d.origin[0]) {
            PD_HIP(hipMemcpyAsync(d.origin[ctx->cur], at, 4 * Nc, hipMemcpyHostToDevice,
                                  ctx->stream));
            at += (4 * Nc + 7) / 8 * 8;
        }
        if (d.ksnap[0]) {
            PD_HIP(hipMemcpyAsync(d.ksnap[ctx->cur], at, 8 * Nc, hipMemcpyHostToDevice,
                                  ctx->stream));
            at += 8 * Nc;
        }
    }
    PD_HIP(hipStreamSynchronize(ctx->stream));
    ctx->beta = (int64_t)h[2];
    ctx->perm = false;
    ctx->stepped = false;
    ctx->anc_valid = false;
    return PD_OK;
}

pd_status pd_set_guide(pd_ctx* ctx, const uint32_t* d_table, size_t n)
{
    if (!ctx) return PD_EINVAL;
    if (!ctx->any_guided) return fail(ctx, PD_EINVAL, "no instance uses guided weights");
    if (!d_table || n != (size_t)kGuideEntries) return fail(ctx, PD_EINVAL, "table must hold 8192 entries");
    if ((reinterpret_cast<uintptr_t>(d_table) & 15u) != 0)
        return fail(ctx, PD_EINVAL, "table must be 16-byte aligned");
    std::vector<uint32_t> h(kGuideEntries);
    PD_HIP(hipMemcpyAsync(h.data(), d_table, sizeof(uint32_t) * h.size(), hipMemcpyDeviceToHost,
                          ctx->stream));
    PD_HIP(hipStreamSynchronize(ctx->stream));
    uint32_t lo = UINT32_MAX, hi = 0;
    for (int u = 0; u < kGuideEntries; ++u) {
        const bool allowed = ((u >> 6) ^ (u >> 7)) & 1;
        if (!allowed) {
            if (h[u] != 0) return fail(ctx, PD_EINVAL, "entries of non-hop neighbourhoods must be 0");
            continue;
        }
        if (h[u] == 0 || h[u] >= (1u << 31)) return fail(ctx, PD_EINVAL, "entries must be in [1, 2^31)");
        lo = std::min(lo, h[u]);
        hi = std::max(hi, h[u]);
    }
    if ((uint64_t)hi > 1024ull * lo) return fail(ctx, PD_EINVAL, "largest/smallest entry must be <= 1024");
    for (int i = 0; i < ctx->n; ++i) {
        const pd_params& p = ctx->params[i];
        if (p.weight_mode != PD_W_GUIDED) continue;
        const double rate = std::exp(-p.s) * ((double)hi / 65536.0) * (double)p.L;
        if (!(rate * p.dt <= kMaxEventsPerInterval))
            return fail(ctx, PD_EINVAL, "guide makes more than 2^24 expected hops per interval");
    }
    // the library's own copy: the caller may change or free its buffer afterwards
    uint32_t* own = (uint32_t*)(ctx->ws + ctx->plan.guide_off);
    PD_HIP(hipMemcpyAsync(own, d_table, sizeof(uint32_t) * kGuideEntries,
                          hipMemcpyDeviceToDevice, ctx->stream));
    for (int i = 0; i < ctx->n; ++i) {
        if (ctx->params[i].weight_mode != PD_W_GUIDED) continue;
        ctx->dev[i].guide = own;
        ctx->dev[i].guide_max = hi;
        // proposals come at e^{-s} hi 2^-16 per allowed bond (thinning)
        ctx->dev[i].guide_scale = 65536.0 / (ctx->dev[i].es * (double)hi);
    }
    PD_HIP(hipMemcpyAsync(ctx->d_insts, ctx->dev.data(), sizeof(InstDev) * (size_t)ctx->n,
                          hipMemcpyHostToDevice, ctx->stream));
    for (int i = 0; i < ctx->n; ++i) {
        const pd_status st = drop_carried_rates(ctx, i);
        if (st != PD_OK) return st;
    }
    PD_HIP(hipStreamSynchronize(ctx->stream));
    ctx->guide_set = true;
    return PD_OK;
}

pd_status pd_reset_origin(pd_ctx* ctx, int32_t inst)
{
    pd_status st = check_inst(ctx, inst);
    if (st != PD_OK) return st;
    if (!ctx->dev[inst].origin[0]) return fail(ctx, PD_ESTATE, "instance does not track origins");
    if (ctx->stepped) return fail(ctx, PD_ESTATE, "reset between pd_step and pd_resample");
    st = materialise(ctx);
    if (st != PD_OK) return st;
    PD_HIP(launch_iota_origin(ctx->d_insts, inst, ctx->params[inst].Nc, ctx->cur, ctx->stream));
    PD_HIP(hipStreamSynchronize(ctx->stream));
    return PD_OK;
}

pd_status pd_get_origin(pd_ctx* ctx, int32_t inst, int32_t* origin)
{
    pd_status st = check_inst(ctx, inst);
    if (st != PD_OK) return st;
    if (!origin) return fail(ctx, PD_EINVAL, "null output");
    if (!ctx->dev[inst].origin[0]) return fail(ctx, PD_ESTATE, "instance does not track origins");
    st = materialise(ctx);
    if (st != PD_OK) return st;
    PD_HIP(hipMemcpyAsync(origin, ctx->dev[inst].origin[ctx->cur],
                          4 * (size_t)ctx->params[inst].Nc, hipMemcpyDeviceToHost, ctx->stream));
    PD_HIP(hipStreamSynchronize(ctx->stream));
    return PD_OK;
}

pd_status pd_hop_counts(pd_ctx* ctx, uint64_t* d_hops)
{
    if (!ctx) return PD_EINVAL;
    if (!d_hops) return fail(ctx, PD_EINVAL, "null output");
    PD_HIP(launch_hop_counts(ctx->d_insts, ctx->n, d_hops, ctx->stream));
    return PD_OK;
}

pd_status pd_descendant_counts(pd_ctx* ctx, int32_t inst, uint32_t* d_counts)
{
    pd_status st = check_inst(ctx, inst);
    if (st != PD_OK) return st;
    if (!d_counts) return fail(ctx, PD_EINVAL, "null output");
    if (!ctx->dev[inst].origin[0]) return fail(ctx, PD_ESTATE, "instance does not track origins");
    if (ctx->stepped) return fail(ctx, PD_ESTATE, "counts between pd_step and pd_resample");
    st = materialise(ctx);
    if (st != PD_OK) return st;
    PD_HIP(launch_descendants(ctx->d_insts, inst, ctx->params[inst].Nc, ctx->cur, d_counts,
                              ctx->stream));
    return PD_OK;
}

pd_status pd_density_mode(pd_ctx* ctx, int32_t inst, int32_t n, double* d_out)
{
    pd_status st = check_inst(ctx, inst);
    if (st != PD_OK) return st;
    if (!d_out) return fail(ctx, PD_EINVAL, "null output");
    if (ctx->stepped) return fail(ctx, PD_ESTATE, "observable between pd_step and pd_resample");
    st = materialise(ctx);
    if (st != PD_OK) return st;
    const pd_params& p = ctx->params[inst];
    PD_HIP(launch_density_mode(words_of(p.L), ctx->d_insts, inst, p.Nc, ctx->cur, n, d_out,
                               ctx->stream));
    return PD_OK;
}

pd_status pd_mean(pd_ctx* ctx, int32_t inst, const double* d_values, int32_t ancestral,
                  double* mean)
{
    pd_status st = check_inst(ctx, inst);
    if (st != PD_OK) return st;
    if (!d_values || !mean) return fail(ctx, PD_EINVAL, "null argument");
    if (ancestral != 0 && ancestral != 1) return fail(ctx, PD_EINVAL, "ancestral must be 0 or 1");
    if (ancestral && !ctx->dev[inst].origin[0])
        return fail(ctx, PD_ESTATE, "instance does not track origins");
    if (ctx->stepped) return fail(ctx, PD_ESTATE, "observable between pd_step and pd_resample");
    st = materialise(ctx);
    if (st != PD_OK) return st;
    const InstDev& d = ctx->dev[inst];
    PD_HIP(launch_mean(ctx->d_insts, inst, ctx->params[inst].Nc, ctx->cur, d_values, ancestral,
                       ctx->stream));
    PD_HIP(hipMemcpyAsync(mean, d.tile_off, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    PD_HIP(hipStreamSynchronize(ctx->stream));
    return PD_OK;
}

pd_status pd_histogram(pd_ctx* ctx, int32_t inst, const double* d_values, int32_t ancestral,
                       double lo, double width, int32_t nbins, uint64_t* d_counts)
{
    pd_status st = check_inst(ctx, inst);
    if (st != PD_OK) return st;
    if (!d_values || !d_counts) return fail(ctx, PD_EINVAL, "null argument");
    if (ancestral != 0 && ancestral != 1) return fail(ctx, PD_EINVAL, "ancestral must be 0 or 1");
    if (nbins < 1 || nbins > kMaxHistBins) return fail(ctx, PD_EINVAL, "nbins must be in [1, 4096]");
    if (!std::isfinite(lo) || !(width > 0.0) || !std::isfinite(width))
        return fail(ctx, PD_EINVAL, "lo must be finite and width finite and positive");
    if (ancestral && !ctx->dev[inst].origin[0])
        return fail(ctx, PD_ESTATE, "instance does not track origins");
    if (ctx->stepped) return fail(ctx, PD_ESTATE, "observable between pd_step and pd_resample");
    st = materialise(ctx);
    if (st != PD_OK) return st;
    PD_HIP(launch_histogram(ctx->d_insts, inst, ctx->params[inst].Nc, ctx->cur, d_values,
                            ancestral, lo, width, nbins, d_counts, ctx->stream));
    return PD_OK;
}

pd_status pd_get_tuning(pd_ctx* ctx, pd_tuning* out)
{
    if (!ctx || !out) return PD_EINVAL;
    *out = ctx->tuning;
    return PD_OK;
}

pd_status pd_set_tuning(pd_ctx* ctx, const pd_tuning* t)
{
    if (!ctx || !t) return PD_EINVAL;
    return apply_tuning(ctx, *t);
}

pd_status pd_autotune(pd_ctx* ctx, int32_t trial_cycles, pd_tuning* best)
{
    if (!ctx || trial_cycles < 1) return PD_EINVAL;
    if (ctx->stepped) return fail(ctx, PD_ESTATE, "autotune between pd_step and pd_resample");
    if (ctx->any_guided && !ctx->guide_set)
        return fail(ctx, PD_ESTATE, "guided instances need pd_set_guide first");
    // the trials advance the population: keep a checkpoint and restore it
    size_t nb = 0;
    pd_status st = pd_save_bytes(ctx, &nb);
    if (st != PD_OK) return st;
    std::vector<char> snap(nb);
    const int64_t beta0 = ctx->beta;
    st = pd_save(ctx, snap.data(), nb);
    if (st != PD_OK) return st;
    const pd_tuning start = ctx->tuning;
    // the trials are not part of a stage timing
    const bool timing = ctx->timing;
    ctx->timing = false;
    struct Restore { pd_ctx* c; bool t; ~Restore() { c->timing = t; } } restore{ctx, timing};
    std::vector<pd_tuning> cands;
    pd_tuning t = start;
    t.step_variant = 0;
    cands.push_back(t);
    t.step_variant = 4;
    for (int f : {12, 13, 14, 15}) {
        t.refill = f;
        cands.push_back(t);
    }
    for (int v : {1, 2, 3})
        for (int rf : {4, 8, 16}) {
            t.step_variant = v;
            t.refill = rf;
            cands.push_back(t);
        }
    t.step_variant = 5;
    for (int f : {13, 14}) {
        t.refill = f;
        cands.push_back(t);
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    PD_HIP(hipEventCreate(&e0));
    PD_HIP(hipEventCreate(&e1));
    // one untimed cycle, then the timed ones (single launches, no graph)
    auto time_one = [&](const pd_tuning& c, float* ms) -> pd_status {
        pd_status s2 = apply_tuning(ctx, c);
        for (int rep = 0; rep <= trial_cycles && s2 == PD_OK; ++rep) {
            if (rep == 1 && hipEventRecord(e0, ctx->stream) != hipSuccess) return PD_EDEVICE;
            s2 = enqueue_cycle(ctx, ctx->perm ? 1 : 0, ctx->cur);
            if (s2 != PD_OK) break;
            ctx->cur ^= 1;
            ctx->perm = true;
        }
        if (s2 != PD_OK) return s2;
        if (hipEventRecord(e1, ctx->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess)
            return PD_EDEVICE;
        if (hipEventElapsedTime(ms, e0, e1) != hipSuccess) return PD_EDEVICE;
        return PD_OK;
    };
    // each list is timed in two interleaved passes and a candidate keeps its
    // faster time, so one disturbed trial does not decide
    auto pick = [&](const std::vector<pd_tuning>& list, pd_tuning* out) -> pd_status {
        std::vector<float> best(list.size(), 1e30f);
        for (int pass = 0; pass < 2; ++pass)
            for (size_t i = 0; i < list.size(); ++i) {
                float ms = 0.0f;
                const pd_status s2 = time_one(list[i], &ms);
                if (s2 != PD_OK) return s2;
                best[i] = std::min(best[i], ms);
            }
        *out = list[std::min_element(best.begin(), best.end()) - best.begin()];
        return PD_OK;
    };
    pd_tuning chosen = start;
    // the dynamical stage's launch configuration, then the cloning stage's scan tiling
    st = pick(cands, &chosen);
    if (st == PD_OK) {
        std::vector<pd_tuning> tilings;
        for (int tpb : {1, 2, 4, 8}) {
            pd_tuning c = chosen;
            c.scan_tiles = tpb;
            tilings.push_back(c);
        }
        st = pick(tilings, &chosen);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != PD_OK) return st;
    st = pd_load(ctx, snap.data(), nb);
    if (st != PD_OK) return st;
    ctx->beta = beta0;
    st = apply_tuning(ctx, chosen);
    if (st != PD_OK) return st;
    if (best) *best = chosen;
    return PD_OK;
}

pd_status pd_time_stages(pd_ctx* ctx, int32_t enable)
{
    if (!ctx) return PD_EINVAL;
    if (enable != 0 && enable != 1) return fail(ctx, PD_EINVAL, "enable must be 0 or 1");
    if (ctx->stepped) return fail(ctx, PD_ESTATE, "stage timing between pd_step and pd_resample");
    PD_HIP(hipStreamSynchronize(ctx->stream));
    for (hipEvent_t e : ctx->ev_step) PD_HIP(hipEventDestroy(e));
    for (hipEvent_t e : ctx->ev_res) PD_HIP(hipEventDestroy(e));
    ctx->ev_step.clear();
    ctx->ev_res.clear();
    ctx->timing = enable == 1;
    return PD_OK;
}

pd_status pd_get_stage_times(pd_ctx* ctx, pd_stage_times* out)
{
    if (!ctx || !out) return PD_EINVAL;
    if (ctx->stepped) return fail(ctx, PD_ESTATE, "stage timing between pd_step and pd_resample");
    PD_HIP(hipStreamSynchronize(ctx->stream));
    std::memset(out, 0, sizeof *out);
    const size_t ns = ctx->ev_step.size() / 3, nr = ctx->ev_res.size() / 2;
    for (size_t k = 0; k < ns; ++k) {
        float a = 0.0f, b = 0.0f;
        PD_HIP(hipEventElapsedTime(&a, ctx->ev_step[3 * k], ctx->ev_step[3 * k + 1]));
        PD_HIP(hipEventElapsedTime(&b, ctx->ev_step[3 * k + 1], ctx->ev_step[3 * k + 2]));
        out->step_ms += a;
        out->prefix_ms += b;
    }
    for (size_t k = 0; k < nr; ++k) {
        float a = 0.0f;
        PD_HIP(hipEventElapsedTime(&a, ctx->ev_res[2 * k], ctx->ev_res[2 * k + 1]));
        out->resample_ms += a;
    }
    if (ns) { out->step_ms /= (double)ns; out->prefix_ms /= (double)ns; }
    if (nr) out->resample_ms /= (double)nr;
    out->steps = (int64_t)ns;
    out->resamples = (int64_t)nr;
    return PD_OK;
}

const char* pd_last_error(const pd_ctx* ctx)
{
    return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

const char* pd_status_str(pd_status s)
{
    switch (s) {
        case PD_OK: return "ok";
        case PD_EINVAL: return "invalid argument";
        case PD_ENOMEM: return "buffer too small";
        case PD_EDEVICE: return "device error";
        case PD_ESTATE: return "call out of order";
        case PD_EUNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

}  // extern "C"
