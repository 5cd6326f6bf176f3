// C ABI of the guide network (include/pd_guide.h): argument checks, then the
// kernels of pd_guide.hip.
#include <hip/hip_runtime.h>

#include <atomic>
#include <cmath>
#include <cstdint>
#include <string>

#include "../../include/pd_guide.h"
#include "pd_guide.hpp"

using namespace pd;

static_assert(PDG_PARAMS == kGuideParams, "parameter count");
static_assert(PDG_MIN_L == kGuideMinL, "smallest ring");
static_assert(PDG_COND_WORK_BYTES == kCondWorkBytes, "conditional distillation workspace");

namespace {

thread_local std::string g_guide_error;

pd_status gfail(pd_status st, const std::string& msg)
{
    g_guide_error = msg;
    return st;
}

pd_status gdev(hipError_t e, const char* what)
{
    if (e == hipSuccess) return PD_OK;
    return gfail(PD_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

bool aligned256(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 255u) == 0; }

std::string check_batch(const void* states, int64_t ld, int32_t L, int64_t n)
{
    if (!states) return "null states";
    if (L < kGuideMinL || L > PD_MAX_L) return "L out of range";
    if (n < 1 || n > INT32_MAX) return "n out of range";
    if (ld < n || ld > INT32_MAX) return "ld must satisfy n <= ld <= 2^31 - 1";
    return "";
}

// A kernel attribute (hipFuncSetAttribute) holds for the device that is current when it is set:
// each flag records, per device, that it has been set there.  Setting it twice is harmless, so
// two threads racing on the first call need no lock.
constexpr int kMaxDevices = 64;
std::atomic<bool> g_net_smem_set[kMaxDevices];
std::atomic<bool> g_stats_smem_set[kMaxDevices];

pd_status once_per_device(std::atomic<bool>* flags, hipError_t (*set)())
{
    int dev = 0;
    pd_status st = gdev(hipGetDevice(&dev), "hipGetDevice");
    if (st != PD_OK) return st;
    if (dev < 0 || dev >= kMaxDevices) return gfail(PD_EDEVICE, "device ordinal beyond 63");
    if (flags[dev].load(std::memory_order_acquire)) return PD_OK;
    st = gdev(set(), "hipFuncSetAttribute");
    if (st == PD_OK) flags[dev].store(true, std::memory_order_release);
    return st;
}

// The sample kernels' dynamic LDS grows with L: the limit is raised once, for the largest ring.
hipError_t net_smem_max_l() { return net_set_smem_limit(PD_MAX_L); }

pd_status smem_limit() { return once_per_device(g_net_smem_set, net_smem_max_l); }

}  // namespace

extern "C" {

pd_status pdg_workspace_bytes(int64_t n, size_t* bytes)
{
    if (!bytes || n < 1 || n > INT32_MAX) return gfail(PD_EINVAL, "null argument or n out of range");
    *bytes = (size_t)guide_blocks(n) * (kGuideParams + 1) * sizeof(float);
    return PD_OK;
}

pd_status pdg_forward(const float* theta, const uint64_t* states, int64_t ld, int32_t L,
                      int64_t n, float* f_out, void* hip_stream)
{
    std::string m = check_batch(states, ld, L, n);
    if (!m.empty()) return gfail(PD_EINVAL, m);
    if (!theta || !f_out) return gfail(PD_EINVAL, "null pointer");
    pd_status st = smem_limit();
    if (st != PD_OK) return st;
    return gdev(launch_net(0, theta, states, ld, nullptr, L, n, f_out, nullptr, nullptr, nullptr,
                           (hipStream_t)hip_stream),
                "forward launch");
}

pd_status pdg_loss_grad(const float* theta, const uint64_t* states, int64_t ld,
                        const float* counts, int32_t L, int64_t n, float* grad, float* loss,
                        void* work, size_t work_bytes, void* hip_stream)
{
    std::string m = check_batch(states, ld, L, n);
    if (!m.empty()) return gfail(PD_EINVAL, m);
    if (!theta || !counts || !grad || !work) return gfail(PD_EINVAL, "null pointer");
    if (!aligned256(work)) return gfail(PD_EINVAL, "workspace must be 256-byte aligned");
    size_t need = 0;
    pdg_workspace_bytes(n, &need);
    if (work_bytes < need) return gfail(PD_ENOMEM, "workspace too small");
    pd_status st = smem_limit();
    if (st != PD_OK) return st;
    return gdev(launch_net(1, theta, states, ld, counts, L, n, nullptr, (float*)work, grad, loss,
                           (hipStream_t)hip_stream),
                "loss/gradient launch");
}

pd_status pdg_adam(float* theta, float* m, float* v, const float* grad, int32_t step, float lr,
                   void* hip_stream)
{
    if (!theta || !m || !v || !grad) return gfail(PD_EINVAL, "null pointer");
    if (step < 1 || !(lr > 0.0f) || !std::isfinite(lr)) return gfail(PD_EINVAL, "step < 1 or lr <= 0");
    return gdev(launch_adam(theta, m, v, grad, step, lr, (hipStream_t)hip_stream), "adam launch");
}

pd_status pdg_train_epoch(float* theta, float* m, float* v, const uint64_t* states, int64_t ld,
                          const float* counts, int32_t L, int64_t n, int64_t batch, int32_t step0,
                          float lr, double* loss_sum, void* work, size_t work_bytes,
                          void* hip_stream)
{
    std::string msg = check_batch(states, ld, L, n);
    if (!msg.empty()) return gfail(PD_EINVAL, msg);
    if (!theta || !m || !v || !counts || !loss_sum || !work) return gfail(PD_EINVAL, "null pointer");
    if (batch < 1) return gfail(PD_EINVAL, "batch < 1");
    if (step0 < 0 || (int64_t)step0 + (n + batch - 1) / batch > INT32_MAX)
        return gfail(PD_EINVAL, "step0 < 0 or step numbers overflow");
    if (!(lr > 0.0f) || !std::isfinite(lr)) return gfail(PD_EINVAL, "lr <= 0");
    if (!aligned256(work)) return gfail(PD_EINVAL, "workspace must be 256-byte aligned");
    size_t need = 0;
    pdg_workspace_bytes(batch < n ? batch : n, &need);
    if (work_bytes < need) return gfail(PD_ENOMEM, "workspace too small");
    pd_status st = smem_limit();
    if (st != PD_OK) return st;
    return gdev(launch_train_epoch(theta, m, v, states, ld, counts, L, n, batch, step0, lr,
                                   loss_sum, (float*)work, (hipStream_t)hip_stream),
                "training launch");
}

pd_status pdg_window_table(const float* theta, float* table, void* hip_stream)
{
    if (!theta || !table) return gfail(PD_EINVAL, "null pointer");
    return gdev(launch_window_table(theta, table, (hipStream_t)hip_stream), "window table launch");
}

pd_status pdg_bond_table(const float* window_table, double gmax, uint32_t* eg, double* G,
                         void* hip_stream)
{
    if (!window_table || !eg) return gfail(PD_EINVAL, "null pointer");
    if (!(gmax >= 0.0) || !(gmax <= PDG_MAX_GMAX)) return gfail(PD_EINVAL, "gmax out of range");
    return gdev(launch_bond_table(window_table, gmax, eg, G, (hipStream_t)hip_stream),
                "bond table launch");
}

pd_status pdg_bond_table_cond(const float* window_table, const uint64_t* states, int64_t ld,
                              int32_t L, int64_t n, int32_t min_count, double gmax, uint32_t* eg,
                              double* G, uint32_t* counts, void* work, size_t work_bytes,
                              void* hip_stream)
{
    std::string m = check_batch(states, ld, L, n);
    if (!m.empty()) return gfail(PD_EINVAL, m);
    if (L < PDG_COND_MIN_L) return gfail(PD_EINVAL, "conditional distillation needs L >= 26");
    if (!window_table || !eg || !work) return gfail(PD_EINVAL, "null pointer");
    if (min_count < 1) return gfail(PD_EINVAL, "min_count must be >= 1");
    if (!(gmax >= 0.0) || !(gmax <= PDG_MAX_GMAX)) return gfail(PD_EINVAL, "gmax out of range");
    if (!aligned256(work)) return gfail(PD_EINVAL, "workspace must be 256-byte aligned");
    if (work_bytes < kCondWorkBytes) return gfail(PD_ENOMEM, "workspace too small");
    pd_status st = once_per_device(g_stats_smem_set, stats_set_smem_limit);
    if (st != PD_OK) return st;
    return gdev(launch_bond_table_cond(window_table, states, ld, L, n, (uint32_t)min_count, gmax,
                                       eg, G, counts, work, (hipStream_t)hip_stream),
                "conditional bond table launch");
}

pd_status pdg_bond_table_cond_noalloc(const float* window_table, const uint64_t* states,
                                      int64_t ld, int32_t L, int64_t n, int32_t min_count,
                                      double gmax, uint32_t* eg, double* G, uint32_t* counts,
                                      void* hip_stream)
{
    std::string m = check_batch(states, ld, L, n);
    if (!m.empty()) return gfail(PD_EINVAL, m);
    if (L < PDG_COND_MIN_L) return gfail(PD_EINVAL, "conditional distillation needs L >= 26");
    if (!window_table || !eg) return gfail(PD_EINVAL, "null pointer");
    if (min_count < 1) return gfail(PD_EINVAL, "min_count must be >= 1");
    if (!(gmax >= 0.0) || !(gmax <= PDG_MAX_GMAX)) return gfail(PD_EINVAL, "gmax out of range");
    // the kernels need kCondWorkBytes of scratch for any n: the library's array holds exactly that
    static_assert(PDG_NOALLOC_SCRATCH_BYTES == kCondWorkBytes, "no-allocation scratch size");
    void* work = nullptr;
    pd_status st = gdev(cond_scratch(&work), "scratch address");
    if (st != PD_OK) return st;
    st = once_per_device(g_stats_smem_set, stats_set_smem_limit);
    if (st != PD_OK) return st;
    return gdev(launch_bond_table_cond(window_table, states, ld, L, n, (uint32_t)min_count, gmax,
                                       eg, G, counts, work, (hipStream_t)hip_stream),
                "conditional bond table launch");
}

const char* pdg_last_error(void) { return g_guide_error.c_str(); }

}  // extern "C"
