// Guide network: constants and kernel launchers shared by its kernels and its
// C ABI.  Internal: not part of the C ABI.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pd {

constexpr int kGuideParams = 5506;  // flat parameter vector (layout in pd_guide.h)
constexpr int kGuideBlocks = 768;   // one-wave blocks of the sample-parallel kernels
constexpr int kGuideMinL = 5;       // the circular halo of 2 sites must not wrap twice

int guide_blocks(int64_t n);
size_t net_smem(int L);
hipError_t net_set_smem_limit(int L);
// mode 0: f_out[i] = f(C_i); mode 1: grad, loss of the Poisson loss (partial:
// guide_blocks(n) * (kGuideParams + 1) floats of workspace)
hipError_t launch_net(int mode, const float* theta, const uint64_t* states, int64_t ld,
                      const float* counts, int L, int64_t n, float* f_out, float* partial,
                      float* grad, float* loss, hipStream_t st);
hipError_t launch_adam(float* theta, float* m, float* v, const float* grad, int step, float lr,
                       hipStream_t st);
// minibatches [a, a + batch) of n samples: partial gradients, then reduction
// fused with Adam (step numbers step0 + 1, ...), minibatch losses added to
// *loss_sum (partial: guide_blocks(batch) * (kGuideParams + 1) floats)
hipError_t launch_train_epoch(float* theta, float* m, float* v, const uint64_t* states,
                              int64_t ld, const float* counts, int L, int64_t n, int64_t batch,
                              int step0, float lr, double* loss_sum, float* partial,
                              hipStream_t st);
hipError_t launch_window_table(const float* theta, float* table, hipStream_t st);
hipError_t launch_bond_table(const float* H, double gmax, uint32_t* eg, double* G,
                             hipStream_t st);
// work: kCondWorkBytes bytes (sums, counts, and G when G is null)
constexpr size_t kCondWorkBytes = 8192 * (2 * sizeof(double) + sizeof(uint32_t));
hipError_t launch_bond_table_cond(const float* H, const uint64_t* states, int64_t ld, int L,
                                  int64_t n, uint32_t min_count, double gmax, uint32_t* eg,
                                  double* G, uint32_t* counts_out, void* work, hipStream_t st);
hipError_t stats_set_smem_limit();
// Device address, on the current device, of the library's own kCondWorkBytes
// of scratch for launch_bond_table_cond (looked up once per device).
hipError_t cond_scratch(void** out);

}  // namespace pd
