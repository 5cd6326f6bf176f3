/*
 * pd_guide.h -- C ABI of the learned guide of the population-dynamics library.
 *
 * Sec. 2.2 of arXiv:1711.05095 shows that running the clones with controlled
 * rates W^ctrl(C -> C') = W_s(C -> C') v(C')/v(C), v the dominant (right)
 * eigenvector of the tilted generator, and compensating weights leaves
 * psi-hat unbiased while the clones' cloning factors become (nearly)
 * constant; Sec. 2.4 relates a clone's expected number of descendants after
 * a long lag to v of its configuration.  The guide here is a translation-
 * equivariant net f(C) ~ ln v(C) + const, trained on the GPU by Poisson
 * regression of descendant counts measured in plain runs (pd_reset_origin /
 * pd_get_origin), then distilled into the 8192-entry bond table that
 * pd_set_guide takes.
 *
 * Network (flat float32 parameter vector theta of PDG_PARAMS entries):
 *   a_j = 2 n_j - 1 (n_j the occupation of site j)
 *   h1[c][j] = tanh(b1[c] + sum_k W1[c][k] a_{j+k-2})                  c < 32, k < 5
 *   h2[c][j] = tanh(b2[c] + sum_{c',k} W2[c][c'][k] h1[c'][j+k-2])
 *   o_j      = b3 + sum_{c,k} W3[c][k] h2[c][j+k-2]
 *   f(C)     = sum_j o_j                                   (site indices mod L)
 * Offsets in theta: W1 0 [32][5], b1 160, W2 192 [32][32][5], b2 5312,
 * W3 5344 [32][5], b3 5504, c0 5505 (the Poisson intercept).  The weights
 * W1, W2, W3 enter the arithmetic rounded to bfloat16 (nearest, ties to
 * even), the layer-2 contractions accumulate in float32 on the matrix cores,
 * everything else is float32.  Gradients are taken with respect to the
 * rounded weights and applied to the float32 master copy.
 *
 * Because every o_j depends on the 13 sites j-6..j+6 only, f(C) = sum_j
 * h(window_j); pdg_window_table evaluates h for all 8192 windows and
 * pdg_bond_table averages the change of f across a hop over the sites the
 * bond table cannot see.
 *
 * Conventions as in pd.h: a pd_status is returned; invalid arguments give
 * PD_EINVAL before any device work; a failing HIP call gives PD_EDEVICE;
 * pdg_last_error() holds the message of the last failure on this host
 * thread.  Every pointer is a caller-owned device pointer unless stated;
 * work is queued on `hip_stream` (NULL: default stream) and not
 * synchronised.
 */
#ifndef PD_GUIDE_H
#define PD_GUIDE_H

#include "pd.h"

#ifdef __cplusplus
extern "C" {
#endif

#define PDG_PARAMS 5506
#define PDG_WINDOWS 8192
#define PDG_MIN_L 5
#define PDG_MAX_GMAX 3.45   /* ln(1024)/2 rounded down: tables pd_set_guide accepts */

/* Bytes of device workspace pdg_loss_grad needs for n samples (n >= 1). */
pd_status pdg_workspace_bytes(int64_t n, size_t* bytes);

/* f_out[i] = f(C_i) for n configurations.  `states` holds uint64 words
 * [W][ld], W = ceil(L/64) (word w of configuration i at w*ld + i; site j is
 * bit j%64 of word j/64, bits >= L ignored): with ld = Nc, the population
 * layout of pd_get_population; a larger ld selects n columns of a wider
 * array.  PDG_MIN_L <= L <= PD_MAX_L, 1 <= n <= ld <= 2^31 - 1. */
pd_status pdg_forward(const float* theta, const uint64_t* states, int64_t ld, int32_t L,
                      int64_t n, float* f_out, void* hip_stream);

/* Poisson regression loss of descendant counts (Sec. 2.4: the expected count
 * is proportional to v(C)):
 *   loss = (1/n) sum_i [exp(f(C_i) + c0) - counts[i] (f(C_i) + c0)]
 * and its gradient grad[PDG_PARAMS] with respect to theta (states as in
 * pdg_forward, counts[i] for column i); `loss` (one float) may be NULL.  `work` is device scratch of pdg_workspace_bytes(n) bytes,
 * 256-byte aligned.  counts[i] >= 0. */
pd_status pdg_loss_grad(const float* theta, const uint64_t* states, int64_t ld,
                        const float* counts, int32_t L, int64_t n, float* grad, float* loss,
                        void* work, size_t work_bytes, void* hip_stream);

/* One Adam step (Kingma and Ba; beta1 0.9, beta2 0.999, eps 1e-8) on the
 * PDG_PARAMS entries of theta with moment buffers m and v (zero before step
 * 1); `step` >= 1 is the step number used in the bias corrections, lr > 0. */
pd_status pdg_adam(float* theta, float* m, float* v, const float* grad, int32_t step, float lr,
                   void* hip_stream);

/* One epoch of training (Sec. 2.4's regression of descendant counts): the n
 * samples (states, ld and counts as in pdg_loss_grad) in minibatches of
 * `batch` columns, [0, batch), [batch, 2 batch), ..., the last one shorter;
 * for the k-th minibatch (k = 0, 1, ...) the gradient of its mean loss and
 * one Adam step with step number step0 + k + 1, as pdg_loss_grad followed by
 * pdg_adam would give them (same results, bit for bit), then its loss added,
 * as a double, to *loss_sum (device memory) in minibatch order.  Everything
 * is enqueued on the stream from the library (two launches per minibatch, no
 * host synchronisation); the caller advances its step count by
 * ceil(n / batch).  work: pdg_workspace_bytes(min(batch, n)) bytes, 256-byte
 * aligned.  batch >= 1, step0 >= 0, lr > 0. */
pd_status pdg_train_epoch(float* theta, float* m, float* v, const uint64_t* states, int64_t ld,
                          const float* counts, int32_t L, int64_t n, int64_t batch, int32_t step0,
                          float lr, double* loss_sum, void* work, size_t work_bytes,
                          void* hip_stream);

/* table[w] = h(w) for the 8192 windows w of 13 sites (site j-6 in bit 0 ...
 * site j+6 in bit 12): the net on the window alone, so f(C) = sum_j h(w_j). */
pd_status pdg_window_table(const float* theta, float* table, void* hip_stream);

/* Bond table for pd_set_guide from a window table (float, 8192 entries): for
 * every neighbourhood u of a bond (b, b+1) (site b-6 in bit 0 ... b+6 in bit
 * 12) whose two bond sites differ, G[u] = the change of f(C) when the
 * particle crosses the bond, i.e. the 14 windows that contain b or b+1
 * evaluated after minus before, averaged (in double precision) over all
 * 8192 settings of the 13 sites b-12..b-7 and b+7..b+13 that u leaves out;
 * eg[u] = rint(2^16 exp(clamp(G[u], -gmax, gmax))), and eg[u] = G[u] = 0
 * for the other u.  0 <= gmax <= PDG_MAX_GMAX; G (double[8192]) may be NULL. */
pd_status pdg_bond_table(const float* window_table, double gmax, uint32_t* eg, double* G,
                         void* hip_stream);

/* Bond table conditioned on a sample of configurations (states as in
 * pdg_forward; L >= PDG_COND_MIN_L so that the windows around a bond span
 * distinct sites): for every configuration and every bond whose two sites
 * differ, d = f(C after the hop) - f(C) exactly (the 14 windows holding b or
 * b+1, after minus before, summed in double precision); G[u] = the mean of d
 * over the pairs with neighbourhood u if there are at least min_count (>= 1)
 * of them, else the uniform-context value of pdg_bond_table; eg as there.
 * The mean over the data is the best table entry in the least-squares sense
 * for configurations drawn like the sample, which the uniform average is not
 * when distant sites are correlated with the neighbourhood (phase-separated
 * populations, Sec. 3.3).  counts (uint32[8192], may be NULL) receives the
 * number of pairs per u; G may be NULL.  `work` is device scratch of
 * PDG_COND_WORK_BYTES bytes, 256-byte aligned. */
#define PDG_COND_MIN_L 26
#define PDG_COND_WORK_BYTES 163840
pd_status pdg_bond_table_cond(const float* window_table, const uint64_t* states, int64_t ld,
                              int32_t L, int64_t n, int32_t min_count, double gmax, uint32_t* eg,
                              double* G, uint32_t* counts, void* work, size_t work_bytes,
                              void* hip_stream);

/* pdg_bond_table_cond without the caller's workspace, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the arguments and results are
 * those of pdg_bond_table_cond, and the function allocates nothing.  Its
 * scratch is the library's own array of PDG_NOALLOC_SCRATCH_BYTES (160 KiB)
 * per GPU, enough for any n (the distillation's scratch does not grow with
 * the sample), held until the process ends.  Every call on a GPU uses that
 * GPU's array: calls that overlap in time on one GPU (two streams, two host
 * threads) race on it and must be serialised by the caller.  The sums and
 * counts are cleared on the device at the start of each call. */
#define PDG_NOALLOC_SCRATCH_BYTES 163840
pd_status pdg_bond_table_cond_noalloc(const float* window_table, const uint64_t* states,
                                      int64_t ld, int32_t L, int64_t n, int32_t min_count,
                                      double gmax, uint32_t* eg, double* G, uint32_t* counts,
                                      void* hip_stream);

const char* pdg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* PD_GUIDE_H */
