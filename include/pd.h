/*
 * pd.h -- C ABI of the MI355X population-dynamics (cloning) library for
 * large deviations of the activity of the periodic symmetric simple
 * exclusion process (SSEP).
 *
 * The method is the cloning algorithm of T. Brewer, S. R. Clark, R. Bradford,
 * R. L. Jack, "Efficient characterisation of large deviations using population
 * dynamics" (arXiv:1711.05095):
 *   - Nc clones of the SSEP (L sites, N particles, hop rate 1 to each empty
 *     neighbour, periodic; Sec. 3.1) evolve independently for an interval
 *     Delta t in continuous time (the dynamical stage, Sec. 2.3 and Sec. 4);
 *   - each clone carries its cloning factor Upsilon^beta (eq. upsbdef): with
 *     the modified dynamics of Sec. 3.2 (every rate times e^{-s}) it is
 *     exp(-(1 - e^{-s}) * integral of r(C) dt) (eq. def-ups-ssep); with the
 *     unmodified dynamics it is e^{-s K^beta} (Sec. 3.1); with a guide g it
 *     is the compensating factor of eqs. modpdef and upsdef (Sec. 2.2);
 *   - the cloning stage replaces the population by Nc clones pulled from the
 *     old one by the [eq] rule of Sec. 4.1 (eq. alpha-Ups) or the [iid] rule;
 *   - after M = t_obs / Delta t repetitions, psi-hat (eq. psihat) estimates
 *     the scaled cumulant generating function and k-hat (eq. khat, divided
 *     also by Nc) the biased activity per site.
 *
 * Conventions for every function:
 *   - The return value is a pd_status: PD_OK (0) or a negative error.  No
 *     C++ exception crosses this boundary.  pd_last_error() returns a
 *     human-readable message for the last failure on a context.
 *   - Invalid arguments return PD_EINVAL before any device work is queued.
 *     A failing HIP call returns PD_EDEVICE.
 *   - Device memory is owned by the caller: pd_workspace_bytes() says how
 *     much, pd_create() takes a device pointer to it (256-byte aligned), and
 *     the memory must outlive the context.  The library allocates no device
 *     memory of its own; pd_destroy() frees only the host-side context.
 *   - All device work is queued on the HIP stream given to pd_create()
 *     (NULL means the default stream).  Calls that return results to the
 *     host (pd_scgf, pd_get_*, pd_save) synchronise that stream.
 *   - A context holds n independent instances (a batch); functions that take
 *     `inst` act on one of them, the others on all.  A context is not
 *     thread-safe; use one context per host thread and stream.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by `seed`; the
 * counter of every draw is (draw index, clone slot, interval beta, tag |
 * instance << 8), so results depend only on the parameters, never on how the
 * GPU schedules the work.
 */
#ifndef PD_H
#define PD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PD_OK = 0,
    PD_EINVAL = -1,       /* invalid argument or parameter set */
    PD_ENOMEM = -2,       /* workspace or host buffer too small */
    PD_EDEVICE = -3,      /* a HIP call failed; see pd_last_error */
    PD_ESTATE = -4,       /* call out of order (e.g. two dynamical stages in a row) */
    PD_EUNSUPPORTED = -5  /* parameter combination not supported by this library */
} pd_status;

typedef enum {
    PD_SEL_EQ = 0,        /* equally spaced points, one offset d per interval (Sec. 4.1) */
    PD_SEL_IID = 1        /* independent uniform points (Sec. 4.1, [iid]) */
} pd_selection;

typedef enum {
    PD_W_MODIFIED = 0,    /* rates x e^{-s}; Ups = exp(-(1-e^{-s}) int r dt) (Sec. 3.2) */
    PD_W_DIRECT = 1,      /* unmodified rates; Ups = e^{-s K^beta} (Sec. 3.1) */
    PD_W_GUIDED = 2       /* rates x e^{-s+g}; exact compensating weight (Sec. 2.2) */
} pd_weight_mode;

#define PD_MAX_L 512      /* states are at most 8 words of 64 sites */

typedef struct {
    int32_t  L;           /* sites, 2 <= L <= PD_MAX_L */
    int32_t  N;           /* particles, 0 <= N <= L (N = 0 or L: no hop, psi-hat = 0) */
    double   s;           /* biasing field, finite */
    int64_t  Nc;          /* clones, 1 <= Nc <= 2^31 - 1 */
    double   t_obs;       /* observation time, > 0 */
    double   dt;          /* cloning interval Delta t, > 0; M = llround(t_obs/dt) >= 1
                             and |M dt - t_obs| <= 1e-9 t_obs, else PD_EINVAL */
    uint64_t seed;        /* Philox key */
    int32_t  selection;   /* pd_selection */
    int32_t  weight_mode; /* pd_weight_mode */
    uint32_t instance;    /* Philox counter tag, < 2^24; distinct per instance of a batch */
    int32_t  log_cycles;  /* >= 0: keep per-interval (ln mean Ups, mean K^beta) for the
                             first log_cycles intervals (see pd_get_log) */
    int64_t  burn_in;     /* >= 0: intervals left out of psi_burn and k_hat_burn
                             (pd_estimates); > 0 adds 16 bytes per clone of workspace */
    int32_t  track_origin;/* 1: every clone carries the slot it descended from at the last
                             pd_reset_origin (ancestral lines, Sec. 2.4); 0: off */
    int32_t  reserved;    /* must be 0 */
} pd_params;

typedef struct {
    double   psi;         /* psi-hat = (1/(beta dt)) sum over completed intervals */
    double   psi_burn;    /* the same sum over intervals beyond burn_in, / ((beta-burn_in) dt);
                             0 until beta > burn_in */
    double   k_hat;       /* sum_j K_j / (Nc L beta dt) over the current population */
    double   t;           /* beta * dt */
    int64_t  cycles;      /* beta: completed (dynamics, cloning) cycles */
    uint64_t hops;        /* every hop performed by every clone so far */
    double   k_hat_burn;  /* k_hat with the transient left out (Sec. 5.1): sum_j K'_j /
                             (Nc L (beta-burn_in) dt), K'_j = the hops of the intervals beyond
                             burn_in along clone j's ancestral line (K_j minus the K its
                             ancestor carried at the end of interval burn_in); equal to k_hat
                             when burn_in = 0; 0 until beta > burn_in.  With burn_in > 0,
                             pd_set_population restarts K' at 0 for the clones it installs */
    uint64_t draws;       /* guided instances: random draws of the guided dynamical stage so
                             far, one per proposed hop (taken or not, Sec. 2.2 by thinning)
                             and one closing draw per clone per interval; 0 for the other
                             forms */
} pd_estimates;

typedef struct pd_ctx pd_ctx;   /* opaque, host-side, owned by the library */

/* Bytes of device workspace for a batch of n instances (n >= 1). */
pd_status pd_workspace_bytes(const pd_params* params, int32_t n, size_t* bytes);

/* Validates the n parameter sets, lays out the workspace, and queues the
 * initial condition on `hip_stream`: every clone a uniform N-subset of the L
 * sites (the steady state at fixed N, Sec. 3.1), K = 0.  `d_workspace` is a
 * caller-owned device buffer of at least pd_workspace_bytes() bytes. */
pd_status pd_create(const pd_params* params, int32_t n, void* d_workspace, size_t bytes,
                    void* hip_stream, pd_ctx** out);

/* Releases the host-side context.  Does not touch the caller's device memory. */
pd_status pd_destroy(pd_ctx* ctx);

/* Dynamical stage of the next interval beta for every instance (Sec. 2.3):
 * each clone runs the continuous-time SSEP for Delta t and gets its hop count
 * K^beta, the integral of r dt and ln Upsilon^beta.  It also forms ln of the
 * population mean of Upsilon^beta (eq. psihat) and adds it to psi.
 * PD_ESTATE if the previous call was also pd_step. Asynchronous. */
pd_status pd_step(pd_ctx* ctx);

/* Cloning stage of interval beta (Sec. 4.1): new clone j is pulled, with its
 * accumulated K, from the old clone whose interval of the cumulative
 * Upsilon line holds the point alpha_j.  PD_ESTATE unless pd_step came
 * immediately before. Asynchronous. */
pd_status pd_resample(pd_ctx* ctx);

/* `cycles` repetitions of (pd_step, pd_resample) -- the cloning algorithm's
 * cycle of Sec. 2.3 -- replayed from captured HIP graphs of graph_cycles
 * cycles (pd_tuning; the remainder as single launches).  Asynchronous.
 * cycles = 0 runs nothing and captures the graphs that later calls replay,
 * uploading them to the device (a graph is otherwise captured and uploaded on
 * its first use).  Graphs need a stream other
 * than the legacy default stream; with NULL every cycle is a single launch.
 * PD_ESTATE if a pd_step is waiting for its pd_resample. */
pd_status pd_run(pd_ctx* ctx, int64_t cycles);

/* Estimates of instance 0 (synchronises the stream): psi-hat = (1/(beta dt))
 * sum over the completed intervals of ln((1/Nc) sum_i Upsilon_i) (eq. psihat),
 * k-hat = sum_j K_j / (Nc L beta dt) (eq. khat, with the 1/Nc the printed
 * formula omits), and beta.  Any output pointer may be NULL. */
pd_status pd_scgf(pd_ctx* ctx, double* psi, double* k_hat, int64_t* cycles_done);

/* Estimates of instance `inst` (synchronises the stream): psi-hat (eq. psihat),
 * k-hat (eq. khat with the 1/Nc the printed formula omits; K carried along
 * the ancestral lines, Sec. 4.2) and both with the first burn_in intervals
 * left out (the transient of Sec. 5.1). */
pd_status pd_estimates_get(pd_ctx* ctx, int32_t inst, pd_estimates* out);

/* The hop counts so far (pd_estimates.hops) of every instance, written to the
 * caller-owned device array d_hops[n] (uint64, n = the context's instances) by
 * a launch queued on the context stream, without synchronising: a progress or
 * throughput probe that leaves the device busy.  PD_EINVAL if d_hops is NULL. */
pd_status pd_hop_counts(pd_ctx* ctx, uint64_t* d_hops);

/* Host image of a population: uint64 state words [W][Nc] (word w of clone j
 * at w*Nc + j; site i is bit i%64 of word i/64, bits >= L are zero), then
 * uint64 K[Nc] (hops accumulated along the clone's ancestry).  W = ceil(L/64). */
pd_status pd_population_bytes(const pd_params* params, size_t* bytes);

/* Copies the current population of instance `inst` to `host` (synchronises). */
pd_status pd_get_population(pd_ctx* ctx, int32_t inst, void* host, size_t bytes);

/* Replaces the current population of instance `inst` (synchronises).
 * Every clone must hold exactly N particles in its first L bits (PD_EINVAL
 * otherwise).  Clears a pending dynamical stage.  Carried origins are left as
 * they were and mean nothing for the new clones until pd_reset_origin. */
pd_status pd_set_population(pd_ctx* ctx, int32_t inst, const void* host, size_t bytes);

/* Per-clone outputs of the last dynamical stage of instance `inst`, indexed
 * by clone slot: K^beta (uint32), integral of r dt (double), ln Upsilon^beta
 * (double).  Any pointer may be NULL.  Synchronises. */
pd_status pd_get_step_outputs(pd_ctx* ctx, int32_t inst, uint32_t* Kb, double* A, double* ell);

/* Ancestor map of the last cloning stage of instance `inst`: anc[j] = old
 * clone that new clone j was pulled from.  PD_ESTATE if no cloning stage has
 * run since the last dynamical stage.  Synchronises. */
pd_status pd_get_ancestors(pd_ctx* ctx, int32_t inst, int32_t* anc);

/* Ancestry (track_origin = 1): pd_reset_origin marks every clone of instance
 * `inst` as its own origin (origin[j] = j); from then on a clone carries the
 * origin of the clone it was pulled from at every cloning stage.
 * pd_get_origin copies the current origins (int32, Nc entries); the number
 * of clones with origin k is the descendant count of the clone that sat in
 * slot k at the reset.  PD_ESTATE if tracking is off.  Both synchronise. */
pd_status pd_reset_origin(pd_ctx* ctx, int32_t inst);
pd_status pd_get_origin(pd_ctx* ctx, int32_t inst, int32_t* origin);

/* Descendant counts (track_origin = 1): d_counts[k] = the number of current
 * clones of instance `inst` whose origin is k, i.e. the descendants of the
 * clone that sat in slot k at the last pd_reset_origin (Sec. 2.4: after a
 * long lag their expectation is proportional to v, the dominant eigenvector
 * of the tilted generator, of that clone's configuration).  d_counts: a
 * caller-owned device array of Nc uint32, overwritten.  Queued on the
 * context stream (no synchronisation).  PD_ESTATE if tracking is off or
 * between pd_step and pd_resample. */
pd_status pd_descendant_counts(pd_ctx* ctx, int32_t inst, uint32_t* d_counts);

/* Observables (Secs. 2.4, 3.3).  pd_density_mode queues, for every clone j of
 * instance `inst` (slot order), d_out[j] = |delta rho_n|^2 with
 * delta rho_n = L^{-1/2} sum over the occupied sites X of e^{-2 pi i n X / L}
 * (eq. fourdens); d_out is a caller-owned device array of Nc doubles.
 * pd_mean returns (1/Nc) sum_j v_j for a caller-owned device array d_values of
 * Nc doubles: v_j = d_values[j] (ancestral = 0: the end-time distribution of
 * the current population) or v_j = d_values[origin_j] (ancestral = 1, needs
 * track_origin: d_values holds a quantity recorded per slot at the last
 * pd_reset_origin, averaged over the ancestors of the current clones, the
 * ancestral distribution of eq. Opave).  pd_mean synchronises.  Both return
 * PD_ESTATE between pd_step and pd_resample. */
pd_status pd_density_mode(pd_ctx* ctx, int32_t inst, int32_t n, double* d_out);
pd_status pd_mean(pd_ctx* ctx, int32_t inst, const double* d_values, int32_t ancestral,
                  double* mean);

/* Histogram of a per-clone quantity, as the distributions p_end and p_ave of
 * Sec. 2.4 are shown (the activity distributions of Sec. 5): d_counts[b] =
 * #{j : floor((v_j - lo) / width) = b} for b = 0 .. nbins-1, with v_j as in
 * pd_mean (d_values[j], or d_values[origin_j] when ancestral = 1, which needs
 * track_origin).  The bin is decided by one FP64 subtraction and one FP64
 * division, then the floor; values outside [lo, lo + nbins width) and NaN
 * are not counted.  d_values: caller-owned device array of Nc doubles;
 * d_counts: caller-owned device array of nbins uint64, overwritten.
 * 1 <= nbins <= 4096, lo finite, width finite and > 0; PD_EINVAL otherwise,
 * PD_ESTATE between pd_step and pd_resample.  Queued on the context stream
 * (no synchronisation). */
pd_status pd_histogram(pd_ctx* ctx, int32_t inst, const double* d_values, int32_t ancestral,
                       double lo, double width, int32_t nbins, uint64_t* d_counts);

/* Per-interval log of instance `inst` (params.log_cycles > 0): for interval
 * beta = 1..n_rows, lbeta[beta-1] = ln((1/Nc) sum_i Upsilon_i^beta) and
 * mean_kb[beta-1] = population mean of K^beta before cloning.  Synchronises. */
pd_status pd_get_log(pd_ctx* ctx, int32_t inst, double* lbeta, double* mean_kb, int32_t n_rows);

/* Checkpoint of the whole context (all instances: populations, estimator sums
 * and, for instances with track_origin, the carried origins) into a host
 * buffer of pd_save_bytes() bytes, and its restore into a context created
 * with the same parameters.  A restored run continues bit-identically.  Both
 * synchronise.  pd_load checks the whole image before it uploads any of it
 * (magic and instance count, every state holding N particles on sites
 * 0..L-1, every origin in [0, Nc)) and returns PD_EINVAL, with the context
 * unchanged, if any check fails. */
pd_status pd_save_bytes(pd_ctx* ctx, size_t* bytes);
pd_status pd_save(pd_ctx* ctx, void* host, size_t bytes);
pd_status pd_load(pd_ctx* ctx, const void* host, size_t bytes);

/* Guide for the PD_W_GUIDED instances of the context (Sec. 2.2: controlled
 * dynamics with a compensating weight).  `d_table` is a caller-owned device
 * array of 8192 uint32 entries eg[u], one per 13-site bond neighbourhood u
 * (site b-6 in bit 0 ... site b+6 in bit 12, so the bond's own sites b, b+1
 * are bits 6 and 7).  The hop across an allowed bond has rate
 * e^{-s} eg[u] / 2^16, i.e. log-ratio g = ln(eg[u] / 2^16) on top of the
 * modified rate; the cloning factor carries the exact compensation
 * -sum_jumps g - integral (r - e^{-s} sum_b eg[u_b] / 2^16) dt, so psi-hat
 * stays unbiased for any table.  Entries of neighbourhoods whose bits 6 and 7
 * are equal must be 0, the others in [1, 2^31) with largest/smallest <= 1024;
 * PD_EINVAL otherwise (the guide in use is then unchanged), and also if
 * d_table is not 16-byte aligned.  The library copies the table into its
 * workspace, so the caller may change or free d_table once the call returns;
 * a changed table takes effect only through another pd_set_guide.
 * Synchronises. */
pd_status pd_set_guide(pd_ctx* ctx, const uint32_t* d_table, size_t n);

/* Launch configuration of the dynamical stage.  It never changes results
 * (every random number is keyed by clone slot, never by lane or block), only
 * speed. */
typedef struct {
    int32_t step_variant; /* 0: one clone per lane; 1, 2, 3: persistent waves,
                             each lane working through a queue of clones,
                             compiled for 4, 6 and 8 waves per SIMD (not with
                             track_origin: variant 0 runs instead); 4: one
                             clone per lane, the unfinished clones of a tile
                             packed into the lowest lanes between rounds of
                             events; 5: as 4, but all plain instances of the
                             context, whatever their word counts, in one
                             persistent launch whose blocks take tiles from a
                             work counter (largest word count and expected
                             work first) */
    int32_t refill;       /* variants 1-3: finished lanes (1..64) that trigger a
                             refill; variants 4, 5: length of the first round of
                             events in sixteenths of the expected number per
                             clone (later rounds: 0.15 of it) */
    int32_t graph_cycles; /* cycles per captured graph in pd_run (even, 0: no graph) */
    int32_t scan_tiles;   /* tiles of 256 clones per wave of the cloning stage: 1, 2, 4
                             or 8 (0 means 1); a wave loads them all before it
                             scans the first */
} pd_tuning;

/* A new context starts with {step_variant 4, refill 13, graph_cycles 16, scan_tiles 1}.
 * pd_autotune times the dynamical stage's configurations first and then the
 * scan tilings with the best of them. */
pd_status pd_get_tuning(pd_ctx* ctx, pd_tuning* out);
pd_status pd_set_tuning(pd_ctx* ctx, const pd_tuning* tuning);

/* Autotuner: times `trial_cycles` cycles of each candidate launch
 * configuration on this context's own instances, restores the population and
 * estimator state exactly as they were, and keeps the fastest configuration
 * (also written to `best` if not NULL).  Synchronises. */
pd_status pd_autotune(pd_ctx* ctx, int32_t trial_cycles, pd_tuning* best);

/* Stage timing, for measurement.  pd_time_stages(ctx, 1) discards earlier
 * records and makes every later pd_step and pd_resample (and the single
 * launches of pd_run, never its graph replays, nor the autotuner's trials)
 * record HIP events on the context stream around its kernels: the dynamical
 * stage's launches, the interval statistics (k_prefix) and the cloning stage.
 * pd_get_stage_times synchronises and returns the mean durations over the
 * recorded calls; pd_time_stages(ctx, 0) stops recording.  Both return
 * PD_ESTATE between pd_step and pd_resample. */
typedef struct {
    double  step_ms;      /* dynamical-stage kernels of one pd_step */
    double  prefix_ms;    /* interval statistics of one pd_step */
    double  resample_ms;  /* cloning-stage kernels of one pd_resample */
    int64_t steps;        /* recorded pd_step calls */
    int64_t resamples;    /* recorded pd_resample calls */
} pd_stage_times;
pd_status pd_time_stages(pd_ctx* ctx, int32_t enable);
pd_status pd_get_stage_times(pd_ctx* ctx, pd_stage_times* out);

/* Human-readable message of the last error on ctx (or of the last failed
 * pd_create when ctx is NULL). */
const char* pd_last_error(const pd_ctx* ctx);
const char* pd_status_str(pd_status status);

#ifdef __cplusplus
}
#endif

#endif /* PD_H */
