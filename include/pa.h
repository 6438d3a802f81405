/*
 * pa.h - population annealing for the 2D Ising ferromagnet on AMD Instinct
 * MI355X (gfx950): the C-ABI of libpa.
 *
 * The method (Weigel, Barash, Shchur & Janke, arXiv:2102.06611, Sec.
 * "Algorithm", steps 1-5): start R replicas at beta_0 = 0 by simple sampling;
 * for each step beta_{i-1} -> beta_i resample the population with the
 * normalised Boltzmann weights tau_i(E_j) = exp[-(beta_i - beta_{i-1}) E_j] /
 * Q_i (Eq. Q), apply theta checkerboard Metropolis sweeps at beta_i, and
 * measure.  The model is H = -sum_<ij> s_i s_j on a periodic L x L lattice
 * (Eq. hamiltonian, J = 1).
 *
 * Conventions for every call:
 *  - All functions return a pa_status (0 = PA_OK, negative = error) and never
 *    throw across the ABI.  On error, pa_last_error() on the same handle (or
 *    NULL for calls that failed before a handle existed) gives a message.
 *  - Pointers named dev_* are device pointers; all others are host pointers.
 *    Host output buffers are owned by the caller; every "cap" argument bounds
 *    the number of elements written, and the call fails with PA_ERR_ARG
 *    rather than write past it.
 *  - The library allocates no device memory for run state: the caller passes
 *    one device workspace (e.g. a torch uint8 tensor) of at least the size
 *    returned by pa_workspace_size(); it must outlive the handle, and the
 *    library neither frees nor reallocates it.
 *  - Work is enqueued on the caller's HIP stream (NULL = the null stream).
 *    Calls on one handle are serialised on its stream; a handle is not
 *    thread-safe.  Only calls documented as "synchronises" wait for the GPU.
 *  - Device-side failures (capacity overflow, a numerically undecidable
 *    resampling decision, a finished schedule) are sticky: the step that
 *    raised them and all later steps do nothing, the population stays that of
 *    the last good step, and the next synchronising call reports the status.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) keyed by the run's
 * 64-bit seed; the map from (replica, site, step, sweep) to counters is fixed
 * (see pa_philox4x32_10), so results do not depend on launch geometry.
 */
#ifndef PA_H
#define PA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pa_status;
enum {
    PA_OK = 0,
    PA_ERR_ARG = -1,      /* invalid argument or configuration */
    PA_ERR_NOMEM = -2,    /* workspace smaller than pa_workspace_size() */
    PA_ERR_DEVICE = -3,   /* a HIP runtime call failed; the handle is only destroyable */
    PA_ERR_CAPACITY = -4, /* nearest-integer or Poisson resampling produced R_i > capacity */
    PA_ERR_DONE = -5,     /* the fixed schedule has no further temperature */
    PA_ERR_STATE = -6,    /* malformed or mismatching snapshot */
    PA_ERR_NUMERIC = -7,  /* a resampling/acceptance integer could not be decided, or a
                             Poisson mean tau_hat_j exceeds 65536 */
    PA_ERR_EXTINCT = -8   /* resampling gave every parent zero copies (R_i = 0) */
};

/* Copy-count rule of the resampling step (Sec. "Algorithm", step 2). */
enum {
    PA_RESAMPLE_NEAREST = 0,     /* Eq. resampling-factors: floor(tau_hat) or +1 */
    PA_RESAMPLE_MULTINOMIAL = 1, /* R draws with probability tau_i(E_j) / R_{i-1} */
    PA_RESAMPLE_NONE = 2,        /* every replica copied once (diagnostic) */
    PA_RESAMPLE_POISSON = 3      /* r_j ~ Poisson(tau_hat_j) (Eq. taus), by inversion of a
                                    64-bit uniform: the smallest k with U < 2^64 F(k), F the
                                    Poisson CDF; fluctuating R_i */
};

/* Single-spin update of the theta sweeps (Sec. "Spin updates"). */
enum {
    PA_UPDATE_METROPOLIS = 0,    /* flip with probability min(1, e^{-beta dE}) */
    PA_UPDATE_HEATBATH = 1       /* flip with probability 1 / (1 + e^{beta dE}) (Glauber) */
};

/* Device layout of the population (replica r is lane r % 64 of group r / 64). */
enum {
    PA_LAYOUT_INT8 = 0, /* int8 spins, +1 / -1, [group][site][64 lanes] */
    PA_LAYOUT_MSC64 = 1 /* multispin: uint64 [group][site], bit lane = 1 means +1 */
};

typedef struct pa_config {
    int32_t L;             /* lattice side, even, 4 <= L <= 128 */
    int32_t R;             /* nominal population size R = R_0, 1 <= R <= 2^24 */
    const double *betas;   /* betas[0..n_steps], betas[0] = 0, non-decreasing;
                              copied at create; NULL selects caller-driven steps
                              (pa_anneal_step_to) with room for n_steps steps */
    int32_t n_steps;       /* number of temperature steps N_T (>= 0) */
    int32_t theta;         /* Metropolis sweeps per step, >= 0 */
    uint64_t seed;         /* Philox key */
    int32_t resample;      /* PA_RESAMPLE_* */
    int32_t layout;        /* PA_LAYOUT_* */
    int32_t capacity;      /* replica slots; 0 = default: R + ceil(10 sqrt R)
                              rounded up to 64 (nearest, Poisson), 64 ceil(R / 64)
                              otherwise */
    int32_t update;        /* PA_UPDATE_*; 0 (Metropolis) in configurations written
                              before the field existed */
} pa_config;

/* Per-temperature record, Sec. "Model and observables" (with N -> R_i as the
 * paper's footnote directs), Eq. free-emergy-estimator and Sec. "Families". */
typedef struct pa_obs {
    int32_t step;         /* i; record 0 is the beta_0 = 0 population */
    int32_t R_i;          /* population size after resampling */
    double beta;          /* beta_i */
    int64_t sum_E, sum_E2, sum_absM, sum_M2; /* exact population sums */
    double e, c_v, m, chi; /* per-spin energy, specific heat, |magnetisation|, susceptibility */
    double ln_Q;          /* ln Q_i of Eq. Q (0 for i = 0) */
    double minus_beta_F;  /* -beta_i F_i = L^2 ln 2 + sum_{k<=i} ln Q_k */
    int64_t n_families;   /* f: surviving families (descendants of one beta_0 replica) */
    int64_t sum_fam2;     /* sum_k c_k^2 over family sizes c_k */
    int64_t sum_cnt2;     /* sum_j r_j^2 over this step's copy counts */
    double rho_t;         /* Eq. rhot: R_i sum_k (c_k / R_i)^2 */
    double rho_s;         /* Eq. rhos: R_i / exp(S_f), S_f = -sum_k n_k ln n_k */
    double rho_t_step;    /* Eq. one-step-Reff: R_i sum_j (r_j / R_i)^2 */
    /* Blocking over the tree-ordered population (Sec. "Effective population
     * size", Eqs. blocks, blocked_variance, neff; Sec. "Statistical errors",
     * Eqs. jackknife-blocks, jackknife-variance): n = min(100, R_i) blocks of
     * consecutive slots, block k = slots [floor(k R_i / n), floor((k+1) R_i / n)).
     * NaN when n < 2; a zero blocked variance gives R_eff = inf (NaN if the
     * values do not vary). */
    double r_eff_E;       /* sigma^2(E) / sigma^2(mean E), sigma^2 unbiased over the replicas */
    double r_eff_absM;    /* the same for |M| */
    double err_e;         /* blocked standard error of e */
    double err_m;         /* blocked standard error of m */
    double err_c_v;       /* jackknife standard error of c_v */
    double err_chi;       /* jackknife standard error of chi */
    /* Single-run jackknife of the free-energy estimator (Sec. "Conclusions",
     * last guideline: variance and covariances involving the free-energy
     * estimator from a jackknife block analysis of the tree-ordered population;
     * Eqs. free-emergy-estimator, jackknife-variance, bias_covariance).  Sample
     * k of -beta_i F_i leaves block k out of every normalisation Q_l, l <= i:
     * block k of the parents of step l is the slot range [floor(k R_{l-1} / n_F),
     * floor((k + 1) R_{l-1} / n_F)) with n_F = min(100, R) for the whole run (the
     * same index range of the tree-ordered populations, so the same lineages).
     * jk_var_beta_F = (n_F - 1)/n_F sum_k (beta F_k - mean)^2 (0 at step 0);
     * jk_cov_O = (n_F - 1)/n_F sum_k (O_k^J - mean O^J)(beta F_k - mean), O_k^J
     * the jackknife sample of e, m, c_v or chi of the current population without
     * its block k (NaN unless min(100, R_i) = n_F).  NaN when n_F < 2.  After
     * pa_set_population the samples start again from the adopted population. */
    double jk_var_beta_F;
    double jk_cov_e, jk_cov_m, jk_cov_c_v, jk_cov_chi;
} pa_obs;

typedef struct pa_ctx pa_ctx;

/* Device workspace bytes for one run with this configuration. */
pa_status pa_workspace_size(const pa_config *cfg, size_t *bytes);

/* Validate cfg, carve the workspace, draw the beta_0 = 0 population (simple
 * sampling, Sec. "Algorithm" step 1) and enqueue record 0.  stream is a
 * hipStream_t or NULL.  On success *out owns host-side state only. */
pa_status pa_create(const pa_config *cfg, void *dev_workspace, size_t bytes, void *stream,
                    pa_ctx **out);

/* One temperature step beta_{i-1} -> beta_i of the fixed schedule: histogram,
 * Q_i, copy counts, offsets, copy/compaction, theta sweeps, measurement and
 * record i.  Asynchronous. */
pa_status pa_anneal_step(pa_ctx *ctx);

/* As pa_anneal_step, to a caller-chosen beta_next >= beta_{i-1} (adaptive and
 * learned schedules).  Asynchronous. */
pa_status pa_anneal_step_to(pa_ctx *ctx, double beta_next);

/* n_steps consecutive steps of the fixed schedule, replayed from one captured
 * HIP graph.  Asynchronous. */
pa_status pa_run(pa_ctx *ctx, int32_t n_steps);

/* Wait for the stream; report any sticky device-side status. */
pa_status pa_sync(pa_ctx *ctx);

/* Record of step `step` (0..current).  Synchronises. */
pa_status pa_observables(pa_ctx *ctx, int32_t step, pa_obs *out);

/* Current step index i and population size R_i.  Synchronises. */
pa_status pa_current(pa_ctx *ctx, int32_t *step, int32_t *R_i);

/* Energy histogram of the current population (the one the next step
 * reweights): counts[k] = #{j : E_j = -2 L^2 + 4 (k_min + k)}, k < n_bins.
 * Synchronises. */
pa_status pa_energy_histogram(pa_ctx *ctx, int32_t *counts, int32_t cap, int32_t *k_min,
                              int32_t *n_bins);

/* Copy counts r_j of the last resampling, j < R_{i-1}.  Synchronises. */
pa_status pa_copy_counts(pa_ctx *ctx, int32_t *cnt, int64_t cap, int64_t *n);

/* Spins of replicas [first, first + count) of the current population as
 * int8 +1 / -1 in replica-major order out[(r - first) * L^2 + y L + x],
 * together with their family labels (index of the beta_0 replica they
 * descend from) and energies/magnetisations.  Any output pointer may be NULL.
 * Synchronises. */
pa_status pa_get_population(pa_ctx *ctx, int32_t first, int32_t count, int8_t *spins,
                            int32_t *fam, int32_t *E, int32_t *M);

/* Checkpoint: the whole run state (population, families, step, R_i, the
 * running sum of ln Q, records) as an opaque byte string.  With buf = NULL
 * only *used is set.  Synchronises. */
pa_status pa_get_state(pa_ctx *ctx, void *buf, size_t cap, size_t *used);

/* Restore a checkpoint written by pa_get_state for the same configuration. */
pa_status pa_set_state(pa_ctx *ctx, const void *buf, size_t len);

/* Replace the current population by caller data (same layout as
 * pa_get_population) at step `step` with running sum -beta F = minus_beta_F;
 * E and M are recomputed on the device.  Used to resume from a snapshot. */
pa_status pa_set_population(pa_ctx *ctx, int32_t step, int32_t R_i, const int8_t *spins,
                            const int32_t *fam, double minus_beta_F);

/* Histogram overlap alpha(beta_i, beta_i + dbeta) = sum_E min(P(E), P'(E)) of
 * the current population, P' its reweighting to beta_i + dbeta; equal to
 * (1/R_i) sum_j min(1, tau(E_j)).  Used by the adaptive schedule (Sec.
 * "Algorithm", self-adaptive temperature steps).  Synchronises. */
pa_status pa_overlap(pa_ctx *ctx, double dbeta, double *alpha);

/* Largest dbeta in (0, dbeta_max] with alpha(beta_i, beta_i + dbeta) >= alpha
 * _target, by a 17-ary bracket search on the device to within dbeta_max
 * 2^-49 (dbeta_max if that already qualifies).  Synchronises. */
pa_status pa_adaptive_dbeta(pa_ctx *ctx, double alpha_target, double dbeta_max, double *dbeta);

/* Phase timing.  enable = 0 turns it off; otherwise every step records HIP
 * events on the run's stream before the resampling (histogram, Q_i, copy
 * counts, offsets, copy/compaction), before the sweeps, before the
 * measurement/record kernel and after it; with the value 2 set in enable
 * the sweeps run a counting build of the sweep kernel, which also counts the
 * Philox4x32-10 calls its words need and the words it updates (about 3 %
 * slower: time with enable = 1, count with enable = 3; changing the value 2
 * drops a captured step graph).  A nonzero enable resets the totals; any
 * other bit set: PA_ERR_ARG.  Synchronises. */
pa_status pa_profile(pa_ctx *ctx, int32_t enable);

/* Totals since profiling was enabled: steps timed, summed milliseconds of the
 * three phases (resampling, sweeps, measurement), Philox calls and 64-replica
 * words updated by the sweeps, and the part of the resampling phase spent in
 * the copy / compaction kernel (ms_copy).  Any output may be NULL.
 * Synchronises. */
pa_status pa_profile_read(pa_ctx *ctx, int32_t *n_steps, double *ms_resample, double *ms_sweep,
                          double *ms_measure, uint64_t *philox_calls, uint64_t *sweep_words,
                          double *ms_copy);

/* Launch geometry of the sweep kernel for the runs of lattice side L: threads
 * per block (a multiple of 64 in [64, 1024]) and 64-replica groups per block
 * (1..8, with groups_per_block * (L + 2)^2 * 8 bytes <= 152 KiB of LDS: each
 * lattice is held with a one-site halo).  variant: the 64-replica words each
 * thread updates at once, their Philox chains interleaved: 1 or 2, or 0 for
 * the default (1); other values give PA_ERR_ARG.  The results do not depend on the geometry
 * (the random numbers are keyed by replica and site); only speed does.
 * Synchronises. */
pa_status pa_set_sweep_launch(pa_ctx *ctx, int32_t L, int32_t threads, int32_t groups_per_block,
                              int32_t variant);
pa_status pa_get_sweep_launch(pa_ctx *ctx, int32_t L, int32_t *threads, int32_t *groups_per_block,
                              int32_t *variant);

/* Release host-side state; NULL-safe; does not free the workspace. */
void pa_destroy(pa_ctx *ctx);

/* Message of the last failing call on ctx (or of the last failure with no
 * handle when ctx is NULL).  Valid until the next call on that handle. */
const char *pa_last_error(const pa_ctx *ctx);

/* ---- batched independent runs (uneven L and R) ---------------------------
 * n_runs configurations in one engine: every step launches each kernel once
 * for all runs, and pa_batch_run replays a captured HIP graph of that step. */
typedef struct pa_batch pa_batch;
pa_status pa_batch_workspace_size(const pa_config *cfgs, int32_t n_runs, size_t *bytes);
pa_status pa_batch_create(const pa_config *cfgs, int32_t n_runs, void *dev_workspace,
                          size_t bytes, void *stream, pa_batch **out);
pa_status pa_batch_run(pa_batch *b, int32_t n_steps);
pa_status pa_batch_observables(pa_batch *b, int32_t run, int32_t step, pa_obs *out);
/* As pa_get_population, for run `run` of the batch.  Synchronises. */
pa_status pa_batch_get_population(pa_batch *b, int32_t run, int32_t first, int32_t count,
                                  int8_t *spins, int32_t *fam, int32_t *E, int32_t *M);
pa_status pa_batch_sync(pa_batch *b);
pa_status pa_batch_set_sweep_launch(pa_batch *b, int32_t L, int32_t threads,
                                    int32_t groups_per_block, int32_t variant);
pa_status pa_batch_get_sweep_launch(pa_batch *b, int32_t L, int32_t *threads,
                                    int32_t *groups_per_block, int32_t *variant);

/* Overlap correlation of the current population along its index (Sec.
 * "Effective population size", Eq. overlap_correlation): with copies of one
 * parent at adjacent indices, C_q(d) = sum_{i < R_i - d} sum_k s_k^(i)
 * s_k^(i+d) / (N (R_i - d)), the mean overlap of the R_i - d pairs at index
 * distance d, for d = 0 .. d_max (C_q(0) = 1) into dev_cq (device memory,
 * d_max + 1 doubles), asynchronously on the run's stream.  It waits for the
 * queued steps to read R_i; 1 <= d_max <= min(R_i - 1, 65536), PA_ERR_ARG
 * otherwise.  The sums over pairs are exact integers. */
pa_status pa_overlap_correlation(pa_ctx *ctx, int32_t d_max, double *dev_cq);

/* Combination of the batch's independent runs at one temperature (Sec.
 * "Weighted averages", Eqs. weighted-averages and modified-weights2; Sec.
 * "Bias with resampling", Eqs. bias_covariance and rho_f).  Each run m
 * contributes its thermal averages <E>, <E^2>, <|M|>, <M^2> at step i (from
 * its exact population sums) with weight
 *   omega_i^m = R_i^m e^{-beta_i F_i^m} / sum_m' (same)           (weighted-averages)
 * or, for a fluctuating population, with the extra factor
 *   prod_{k=1}^{i} R_{k-1}^m / R^m, R^m the run's nominal size     (modified-weights2);
 * e = <E>/N, m = <|M|>/N, c_v = beta^2 (<E^2> - <E>^2)/N and chi = beta
 * (<M^2> - <|M|>^2)/N are formed from the combined averages.  The plain
 * average uses omega = 1/M.  The spread of the runs: sigma^2(beta F), the
 * sample variance over the runs of beta_i F_i^m; rho_f = R sigma^2(beta F)
 * with R the mean nominal size; cov_*: the sample covariance over the runs of
 * each run's own e, m, c_v, chi with its beta_i F_i^m (the bias estimate). */
typedef struct pa_weighted {
    int32_t step;          /* i */
    int32_t n_runs;        /* M; 0 when the runs do not share beta_i or one stopped (on a
                              device status) before step i: every field NaN */
    double beta;           /* beta_i */
    double e, m, c_v, chi;                          /* Eq. weighted-averages */
    double e_mod, m_mod, c_v_mod, chi_mod;          /* Eq. modified-weights2 */
    double e_plain, m_plain, c_v_plain, chi_plain;  /* omega = 1/M */
    double omega_max;      /* largest omega_i^m of Eq. weighted-averages */
    double n_eff_runs;     /* 1 / sum_m (omega_i^m)^2 */
    double var_beta_F;     /* sigma^2(beta F) over the runs; NaN for M < 2 (so are rho_f, cov_*) */
    double rho_f;          /* Eq. rho_f */
    double cov_e, cov_m, cov_c_v, cov_chi;          /* Eq. bias_covariance */
} pa_weighted;

/* Steps first .. first + count - 1 of all runs of b, one pa_weighted each,
 * into dev_out (device memory, count elements), asynchronously on the
 * batch's stream (after the steps queued before it).  The runs must have one
 * lattice size L and the last step must be queued for every run; PA_ERR_ARG
 * otherwise, or for count < 1 or first < 0. */
pa_status pa_batch_weighted(pa_batch *b, int32_t first, int32_t count, pa_weighted *dev_out);
void pa_batch_destroy(pa_batch *b);
const char *pa_batch_last_error(const pa_batch *b);

/* ---- random numbers -------------------------------------------------------
 * Philox4x32-10 on the device for n counters: out[4 k + m] = word m of the
 * output for counter (ctr[4 k .. 4 k + 3]) under key (key0, key1).  All
 * pointers are device pointers.  Asynchronous. */
pa_status pa_philox4x32_10(uint32_t key0, uint32_t key1, const uint32_t *dev_ctr, int64_t n,
                           uint32_t *dev_out, void *stream);

/* ---- learned temperature steps --------------------------------------------
 * A multilayer perceptron 35 -> 64 -> 64 -> 1 (tanh hidden layers, FP32)
 * proposes the next dbeta from the energy histogram of the population; the
 * histogram-overlap criterion (pa_overlap) is the fallback and decides
 * whether a proposal is taken.
 * Parameters live in one caller-owned device array of PA_MLP_PARAMS floats:
 * W1[64][35], b1[64], W2[64][64], b2[64], w3[64], b3. */
#define PA_MLP_IN 35
#define PA_MLP_HIDDEN 64
#define PA_MLP_PARAMS (64 * 35 + 64 + 64 * 64 + 64 + 64 + 1)

/* Features of the current population into dev_feat[35]: the energy histogram
 * on 32 bins of z = (E - <E>) / sigma_E over [-4, 4) normalised to sum 1,
 * then beta_i, <E> / L^2 and Var(E) / L^2.  Asynchronous. */
pa_status pa_features(pa_ctx *ctx, float *dev_feat);

/* y[k] = MLP(x[k]) for n rows of 35 features.  Asynchronous. */
pa_status pa_mlp_forward(const float *dev_params, const float *dev_x, int32_t n, float *dev_y,
                         void *stream);

/* Gradient of the mean squared error (1/n) sum_k (MLP(x_k) - t_k)^2 with
 * respect to the parameters, into dev_grad[PA_MLP_PARAMS]; the loss into
 * dev_loss[0].  Asynchronous. */
pa_status pa_mlp_backward(const float *dev_params, const float *dev_x, const float *dev_t,
                          int32_t n, float *dev_grad, float *dev_loss, void *stream);

/* One Adam step (beta1 = 0.9, beta2 = 0.999, eps = 1e-8) at iteration t >= 1:
 * gradient as pa_mlp_backward, then update dev_params in place using the
 * moment buffers dev_adam[2 * PA_MLP_PARAMS] (zero before the first step).
 * Asynchronous. */
pa_status pa_mlp_train_step(float *dev_params, float *dev_adam, const float *dev_x,
                            const float *dev_t, int32_t n, float lr, int32_t t, float *dev_loss,
                            void *stream);

/* One step whose temperature is chosen on the device (no host round trip):
 * dbeta* = largest step in (0, beta_final - beta_{i-1}] with histogram overlap
 * alpha(beta_{i-1}, beta_{i-1} + dbeta*) >= alpha_target (the self-adaptive
 * schedule of Sec. "Algorithm"), then the step to beta_i = beta_{i-1} +
 * dbeta*.  When beta_{i-1} has reached beta_final the run reports
 * PA_ERR_DONE.  Asynchronous. */
pa_status pa_anneal_step_adaptive(pa_ctx *ctx, double alpha_target, double beta_final);

/* As pa_anneal_step_adaptive, but the step is the perceptron's proposal
 * (see pa_learned_dbeta) when its overlap is >= alpha_min, and dbeta*
 * otherwise.  Asynchronous. */
pa_status pa_anneal_step_learned(pa_ctx *ctx, const float *dev_params, double alpha_min,
                                 double alpha_target, double beta_final);

/* Per-step log of the device-chosen schedule, for steps 1..n (n = current
 * step): the features of the population that entered step i
 * (dev_feat[35 (i - 1) ..]), the training target log(dbeta*_i sigma_E)
 * (dev_target[i - 1]; NaN on learned steps whose proposal was taken, where
 * dbeta* is not searched for), whether the learned proposal was taken (accepted[i -
 * 1], host) and the overlap of the step actually taken (alpha[i - 1], host).
 * Rows of steps not chosen on the device are zero.  Any output may be NULL;
 * cap bounds the rows written.  Synchronises. */
pa_status pa_schedule_log(pa_ctx *ctx, float *dev_feat, float *dev_target, int32_t *accepted,
                          double *alpha, int32_t cap, int32_t *n);

/* Learned step with the overlap guard, all on the device: features of the
 * current population, y = MLP(features), proposal dbeta = exp(y) / sigma_E
 * clipped to (0, dbeta_max]; accepted (*accepted = 1) iff alpha(beta_i,
 * beta_i + dbeta) >= alpha_min, otherwise replaced by pa_adaptive_dbeta's
 * answer for alpha_target (*accepted = 0); dbeta* is searched for only when
 * the proposal is rejected.  dev_feat (35 floats, may be NULL)
 * receives the features.  Synchronises. */
pa_status pa_learned_dbeta(pa_ctx *ctx, const float *dev_params, double alpha_min,
                           double alpha_target, double dbeta_max, float *dev_feat,
                           double *dbeta, int32_t *accepted);

/* ---- allocation-free variant ---------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * answer as pa_adaptive_dbeta, for a population given as its energies instead
 * of a handle, with no workspace and no allocation.  dev_E[0..n) are the
 * energies E_j = -sum_<ij> s_i s_j of n replicas of an L x L torus (device
 * memory, any order); dev_out[0] receives the largest dbeta in (0, dbeta_max]
 * whose histogram overlap is >= alpha_target and dev_out[1] that overlap
 * (device memory, two doubles; both NaN when an energy is not -2 L^2 + 4k
 * with 0 <= k <= L^2).  Asynchronous on stream, which belongs to the current
 * device, as do dev_E and dev_out.  The energy histogram lives in a
 * library-owned scratch array of 16448 + 64 int32 (66 KiB) per device, kept
 * until the process ends and cleared by every call, so L is limited to 128
 * (PA_ERR_ARG beyond, or for odd L, n < 1, alpha_target outside (0, 1), or
 * dbeta_max not finite and positive).  Calls that overlap in time on one
 * device share that array and race: serialise them (one stream, or events). */
pa_status pa_adaptive_dbeta_noalloc(const int32_t *dev_E, int32_t n, int32_t L,
                                    double alpha_target, double dbeta_max, double *dev_out,
                                    void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PA_H */
