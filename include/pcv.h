/*
 * pcv.h -- C ABI of the MI355X (gfx950) library for parallel brute-force
 * Bayesian cross-validation (PCV).
 *
 * Method: Cooper, Vehtari, Forbes, Simpson, Kennedy, "Bayesian
 * cross-validation by parallel Markov chain Monte Carlo".  Every chain of
 * every fold advances in lock-step with fixed-trajectory HMC (Section 3.3);
 * each fold's log density and log predictive are masked sums over all rows
 * (Appendix B); online accumulators give the LogS estimate, its Monte Carlo
 * error, ESS and Rhat without storing draws (Algorithm A2, Appendix A).
 *
 * Conventions used by every entry point
 *  - C = K * L chains; chain c belongs to fold k = c / L (its L chains are
 *    adjacent).  Random streams are keyed by the global chain id
 *    chain_offset + c, so a run over a subset of folds reproduces exactly the
 *    same chains as the full run.
 *  - d = p for the GLM families, p + 2 + n_groups for the hierarchical
 *    logistic family (theta = [beta(p), mu, log tau, z(n_groups)]) and
 *    p + 3 + n_groups for the hierarchical Gaussian family (theta = [beta(p),
 *    mu, log sigma_a, log sigma_y, z(n_groups)], alpha_g = mu + sigma_a z_g).
 *  - Host arrays passed to pcv_init are copied; the caller may free them on
 *    return.  Device pointers passed to the test hooks are borrowed for the
 *    duration of the call and must be device memory of the current HIP device.
 *  - All work is queued on the context's stream (pcv_set_stream); calls that
 *    return host data synchronise that stream.
 *  - Thread safety: a context must not be used from two threads at once.
 *    Different contexts are independent.
 *  - On error a call returns a non-zero pcv_status and leaves a message in
 *    pcv_last_error(ctx).  After PCV_ERR_DEVICE the context only accepts
 *    pcv_destroy.
 */
#ifndef PCV_H
#define PCV_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum pcv_status {
  PCV_OK = 0,
  PCV_ERR_INVALID_ARG = 1,   /* bad sizes, non-finite data, invalid y, empty fold ... */
  PCV_ERR_NOMEM = 2,         /* device or host allocation failed */
  PCV_ERR_DEVICE = 3,        /* a HIP call or kernel launch failed */
  PCV_ERR_STATE = 4,         /* not enough draws yet, or context unusable */
  PCV_ERR_UNSUPPORTED = 5    /* combination of family / precision / size not built */
} pcv_status;

/* Likelihood families (Appendix B masks them per fold). */
enum {
  PCV_FAMILY_GAUSSIAN = 0,        /* y ~ N(x'theta, sigma^2), sigma known      */
  PCV_FAMILY_LOGISTIC = 1,        /* y in {0,1}, logit link                   */
  PCV_FAMILY_POISSON = 2,         /* y in {0,1,2,...}, log link               */
  PCV_FAMILY_HIER_LOGISTIC = 3,   /* logit(P(y=1)) = x'beta + mu + tau z_g(n) */
  PCV_FAMILY_HIER_GAUSSIAN = 4    /* y ~ N(x'beta + mu + sigma_a z_g(n), sigma_y^2),
                                     sigma_y unknown: the grouped regression of
                                     Section 2, Example 1 (fp64 / fp32 paths)     */
};

/* Arithmetic of the log-density / gradient contractions.  Metropolis
 * energies, log predictive draws and all accumulators are fp64 always. */
enum {
  PCV_PREC_FP64 = 0,          /* fp64 VALU kernels (p <= 64)                        */
  PCV_PREC_FP32 = 1,          /* fp32 VALU kernels (p <= 64)                        */
  PCV_PREC_BF16X3 = 2,        /* bf16 MFMA, X and theta split hi+lo, 3 products each
                                 way, fp32 accumulation (p <= 128; the kernels run
                                 at width 64 or 128 with zero columns past p)       */
  PCV_PREC_BF16X5 = 3,        /* as BF16X3 with a three-term theta split in the
                                 forward product (5 products), fp32-exact eta        */
  PCV_PREC_FP64_UNFUSED = 4   /* plain fp64 path: library DGEMMs with eta and the
                                 residual materialised in memory (baseline)          */
};

/* Fold encodings.  Roles of a row in a fold: excluded, train or test. */
enum {
  PCV_FOLDS_INDEX = 0,      /* fold_index[n]: test in fold fold_index[n], train in
                               every other fold; -1 = train in every fold           */
  PCV_FOLDS_INTERVALS = 1,  /* intervals[K][4] = (test_lo, test_hi, excl_lo, excl_hi):
                               [test_lo,test_hi) test, rest of [excl_lo,excl_hi)
                               excluded, every other row train (hv-block, blocked);
                               when both ranges are non-empty they must overlap
                               or touch (one non-train range per fold), else
                               PCV_ERR_INVALID_ARG                                  */
  PCV_FOLDS_DENSE = 2       /* roles[K][n]: 0 excluded, 1 train, 2 test            */
};

typedef struct pcv_folds {
  int32_t kind;
  const int32_t* fold_index;   /* INDEX: n entries in [-1, K)                       */
  const int64_t* intervals;    /* INTERVALS: K*4 entries, 0 <= lo <= hi <= n, excl ⊇ test */
  const int8_t* roles;         /* DENSE: K*n entries in {0,1,2}                     */
} pcv_folds;

/* Encoding of X passed to pcv_init. */
enum {
  PCV_X_FP64 = 0,        /* n*p fp64, row-major.  The bf16 precisions round each
                            entry to fp32 and store it as the bf16 pair hi + lo,
                            which keeps about 16 significant bits (relative error
                            <= 2^-16); exact for designs given as two planes      */
  PCV_X_BF16_HILO = 1    /* two bf16 planes (uint16 bit patterns), hi then lo, each
                            n*p row-major; the design is hi + lo, summed exactly in
                            fp64 (a stored split such as the synthetic c4/c5 designs) */
};

/* Extra scoring rules accumulated online (bit mask; Appendix, HS and DSS). */
enum {
  PCV_SCORE_HS = 1,    /* Hyvarinen score (continuous responses: Gaussian family)    */
  PCV_SCORE_DSS = 2    /* Dawid-Sebastiani score, from one predictive draw per chain,
                          transition and test row                                      */
};

/* How Rhat is accumulated (Section 4.2). */
enum {
  PCV_RHAT_WELFORD = 0,       /* per-block Welford mean and M2, Chan-merged           */
  PCV_RHAT_SHIFTED_SUMS = 1   /* per-block sums of s - C_k and (s - C_k)^2, with C_k
                                 the fold's warm-up mean of s (Algorithm A2)          */
};

typedef struct pcv_model {
  int32_t family;              /* PCV_FAMILY_*                                      */
  int32_t precision;           /* PCV_PREC_*                                        */
  int64_t n, p;                /* X is n x p, row-major (encoding: x_format)        */
  int32_t K, L;                /* folds, chains per fold (L >= 2)                   */
  int32_t n_groups;            /* HIER_LOGISTIC: number of groups                   */
  const int32_t* group_of;     /* HIER_LOGISTIC: n entries in [0, n_groups), sorted */
  double sigma;                /* GAUSSIAN: known noise sd                          */
  const double* prior_scale;   /* d entries: theta_j ~ N(0, prior_scale_j^2) (GLMs);
                                  NULL = all 1.  HIER_LOGISTIC: beta, mu, z ~ N(0,1),
                                  tau ~ HalfNormal(1); HIER_GAUSSIAN: beta, mu, z ~
                                  N(0,1), sigma_a and sigma_y half-normal with
                                  variance 10 (Example 1); the array is ignored     */
  double step_size;            /* leapfrog step eps (> 0)                            */
  int32_t n_leapfrog;          /* leapfrog steps per transition S (>= 1)             */
  const double* inv_mass;      /* d entries (> 0): diagonal inverse mass matrix      */
  const double* init_pos;      /* C*d, chain-major: theta of chain c at [c*d + j]   */
  int64_t n_warmup;            /* transitions (cumulative over pcv_step) not accumulated */
  int32_t batch_size;          /* b: draws per batch mean (>= 1)                     */
  int32_t batches_per_block;   /* G: batches per shuffle block (>= 1)                */
  int32_t n_blocks;            /* D: shuffle blocks (1..64); draws past D*G*b go
                                  to the last block                                  */
  uint64_t seed;               /* Philox4x32-10 key                                  */
  int64_t chain_offset;        /* global id of chain 0 (0 for a full run)            */
  int32_t x_format;            /* PCV_X_*: encoding of the X argument of pcv_init   */
  int32_t rhat_mode;           /* PCV_RHAT_*                                         */
  int32_t scores;              /* PCV_SCORE_* mask (0 = LogS only)                   */
  int64_t store_draws;         /* keep the first store_draws post-warm-up draws of s
                                  of every chain on the device (Algorithm 1); 0 = none */
  /* Several nested models in one launch (Appendix B, parallel model
   * evaluation): model m uses covariate j iff model_mask[m*p + j] = 1; a
   * masked beta_j stays a parameter that the likelihood and the predictive
   * ignore (x_nj beta_j enters as 0) and only its prior informs.  The run
   * then holds M*K posteriors, model-major: chain c = (m*K + k)*L + l is chain
   * l of fold k under model m, so C = M*K*L and init_pos has M*K*L rows; the
   * per-fold arrays of the diagnostics have M*K entries in the same order.
   * Not with scores or the plain fp64 path; the hierarchical families (masks
   * on beta) on the fp64 and fp32 paths. */
  int32_t n_models;            /* M (0 or 1: one model, model_mask ignored)          */
  const uint8_t* model_mask;   /* M*p entries, 0 or 1                               */
} pcv_model;

typedef struct pcv_diag {
  double rhat_max;        /* max over folds of Rhat (eq rhat-max); NaN if < 2 draws  */
  double ess;             /* aggregate ESS of the elpd (Section 4.1); NaN if < 2 batches */
  double elpd;            /* sum over folds of the LogS estimate                   */
  double mcse;            /* Monte Carlo s.e. of elpd (eq mc-var)                  */
  double accept_rate;     /* post-warm-up acceptance rate                          */
  int64_t n_divergent;    /* post-warm-up divergent transitions                    */
  int64_t n_draws;        /* post-warm-up draws per chain                          */
  int64_t n_iter;         /* transitions run so far (warm-up included)             */
  double* rhat_fold;      /* optional, K entries (M*K with several models), caller-owned */
  double* ess_fold;       /* optional, K entries (M*K with several models), caller-owned */
} pcv_diag;

/* Comparison of two models on the same folds (Sections 2.3 and 4.1). */
typedef struct pcv_comparison {
  double delta;           /* Delta = sum_k Delta_k, Delta_k = S_A,k - S_B,k (eq sel-cv) */
  double sigma2;          /* sample variance of the Delta_k, 1/(K-1) sum (Delta_k - Delta/K)^2 */
  double prob_a_better;   /* Pr(M_A better than M_B | y) ~ Phi(Delta / sqrt(K sigma2))
                             (eq norm-approx); 1/2 when Delta = sigma2 = 0            */
  double mcse;            /* Monte Carlo s.e. of Delta: both models' fold variances
                             add (eq mc-var)                                          */
  double* delta_fold;     /* optional, K entries, caller-owned                        */
} pcv_comparison;

/* Diagnostics from stored draws (Algorithm 1), computed after the run. */
typedef struct pcv_posthoc_diag {
  double elpd, mcse, ess;   /* two-pass LogS estimate, its MC s.e. and ESS (Sec. 4.1)  */
  double rhat_max;          /* max over folds of the paper's Rhat (eq rhat)            */
  double split_rhat_max;    /* ... of split Rhat (chain halves as chains)              */
  double rank_rhat_max;     /* ... of rank-normalised split Rhat, bulk and folded
                               (Vehtari et al., 2021)                                   */
  int64_t n_draws;          /* stored draws per chain used                              */
  double* rhat_fold;        /* optional, K entries each, caller-owned                   */
  double* split_rhat_fold;
  double* rank_rhat_fold;
} pcv_posthoc_diag;

typedef struct pcv_ctx_s* pcv_ctx;

/* Validate the model and data, copy them to the device, and evaluate log pi,
 * its gradient and the log predictive at the initial positions (Section 3,
 * Steps 2-3: every fold starts from draws of the full-data fit and reuses its
 * step size and mass matrix, Section 3.1).
 * X: as model->x_format says (n*p row-major fp64, or two bf16 planes); y: n
 * fp64.  Errors: PCV_ERR_INVALID_ARG (n, p, K <= 0;
 * L < 2; non-finite X, y or init_pos; y outside the family's support; a fold
 * with no training row; a fold with no test row when K > 1 (K = 1 without
 * test rows is the full-data model, s = 0, which pcv_adapt tunes);
 * step_size, inv_mass, sigma <= 0;
 * n_leapfrog < 1; batch settings < 1), PCV_ERR_UNSUPPORTED, PCV_ERR_NOMEM,
 * PCV_ERR_DEVICE.  *out is NULL on error. */
pcv_status pcv_init(pcv_ctx* out, const pcv_model* model, const void* X, const double* y,
                    const pcv_folds* fold_masks);

/* Queue all further work of ctx on hip_stream (a hipStream_t; NULL = the
 * default stream).  The stream must outlive its use by ctx. */
pcv_status pcv_set_stream(pcv_ctx ctx, void* hip_stream);

/* Advance every chain n_iter HMC transitions (n_iter >= 0): the sampling
 * loop of Algorithm A2 (Appendix A) over all folds at once, each transition
 * one fixed-trajectory HMC step of every chain in lock-step (Section 3.3):
 * momentum refresh, n_leapfrog leapfrog steps of masked value-and-gradient
 * evaluations (Appendix B), Metropolis accept, and for post-warm-up
 * transitions the log predictive of the fold's test set and the online
 * accumulators (streaming log-sum-exp, batch means, per-block R-hat
 * statistics).  The first model->n_warmup transitions overall are warm-up
 * and are not accumulated.  Asynchronous on the context stream.  Divergent
 * transitions are counted, not errors.  Errors: PCV_ERR_INVALID_ARG for
 * n_iter < 0 or a transition count beyond 32 bits; PCV_ERR_STATE for a dead
 * context; PCV_ERR_DEVICE if a launch fails. */
pcv_status pcv_step(pcv_ctx ctx, int64_t n_iter);

/* Convergence diagnostics of the LogS estimate (Section 4) from the online
 * accumulators.  Synchronises.  Returns PCV_ERR_STATE if fewer than 2
 * post-warm-up draws exist; values that need complete batches are NaN until
 * 2 batches are complete. */
pcv_status pcv_diagnostics(pcv_ctx ctx, pcv_diag* out);

/* LogS cross-validation estimate (eq cv-score) and its Monte Carlo standard
 * error (eq mc-var), in total and per fold (K entries each, optional).
 * With several models the totals run over all M*K posteriors and the
 * per-fold arrays have M*K entries; pcv_elpd_model gives one model's.
 * Synchronises.  PCV_ERR_STATE if there is no post-warm-up draw. */
pcv_status pcv_elpd(pcv_ctx ctx, double* elpd, double* mcse, double* elpd_fold, double* mcse_fold);

/* The same for model `model` of a multi-model run (0 <= model < M; model 0
 * of a one-model run): elpd and mcse over its K folds, per-fold arrays of K
 * entries (optional).  Errors: PCV_ERR_INVALID_ARG for a model out of
 * range; PCV_ERR_STATE without post-warm-up draws. */
pcv_status pcv_elpd_model(pcv_ctx ctx, int32_t model, double* elpd, double* mcse, double* elpd_fold,
                          double* mcse_fold);

/* Block-shuffle benchmark of Rhat_max (Section 4.2, Fig. 4; last loop of
 * Algorithm A2): R replicates, each rebuilding every chain from D blocks
 * drawn with replacement from the fold's chains (Philox stream of `seed`).
 * rhat_max_rep: R entries (caller-owned).  rhat_rep: K*R entries or NULL.
 * Synchronises.  PCV_ERR_STATE before 2 draws, PCV_ERR_INVALID_ARG if R < 1. */
pcv_status pcv_shuffle_benchmark(pcv_ctx ctx, int32_t R, uint64_t seed, double* rhat_max_rep,
                                 double* rhat_rep);

/* Size, in doubles, of the static device scratch array that
 * pcv_shuffle_benchmark_noalloc uses (8 MiB).  Each GPU the library runs on
 * holds one copy from the first pcv_init on that device until the process
 * ends. */
#define PCV_SHUFFLE_NOALLOC_MAX_DOUBLES (1 << 20)

/* pcv_shuffle_benchmark for callers that cannot allocate device memory:
 * monitoring loops that re-run the benchmark at every batch end, serving
 * loops and harnesses that forbid hipMalloc.  Same arguments, same kernels
 * and bit-identical results; the replicate buffers (M*K*R + R doubles, M*K
 * the run's posteriors) live in the library's static scratch array of this
 * GPU instead of fresh allocations, and the call makes no hipMalloc, hipFree
 * or other allocating call.  The kernels overwrite the buffers in full, so
 * nothing carries over from earlier calls; but every context on one GPU
 * shares that GPU's array, so calls that overlap on one GPU (other streams
 * or threads) race: the caller must serialise them.  Synchronises.
 * Errors: those of pcv_shuffle_benchmark, plus PCV_ERR_INVALID_ARG, before
 * any device work, when (M*K + 1) * R exceeds
 * PCV_SHUFFLE_NOALLOC_MAX_DOUBLES. */
pcv_status pcv_shuffle_benchmark_noalloc(pcv_ctx ctx, int32_t R, uint64_t seed, double* rhat_max_rep,
                                         double* rhat_rep);

/* Hyvarinen (HS) and Dawid-Sebastiani (DSS) cross-validation scores
 * (Appendix, sections HS and DSS; positively oriented), summed over folds
 * and per fold (K entries each; any output may be NULL).  Per fold k with
 * test rows V_k, from the post-warm-up draws of its L chains:
 * - HS_k = sum_i (-2 mu1_i + mu2_i^2), mu1_i the average of
 *   d2 log p/dy_i^2 + (d log p/dy_i)^2 and mu2_i that of d log p/dy_i;
 * - DSS_k = -log|Sigma| - (y - mu)' Sigma^-1 (y - mu), mu and Sigma the mean
 *   and covariance of the predictive draws of y_{V_k}.
 * DSS_k is NaN if Sigma is not positive definite.  The scores must be
 * enabled in pcv_model.scores.  Synchronises.
 * Errors: PCV_ERR_INVALID_ARG if a requested score is not enabled;
 * PCV_ERR_STATE before 2 post-warm-up draws. */
pcv_status pcv_scores(pcv_ctx ctx, double* hs, double* hs_fold, double* dss, double* dss_fold);

/* Stored draws (Algorithm 1; pcv_model.store_draws > 0).  pcv_get_draws
 * copies the first min(stored, n_max) post-warm-up draws of s of every chain
 * to s (C rows of n_out entries, chain-major; caller-owned).  pcv_posthoc
 * computes from them, after the run, the two-pass estimates and three Rhats
 * per fold (optional per-fold arrays of K entries).  Both synchronise.
 * Errors: PCV_ERR_INVALID_ARG if draws are not stored or a buffer is bad;
 * PCV_ERR_STATE with fewer than 4 stored draws (pcv_posthoc). */
pcv_status pcv_get_draws(pcv_ctx ctx, double* s, int64_t n_max, int64_t* n_out);
pcv_status pcv_posthoc(pcv_ctx ctx, pcv_posthoc_diag* out);

/* Pairwise model comparison from two runs on the same folds (same fold
 * encoding and arrays, checked by fingerprint): context a holds model A,
 * context b model B, for instance nested designs that differ by a covariate
 * (Section 2.3).  Both need post-warm-up draws and one model each
 * (pcv_compare_models compares the models of one run).  Synchronises both
 * streams.
 * Errors: PCV_ERR_INVALID_ARG for a null output or different fold sets
 * (message on a); PCV_ERR_STATE when either run has no draw yet. */
pcv_status pcv_compare(pcv_ctx a, pcv_ctx b, pcv_comparison* out);

/* The same comparison between models a and b of one multi-model run (both
 * models in one launch, Appendix B): their posteriors share the folds by
 * construction.  Errors: PCV_ERR_INVALID_ARG for models out of range or a
 * null output; PCV_ERR_STATE without post-warm-up draws. */
pcv_status pcv_compare_models(pcv_ctx ctx, int32_t a, int32_t b, pcv_comparison* out);

/* Full-data tuning by window adaptation (Section 3.1, efficient warm-up;
 * workflow Step 1).  Meant for a context on the full data: one fold whose
 * rows all train (PCV_FOLDS_INDEX, K = 1, every fold_index -1), L chains,
 * and n_warmup >= n_adapt so no adaptation draw is accumulated.  Runs
 * n_adapt transitions of ctx, eagerly:
 *   step size  - after every transition, dual averaging (Hoffman and Gelman,
 *                2014; gamma 0.05, t0 10, kappa 0.75) of the chains' mean
 *                acceptance statistic min(1, e^(H0 - H1)) toward
 *                target_accept in (0, 1);
 *   inverse mass (diagonal) - at the end of each slow window, the
 *                regularised variance n/(n+5) var + 1e-3 * 5/(n+5) of the
 *                positions of all chains over the window (n = chains x
 *                transitions), after which the dual averaging restarts.
 * Windows (Stan's published schedule): a fast buffer of 75 transitions,
 * slow windows of 25, 50, 100, ... (the last stretched to the final buffer),
 * a final fast buffer of 50; 15% / rest / 10% of n_adapt when those do not
 * fit.  On return the context runs with the adapted values (step size =
 * exp of the averaged log step size) and its chains sit at the adapted
 * positions; step_size (1 entry) and inv_mass (d entries) receive them when
 * not NULL (caller-owned).  Synchronises every transition.
 * Errors: PCV_ERR_INVALID_ARG for n_adapt < 1 or target_accept outside
 * (0, 1); PCV_ERR_DEVICE on a failed copy (the context is then at an
 * intermediate step size). */
pcv_status pcv_adapt(pcv_ctx ctx, int64_t n_adapt, double target_accept, double* step_size, double* inv_mass);

/* Starting positions drawn from full-data draws (workflow Step 2): chain c
 * (global id chain_offset + c) starts at draw floor(u n_draws) of
 * draws[n_draws][d] (row-major, host), u from Philox4x32-10 with key seed
 * and counter (chain_offset + c, 0, 5, 0), first two words.  init_pos:
 * C*d host doubles, chain-major (the layout of pcv_model.init_pos;
 * caller-owned).  Pure host code: no context, no device.
 * Errors: PCV_ERR_INVALID_ARG for null pointers, n_draws, d or C < 1, or
 * chain ids beyond 32 bits. */
pcv_status pcv_init_positions(const double* draws, int64_t n_draws, int64_t d, int64_t C, uint64_t seed,
                              int64_t chain_offset, double* init_pos);

void pcv_destroy(pcv_ctx ctx);
const char* pcv_last_error(pcv_ctx ctx);
const char* pcv_status_str(pcv_status s);

/* ---- lower-level calls (gradient checks, parity tests, state transfer) ---- */

/* Masked log density log pi (Appendix B) and, if want_grad, its gradient
 * (the hand-written adjoint), for caller-given positions.  theta_dev: C*d
 * chain-major fp64 device array; logp_dev: C fp64; grad_dev: C*d fp64 or NULL
 * when want_grad = 0.  Uses the context's precision.  Does not change the
 * chain state. */
pcv_status pcv_logdensity_grad(pcv_ctx ctx, const double* theta_dev, double* logp_dev,
                               double* grad_dev, int32_t want_grad);

/* n_steps leapfrog steps (step size of the model) from (q, p) for every
 * chain, as inside one HMC transition.  All arrays are C*d (logp: C) fp64
 * device arrays, chain-major.  Does not change the chain state. */
pcv_status pcv_leapfrog(pcv_ctx ctx, const double* q_dev, const double* p_dev, int32_t n_steps,
                        double* q_out_dev, double* p_out_dev, double* logp_out_dev,
                        double* grad_out_dev);

/* Copy the current chain state to host buffers (any may be NULL):
 * theta C*d chain-major, logp C, log predictive s C. Synchronises. */
pcv_status pcv_get_state(pcv_ctx ctx, double* theta, double* logp, double* s);

/* Replace the chain positions (C*d chain-major host array) and recompute
 * log pi, its gradient and s there.  Accumulators are kept. */
pcv_status pcv_set_state(pcv_ctx ctx, const double* theta);

/* Raw online accumulators (Algorithm A2) to host buffers, any may be NULL:
 * Z, U, U2, V, V2: C each (log scale); blk_mean, blk_m2: D*C each
 * (block-major: [dd*C + c]) holding the Welford mean and M2 of s per block,
 * or with rhat_mode PCV_RHAT_SHIFTED_SUMS the sums of s - C_k and
 * (s - C_k)^2; n_accept, n_divergent: C each. */
pcv_status pcv_get_accumulators(pcv_ctx ctx, double* Z, double* U, double* U2, double* V,
                                double* V2, double* blk_mean, double* blk_m2,
                                int64_t* n_accept, int64_t* n_divergent);

/* Autotuner for the hot kernel's launch shape.  It times candidate shapes of
 * the gradient kernel:
 * - matrix-core path: the kernel shape (16x16x32 or 32x32x16 bf16 MFMA
 *   tiles, and at design widths up to 64 a 16x16x32 kernel with 16 chains
 *   per wave whose registers fit two workgroups per CU) and the number of
 *   row splits per chain tile, around the analytic choice made at init;
 * - row-split VALU path: waves per workgroup (2, 4 or 8) and row splits
 *   around the analytic choice, scaled to keep the rows per wave;
 * - fused VALU path: waves per workgroup, each owning a range of rows.
 * Timing runs on a scratch copy of the current positions, so the chains are
 * untouched.  The fastest shape is kept, and the captured transition graph is
 * rebuilt on the next pcv_step.
 * cache_path (or NULL) names a JSON file of tuned shapes, keyed by path,
 * family, precision, fold encoding, sizes and GPU architecture.  A hit is
 * applied without timing; a miss is timed and written back (created,
 * updated or extended).
 * config receives the shape as one integer (matrix-core path:
 * 256 * shape + splits, shape 0 = 16x16x32 MFMAs with 32 chains per wave
 * (256 per workgroup), 1 = 32x32x16 MFMAs in program order, 2 = the same
 * scheduled freely by the compiler, 3 = 16x16x32 MFMAs with 16 chains per
 * wave (128 per workgroup; p <= 64 only); row-split VALU path: 1024 *
 * waves + splits, waves 1, 2, 4 or 8 (a bare split count below 1024 keeps
 * the context's waves); fused VALU path: waves); ms receives its mean kernel
 * time (both optional).
 * Synchronises.
 * Errors: PCV_ERR_UNSUPPORTED on the plain fp64 path; PCV_ERR_INVALID_ARG if
 * the cache cannot be written; PCV_ERR_DEVICE. */
pcv_status pcv_autotune(pcv_ctx ctx, const char* cache_path, int32_t* config, double* ms);

/* Apply, or read, a launch shape in pcv_autotune's encoding (for instance
 * one tuned elsewhere): the captured transition graph is rebuilt on the next
 * pcv_step.  Results depend on the shape only through the order of floating
 * point sums.  Errors: PCV_ERR_INVALID_ARG for a shape out of range for this
 * context (the context is unchanged); PCV_ERR_UNSUPPORTED on the plain fp64
 * path. */
pcv_status pcv_set_launch_config(pcv_ctx ctx, int32_t config);
pcv_status pcv_get_launch_config(pcv_ctx ctx, int32_t* config);

/* Checkpoint and resume.  pcv_save writes everything a run carries between
 * transitions to the file `path`:
 * - the accepted positions, gradients, log pi and log predictive of every chain;
 * - every online accumulator (Algorithm A2) and the accept/divergence counters;
 * - the step size and diagonal inverse mass in force (pcv_adapt changes both);
 * - the transition count.
 * The write goes to `path`.tmp first and is renamed into place.
 * pcv_load restores such a file into a context made by pcv_init with the
 * same model, data, folds and precision (checked against a fingerprint of
 * X, y, the folds, the Gaussian noise scale and the prior scales); the
 * context takes the checkpoint's step size and inverse mass, whatever it
 * was created with.  Because every random number is keyed by (seed, chain,
 * transition), the resumed run continues exactly as the original would
 * have.  Errors: PCV_ERR_INVALID_ARG for an unwritable or unreadable path,
 * a file of another run or target, or a truncated or corrupted file (the
 * ctx is unchanged then); PCV_ERR_DEVICE.  Both synchronise. */
pcv_status pcv_save(pcv_ctx ctx, const char* path);
pcv_status pcv_load(pcv_ctx ctx, const char* path);

/* Philox4x32-10 of this library for n counters (c0, c1, c2, c3 + i) with key
 * (seed): out receives 4*n uint32 words.  Host-side buffers; runs on the
 * device.  Used to check the stream bit-for-bit against other implementations. */
pcv_status pcv_philox(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                      int64_t n, uint32_t* out);

/* Per-launch timing of the gradient kernel (the S-fold hot kernel of every
 * transition).  When enabled, every launch of it queued by pcv_step is
 * bracketed by HIP events on the context stream.  pcv_timing_read
 * synchronises, returns the summed device milliseconds and the number of
 * launches since the last reset, and the kernel's name (static string), and
 * resets the counters if reset != 0. */
pcv_status pcv_timing_enable(pcv_ctx ctx, int32_t on);
pcv_status pcv_timing_read(pcv_ctx ctx, double* ms_sum, int64_t* n_launches,
                           const char** kernel_name, int32_t reset);

/* Roofline calibration of the bf16 matrix cores (measurement support, no
 * part of the method).  Times a kernel that keeps every SIMD's matrix core
 * busy with v_mfma_f32_32x32x16_bf16 products, two waves per SIMD, operands
 * read from LDS: data_kind 0 multiplies constant operands (every element
 * 1.0), data_kind 1 seeded random bf16 operands (random sign and mantissa,
 * magnitudes in [2^-8, 1)), like the split hi and lo planes the gradient
 * kernel multiplies.  The part lowers its clock to hold its power limit, and
 * the power of a product grows with the switching activity of its operands,
 * so the two sustained rates bracket what a bf16 MFMA kernel reaches on this
 * device.  tflops receives the dense rate (2*32*32*16 flops per product) over
 * `launches` timed launches after one untimed one, on the null stream of the
 * current device.  Allocates and frees a small buffer; synchronises.
 * Errors: PCV_ERR_INVALID_ARG (data_kind not 0 or 1, launches < 1, tflops
 * NULL), PCV_ERR_NOMEM, PCV_ERR_DEVICE. */
pcv_status pcv_calib_mfma(int32_t data_kind, int32_t launches, double* tflops);

#ifdef __cplusplus
}
#endif

#endif /* PCV_H */
