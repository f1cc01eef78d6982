/*
 * nss.h -- C ABI of the MI355X (gfx950) Nested Slice Sampling library (libnss.so).
 *
 * The library runs the data-parallel hot path of Nested Slice Sampling (NSS, arXiv 2601.23252)
 * on one GPU: batched delete-k nested sampling whose k replacements are produced in parallel by
 * Hit-and-Run Slice Sampling (HRSS) chains under the hard constraint logL(x) > L*, with batched
 * likelihood evaluation inside each chain step and log-sum-exp evidence accumulation.
 *
 * Problem statement (Sec. 1, eq. target / integral_Z): a prior (reference density) Pi and an
 * energy E = -log L; the evidence is Z = integral of L(x) Pi(x) dx.  Run shape (Sec. 3.1,
 * Alg. "Nested Sampling outer kernel"; Sec. 3.2): n_live = m live points, k deletions per
 * iteration (1 <= k <= m-1), chain length p HRSS steps per replacement.
 *
 * Conventions for every call:
 *  - Ownership: all array arguments are HOST pointers.  ns_init copies everything it needs; the
 *    caller may free its arrays on return.  The context owns all device memory until ns_free.
 *  - Layout: points are row-major host arrays, x[i*d + j] = coordinate j of point i.
 *    Matrices are row-major, cov[(c*d + r)*d + s] = entry (r, s) of component c.
 *  - Streams: work is enqueued on the hipStream_t passed to ns_init (NULL = the library's own
 *    stream).  Calls returning host values (ns_step's done flag, ns_run, ns_logz, ns_stats,
 *    state access) synchronise that stream.
 *  - Errors: a call returns an ns_status; nothing throws across the ABI.  On failure,
 *    ns_last_error(ctx) describes it (ns_init failures: ns_last_error(NULL)).  A failed call
 *    leaves the context usable unless it returned NS_EDEVICE.
 *  - Threading: calls on one context are not thread-safe; separate contexts are independent.
 *  - Numerics: a NaN or +inf log-likelihood is treated as -inf (the candidate is rejected) and
 *    counted in ns_stats_t.nonfinite.
 */
#ifndef NSS_H
#define NSS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ns_ctx ns_ctx;

typedef enum {
    NS_OK = 0,
    NS_DONE = 1,            /* ns_step: the run had already terminated; nothing was done */
    NS_EINVAL = -1,         /* invalid argument */
    NS_ENOMEM = -2,         /* device or host allocation failed */
    NS_EDEVICE = -3,        /* a HIP call failed; the context should be freed */
    NS_ESTATE = -4,         /* no survivor lies strictly above L* (likelihood plateau) */
    NS_EUNSUPPORTED = -5    /* valid but outside what this library supports (sizes, kinds) */
} ns_status;

/* Prior Pi, one factor per coordinate (Sec. 1, the reference density). */
typedef enum {
    NS_PRIOR_BOX = 0,        /* uniform on [a_j, b_j] */
    NS_PRIOR_GAUSS_DIAG = 1  /* normal with mean a_j and standard deviation b_j > 0 */
} ns_prior_kind;

/* Likelihood families L = exp(-E). */
typedef enum {
    /* log L(x) = log sum_c exp(logw_c) N(x; mean_c, cov_c): normalised Gaussian mixture,
     * n_comp >= 1 components (n_comp = 1: a single, possibly correlated, Gaussian). */
    NS_LIK_MIXTURE = 1,
    /* Neal's funnel: v = x_0 ~ N(0, 9), x_j | v ~ N(0, e^v) for j = 1..d-1, normalised. */
    NS_LIK_FUNNEL = 2,
    /* GP hyperparameter marginalisation (Sec. 5 GP experiments; App. "Gaussian Process
     * Hyperparameter Marginalization"): d = 6 coordinates u = log theta,
     * theta = (sigma_f, l_1, l_2, l_p, P, sigma_n); log L(u) = log N(y; 0, K + sigma_n^2 I)
     * over n_obs observations (x_obs[i] in R^2, y_obs[i]) with the product kernel
     * K_ab = sigma_f^2 exp(-1/2 sum_j (a_j - b_j)^2 / l_j^2 - 2 sum_j sin^2(pi (a_j - b_j)/P)
     * / l_p^2), j = 1, 2.  A Cholesky factorisation that breaks down gives log L = -inf. */
    NS_LIK_GP = 3,
    /* Gaussian-Rastrigin test likelihood (the evidence comparison of constrained samplers):
     * L = alpha exp(-|x|^2 / 2) + (1 - alpha) exp(-A d + A sum_i cos(2 pi x_i)), alpha in
     * [0, 1], A = amp >= 0 (the paper: A = 10, uniform prior on [-5.14, 5.14]^d).  FP64. */
    NS_LIK_GAUSS_RASTRIGIN = 4
} ns_lik_kind;

/* Arithmetic of the likelihood evaluations inside the chains. */
typedef enum {
    NS_FP64 = 0,       /* everything in FP64 (the plain form) */
    NS_MIXED_BF16 = 1, /* mixture quadratic forms as BF16 MFMA products with FP32 accumulation
                        * and FP32 log-sum-exp; a candidate whose estimate falls within a guard
                        * band of L* is re-evaluated in FP64 before the decision; stored logL,
                        * L*, and the evidence are FP64 (App. A.6 "Reduced-precision
                        * execution": HRSS only compares log densities) */
    NS_MIXED_FP16 = 2, /* as NS_MIXED_BF16 with FP16 operands (8x smaller rounding error) */
    NS_MIXED_BF16X3 = 3, /* split precision: W and the residual are each a 16-bit value plus a
                          * 16-bit remainder; W_hi r_hi + W_hi r_lo + W_lo r_hi on three BF16
                          * MFMAs (~600x smaller error than NS_MIXED_BF16, so FP64 re-checks
                          * near L* become rare) */
    NS_MIXED_FP16X3 = 4, /* as NS_MIXED_BF16X3 with FP16 parts */
    NS_MIXED_FP32 = 5  /* NS_LIK_GP only: kernel matrix and Cholesky factorisation in FP32 on
                        * MFMA (FP64 log-determinant and |z|^2 sums); a candidate whose
                        * estimate falls within a guard band of L*, or whose FP32
                        * factorisation breaks down, is re-evaluated in FP64 */
} ns_precision;

typedef struct {
    int32_t kind;       /* ns_prior_kind */
    int32_t d;          /* dimension, 1 <= d <= 128; up to 320 for NS_LIK_FUNNEL and
                         * NS_LIK_GAUSS_RASTRIGIN in FP64 with the direction buffer */
    const double *a;    /* [d] box lower bound | Gaussian mean */
    const double *b;    /* [d] box upper bound | Gaussian standard deviation */
} ns_prior;

typedef struct {
    int32_t kind;       /* ns_lik_kind */
    int32_t d;          /* must equal the prior's d (NS_LIK_GP: 6) */
    int32_t n_comp;     /* NS_LIK_MIXTURE: number of components, 1 <= n_comp <= 64 */
    const double *logw; /* [n_comp] log weights (normalised by the caller if Z must be) */
    const double *mean; /* [n_comp * d] component means */
    const double *cov;  /* [n_comp * d * d] symmetric positive-definite covariances */
    int32_t n_obs;      /* NS_LIK_GP: observations, 1 <= n_obs <= 256 */
    const double *x_obs;/* NS_LIK_GP: [n_obs * 2] inputs, row-major */
    const double *y_obs;/* NS_LIK_GP: [n_obs] targets */
    double alpha;       /* NS_LIK_GAUSS_RASTRIGIN: weight of the Gaussian term, 0..1 */
    double amp;         /* NS_LIK_GAUSS_RASTRIGIN: amplitude A >= 0 */
} ns_energy;

typedef struct {
    int32_t n_live;       /* m, 2 <= m <= 8192 */
    int32_t k;            /* deletions per iteration, 1 <= k <= m-1 (Sec. 3.1) */
    int32_t chain_len;    /* p >= 1 HRSS steps per replacement (Sec. 3.2) */
    double width;         /* slice width in whitened units; <= 0 selects the tuning rule
                           * w = 4 kappa R sqrt(2/(pi d)) for the unit-covariance ball,
                           * R = sqrt(d+2), kappa = 1.3035 (Sec. 3.3; App. E ball corollary) */
    int32_t stepout_cap;  /* expansions per side, default 10 (App. A.6) */
    int32_t shrink_cap;   /* shrink proposals before a null move, default 100 (App. A.6) */
    double term_frac;     /* stop when logX + max logL_live - logZ < ln(term_frac) (Sec. 2.1);
                           * <= 0 never stops */
    uint64_t seed;        /* Philox key: (seed_lo, seed_hi ^ run_id) */
    uint32_t run_id;
    int32_t precision;    /* ns_precision */
    int32_t max_iter;     /* upper bound of the dead-point record in iterations (>= 1): the
                           * record starts at min(max_iter + 1, 512) iterations and doubles
                           * between launches as the run proceeds (ns_step / ns_run return
                           * NS_ENOMEM if that allocation fails) */
    int32_t flags;        /* NS_FLAG_* */
    int32_t replacement;  /* ns_replacement: the constrained kernel that replaces deleted
                           * points (Sec. 3.1 "Replacement strategies"); default HRSS */
    int32_t outer;        /* ns_outer: nested sampling (default) or adaptive tempered SMC */
    double ess_frac;      /* NS_OUTER_SMC: ESS target rho in (0, 1) of each next temperature,
                           * default 0.5 */
} ns_config;

/* Outer loops.  NS_OUTER_SMC is adaptive tempered SMC with the slice-sampling mutation
 * (App. "Adaptive Tempered SMC"; SMC-SS in App. "Adaptive non-equilibrium samplers"): n_live
 * particles start from the prior at beta = 0; each ns_step picks the next inverse temperature
 * by 50 bisection steps so that the ESS of the incremental weights exp((b - beta) log L) is
 * ess_frac * n_live (or beta = 1), adds the log mean incremental weight to log Z, resamples
 * systematically, whitens with the covariance of all particles and moves every particle by
 * chain_len HRSS steps on Pi L^beta without a hard constraint (slice height
 * log Pi + beta log L - Exp(1)).  The run is done after the step that reaches beta = 1.
 * k, term_frac and the dead record are unused; ns_get_state's Lstar holds beta; ns_logz
 * returns the accumulated log Z with NaN error and H; ns_set_state, ns_geom_uncertainty and
 * NS_REPLACE_RW are not available; FP64 only; not for NS_LIK_GP.  All runs of a context share
 * the outer loop. */
typedef enum {
    NS_OUTER_NESTED = 0,
    NS_OUTER_SMC = 1
} ns_outer;

/* Replacement kernels.  NS_REPLACE_RW runs chain_len constrained Gaussian random-walk
 * Metropolis steps per replacement (App. "Slice Sampling vs Random Walk"): the proposal is
 * x' = x + s L_Sigma z, z ~ N(0, I) (Gaussian with the live-set covariance scaled by s^2),
 * accepted if x' lies in the prior support, passes the Metropolis test of the prior ratio
 * (non-uniform priors: log Pi(x') > log Pi(x) + log uh) and has logL > L*; otherwise the
 * chain stays.  For it `width` is s (<= 0 selects 2.38 / sqrt(d)); the step-out and shrink
 * caps are unused; traces record (0, 0, evaluated, accepted) per step.  Not available for
 * NS_LIK_GP or with NS_FLAG_INLINE_DIRECTIONS (the proposals come from the per-iteration
 * direction buffer, which must fit in 32 GiB). */
typedef enum {
    NS_REPLACE_HRSS = 0,
    NS_REPLACE_RW = 1
} ns_replacement;

#define NS_FLAG_TRACE  1  /* record per-chain, per-step (left, right, shrinks, accepted) */
#define NS_FLAG_TIMING 2  /* time every HRSS kernel with HIP events on the context's stream */
#define NS_FLAG_INLINE_DIRECTIONS 4  /* chains draw their directions and step uniforms
                                      * themselves instead of reading a per-iteration buffer
                                      * of k*p*(d+8) doubles (the buffer is also skipped when
                                      * it would exceed 32 GiB; not for d > 128) */
#define NS_FLAG_RECORD_POINTS 16  /* keep the dead points' coordinates beside their logL
                                  * (k d doubles per iteration, grown like the dead
                                  * record) for ns_posterior_samples */
#define NS_FLAG_AUTOTUNE 32  /* choose the launch shape of each compiled kernel group's
                              * chains by timing: chains per workgroup (1..4) and, for mixture
                              * chains in a 16-bit mode, tests planned per round (4, 8 or 16).
                              * At the context's iterations 0, 32 and 96 (counted from the
                              * runs' start or reset; the later points are skipped once one
                              * candidate's sum is 25% below every other's after the first
                              * point or 5% below after the second), after whitening and
                              * directions, the state
                              * the chains change is saved, every candidate's chain launch is
                              * timed twice on it (the state restored each time), each
                              * candidate's best time is added to its sum, and the iteration
                              * completes with the shape of least sum so far: the chains'
                              * behaviour changes over a run, so one early iteration would
                              * mislead.  The current choice is cached for later contexts of
                              * the same shape (padded dimension, likelihood, precision,
                              * fragment capacity, replacement, total chains, plan kernel
                              * allowed) in this process, which then do not tune.  Results are
                              * identical with and without it.  Not used by NS_LIK_GP (one chain
                              * per workgroup). */
#define NS_FLAG_SHALLOW_PLAN 64  /* mixture chains in a 16-bit mode plan at most 4 tests per
                                 * round (the two bracket ends, then shrink proposals) instead
                                 * of 16 (the next two stepping-out tests of each open end and
                                 * the shrink proposals of the likeliest expansion outcomes).
                                 * Decisions, trajectories and counters are identical. */
#define NS_FLAG_PLAN8 128  /* mixture chains in a 16-bit mode plan 8 tests per round (the
                           * next two stepping-out tests of each open end and the shrink
                           * proposals of the three likeliest expansion outcomes) instead of
                           * 16; identical results.  NS_FLAG_SHALLOW_PLAN takes precedence. */
#define NS_FLAG_GP_NO_WAIT 256  /* testing the failure path of NS_LIK_GP chains: the
                                * factorisation's bounded wait for each diagonal tile gives up
                                * at once, so every chain evaluation fails (log L = -inf, a
                                * rejection) and is counted in gp_wait_timeouts; every kernel
                                * still exits normally.  The initial evaluation is unaffected. */
#define NS_FLAG_FREEZE_WHITENING 512  /* the whitening factor (and with it the direction
                                      * metric, and the random walk's proposal covariance) is
                                      * computed at the first iteration only and kept for the
                                      * run: a proposal scale fixed over the run, the variant
                                      * the slice-versus-random-walk comparison contrasts with
                                      * the adaptive default.  Not for NS_OUTER_SMC. */
#define NS_FLAG_DIAGONAL_METRIC 1024  /* the direction metric (whitening) from the
                                      * survivors' variances alone, a diagonal conditioning
                                      * matrix, instead of their full covariance: the
                                      * restriction Sec. 3.2 suggests for high dimensions.
                                      * Applies to slice and random-walk chains and to the
                                      * tempered-SMC mutation. */
#define NS_FLAG_SERIAL_GROUPS 2048  /* (read from the first run's config) a batch whose runs
                                    * compile to several chain kernels launches them one after
                                    * the other on the context's stream; by default the second
                                    * and later ones run concurrently on side streams of the
                                    * library's own (default priority), forked and joined with
                                    * events around the chain phase of each iteration (eager
                                    * iterations only: iterations captured as a HIP graph run
                                    * the groups in sequence).  Results are identical either
                                    * way. */
#define NS_FLAG_GRAPH  8  /* ns_run captures each batch of 16 iterations as a HIP graph and
                           * replays it (re-captured when a run of the batch finishes); not
                           * used together with NS_FLAG_TIMING.  Results are identical. */

typedef struct {
    int64_t iterations;     /* completed ns_step iterations */
    int64_t evals;          /* likelihood evaluations inside chains (candidates that passed the
                             * prior support and height tests); speculative / padded rows and
                             * FP64 re-checks are not counted */
    int64_t tests;          /* all slice-membership tests, including prior rejections */
    int64_t prior_rejects;
    int64_t stepout_caps;   /* sides that stopped at the expansion cap */
    int64_t shrink_caps;    /* null moves from the shrink cap */
    int64_t nonfinite;      /* NaN/+inf log-likelihoods treated as -inf */
    int64_t rechecks;       /* mixed precision: decisions taken on an FP64 re-evaluation
                             * because the 16-bit estimate was within the guard band of L* */
    int64_t band_violations;/* mixed precision: accepted points whose FP64 logL <= L* */
    int64_t whiten_fallbacks; /* iterations whose covariance factorisation failed (diagonal used) */
    int64_t n_dead;         /* dead points recorded */
    double hrss_ms;         /* NS_FLAG_TIMING: summed HRSS kernel time (HIP events) */
    int64_t hrss_launches;
    double width;           /* slice width in use */
    int64_t tune_launches;  /* NS_FLAG_AUTOTUNE: HRSS launches the tuner timed in this context
                             * (0 when every shape came from the cache) */
    int64_t gp_wait_timeouts; /* NS_LIK_GP: chain evaluations whose factorisation gave up a
                               * bounded wait for a diagonal tile (the candidate then counts as
                               * log L = -inf); never expected outside NS_FLAG_GP_NO_WAIT */
} ns_stats_t;

/* Host arrays for state access (any pointer may be NULL to skip it). */
typedef struct {
    double *x;        /* [m*d] live points, row-major */
    double *logL;     /* [m] */
    int32_t *perm;    /* [m] live indices in ascending (logL, index) order; first k = deleted */
    double *Lsig;     /* [d*d] lower Cholesky factor of the last direction covariance */
    int32_t *parents; /* [k] live indices resampled as parents in the last iteration */
    double Lstar;     /* threshold: logL of the k-th worst live point */
    double logZ;      /* evidence of the dead points so far */
    double logX;      /* log prior volume after the recorded deaths */
    double M;         /* posterior mean of logL over the dead points; H = M - logZ */
    int64_t iter;
    int32_t done;
} ns_state_view;

/* Create a run: copy the problem to the device, draw m points from the prior (Philox purpose
 * INIT), evaluate them in FP64, delete the k worst and account their evidence (Alg. outer
 * kernel, first evaluate-sort-record).  Returns NS_EINVAL for inconsistent arguments,
 * NS_EUNSUPPORTED for sizes beyond this library. */
ns_status ns_init(const ns_prior *prior, const ns_energy *energy, const ns_config *cfg,
                  void *hip_stream, ns_ctx **out);

/* Restart the run on an existing context with a new Philox key (seed, run_id): the problem
 * stays on the device; the live set is redrawn from the prior and evaluated, the evidence,
 * counters, dead record and timing are cleared, and the first delete-k is accounted, exactly
 * as ns_init does.  Lets a caller time runs without the problem upload. */
ns_status ns_reset(ns_ctx *ctx, uint64_t seed, uint32_t run_id);

/* One outer iteration (Sec. 3.1 (ii)-(iv) then (i)): whiten (survivor covariance, Sec. 3.2
 * "Direction metric"), resample k parents uniformly among survivors with logL > L*, run the k
 * HRSS chains of p steps, replace the deleted points, delete the next k worst, accumulate the
 * evidence (Sec. 2.1, App. D.2.1), test termination.  *done = 1 once terminated.
 * Returns NS_DONE (and does nothing) if the run had already terminated. */
ns_status ns_step(ns_ctx *ctx, int32_t *done);

/* Iterate until termination or max_iter further iterations; *iters = iterations done in this
 * call.  The stop iteration is the same as with repeated ns_step calls. */
ns_status ns_run(ns_ctx *ctx, int32_t max_iter, int32_t *iters);

/* Evidence including the live set's remaining contribution X * mean(L_live) (non-destructive):
 * ln Z, its error sqrt(H/m) and the information H (Sec. 2.1). */
ns_status ns_logz(ns_ctx *ctx, double *logz, double *logz_err, double *H);

ns_status ns_stats(ns_ctx *ctx, ns_stats_t *out);

/* Copy the state to host arrays / overwrite it from host arrays.  ns_set_state takes x, logL,
 * logZ, logX, M and iter; it recomputes the delete-k order and L* without re-accounting.  A
 * logL entry that is NaN or +inf is stored as -inf and counted in ns_stats_t.nonfinite, as a
 * computed one would be.  If after this no live point lies strictly above L* (a total
 * plateau), the next ns_step returns NS_ESTATE.  On a run with NS_FLAG_FREEZE_WHITENING a
 * non-null Lsig (d x d row-major, lower triangle read) becomes the whitening factor kept for
 * the rest of the run (until ns_reset) in place of any computed one, e.g. the Cholesky
 * factor of the target's covariance; a non-finite entry is NS_EINVAL.  Without that flag Lsig
 * is ignored. */
ns_status ns_get_state(ns_ctx *ctx, ns_state_view *view);
ns_status ns_set_state(ns_ctx *ctx, const ns_state_view *view);

/* Copy the dead-point log-likelihoods (ascending death order) to out[0..cap); *n = total. */
ns_status ns_get_dead(ns_ctx *ctx, double *out, int64_t cap, int64_t *n);

/* Post-hoc geometric uncertainty of run `run` (App. "Estimation of prior volumes and
 * propagation of geometric uncertainty"; the within-batch live counts of the unrolled
 * evidence, Sec. 2.1).  The deaths, in likelihood order, are the dead record followed by the
 * run's current survivors (the m - k live points not yet accounted) in ascending logL; the
 * j-th death of a batch sees m - j live points (j = 0..k-1) and the q-th survivor m - k - q.
 * Each of R replicas draws the shrinkages t = u^(1/n) (u uniform: deaths 2h+1 and 2h+2 take the
 * two uniforms of Philox block (purpose 6, replica, h), keyed by (seed, run_id) as the run's
 * own draws), forms the trapezoid elements dX_i = (X_{i-1} - X_{i+1}) / 2 with X_0 = 1 and
 * X_{N+1} = 0, and the weights w_i = L_i^beta dX_i (L^0 = 1, also where L = 0).
 * Outputs (host pointers; the call waits for the device):
 *   logz[R]       log sum_i w_i per replica (required); its spread is the error of ln Z;
 *   logw_mean     if not NULL, the first min(N, cap) geometric-mean log weights
 *                 (1/R) sum_r log w_i^(r), in death order (unnormalised);
 *   ess           if not NULL, the Kish effective sample size (sum w~)^2 / sum w~^2 of the
 *                 geometric-mean weights w~;
 *   n_deaths      if not NULL, N;
 *   device_ms     if not NULL, the device time of the computation (events around it).
 * Any beta >= 0 reweights the same run (beta-reweighting); nothing of size R x N is stored.
 * The library keeps one device buffer of about (R / 8 + 2) N doubles per context.
 * Errors: NS_EINVAL (NULL ctx or logz, run out of range, R outside [1, 65535], beta negative,
 * infinite or NaN, cap < 0), NS_ESTATE if the dead record was truncated (more deaths than
 * max_iter + 1 iterations hold), NS_EUNSUPPORTED for N >= 2^31, NS_EDEVICE. */
ns_status ns_geom_uncertainty(ns_ctx *ctx, int32_t run, int32_t R, double beta, uint64_t seed,
                              uint32_t run_id, double *logz, double *logw_mean, int64_t cap,
                              double *ess, int64_t *n_deaths, double *device_ms);

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): ns_geom_uncertainty with caller-owned DEVICE outputs and
 * the partial results in a fixed workspace compiled into the library, one copy of
 * NS_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends (its address is looked up by
 * ns_init / ns_init_batch).  It calls no hipMalloc, hipFree or allocating library routine.
 *   logz[R], logw_mean[cap], ess[1]: device pointers on the context's device, all required;
 *   the values equal ns_geom_uncertainty's (logw_mean: all N of them, so cap >= N);
 *   n_deaths: host pointer, if not NULL set to N (also when cap is too small).
 * The work is enqueued on the context's stream after one wait for the run's death count; the
 * outputs are ready when the stream reaches that point (the call does not wait for them).
 * Every call on one GPU shares that GPU's workspace: calls that overlap on one GPU (other
 * streams, other threads, other contexts) race and must be serialised by the caller.
 * Errors: those of ns_geom_uncertainty, NS_EINVAL for a NULL output, cap < N, or a workspace
 * needing more than NS_NOALLOC_SCRATCH_BYTES (a run with 312,000 deaths and R = 100 needs
 * about 19 MiB; about 4 million deaths fit at R = 100), NS_EDEVICE if the workspace address
 * could not be looked up. */
#define NS_NOALLOC_SCRATCH_BYTES (64u << 20)
ns_status ns_geom_uncertainty_noalloc(ns_ctx *ctx, int32_t run, int32_t R, double beta,
                                      uint64_t seed, uint32_t run_id, double *logz,
                                      double *logw_mean, int64_t cap, double *ess,
                                      int64_t *n_deaths);

/* Weighted posterior samples of run `run` (App. "Estimation of prior volumes and propagation
 * of geometric uncertainty": resampling with the geometric-mean weights): the weights of
 * ns_geom_uncertainty(run, R, beta, seed, run_id), then n samples by systematic resampling of
 * the deaths (one uniform: Philox purpose 7, counter 0, the same key).  x[n * d] (host)
 * receives the samples' coordinates, row by row; idx[n] (host, may be NULL) their death
 * indices (dead record first, then the survivors in ascending logL).  Needs a context created
 * with NS_FLAG_RECORD_POINTS.  Errors: as ns_geom_uncertainty, NS_EINVAL for NULL x or
 * n < 1, NS_ESTATE if the coordinates were not recorded. */
ns_status ns_posterior_samples(ns_ctx *ctx, int32_t run, int32_t R, double beta, uint64_t seed,
                               uint32_t run_id, int32_t n, double *x, int64_t *idx);

/* NS_FLAG_TRACE: copy the last iteration's trace, out[(j*p + s)*4 + {0,1,2,3}] = left
 * expansions, right expansions, shrink proposals, accepted, for chain j and step s. */
ns_status ns_get_trace(ns_ctx *ctx, int32_t *out);

/* Evaluate the likelihood at n host points x[n*d] with the given precision (NS_FP64 or a mixed
 * mode), writing out[n].  Runs the same device evaluators as the chains; for tests. */
ns_status ns_eval_loglik(ns_ctx *ctx, const double *x, int32_t n, int32_t precision,
                         double *out);

/* Batched serving of independent runs (many runs of uneven dimension and likelihood on one
 * GPU).  Run r has its own prior priors[r], energy energies[r] and configuration cfgs[r]
 * (dimension, n_live, k, chain length, precision, seed, run_id, flags; NS_FLAG_TIMING on any
 * run times the whole batch).  Every kernel of an outer iteration is one launch over all
 * unfinished runs that share its compiled shape (padded dimension, likelihood, precision);
 * runs that have terminated drop out of the launches.  Each run follows exactly the trajectory
 * it has alone (ns_init with the same arguments): chains draw from counters keyed by their
 * own run's (seed, run_id) and runs share no state.
 * On a batch context: ns_step and ns_run advance every unfinished run (ns_step's *done = 1 and
 * NS_DONE once all have terminated; ns_run's *iters = the most iterations any run advanced);
 * ns_reset restarts run r with (seed, run_id + r); NS_ESTATE from ns_step or ns_run means
 * some run stopped on a plateau (it is finished; the others continue).  ns_logz, ns_stats,
 * ns_get_state, ns_set_state, ns_get_dead, ns_get_trace and ns_eval_loglik address run 0.
 * Arrays have n_runs entries; all pointers are host pointers copied as by ns_init.
 * Errors: NS_EINVAL if n_runs < 1 or any run's arguments are invalid (ns_last_error(NULL)
 * names the run), NS_EUNSUPPORTED for n_runs > 65536 or a run beyond this library. */
ns_status ns_init_batch(int32_t n_runs, const ns_prior *priors, const ns_energy *energies,
                        const ns_config *cfgs, void *hip_stream, ns_ctx **out);

/* Number of runs of a context (0 for NULL). */
int32_t ns_num_runs(const ns_ctx *ctx);

/* Chains per HRSS workgroup that run `run`'s next iteration uses (1..4; under
 * NS_FLAG_AUTOTUNE the tuned value once tuning has finished); 0 for a NULL context or a run
 * index out of range. */
int32_t ns_chains_per_workgroup(const ns_ctx *ctx, int32_t run);

/* NS_FLAG_AUTOTUNE's process-wide cache of tuned launch shapes, as a JSON file:
 * {"nss_tune": 2, "entries": [{"D", "lik", "mode", "upw", "rw", "chains", "planned", "C",
 * "plan"}, ...]} (the group shape: padded dimension, likelihood, precision, fragment capacity,
 * replacement, total chains, whether the plan kernel is allowed; the choice: chains per
 * workgroup and tests per round, 0 meaning the 4-test kernel).  ns_tune_save writes the cache
 * to path; ns_tune_load merges a file in the format ns_tune_save writes (its entries replace
 * cached ones of the same shape); ns_tune_clear empties the cache; contexts created
 * afterwards with NS_FLAG_AUTOTUNE start with the cached value.  *n (may be NULL) receives the
 * number of cached entries afterwards (before, for ns_tune_clear).  Errors: NS_EINVAL for a
 * NULL path, a file that cannot be opened or written, or a file that is not a tuning cache or
 * holds a malformed entry (unknown shape values, extra keys, non-integer values: then nothing
 * is merged); the message is in ns_last_error(NULL).  Host only: no device is needed. */
ns_status ns_tune_save(const char *path, int32_t *n);
ns_status ns_tune_load(const char *path, int32_t *n);
ns_status ns_tune_clear(int32_t *n);

/* The launch shape run `run`'s chains use now: chains per workgroup and tests planned per
 * round (4 for the k_hrss kernel, 8 or 16 for the hypothesis-plan kernel, 1 for NS_LIK_GP).
 * Either output may be NULL.  Errors: NS_EINVAL for a NULL context or a run out of range. */
ns_status ns_launch_shape(const ns_ctx *ctx, int32_t run, int32_t *chains_per_wg,
                          int32_t *plan_tests);

/* ns_logz for every run: logz[r], logz_err[r], H[r] (any array may be NULL). */
ns_status ns_logz_batch(ns_ctx *ctx, double *logz, double *logz_err, double *H);

/* ns_stats / ns_get_state of run `run` (0 <= run < n_runs, else NS_EINVAL); hrss_ms and
 * hrss_launches are the batch's. */
ns_status ns_stats_run(ns_ctx *ctx, int32_t run, ns_stats_t *out);
ns_status ns_get_state_run(ns_ctx *ctx, int32_t run, ns_state_view *view);

void ns_free(ns_ctx *ctx);

const char *ns_last_error(const ns_ctx *ctx);

/* Default configuration values (caps 10/100, term_frac 1e-3, width rule, FP64). */
void ns_config_default(ns_config *cfg);

#ifdef __cplusplus
}
#endif
#endif /* NSS_H */
