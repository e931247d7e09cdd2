/*
 * sim.h -- C ABI of the MI355X batched stochastic Frank-Wolfe simulator.
 *
 * The library runs Algorithm 1 of He, Liu, Wu, Zheng and Zhu, "A Preliminary Study on
 * Accelerating Simulation Optimization with GPU Implementation" (Section 3.1), over R
 * independent replications on one gfx950 GPU and reduces the paths to FP64 statistics.
 *
 *   problem (Eq. (3)):   min_w f(w) = lambda w' Sigma w - w' mu   on W = {w >= 0, 1'w <= 1},
 *                        returns R ~ N(mu, Sigma) with Sigma = L L' (diag(sigma^2) by default);
 *                        lambda = 1/2 is Eq. (3), lambda = 1 is the sample objective Eq. (4).
 *   estimator (Eq. (4)-(5)): N fresh samples every M iterations; gradient 2 lambda Sigma_hat w - Rbar
 *                        with the centred sample covariance (divisor N-1) and the sample mean.
 *   algorithm (Alg. 1):  linear subproblem over the vertices {0, e_1..e_d} of W (lowest index
 *                        among equal minima; the origin when the smallest entry is >= 0), step
 *                        2/(t+2) with t = kM+m, update w + gamma (s - w), outcome Y = f(w_T).
 *
 * Noise: replication r, epoch k = t div M, uses standard normals number q = 0, 1, ... of the
 * Philox4x32-10 stream with key (seed lo, seed hi) and counter (q/4, k, r, instance_id), words
 * (x0,x1) and (x2,x3) of each block mapped to Box-Muller pairs through u = (2 (x mod 2^23)+1) 2^-24.
 * Sample i, asset j takes normal q = i d + j; Student-t noise scales sample i by
 * sqrt((nu-2)/chi2) with chi2 the sum of squares of normals N d + nu i + k, k < nu.
 *
 * Conventions for every entry point:
 *   - Input pointers are host pointers owned by the caller, read during the call only.
 *   - Results live in device memory owned by the context until the next run or sim_destroy.
 *   - Return 0 on success or a negative sim_status. Validation happens before any launch; a
 *     rejected call changes nothing. No C++ exception crosses this boundary.
 *   - A context is not thread-safe; calls that launch work are asynchronous on its stream, and
 *     the calls that return results synchronise that stream.
 */
#ifndef PAPER_2404_11631_AMD_SIM_H
#define PAPER_2404_11631_AMD_SIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIM_ABI_VERSION 4u
#define SIM_MAX_D 64u          /* assets per instance */
#define SIM_MAX_CKPT 8u        /* checkpoints per run */
#define SIM_TAU_NONE 0xFFFFFFFFu
#define SIM_WIDE_MAX_D 4194304u    /* assets per instance on the wide path (sim_run_wide) */
#define SIM_WIDE_MAX_R 64u         /* replications per wide run */
#define SIM_WIDE_MAX_N 1024u       /* samples per resample on the wide path */
#define SIM_NV_MAX_N 16777216u     /* products of a newsvendor instance (sim_run_newsvendor) */
#define SIM_NV_MAX_S 1024u         /* demand samples per product and resample */
#define SIM_SQN_MAX_N 8192u        /* features of the classification data (sim_sqn_load) */
#define SIM_SQN_MAX_M 32u          /* stored correction pairs */
#define SIM_SQN_MAX_B 1024u        /* gradient and Hessian sample sizes b, b_H */
#define SIM_SQN_MAX_R 4096u        /* replications of sim_run_sqn */

typedef struct sim_ctx sim_ctx;

typedef enum {
    SIM_OK = 0,
    SIM_EINVAL = -1,        /* an argument violates its stated range */
    SIM_ENOMEM = -2,        /* device or host allocation failed */
    SIM_EDEVICE = -3,       /* a HIP call failed; sim_last_error has its message */
    SIM_ESTATE = -4,        /* call out of order (e.g. results before any run) */
    SIM_EUNSUPPORTED = -5   /* a combination the library does not implement */
} sim_status;

typedef enum { SIM_NOISE_GAUSS = 0, SIM_NOISE_T = 1 } sim_noise;
typedef enum { SIM_FP32 = 0, SIM_FP64 = 1 } sim_precision;

typedef enum {
    SIM_KEEP_PATHS = 1u,    /* keep per-path records (Y, checkpoints, cnt, wsum, tau) */
    SIM_DECISION_LOG = 2u,  /* log every decision of replications [log_rep_begin, +log_rep_count) */
    SIM_CV_FEATURES = 4u    /* write each path's d+2 control-variate features (see sim_path_view.x) */
} sim_flag;

/* One problem instance (Eq. (3)) and the sampling knobs of Algorithm 1. */
typedef struct {
    uint32_t abi_version;       /* SIM_ABI_VERSION */
    uint32_t d;                 /* assets, 1..SIM_MAX_D */
    const double *mu;           /* [d] mean returns */
    const double *sigma;        /* [d] standard deviations >= 0, used when chol is NULL */
    const double *chol;         /* [d*d] row-major lower-triangular L (Sigma = L L'), or NULL */
    double risk_coef;           /* lambda > 0 */
    const double *w0;           /* [d] starting point in W, or NULL for the origin */
    uint32_t n_samples;         /* N >= 2 */
    uint32_t resample_every;    /* M >= 1 */
    uint32_t noise;             /* sim_noise */
    uint32_t nu;                /* Student-t degrees of freedom, integer >= 3 (noise == SIM_NOISE_T) */
    uint32_t state_precision;   /* sim_precision of normals, sums and iterate */
    uint32_t n_checkpoints;     /* 0..SIM_MAX_CKPT */
    uint64_t checkpoints[SIM_MAX_CKPT]; /* strictly increasing iterate counts in [1, T] */
    double gap_eps;             /* Frank-Wolfe gap threshold of the hitting time tau, >= 0 */
    uint32_t flags;             /* sim_flag bits */
    uint32_t instance_id;       /* stream domain of this instance, < 2^24 */
    uint64_t log_rep_begin;     /* SIM_DECISION_LOG: first logged replication */
    uint64_t log_rep_count;     /* SIM_DECISION_LOG: number of logged replications (<= 65536) */
    const double *cv_ref;       /* SIM_CV_FEATURES: [d] reference gradient b of the features */
    const uint32_t *n_schedule; /* sample size N_k of every epoch k < ceil(T / M) (Algorithm 1's
                                   resampling step lets the size adapt to k), each in [2, 2^24] for
                                   sim_run (diagonal Sigma, no control-variate features) and in
                                   [2, SIM_WIDE_MAX_N] for sim_run_wide; NULL: n_samples in every
                                   epoch. A dense factor, features, batches and sim_run_noalloc
                                   reject a schedule with SIM_EUNSUPPORTED */
} sim_params;

/* FP64 statistics of one run. Means, variances and sums use compensated (double-double)
 * accumulation over a fixed reduction tree, so they do not depend on scheduling. */
typedef struct {
    uint64_t R, T;
    double mean, var, ci95_halfwidth, min, max;     /* of Y = f(w_T); var unbiased; 1.96 sqrt(var/R) */
    double f_star;                                  /* min over W of f (diagonal Sigma), else NaN */
    uint32_t n_checkpoints;
    uint32_t pad_;
    uint64_t checkpoints[SIM_MAX_CKPT];
    double f_mean[SIM_MAX_CKPT], f_sd[SIM_MAX_CKPT];        /* f(w_c) across paths */
    double rse_mean[SIM_MAX_CKPT], rse_sd[SIM_MAX_CKPT];    /* ((f(w_c) - Y)/f(w_c))^2, Table 2 */
    uint64_t rse_undefined[SIM_MAX_CKPT];                   /* paths with f(w_c) == 0 */
    uint64_t decision_total[SIM_MAX_D + 1];                 /* [0] origin, [j+1] vertex e_j */
    uint64_t tau_count;                                     /* paths whose FW gap reached gap_eps */
    double tau_mean;                                        /* mean hitting step over those paths */
    double kernel_ms;                                       /* device time of the run (HIP events) */
    double path_steps_per_s;                                /* R T / kernel time */
} sim_stats_out;

/* Control-variate features (SIM_CV_FEATURES). A variance-reduction layer over the Monte Carlo
 * estimate of E f(w_T); not part of the paper's method. With zbar_e the sample mean of the Gaussian
 * numerators a path draws in epoch e (for t noise, before the chi-square scaling), E = ceil(T/M):
 *   J_e  = the vertex the linear subproblem over W picks for the gradient b - sigma .* zbar_e, with
 *          b = cv_ref fixed before the run (lowest index among equal minima, the origin when the
 *          minimum is >= 0): i.i.d. categorical over epochs with probabilities p_c (c = 0 origin,
 *          c = j+1 vertex e_j), p_c one-dimensional normal integrals;
 *   K_c  = sum over iterations t of (t+1)^2 [J_e(t) = c],  K1 = sum_t (t+1) [J_e(t) = c*], c* the
 *          most probable category;  per epoch W2_e, W1_e = sums of (t+1)^2, (t+1) over it;
 *          S2 = sum W2_e, S4 = sum W2_e^2, S1 = sum W1_e, S11 = sum W1_e^2.
 * Features: x_j = (K_{j+1} - p_{j+1} S2) / sqrt(S4 max(p(1-p), 1e-4)) for j < d, x_d the same for
 * the origin, x_{d+1} = (K1 - p_c* S1) / sqrt(S11 max(p_c* (1 - p_c*), 1e-4)). The law is exact
 * for exact arithmetic; the device takes J_e from binary32 sample means, which moves it only by
 * near-ties at the rounding level. Supported with FP32 state, diagonal Sigma with every
 * sigma_j > 0, d <= 32 and T <= 92681. */

/* Device pointers (owned by the context) to the per-path records of the last run, structure of
 * arrays indexed [field][r]. Fields not produced by the run are NULL. */
typedef struct {
    uint64_t R, T;
    uint32_t d, n_checkpoints;
    const double *y;            /* [R] f(w_T) */
    const double *f_ckpt;       /* [n_checkpoints][f_ckpt_stride], first R of each row */
    const uint32_t *cnt;        /* [d+1][R] decision counts */
    const uint64_t *wsum;       /* [d][R] sum of (t+1) over steps choosing e_j */
    const uint32_t *tau;        /* [R] hitting step or SIM_TAU_NONE */
    const uint8_t *decisions;   /* [T][log_rep_count] decisions, 0 = origin, j+1 = e_j */
    uint64_t log_rep_begin, log_rep_count;
    uint64_t f_ckpt_stride;     /* elements between checkpoint rows (R, or the batch total) */
    const float *x;             /* SIM_CV_FEATURES: [d+2][R] features xi_0..xi_{d-1}, eta, zeta */
    uint32_t n_features;        /* d+2 when x is set, else 0 */
    uint32_t pad_;
} sim_path_view;

/* Creates a context on HIP device `device`, launching on `hip_stream` (a hipStream_t, or NULL
 * for the null stream). */
int sim_create(int device, void *hip_stream, sim_ctx **out);

/* sim_create with a cap on the context's device memory: every buffer later calls allocate for it
 * (per-path records, partial sums, staging of every path) may total at most workspace_bytes
 * (0: no cap). A call that would go past it returns SIM_ENOMEM before launching anything and leaves
 * the context as it was, usable with smaller inputs. SIM_ENOMEM here also when the context's own
 * set-up buffers do not fit. */
int sim_create_ex(int device, void *hip_stream, uint64_t workspace_bytes, sim_ctx **out);

/* The bytes of device memory the context's buffers hold now. */
int sim_workspace_bytes(sim_ctx *ctx, uint64_t *used);

/* Replaces the stream later calls launch on. */
int sim_set_stream(sim_ctx *ctx, void *hip_stream);

/* Runs R replications of Algorithm 1 for T iterations (Section 3.1) with noise seed `seed`,
 * fused with the cross-path reduction in one launch. Asynchronous on the context's stream.
 * Ranges: 1 <= R < 2^32, 1 <= T <= 2^32 - 2. One lane (diagonal Sigma) or four lanes (dense L) hold
 * a replication's state, so the shapes are: diagonal Sigma with d <= 32 in FP32 state or d <= 16 in
 * FP64; a dense factor with d = 32 or 64, FP32, T <= 65535. Others return SIM_EUNSUPPORTED (many
 * assets on a few replications: sim_run_wide). */
int sim_run(sim_ctx *ctx, const sim_params *p, uint64_t R, uint64_t T, uint64_t seed);

/* sim_run with its results in caller device memory (for instance tensors of the caller's framework)
 * instead of the context's, launched on the context's stream (sim_set_stream):
 *   f_ckpt  [n_checkpoints][R] f(w_c) per path (may be NULL when n_checkpoints == 0);
 *   stats_f [(1 + 2 n_checkpoints) * 5 + 2] and stats_i [d + 3]: the FP64 reduction fields and the
 *           decision totals, hitting count and hitting-step sum, in sim_run_noalloc's layouts
 *           (sim_stats_from_raw turns host copies of them into sim_stats_out).
 * Partial sums and the per-path records that flags ask for stay in the context; sim_paths serves
 * the records as after sim_run (with f_ckpt NULL), and sim_stats returns SIM_ESTATE until the next
 * sim_run. The caller's buffers must stay valid until the stream has passed the run. Same shapes,
 * checks and errors as sim_run. */
int sim_run_into(sim_ctx *ctx, const sim_params *p, uint64_t R, uint64_t T, uint64_t seed, double *f_ckpt,
                 double *stats_f, uint64_t *stats_i);

/* Draws an instance's mu[d] and sigma[d] from `seed` on the host: SIM_REGIME_UNIT, mu_j and sigma_j
 * ~ U(0, 1); SIM_REGIME_PAPER, Section 4.1's mu_j ~ U(-1, 1) and sigma_j ~ U(0, 0.025). The
 * generator is SplitMix64 (Steele, Lea and Flood, 2014), 53-bit uniforms, all of mu before sigma.
 * Returns SIM_EINVAL for d = 0, NULL outputs or an unknown regime. */
#define SIM_REGIME_UNIT 0
#define SIM_REGIME_PAPER 1
int sim_param_gen(uint32_t d, int regime, uint64_t seed, double *mu, double *sigma);

/* Checks a parameter set exactly as sim_run does, without a device. Returns 0 or the code sim_run
 * would return, and writes the reason into msg (may be NULL). */
int sim_validate(const sim_params *p, uint64_t R, uint64_t T, char *msg, size_t len);

/* sim_batch_config.flags bit: the tile launch and the reduction are captured once into a HIP graph
 * (kernel nodes only, captured on a library stream) and launched as one graph on the context's
 * stream; the executable graph is kept and replayed while later calls have the same plan and
 * buffers (new seeds and parameters travel in the uploaded descriptors). */
#define SIM_BATCH_GRAPH 0x100u

/* Knobs of a batched run (sim_run_batch); zero fields take the built-in cost model's choice. */
typedef struct {
    uint32_t reserved;              /* must be 0 */
    uint32_t flags;                 /* SIM_KEEP_PATHS for per-path records of every instance;
                                       SIM_BATCH_GRAPH to launch through a captured HIP graph */
    double heavy_factor;            /* theta > 0: replications are split across lanes until one
                                       tile needs at most theta x the balanced run time (0: 0.5) */
    const uint8_t *lanes_per_rep;   /* [n_inst] lanes per replication, each 0 (model) or a power of
                                       two <= 64, or NULL */
} sim_batch_config;

/* Runs n_inst instances (Eq. (3) each, own d, N, T, R) of Algorithm 1 as wavefront tiles: one
 * launch of every tile, longest first (the hardware dispatcher is the work queue), replications of
 * heavy instances split across several lanes (assets x sample chunks), then one per-instance
 * reduction in fixed order. When every instance asks for 64 lanes per replication, has Gaussian
 * noise and N d + 3 <= 2112, each replication instead runs on a workgroup of its own: a wavefront
 * with an asset per lane, and a second one that draws the next epoch's normals (the latency form,
 * for few replications); the results follow the same protocol.
 * Each instance uses its instance_id as stream domain and the common noise `seed`.
 * Supported: FP32 state, diagonal Sigma, d <= 32, T <= 131071 (the signature is held in 33 bits),
 * per-instance R < 2^32, 1 <= n_inst <= 65536. Decision logs follow each instance's
 * log_rep_begin/log_rep_count. Asynchronous on the context's stream. cfg may be NULL. The plan is
 * checked on the host (tile ranges, lanes and replications per tile, slots, normal numbering)
 * before anything is uploaded. */
int sim_run_batch(sim_ctx *ctx, uint32_t n_inst, const sim_params *p, const uint64_t *R,
                  const uint64_t *T, uint64_t seed, const sim_batch_config *cfg);

/* Computes, without a device, the plan sim_run_batch would use on a GPU with n_cu compute units:
 * the lanes per replication and the tile count of every instance (arrays of n_inst, may be NULL).
 * Returns 0 or the code sim_run_batch would return, with the reason in msg (may be NULL). */
int sim_plan_batch(uint32_t n_inst, const sim_params *p, const uint64_t *R, const uint64_t *T,
                   const sim_batch_config *cfg, uint32_t n_cu, uint32_t *lanes_per_rep, uint32_t *n_tiles,
                   char *msg, size_t len);

/* ---- no device allocation ------------------------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. sim_run_noalloc runs sim_run's fused path (diagonal
 * Sigma, FP32 state, no per-path records, logs or features) with every intermediate (instance
 * descriptor, per-workgroup partial sums, finishing counter) in a library-owned static device
 * array of SIM_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends; its device address is
 * taken once per device on the first call there. Nothing is allocated, no memset is issued: the
 * call enqueues kernel launches only, asynchronously on hip_stream (NULL: the null stream) of
 * `device`. R <= SIM_NOALLOC_MAX_R (larger R: SIM_EINVAL).
 * Outputs (device memory, caller-owned, written by the launch):
 *   f_ckpt  [n_checkpoints][R] f(w_c) per path (may be NULL when n_checkpoints == 0);
 *   stats_f [(1 + 2 n_checkpoints) * 5 + 2] FP64 reduction fields (per stream Y, f(w_c), RSE_c:
 *           sum hi, sum lo, squares hi, squares lo, count; then min Y, max Y);
 *   stats_i [d + 3] decision totals (origin first), hitting count, hitting-step sum.
 * sim_stats_from_raw turns host copies of stats_f and stats_i into sim_stats_out (kernel_ms 0).
 * Every call on one GPU shares that GPU's array, which keeps the last call's contents: calls that
 * overlap on one GPU (two streams, two threads) race and must be serialised by the caller.
 * Errors are returned as codes; sim_noalloc_last_error gives the calling thread's last message. */
#define SIM_NOALLOC_MAX_R 1048576u
#define SIM_NOALLOC_SCRATCH_BYTES 4194304u
int sim_run_noalloc(int device, void *hip_stream, const sim_params *p, uint64_t R, uint64_t T, uint64_t seed,
                    double *f_ckpt, double *stats_f, uint64_t *stats_i);
int sim_noalloc_last_error(char *buf, size_t len);
int sim_stats_from_raw(const sim_params *p, uint64_t R, uint64_t T, const double *stats_f,
                       const uint64_t *stats_i, sim_stats_out *out);

/* Measured choice of the batched plan's knob theta (sim_batch_config.heavy_factor: how far heavy
 * instances are split over lanes). Every candidate of SIM_TUNE_THETAS is timed (device time between
 * HIP events, best of two runs) on the same instances with each horizon divided by t_scale (>= 1;
 * per-tile work then shrinks by the same factor for every instance, which keeps the plan's balance),
 * without checkpoints, logs or per-path records; the fastest is returned. Results are cached as one
 * JSON object per line in cache_path (may be NULL: no cache), keyed by a hash of the device name,
 * the ABI version, the candidate list and every instance's (d, N, T, R, noise, nu); a call whose
 * key is in the cache reads it and launches nothing. The tuning runs replace the context's last
 * batched run. Synchronous. */
#define SIM_TUNE_MAX_CAND 16u
typedef struct {
    double heavy_factor;                 /* the fastest theta */
    uint32_t from_cache;                 /* 1: read from cache_path, nothing was run */
    uint32_t n_candidates;
    double cand_theta[SIM_TUNE_MAX_CAND];
    double cand_ms[SIM_TUNE_MAX_CAND];   /* device ms of each candidate at the reduced horizons */
    uint64_t key;                        /* the cache key */
} sim_tune_out;
int sim_tune_batch(sim_ctx *ctx, uint32_t n_inst, const sim_params *p, const uint64_t *R, const uint64_t *T,
                   uint64_t seed, uint32_t t_scale, const char *cache_path, sim_tune_out *out);

/* Statistics of instance `instance` of the last batched run (kernel_ms and path_steps_per_s
 * describe the whole batch); synchronises the stream. */
int sim_batch_stats(sim_ctx *ctx, uint32_t instance, sim_stats_out *out);

/* Per-path records of one instance of the last batched run (device pointers, see sim_paths), and
 * the lanes per replication and tile count the plan gave it; synchronises the stream. */
int sim_batch_paths(sim_ctx *ctx, uint32_t instance, sim_path_view *out, uint32_t *lanes_per_rep,
                    uint32_t *n_tiles);

/* ---- control variate ----------------------------------------------------------------------
 * A variance-reduction layer over the Monte Carlo estimate of E f(w_T) (not part of the paper's
 * method): a surrogate h(x) of Y = f(w_T) from the path's features x (SIM_CV_FEATURES), trained
 * on pairs the simulation generates, and the estimator
 *   Y_cv = mean_r (Y_r - beta h(x_r)) + beta mean_k h(x'_k),
 * with x'_k drawn from the features' exact law. Y_cv is unbiased for E Y whatever h and beta
 * (both fixed before the run); the plain mean stays the fallback and the check on its bias.
 * The surrogate: F = d + 2 inputs -> 64 -> 64 -> 1, exact GELU (x Phi(x)), parameters flat
 * theta = W1 [64][F], b1 [64], W2 [64][64], b2 [64], w3 [64], b3 (P = 64 F + 4289 floats), matrix
 * products on the matrix cores with bfloat16 operands and FP32 accumulation, FP32 master weights,
 * Adam. */

typedef struct {
    uint32_t n_runs;        /* training simulations, seeds seed, seed+1, ...; >= 1 */
    uint32_t epochs;        /* passes over the training pairs, >= 1 */
    uint64_t R_train;       /* replications per training simulation, >= batch */
    uint64_t R_pilot;       /* replications of the held-out simulation (seed + n_runs) fitting beta */
    uint32_t batch;         /* minibatch rows, a multiple of 128 in [128, 65536] */
    uint32_t reinit;        /* 1: fresh weights (Philox stream domain 3 of seed); 0: continue */
    double lr;              /* Adam step size (beta1 0.9, beta2 0.999, eps 1e-8) */
} sim_cv_opts;

typedef struct {
    uint64_t n_train, steps;
    double ref[SIM_MAX_D];  /* the reference gradient b used for the features: 2 lambda Sigma wbar - mu,
                               wbar the mean of w_T over a plain pilot run (seed + n_runs + 1) */
    double y_mean, y_sd;    /* standardization of the training target */
    double loss_first_epoch, loss_last_epoch;   /* mean squared error of the standardized target */
    double beta, rho2;      /* Cov(Y, h) / Var(h) and Corr(Y, h)^2 on the pilot */
    double pilot_var_y;
    double sim_ms, train_ms, pilot_ms;          /* device time of each phase (HIP events) */
} sim_cv_fit_out;

typedef struct {
    uint64_t R, R_aux;
    double beta;
    double mean_plain, var_plain, ci95_plain;   /* plain Monte Carlo over the same paths */
    double mean_resid, var_resid;               /* Y - beta h(x) */
    double mean_h_aux, var_h_aux;               /* h over the aux draws */
    double mean_cv, var_est, ci95_cv;           /* estimate, its variance, 95% half-width */
    double rho2;                                /* Corr(Y, h)^2 on this run */
    double kernel_ms;                           /* device time: paths, features, h, aux, reductions */
    double paths_ms, aux_ms;                    /* of which the path kernel, and the aux draws with h */
} sim_cv_stats_out;

/* Trains the surrogate for problem p (with T iterations) on the device: fixes the features'
 * reference gradient from a plain pilot run, runs n_runs simulations of R_train replications with
 * features, standardizes Y, takes epochs x (n / batch) Adam steps
 * over minibatches in a fresh affine permutation of the pairs per epoch, then fits beta on a
 * held-out pilot run. Synchronous. Supported problems: those SIM_CV_FEATURES supports. */
int sim_cv_fit(sim_ctx *ctx, const sim_params *p, uint64_t T, uint64_t seed, const sim_cv_opts *o,
               sim_cv_fit_out *out);

/* Control-variate estimate of E f(w_T) from R replications (seed `seed`) and R_aux draws from the
 * features' law (stream domain 2 of `seed`), with the fitted surrogate, beta and reference gradient
 * (p->cv_ref is not read). Synchronous. */
int sim_run_cv(sim_ctx *ctx, const sim_params *p, uint64_t R, uint64_t T, uint64_t seed, uint64_t R_aux,
               sim_cv_stats_out *out);

/* Device pointers to the last sim_run_cv: Y [R], h(x_r) [R], x [F][R], and the last chunk of aux
 * draws x' [F][n_aux] with h(x') [n_aux] (all of them when R_aux <= 4,194,304). */
typedef struct {
    uint64_t R, n_aux;
    uint32_t F, pad_;
    const double *y;
    const float *h, *x, *x_aux, *h_aux;
} sim_cv_view;
int sim_cv_paths(sim_ctx *ctx, sim_cv_view *out);

/* Surrogate primitives (host arrays). set/get: P = 64 F + 4289 parameters, F in [3, 66];
 * forward: raw network outputs of n rows of features x [F][n] (feature-major); grad: the mean
 * squared error against y [n] and its gradient [P] at the current parameters. */
int sim_mlp_set_params(sim_ctx *ctx, uint32_t F, const float *theta);
int sim_mlp_get_params(sim_ctx *ctx, uint32_t F, float *theta);
int sim_mlp_forward(sim_ctx *ctx, const float *x, uint64_t n, float *out);
int sim_mlp_grad(sim_ctx *ctx, const float *x, const float *y, uint64_t n, float *grad, double *loss);

/* Draws k0 .. k0+n-1 from the exact law of the features of problem p (reference gradient
 * p->cv_ref) with T iterations into host x [F][n]: per epoch one 53-bit uniform from Philox block
 * (e/2, 1, k, domain 2 | instance) picks the category by the cumulative p_0, p_1, .... */
int sim_cv_aux_draws(sim_ctx *ctx, const sim_params *p, uint64_t T, uint64_t seed, uint64_t k0, uint64_t n,
                     float *x);

/* The features' law for problem p (reference gradient p->cv_ref) with T iterations, without a
 * device: probs [d+1] (0 origin, j+1 vertex e_j), S2 and S4 (may be NULL). Returns 0 or the code
 * sim_run with SIM_CV_FEATURES would return. */
int sim_cv_law(const sim_params *p, uint64_t T, double *probs, double *S2, double *S4, char *msg, size_t len);

/* ---- Algorithm 1 at the paper's experimental shape -------------------------------------------
 * Section 4.1 runs Algorithm 1 on a single replication of an instance with many assets: d from 5e2
 * to 1e5, N = 25 (50 at d = 1e5) samples per gradient, K = 1500 iterations, mu_j ~ U(-1,1),
 * sigma_j ~ U(0, 0.025), Sigma diagonal. The wide path runs that shape with the parallelism inside a
 * replication: each iteration is four launches (samples and their dot products with v = sigma .* w,
 * the cross-workgroup sums, the gradient of Eq. (4)-(5) with the per-workgroup vertex search, and
 * the global vertex with the update), all sums in a fixed order. The noise is the stream of sim_run:
 * standard normal i d + j of (replication, epoch) for sample i and asset j.
 * Supported: 4 <= d <= SIM_WIDE_MAX_D with d a multiple of 4, diagonal Sigma (chol NULL), Gaussian
 * noise, FP32 state, 2 <= N <= SIM_WIDE_MAX_N, any M, 1 <= R <= SIM_WIDE_MAX_R, R T <= 2^30; flags
 * may hold SIM_KEEP_PATHS and SIM_DECISION_LOG, and the run keeps every per-path record and
 * decision either way. Asynchronous on the context's stream; the host enqueues 4 T (+ checkpoint)
 * launches before returning. */
int sim_run_wide(sim_ctx *ctx, const sim_params *p, uint64_t R, uint64_t T, uint64_t seed);

/* Checks a parameter set exactly as sim_run_wide does, without a device. */
int sim_validate_wide(const sim_params *p, uint64_t R, uint64_t T, char *msg, size_t len);

/* Statistics of the last wide run (as sim_stats; decision_total holds only the origin's total, the
 * per-asset counts are in sim_wide_paths); synchronises the stream. */
int sim_wide_stats(sim_ctx *ctx, sim_stats_out *out);

/* Device pointers (owned by the context) to the records of the last wide run, replication-major. */
typedef struct {
    uint64_t R, T;
    uint32_t d, n_checkpoints;
    const double *y;            /* [R] f(w_T) */
    const double *f_ckpt;       /* [n_checkpoints][R] */
    const uint32_t *cnt;        /* [R][d+1] decision counts, origin first */
    const uint64_t *wsum;       /* [R][d] sum of (t+1) over the steps choosing e_j */
    const uint32_t *tau;        /* [R] hitting step or SIM_TAU_NONE */
    const uint32_t *decisions;  /* [R][T] decisions, 0 = origin, j+1 = e_j */
} sim_wide_view;

int sim_wide_paths(sim_ctx *ctx, sim_wide_view *out);

/* ---- Algorithm 2: the multi-product newsvendor (Section 3.2, Task 2) -------------------------
 * Products j = 1..n with demand N(mu_j, sigma_j^2), unit cost k_j, holding cost h_j (negative: a
 * scrap value) and selling value v_j; cost Eq. (6) f_j(x) = k x + h E(x - xi)^+ + v E(xi - x)^+;
 * problem Eq. (7) over X = {c'x <= C, x >= 0} (one resource row, c > 0), whose vertices are the
 * origin and (C/c_j) e_j; gradient Eq. (9): k_j - v_j + (h_j + v_j) #{s : d_j^(s) <= x_j} / S from S
 * demand samples per product, d_j^(s) = mu_j + sigma_j z with z the standard normal s n + j of the
 * (replication, epoch) stream in domain 4; Algorithm 2 with the vertex of smallest g_j / c_j when it
 * is negative (else the origin, lowest index among equal values), step 2/(t+2). Y = f(x_T) and the
 * checkpoints f(x_c) in FP64 from Eq. (6) in closed form. The parallelism is inside a replication
 * (a thread per four products), two launches per iteration. */
typedef struct {
    uint32_t abi_version;       /* SIM_ABI_VERSION */
    uint32_t n;                 /* products, a multiple of 4 in [4, SIM_NV_MAX_N] */
    const double *mu;           /* [n] demand means */
    const double *sigma;        /* [n] demand standard deviations >= 0 */
    const double *k;            /* [n] unit costs */
    const double *h;            /* [n] holding costs per unit */
    const double *v;            /* [n] selling values per unit */
    const double *c;            /* [n] resource use per unit, > 0 */
    double C;                   /* resource level, > 0 */
    const double *x0;           /* [n] starting point in X, or NULL for the origin */
    uint32_t n_samples;         /* S: demand samples per product and resample, 1..SIM_NV_MAX_S */
    uint32_t resample_every;    /* M >= 1 */
    uint32_t n_checkpoints;     /* 0..SIM_MAX_CKPT */
    uint32_t instance_id;       /* stream instance, < 2^24 */
    uint64_t checkpoints[SIM_MAX_CKPT]; /* strictly increasing iterate counts in [1, T] */
    double gap_eps;             /* Frank-Wolfe gap threshold of tau, >= 0 */
} sim_nv_params;

/* Runs R replications (1 <= R <= SIM_WIDE_MAX_R, R T <= 2^30) of Algorithm 2 for T iterations with
 * noise seed `seed`. Asynchronous on the context's stream. Results: sim_nv_stats (f_star NaN,
 * decision_total holds the origin's total only) and sim_nv_paths (the records of sim_wide_view, with
 * products in place of assets: cnt [R][n+1], wsum [R][n], x_T = (C/c) .* 2 wsum / (T (T+1))). */
int sim_run_newsvendor(sim_ctx *ctx, const sim_nv_params *p, uint64_t R, uint64_t T, uint64_t seed);

/* Checks a parameter set exactly as sim_run_newsvendor does, without a device. */
int sim_validate_newsvendor(const sim_nv_params *p, uint64_t R, uint64_t T, char *msg, size_t len);

int sim_nv_stats(sim_ctx *ctx, sim_stats_out *out);
int sim_nv_paths(sim_ctx *ctx, sim_wide_view *out);

/* Algorithm 2 over Eq. (7)'s general constraint set X = {A x <= C, x >= 0} with M resource rows.
 * The linear subproblem min_{s in X} s'g is solved on the device each iteration. The solver is the
 * revised simplex in FP64 on the standard form [A I][s; slack] = C, one workgroup per replication,
 * started from the slack basis each iteration. It
 * enters the column of most negative reduced cost (lowest index among equal ones), switching to the
 * lowest index with a negative reduced cost (Bland's rule) after 2M + 2 degenerate pivots in a row.
 * It leaves by the smallest ratio (lowest basis position among equal ones), with at most
 * SIM_NV_LP_MAX_PIVOTS pivots per iteration. The gradient is Eq. (9) in FP64 from the same demand
 * samples as sim_run_newsvendor, compared with x_j in FP64. The iterate x is kept in FP64 and
 * updated as x + gamma (s - x) with gamma = 2/(t+2), separately rounded (no fused operations).
 * Y = f(x_T) and the checkpoints f(x_c) come from Eq. (6).
 * The params' c and C are not used (c may be NULL). Requires: 1 <= M <= SIM_NV_MAX_RES, A >= 0
 * with a positive entry in every column (X is then bounded), C > 0, x0 in X, n <= SIM_NV_LP_MAX_N,
 * R T <= 2^24. Asynchronous on the context's stream. Results: sim_nv_lp_stats (f_star NaN;
 * decision_total[0] counts the iterations whose vertex is the origin) and sim_nv_lp_paths. */
#define SIM_NV_MAX_RES 8u
#define SIM_NV_LP_MAX_N 262144u
#define SIM_NV_LP_MAX_PIVOTS 64u
typedef struct {
    uint32_t n_resources;       /* M */
    uint32_t pad_;
    const double *A;            /* [M][n] row-major resource use per unit */
    const double *C;            /* [M] resource levels */
} sim_nv_constraints;

int sim_run_newsvendor_lp(sim_ctx *ctx, const sim_nv_params *p, const sim_nv_constraints *con, uint64_t R,
                          uint64_t T, uint64_t seed);
int sim_validate_newsvendor_lp(const sim_nv_params *p, const sim_nv_constraints *con, uint64_t R, uint64_t T,
                               char *msg, size_t len);

typedef struct {
    uint64_t R, T;
    uint32_t n, n_resources, n_checkpoints, pad_;
    const double *y;            /* [R] f(x_T) */
    const double *f_ckpt;       /* [n_checkpoints][R] */
    const double *x;            /* [R][n] x_T */
    const uint32_t *tau;        /* [R] first iteration with Frank-Wolfe gap <= gap_eps, or SIM_TAU_NONE */
    const uint32_t *basis;      /* [R][T][M] the optimal basis of each iteration: j < n product j, n + i slack i */
    const double *value;        /* [R][T][M] the basic variables' values: the vertex s has s_j = value where basis = j */
    const uint32_t *pivots;     /* [R][T] pivots taken; SIM_NV_LP_MAX_PIVOTS + 1 marks a subproblem left unsolved */
} sim_nv_lp_view;

int sim_nv_lp_stats(sim_ctx *ctx, sim_stats_out *out);
int sim_nv_lp_paths(sim_ctx *ctx, sim_nv_lp_view *out);

/* ---- Algorithms 3-4: stochastic quasi-Newton classification (Section 3.3, Task 3) ------------
 * Logistic loss Eq. (10)-(11), F(w) = (1/N) sum_i log(1 + e^{-x_i'w}) + (1 - z_i) x_i'w, over N rows
 * of n binary features; mini-batch gradient Eq. (12) over b rows; sub-sampled Hessian Eq. (13) over
 * b_H rows, applied to s; Algorithm 3 with alpha_k = beta / k, plain gradient steps for k <= 2L,
 * steps along -H_t g after that, a correction pair (s_t, y_t) every L iterations from the second
 * window on, the M newest kept; H_t is Algorithm 4's BFGS matrix from gamma I, gamma = s_t'y_t /
 * y_t'y_t (applied to g through its compact representation, never formed). Rows are drawn
 * uniformly with replacement: index floor(u N / 2^32) for the 32-bit Philox words u of counter
 * (q/4, k, replication, 5 << 24 | instance) for the gradient rows of iteration k and
 * (q/4, k, replication, 6 << 24 | instance) for the Hessian rows of the pair closed at iteration k.
 * w^1 = 0. FP64 throughout. */

/* Uploads the data set (host memory, copied; the previous one is replaced): X [N][n] row-major
 * features, each 0 or 1, and z [N] labels, each 0 or 1. 1 <= n <= SIM_SQN_MAX_N, 1 <= N < 2^31,
 * N n < 2^40. Errors: SIM_EINVAL for sizes or any other byte value (nothing is uploaded),
 * SIM_ENOMEM, SIM_EDEVICE. Synchronous. */
int sim_sqn_load(sim_ctx *ctx, const uint8_t *X, const uint8_t *z, uint64_t N, uint32_t n);

typedef struct {
    uint32_t abi_version;       /* SIM_ABI_VERSION */
    uint32_t L;                 /* iterations per window, >= 1 */
    uint32_t M;                 /* pairs kept, 1..SIM_SQN_MAX_M */
    uint32_t b, b_H;            /* sample sizes, 1..SIM_SQN_MAX_B */
    uint32_t n_checkpoints;     /* 0..SIM_MAX_CKPT */
    uint32_t instance_id;       /* stream instance, < 2^24 */
    uint32_t pairs_fp32;        /* 1: keep the correction pairs in binary32 (s rounded before y is
                                   formed from it, y rounded when stored; half the bytes of the two
                                   passes over them per iteration), 0: binary64 */
    double beta;                /* step alpha_k = beta / k, finite and > 0 */
    uint64_t checkpoints[SIM_MAX_CKPT]; /* strictly increasing iterations k in [1, K]: F(w^{k+1}) */
} sim_sqn_params;

/* Runs R replications (1 <= R <= SIM_SQN_MAX_R) of Algorithm 3 for K iterations (1 <= K < 2^32) on
 * the loaded data with sample seed `seed`, then evaluates F at every checkpoint and at w^{K+1}.
 * Asynchronous on the context's stream. SIM_ESTATE without data. */
int sim_run_sqn(sim_ctx *ctx, const sim_sqn_params *p, uint64_t R, uint64_t K, uint64_t seed);

/* The same run (Algorithm 3 with Algorithm 4's H_t, Section 3.3) for few replications, each spread
 * over many workgroups: every workgroup owns a 256-feature slice of w, of the gradient and of the
 * stored pairs, and the dot products that need the whole vector (the sampled rows' x_i'w, S'g and
 * Y'g, the new pair's products) are summed over the slices in a following launch, in slice order.
 * One to two launches per iteration and three more at the end of a window. sim_run_sqn keeps one
 * workgroup per replication, which streams the stored pairs through a single compute unit; this
 * entry point is for the paper's single runs. Results differ from sim_run_sqn's only in the order
 * of those sums (the sampled rows are the same). Same parameters, outputs (sim_sqn_stats,
 * sim_sqn_paths, sim_sqn_hessian) and errors as sim_run_sqn, and 1 <= R <= SIM_SQN_SPLIT_MAX_R
 * (else SIM_EINVAL). Asynchronous on the context's stream; the host issues every launch. */
#define SIM_SQN_SPLIT_MAX_R 64
int sim_run_sqn_split(sim_ctx *ctx, const sim_sqn_params *p, uint64_t R, uint64_t K, uint64_t seed);

/* Checks a parameter set exactly as sim_run_sqn does for data of N rows and n features, without a
 * device. */
int sim_validate_sqn(const sim_sqn_params *p, uint64_t N, uint32_t n, uint64_t R, uint64_t K, char *msg,
                     size_t len);

/* Statistics of the last SQN run over replications: Y = F(w^{K+1}), f_mean / f_sd at the
 * checkpoints, rse of Table 2 ((F_c - Y) / F_c)^2; T holds K, f_star is NaN, kernel_ms the
 * iterations' device time (the loss evaluations excluded), path_steps_per_s R K / that time.
 * Synchronises the stream. */
int sim_sqn_stats(sim_ctx *ctx, sim_stats_out *out);

/* Device pointers (owned by the context) to the records of the last SQN run. */
typedef struct {
    uint64_t R, K;
    uint32_t n, ld;             /* features; stride of w (a multiple of 4, entries n..ld-1 are 0) */
    uint32_t n_checkpoints, pad_;
    const double *F;            /* [R] F(w^{K+1}) */
    const double *F_ckpt;       /* [n_checkpoints][R] */
    const double *w;            /* [R][ld] w^{K+1} */
    const double *w_ckpt;       /* [n_checkpoints][R][ld] */
    const uint32_t *pairs;      /* [R] correction pairs computed */
    uint32_t M;                 /* ring slots per replication */
    uint32_t pairs_fp32;        /* element type of S and Y: 1 float, 0 double */
    const void *S, *Y;          /* [R][M][ld] the stored pairs; with P = pairs[r], the min(P, M) newest,
                                   the oldest at slot (P >= M ? P mod M : 0), then cyclically */
} sim_sqn_view;

int sim_sqn_paths(sim_ctx *ctx, sim_sqn_view *out);

/* Algorithm 4's matrix H_t formed explicitly: gamma I and the BFGS updates over the m = min(P, M)
 * pairs that replication `rep` of the last SQN run holds (the matrix its next iteration would
 * apply), as H = gamma I + U W U' with U = [S, gamma Y] and the 2m x 2m middle matrix W of the
 * compact representation, the n x n product on the FP64 matrix cores. Synchronous. Errors:
 * SIM_ESTATE without a run or when the replication has no pair yet, SIM_EINVAL for rep >= R. */
typedef struct {
    uint32_t n, m;
    uint32_t ld, pad_;          /* row stride of H: n rounded up to a multiple of 16 (128-byte rows) */
    double gamma;               /* s_t'y_t / y_t'y_t of the newest pair */
    const double *H;            /* device, [n][ld] row-major (columns n..ld-1 unset), owned by the
                                   context until the next call */
    double device_ms;           /* the four launches, HIP events */
} sim_sqn_hessian_view;

int sim_sqn_hessian(sim_ctx *ctx, uint64_t rep, sim_sqn_hessian_view *out);

/* Statistics of the last run; synchronises the stream. */
int sim_stats(sim_ctx *ctx, sim_stats_out *out);

/* Per-path records of the last run (device pointers); synchronises the stream. */
int sim_paths(sim_ctx *ctx, sim_path_view *out);

/* Copies `bytes` from a device pointer returned by sim_paths into host memory. */
int sim_copy_to_host(sim_ctx *ctx, void *host_dst, const void *device_src, size_t bytes);

/* Static description of an error code, and the last detailed message of a context. */
const char *sim_strerror(int code);
int sim_last_error(sim_ctx *ctx, char *buf, size_t len);

/* Frees every device allocation of the context. Safe on NULL. */
void sim_destroy(sim_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
