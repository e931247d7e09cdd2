/*
 * oracle.h -- plain serial FP64 CPU oracle for the batched stochastic
 * Frank-Wolfe mean-variance simulation of He, Liu, Wu, Zheng and Zhu,
 * "A Preliminary Study on Accelerating Simulation Optimization with GPU
 * Implementation" (Section 3.1: problem Eq. (3), sample objective Eq. (4),
 * sample mean Eq. (5), Algorithm 1).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. It shares no code,
 * header, table or constant with the HIP library; both sides implement the
 * counter-based generator (Philox4x32-10, Salmon et al., SC'11) from its
 * published definition.
 *
 * The same library holds the oracles of the paper's other tasks: the wide
 * (one replication, many assets) form of Algorithm 1 (wide.c), Algorithm 2,
 * the multi-product newsvendor (newsvendor.c), Algorithms 3-4, stochastic
 * quasi-Newton classification (sqn.c), and the control-variate pieces (cv.c).
 *
 * Everything here is slow on purpose: one replication at a time, the sample
 * matrix R_i = mu + L y_i formed explicitly, the sample mean and the centred
 * sample covariance applied to w exactly as Eq. (4)-(5) write them, and the
 * iterate updated with the recurrence of Algorithm 1.
 */
#ifndef PAPER_2404_11631_ORACLE_H
#define PAPER_2404_11631_ORACLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MAX_D 64
#define OR_MAX_CKPT 8
#define OR_TAU_NONE 0xFFFFFFFFu

enum { OR_NOISE_GAUSS = 0, OR_NOISE_T = 1 };
enum { OR_DOMAIN_PATH = 0, OR_DOMAIN_PARAM = 1, OR_DOMAIN_CV_AUX = 2, OR_DOMAIN_MLP = 3, OR_DOMAIN_NEWSVENDOR = 4,
       OR_DOMAIN_SQN_GRAD = 5, OR_DOMAIN_SQN_HESS = 6 };

/* One instance of problem Eq. (3) plus the sampling knobs of Algorithm 1. */
typedef struct {
    int32_t d;              /* number of assets, 1..64 */
    int32_t N;              /* samples per resample, >= 2 (Eq. (4) divides by N-1) */
    int32_t M;              /* iterations between resamples, >= 1 */
    int32_t noise;          /* OR_NOISE_GAUSS or OR_NOISE_T */
    int32_t nu;             /* t degrees of freedom (integer >= 3) when noise == OR_NOISE_T */
    int32_t n_ckpt;         /* number of checkpoints, 0..8 */
    uint32_t instance;      /* stream domain for batched instances, < 2^24 */
    uint32_t pad_;
    uint64_t seed;          /* Philox key */
    double lambda;          /* risk coefficient: f(w) = lambda w'Sigma w - mu'w */
    double gap_eps;         /* Frank-Wolfe gap threshold for the hitting time */
    const double *mu;       /* d mean returns */
    const double *chol;     /* d*d row-major lower-triangular L, Sigma = L L' */
    const double *w0;       /* d starting point in W, or NULL for the origin */
    int64_t ckpt[OR_MAX_CKPT]; /* iterate counts in [1, T] at which f(w_t) is recorded */
    const double *cv_ref;   /* d reference gradient of the control-variate features, or NULL */
    /* Algorithm 1 lets the sample size N_k of epoch k adapt to k (the remark on its resampling
     * step): n_sched[k] (>= 2) for every epoch k < ceil(T / M) of a run, or NULL for N throughout */
    const int32_t *n_sched;
} or_problem;

/* reference decisions whose margin is below this are reported as ambiguous (cv_amb) */
#define OR_CV_AMBIGUOUS 1e-4

/* Everything one replication produces. */
typedef struct {
    double y;                       /* f(w_T), Eq. (3) at the returned point */
    double f_ckpt[OR_MAX_CKPT];     /* f(w_c) for each checkpoint c */
    uint32_t cnt[OR_MAX_D + 1];     /* cnt[0]: origin chosen; cnt[j+1]: vertex e_j chosen */
    uint64_t wsum[OR_MAX_D];        /* sum of (t+1) over the steps that chose e_j */
    uint32_t tau;                   /* first step with FW gap <= eps, or OR_TAU_NONE */
    uint32_t tau_lo, tau_hi;        /* range of hitting times consistent with the rounding bound */
    uint64_t n_ambiguous;           /* steps whose LMO margin is within the rounding bound */
    uint64_t n_replayed;            /* ambiguous steps where the replayed decision was adopted */
    uint64_t n_mismatch;            /* unambiguous steps where the replayed decision differs */
    int64_t first_mismatch;         /* step of the first mismatch, or -1 */
    double identity_err;            /* max_j |w_T - 2 wsum/(T(T+1))| (recurrence vs closed form) */
    double min_margin;              /* smallest LMO margin seen along the path */
    /* control-variate raw summaries (cv_ref set): per category c (0 origin, j+1 vertex e_j) the sums
     * of (t+1)^2 and of (t+1) over iterations whose epoch's reference decision is c; the (t+1)^2
     * weight of iterations whose reference margin is below OR_CV_AMBIGUOUS */
    double cv_count[OR_MAX_D + 1];
    double cv_count1[OR_MAX_D + 1];
    double cv_amb;
} or_path_out;

typedef struct {
    uint64_t R, T;
    double mean, var, ci95, ymin, ymax;
    double f_mean[OR_MAX_CKPT], f_sd[OR_MAX_CKPT];
    double rse_mean[OR_MAX_CKPT], rse_sd[OR_MAX_CKPT];
    uint64_t rse_undef[OR_MAX_CKPT];
    uint64_t decision_total[OR_MAX_D + 1];
    uint64_t tau_count;
    double tau_mean;
} or_stats;

/* Philox4x32-10 block function: out = philox(ctr, key). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Uniform in (0,1) from one 32-bit word: (2 (x mod 2^23) + 1) 2^-24. */
double or_uniform(uint32_t x);

/* Standard normals number q0 .. q0+n-1 of stream (seed, domain, instance, rep, epoch). */
void or_normals(uint64_t seed, uint32_t domain, uint32_t instance, uint64_t rep,
                uint64_t epoch, uint64_t q0, uint64_t n, double *out);

/* The N x d sample matrix R_i = mu + L y_i of replication `rep`, epoch `epoch` (row-major). */
void or_draw_returns(const or_problem *p, uint64_t rep, uint64_t epoch, double *Rmat);

/* Sample mean Eq. (5), Sigma_hat w from Eq. (4) and the gradient 2 lambda Sigma_hat w - Rbar
 * for replication `rep`, epoch `epoch`, at a fixed point w. */
void or_sample_gradient(const or_problem *p, uint64_t rep, uint64_t epoch, const double *w,
                        double *grad, double *rbar, double *sigma_w);

/* The same gradient and the rounding bound or_path applies at that point for a system with unit
 * roundoff uroff (2^-24 binary32, 2^-53 binary64): a bound on the error of any evaluation order
 * of Eq. (4)-(5), in return or noise coordinates. */
void or_sample_gradient_bound(const or_problem *p, uint64_t rep, uint64_t epoch, const double *w, double uroff,
                              double *grad, double *bound);

/* True objective Eq. (3) with the risk coefficient lambda: lambda |L'w|^2 - mu'w. */
double or_objective(const or_problem *p, const double *w);

/* One replication of Algorithm 1 for T iterations.
 * replay: NULL, or T decisions (0 = origin, j+1 = e_j) from the system under test. At a step
 *         whose margin is within the rounding bound the replayed decision is adopted when it is
 *         a near-optimal vertex; elsewhere a differing replayed decision is counted as a mismatch
 *         and the oracle keeps its own.
 * uroff:  unit roundoff of the system under test (2^-24 for FP32, 2^-53 for FP64); 0 disables
 *         the bound (exact comparison).
 * decisions: NULL or T bytes receiving the decisions taken. */
int or_path(const or_problem *p, uint64_t rep, uint64_t T, const uint8_t *replay, double uroff,
            or_path_out *out, uint8_t *decisions);

/* Replications [r0, r1): per-path outputs into out[r - r0] (array of r1 - r0). */
int or_run_range(const or_problem *p, uint64_t r0, uint64_t r1, uint64_t T, or_path_out *out);

/* Cross-path statistics of n per-path outputs. */
void or_reduce(const or_problem *p, uint64_t T, const or_path_out *paths, uint64_t n,
               or_stats *st);

/* ---- Algorithm 1 at the paper's experimental shape (wide.c) ----------------------------
 * Many assets (Section 4.1: d up to 1e5), diagonal Sigma = diag(sigma^2), Gaussian noise; the
 * same method and noise streams as or_path, with per-path arrays sized by the caller. */
typedef struct {
    int64_t d;              /* assets, >= 1 */
    int32_t N, M;           /* samples per resample (>= 2), iterations between resamples (>= 1) */
    uint32_t instance;      /* stream domain, < 2^24 */
    int32_t n_ckpt;         /* checkpoints, 0..8 */
    uint64_t seed;          /* Philox key */
    double lambda, gap_eps;
    const double *mu;       /* [d] */
    const double *sigma;    /* [d] */
    const double *w0;       /* [d] or NULL */
    int64_t ckpt[OR_MAX_CKPT];
    /* Algorithm 1 lets the sample size N_k of epoch k adapt to k: n_sched[k] (>= 2) for every
     * epoch k < ceil(T / M) of a run, or NULL for N in every epoch */
    const int32_t *n_sched;
} or_wide_problem;

typedef struct {
    double y;
    double f_ckpt[OR_MAX_CKPT];
    uint32_t *cnt;          /* caller-allocated [d+1]: [0] origin, [j+1] vertex e_j */
    uint64_t *wsum;         /* caller-allocated [d]: sum of (t+1) over the steps choosing e_j */
    uint32_t tau, tau_lo, tau_hi;
    uint32_t pad_;
    uint64_t n_ambiguous, n_replayed, n_mismatch;
    int64_t first_mismatch;
    double identity_err, min_margin;
} or_wide_out;

/* One replication (see or_path for replay, uroff and decisions; decisions here are 32-bit). */
int or_wide_path(const or_wide_problem *p, uint64_t rep, uint64_t T, const uint32_t *replay, double uroff,
                 or_wide_out *out, uint32_t *decisions);

/* The sample gradient of (rep, epoch) at w, and the rounding bound of a system with unit
 * roundoff uroff at that point (NULL to skip). */
void or_wide_gradient(const or_wide_problem *p, uint64_t rep, uint64_t epoch, const double *w, double *g,
                      double uroff, double *bound);

double or_wide_objective(const or_wide_problem *p, const double *w);

/* ---- Algorithm 2: the multi-product newsvendor (newsvendor.c) ---------------------------
 * Section 3.2: products j with demand N(mu_j, sigma_j^2), costs k_j, h_j, v_j (Eq. (6)), one
 * resource row c'x <= C with c > 0 (Eq. (7)), gradient estimate Eq. (9) from S demand samples per
 * product, resampled every M iterations. */
typedef struct {
    int64_t n;              /* products */
    int32_t S, M;           /* samples per product, iterations between resamples */
    uint32_t instance;      /* stream domain, < 2^24 */
    int32_t n_ckpt;
    uint64_t seed;
    double C, gap_eps;      /* resource level, Frank-Wolfe gap threshold */
    const double *mu, *sigma, *k, *h, *v, *c;   /* [n] each */
    const double *x0;       /* [n] starting point in X, or NULL for the origin */
    int64_t ckpt[OR_MAX_CKPT];
} or_nv_problem;

typedef struct {
    double y;               /* f(x_T), Eq. (7) with Eq. (6) in closed form for normal demand */
    double f_ckpt[OR_MAX_CKPT];
    uint32_t *cnt;          /* caller-allocated [n+1]: [0] origin, [j+1] vertex (C/c_j) e_j */
    uint64_t *wsum;         /* caller-allocated [n]: sum of (t+1) over the steps choosing vertex j */
    uint32_t tau, tau_lo, tau_hi;
    uint32_t pad_;
    uint64_t n_ambiguous, n_replayed, n_mismatch;
    int64_t first_mismatch;
    double identity_err, min_margin;
} or_nv_out;

/* One replication of Algorithm 2 (replay, uroff and decisions as in or_path; the bound covers a
 * system that draws the normals and forms x in binary32). */
int or_nv_path(const or_nv_problem *p, uint64_t rep, uint64_t T, const uint32_t *replay, double uroff,
               or_nv_out *out, uint32_t *decisions);

/* The uncertainty of each g_j of Eq. (9) at x for a system that draws the normals in binary32
 * (unit roundoff u): e_j = |h_j + v_j| / S times the number of samples whose normal lies within binary32
 * reach of the threshold (x_j - mu_j)/sigma_j, plus the rounding of g_j itself. */
void or_nv_gradient_bound(const or_nv_problem *p, uint64_t rep, uint64_t epoch, const double *x, double u,
                          double *e);
/* Eq. (9) at x for (rep, epoch): the gradient estimate and (count may be NULL) the sample counts. */
void or_nv_gradient(const or_nv_problem *p, uint64_t rep, uint64_t epoch, const double *x, double *g,
                    uint32_t *count);

/* f(x) = sum_j f_j(x_j), Eq. (6) in closed form for normal demand. */
double or_nv_cost(const or_nv_problem *p, const double *x);

/* ---- Algorithms 3-4: stochastic quasi-Newton classification (sqn.c) ---------------------
 * Section 3.3: logistic loss Eq. (10)-(11) over N rows of n binary features, mini-batch gradient
 * Eq. (12), sub-sampled Hessian Eq. (13), SQN (Algorithm 3) with the explicit BFGS matrix of
 * Algorithm 4. */
typedef struct {
    int64_t n, N;           /* features, rows */
    int32_t L, M, b, bH;    /* window, pair memory, gradient and Hessian sample sizes */
    double beta;            /* step alpha_k = beta / k */
    uint32_t instance;      /* stream instance, < 2^24 */
    int32_t n_ckpt;
    uint64_t seed;
    const uint8_t *X;       /* [N][n] features in {0, 1} */
    const uint8_t *z;       /* [N] labels in {0, 1} */
    int64_t ckpt[OR_MAX_CKPT];   /* iterations k after which F(w^{k+1}) is recorded */
    int32_t pairs_fp32;     /* 1: every stored pair is rounded to binary32 (s before y is formed
                               from it, then y); 0: binary64 */
    int32_t pad_;
} or_sqn_problem;

typedef struct {
    double F;               /* F(w^{K+1}) */
    double F_ckpt[OR_MAX_CKPT];
    double *w;              /* caller-allocated [n]: w^{K+1} */
    int64_t pairs;          /* correction pairs computed */
} or_sqn_out;

/* The sampled rows of iteration k: domain OR_DOMAIN_SQN_GRAD (gradient) or OR_DOMAIN_SQN_HESS. */
void or_sqn_indices(const or_sqn_problem *p, uint64_t rep, uint64_t k, uint32_t domain, uint32_t count,
                    uint32_t *idx);
double or_sqn_loss(const or_sqn_problem *p, const double *w);
void or_sqn_gradient(const or_sqn_problem *p, const uint32_t *idx, uint32_t b, const double *w, double *g);
void or_sqn_hessian_vector(const or_sqn_problem *p, const uint32_t *idx, uint32_t bh, const double *w,
                           const double *v, double *out);
/* Algorithm 4's H_t (n x n, row-major) from m pairs S, Y [m][n], oldest first. */
void or_sqn_hessian_approx(int64_t n, int m, const double *S, const double *Y, double *H);
/* One run of Algorithm 3 for K iterations (replication rep picks the sample streams). */
int or_sqn_run(const or_sqn_problem *p, uint64_t rep, uint64_t K, or_sqn_out *out);

/* ---- control-variate pieces (cv.c) ------------------------------------------------------ */

typedef struct {
    uint64_t n, n_aux;
    double beta;
    double mean_plain, var_plain, ci95_plain;   /* plain Monte Carlo: mean, variance of Y, CI */
    double mean_resid, var_resid;               /* Y - beta h(x) over the paths */
    double mean_h_aux, var_h_aux;               /* h over the draws from the law of x */
    double mean_cv, var_est, ci95_cv;           /* the estimate, its variance, 95% half-width */
} or_cv_stats;

/* Probabilities of the reference decision, p[0] the origin and p[j+1] vertex e_j, for a gradient
 * b - s .* Z with Z ~ N(0, I_d) (s > 0: the standard deviations of the sample-mean noise, sigma / sqrt(N)). */
double or_cv_pick_probs(int d, const double *b, const double *s, double *p);
/* Weights of T iterations in epochs of M: W2_e, W1_e = sums of (t+1)^2 and (t+1) over epoch e;
 * w[0] = S2 = sum_e W2_e, w[1] = S4 = sum_e W2_e^2, w[2] = S1 = sum_e W1_e, w[3] = S11 = sum_e W1_e^2,
 * w[4] = S12 = sum_e W1_e W2_e. */
void or_cv_weights(uint64_t T, int M, double *w);
/* The most probable category (lowest index among equal probabilities). */
int or_cv_top(int d, const double *probs);
/* Standardized features x[0..d+1] from raw summaries: x_j (j < d) for category j+1 and x_d for the
 * origin, (count_c - p_c S2) / sqrt(S4 max(p_c (1 - p_c), 1e-4)); x_{d+1} for the most probable
 * category c*, (count1_c* - p_c* S1) / sqrt(S11 max(p_c* (1 - p_c*), 1e-4)). */
void or_cv_features(int d, const double *probs, const double *w, const double *count, const double *count1,
                    double *x);
/* Draw k (stream domain 2) from the exact joint law of the raw summaries: per epoch a category from
 * probs (one 53-bit uniform). */
void or_cv_aux(const or_problem *p, uint64_t T, const double *probs, uint64_t k, double *count, double *count1);

/* bfloat16 rounding (to nearest even, through binary32). */
double or_bf16(double v);
/* Parameters of the F -> 64 -> 64 -> 1 surrogate: 64 F + 4289. */
size_t or_mlp_param_count(int F);
/* h(x_r) for n rows of F features (row-major). quantize: round matrix-product operands to bf16. */
void or_mlp_forward(const double *theta, int F, const double *x, uint64_t n, int quantize, double *out);
/* Mean squared error of h over n rows against y, and its gradient with respect to theta. */
double or_mlp_grad(const double *theta, int F, const double *x, const double *y, uint64_t n, int quantize,
                   double *grad);

/* beta = Cov(Y, H) / Var(H) and rho^2 = Corr(Y, H)^2. */
void or_cv_beta(const double *Y, const double *H, uint64_t n, double *beta, double *rho2);
/* The control-variate estimate from path outcomes Y, surrogate values H = h(x_r), and surrogate
 * values Haux at draws from the law of x. */
void or_cv_estimate(const double *Y, const double *H, uint64_t n, const double *Haux, uint64_t n_aux,
                    double beta, or_cv_stats *st);

#ifdef __cplusplus
}
#endif
#endif
