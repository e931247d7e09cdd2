/*
 * cv.c -- plain serial FP64 CPU oracle for the control-variate pieces (test infrastructure only;
 * see oracle.h): the law of the path features, draws from that law, the small MLP surrogate
 * (forward and backward written as plain loops), and the control-variate estimator.
 *
 * The surrogate is not part of the paper's method; it is a variance-reduction layer over the
 * Monte Carlo estimate of E f(w_T) from Algorithm 1. Its features summarize the noise each path
 * consumed so that their joint law is known exactly. Per epoch e (E = ceil(T/M) epochs), with
 * zbar_e the sample mean of the epoch's Gaussian numerators:
 *   J_e = the vertex the linear subproblem over W picks for the fixed gradient b - diag(L) zbar_e
 *         (b a reference gradient fixed before the run; diag(L) = sigma for a diagonal factor, each
 *         noise coordinate against its own diagonal entry for a dense one): lowest index among
 *         equal minima, the origin when the minimum is >= 0. zbar_e ~ N(0, I/N) i.i.d. over
 *         epochs, so the J_e are i.i.d. categorical with probabilities p_c given by one-
 *         dimensional integrals (or_cv_pick_probs);
 *   q_e = sum_j sum_i (z_eij - zbar_ej)^2 ~ chi-square(d (N-1)), independent of zbar_e.
 * The summaries are count_c = sum_t (t+1)^2 [J_e(t) = c] (the late iterations weigh most, as in
 * w_T) and count1_c = sum_t (t+1) [J_e(t) = c]; their joint law is that of weighted sums of i.i.d.
 * categorical indicators.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static double std_normal_cdf(double x) { return 0.5 * erfc(-x / sqrt(2.0)); }

/* p_0 = prod_k P(b_k - s_k Z_k >= 0) = prod_k Phi(b_k / s_k);
 * p_{a+1} = P(b_a - s_a Z_a < 0 and below every other value)
 *         = integral over z > b_a / s_a of phi(z) prod_{k != a} Phi((b_k - b_a + s_a z) / s_k) dz,
 * by composite Simpson's rule on [max(b_a/s_a, -12), 12] with 24,000 intervals. */
double or_cv_pick_probs(int d, const double *b, const double *s, double *p)
{
    const double inv_sqrt_2pi = 0.39894228040143267793994605993438;
    double p0 = 1.0;
    for (int k = 0; k < d; ++k) p0 *= std_normal_cdf(b[k] / s[k]);
    p[0] = p0;
    double total = p0;
    for (int a = 0; a < d; ++a) {
        double lo = b[a] / s[a];
        if (lo < -12.0) lo = -12.0;
        const double hi = 12.0;
        double acc = 0.0;
        if (lo < hi) {
            const int n = 24000;
            const double h = (hi - lo) / n;
            for (int i = 0; i <= n; ++i) {
                const double z = lo + h * i;
                double f = inv_sqrt_2pi * exp(-0.5 * z * z);
                for (int k = 0; k < d; ++k)
                    if (k != a) f *= std_normal_cdf((b[k] - b[a] + s[a] * z) / s[k]);
                const double wgt = (i == 0 || i == n) ? 1.0 : ((i % 2) ? 4.0 : 2.0);
                acc += wgt * f;
            }
            acc *= h / 3.0;
        }
        p[a + 1] = acc;
        total += acc;
    }
    return total;
}

void or_cv_weights(uint64_t T, int M, double *w)
{
    for (int i = 0; i < 5; ++i) w[i] = 0.0;
    for (uint64_t t0 = 0; t0 < T; t0 += (uint64_t)M) {
        double w2 = 0.0, w1 = 0.0;
        for (uint64_t t = t0; t < t0 + (uint64_t)M && t < T; ++t) {
            w2 += (double)(t + 1) * (double)(t + 1);
            w1 += (double)(t + 1);
        }
        w[0] += w2;
        w[1] += w2 * w2;
        w[2] += w1;
        w[3] += w1 * w1;
        w[4] += w1 * w2;
    }
}

int or_cv_top(int d, const double *probs)
{
    int top = 0;
    for (int c = 1; c <= d; ++c)
        if (probs[c] > probs[top]) top = c;
    return top;
}

static double standardized(double count, double p, double mean_w, double var_w)
{
    double v = p * (1.0 - p);
    if (v < 1e-4) v = 1e-4;
    return (count - p * mean_w) / sqrt(var_w * v);
}

void or_cv_features(int d, const double *probs, const double *w, const double *count, const double *count1,
                    double *x)
{
    for (int c = 0; c <= d; ++c) x[c == 0 ? d : c - 1] = standardized(count[c], probs[c], w[0], w[1]);
    const int top = or_cv_top(d, probs);
    x[d + 1] = standardized(count1[top], probs[top], w[2], w[3]);
}

/* A uniform in (0,1) with 53 random bits from two words: ((a >> 5) 2^26 + (b >> 6) + 1/2) 2^-53. */
static double uniform53(uint32_t a, uint32_t b)
{
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 0.5) * (1.0 / 9007199254740992.0);
}

void or_cv_aux(const or_problem *p, uint64_t T, const double *probs, uint64_t k, double *count, double *count1)
{
    const int d = p->d, M = p->M;
    uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    for (int c = 0; c <= d; ++c) count[c] = count1[c] = 0.0;
    uint64_t e = 0;
    for (uint64_t t0 = 0; t0 < T; t0 += (uint64_t)M, ++e) {
        /* epoch e: words (2 (e mod 2), 2 (e mod 2) + 1) of block e / 2, epoch word 1 */
        uint32_t ctr[4] = {(uint32_t)(e / 2), 1u, (uint32_t)k, (OR_DOMAIN_CV_AUX << 24) | (p->instance & 0xFFFFFFu)};
        uint32_t w[4];
        or_philox4x32_10(ctr, key, w);
        const double u = (e % 2 == 0) ? uniform53(w[0], w[1]) : uniform53(w[2], w[3]);
        int cat = d;                       /* the smallest c with u < p_0 + ... + p_c */
        double cum = 0.0;
        for (int c = 0; c < d; ++c) {
            cum += probs[c];
            if (u < cum) {
                cat = c;
                break;
            }
        }
        for (uint64_t t = t0; t < t0 + (uint64_t)M && t < T; ++t) {
            count[cat] += (double)(t + 1) * (double)(t + 1);
            count1[cat] += (double)(t + 1);
        }
    }
}

/* ---------------------------------------------------------------------------------------------
 * The surrogate h: F -> 64 -> 64 -> 1 with exact GELU, x Phi(x). Parameters theta, flat:
 *   W1 [64][F], b1 [64], W2 [64][64], b2 [64], w3 [64], b3.
 * With quantize != 0 every operand of the two matrix products (x, W1, h1, W2 in the forward
 * pass; the back-propagated pre-activation gradients, h1, x and W2 in the backward pass) is
 * rounded to bfloat16 (round to nearest even, through binary32), as the matrix cores take them;
 * everything else stays FP64.
 * ------------------------------------------------------------------------------------------- */
double or_bf16(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return v;     /* inf / nan: unchanged */
    u += 0x7FFFu + ((u >> 16) & 1u);
    u &= 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double gelu(double a) { return 0.5 * a * (1.0 + erf(a / sqrt(2.0))); }

static double gelu_grad(double a)
{
    const double inv_sqrt_2pi = 0.39894228040143267793994605993438;
    return 0.5 * (1.0 + erf(a / sqrt(2.0))) + a * inv_sqrt_2pi * exp(-0.5 * a * a);
}

size_t or_mlp_param_count(int F) { return (size_t)64 * F + 64 + 64 * 64 + 64 + 64 + 1; }

typedef struct {
    const double *W1, *b1, *W2, *b2, *w3, *b3;
} mlp_view;

static mlp_view view_of(const double *th, int F)
{
    mlp_view v;
    v.W1 = th;
    v.b1 = v.W1 + 64 * F;
    v.W2 = v.b1 + 64;
    v.b2 = v.W2 + 64 * 64;
    v.w3 = v.b2 + 64;
    v.b3 = v.w3 + 64;
    return v;
}

/* forward of one row; keeps the pre-activations for the backward pass */
static double forward_row(const mlp_view *m, int F, const double *x, int qz, double *a1, double *a2,
                          double *h1, double *h2)
{
    for (int o = 0; o < 64; ++o) {
        double acc = 0.0;
        for (int f = 0; f < F; ++f) {
            const double w = qz ? or_bf16(m->W1[o * F + f]) : m->W1[o * F + f];
            const double xv = qz ? or_bf16(x[f]) : x[f];
            acc += w * xv;
        }
        a1[o] = acc + m->b1[o];
        h1[o] = gelu(a1[o]);
    }
    for (int o = 0; o < 64; ++o) {
        double acc = 0.0;
        for (int i = 0; i < 64; ++i) {
            const double w = qz ? or_bf16(m->W2[o * 64 + i]) : m->W2[o * 64 + i];
            const double hv = qz ? or_bf16(h1[i]) : h1[i];
            acc += w * hv;
        }
        a2[o] = acc + m->b2[o];
        h2[o] = gelu(a2[o]);
    }
    double out = m->b3[0];
    for (int o = 0; o < 64; ++o) out += m->w3[o] * h2[o];
    return out;
}

void or_mlp_forward(const double *theta, int F, const double *x, uint64_t n, int quantize, double *out)
{
    const mlp_view m = view_of(theta, F);
    double a1[64], a2[64], h1[64], h2[64];
    for (uint64_t r = 0; r < n; ++r) out[r] = forward_row(&m, F, x + r * (uint64_t)F, quantize, a1, a2, h1, h2);
}

double or_mlp_grad(const double *theta, int F, const double *x, const double *y, uint64_t n, int quantize,
                   double *grad)
{
    const mlp_view m = view_of(theta, F);
    const size_t P = or_mlp_param_count(F);
    for (size_t i = 0; i < P; ++i) grad[i] = 0.0;
    double *gW1 = grad, *gb1 = gW1 + 64 * F, *gW2 = gb1 + 64, *gb2 = gW2 + 64 * 64, *gw3 = gb2 + 64,
           *gb3 = gw3 + 64;
    double a1[64], a2[64], h1[64], h2[64], da2[64], da1[64];
    double loss = 0.0;
    for (uint64_t r = 0; r < n; ++r) {
        const double *xr = x + r * (uint64_t)F;
        const double out = forward_row(&m, F, xr, quantize, a1, a2, h1, h2);
        const double e = out - y[r];
        loss += e * e;
        const double dout = 2.0 * e / (double)n;       /* d/d out of the mean squared error */
        gb3[0] += dout;
        for (int o = 0; o < 64; ++o) {
            gw3[o] += dout * h2[o];
            da2[o] = dout * m.w3[o] * gelu_grad(a2[o]);
            gb2[o] += da2[o];
        }
        for (int o = 0; o < 64; ++o) {
            const double g = quantize ? or_bf16(da2[o]) : da2[o];
            for (int i = 0; i < 64; ++i) gW2[o * 64 + i] += g * (quantize ? or_bf16(h1[i]) : h1[i]);
        }
        for (int i = 0; i < 64; ++i) {
            double acc = 0.0;
            for (int o = 0; o < 64; ++o) {
                const double w = quantize ? or_bf16(m.W2[o * 64 + i]) : m.W2[o * 64 + i];
                acc += w * (quantize ? or_bf16(da2[o]) : da2[o]);
            }
            da1[i] = acc * gelu_grad(a1[i]);
            gb1[i] += da1[i];
        }
        for (int o = 0; o < 64; ++o) {
            const double g = quantize ? or_bf16(da1[o]) : da1[o];
            for (int f = 0; f < F; ++f) gW1[o * F + f] += g * (quantize ? or_bf16(xr[f]) : xr[f]);
        }
    }
    return loss / (double)n;
}

/* ---------------------------------------------------------------------------------------------
 * Control-variate estimator: with h(x) the surrogate, Y_r the outcomes and x'_k independent draws
 * from the exact law of x,
 *   Y_cv = mean_r (Y_r - beta h(x_r)) + beta mean_k h(x'_k),
 * unbiased for E Y whatever h and beta (fixed before the run); its variance is estimated by
 * var(Y - beta h) / R + beta^2 var(h(x')) / R_aux.
 * ------------------------------------------------------------------------------------------- */
static void mean_var(const double *v, uint64_t n, double *mean, double *var)
{
    double s = 0.0;
    for (uint64_t i = 0; i < n; ++i) s += v[i];
    const double m = n ? s / (double)n : 0.0;
    double q = 0.0;
    for (uint64_t i = 0; i < n; ++i) q += (v[i] - m) * (v[i] - m);
    *mean = m;
    *var = n > 1 ? q / (double)(n - 1) : 0.0;
}

void or_cv_beta(const double *Y, const double *H, uint64_t n, double *beta, double *rho2)
{
    double my, vy, mh, vh;
    mean_var(Y, n, &my, &vy);
    mean_var(H, n, &mh, &vh);
    double c = 0.0;
    for (uint64_t i = 0; i < n; ++i) c += (Y[i] - my) * (H[i] - mh);
    c = n > 1 ? c / (double)(n - 1) : 0.0;
    *beta = vh > 0.0 ? c / vh : 0.0;
    *rho2 = (vh > 0.0 && vy > 0.0) ? c * c / (vh * vy) : 0.0;
}

void or_cv_estimate(const double *Y, const double *H, uint64_t n, const double *Haux, uint64_t n_aux,
                    double beta, or_cv_stats *st)
{
    memset(st, 0, sizeof(*st));
    st->n = n;
    st->n_aux = n_aux;
    st->beta = beta;
    mean_var(Y, n, &st->mean_plain, &st->var_plain);
    double *D = (double *)malloc(sizeof(double) * (size_t)(n ? n : 1));
    for (uint64_t i = 0; i < n; ++i) D[i] = Y[i] - beta * H[i];
    mean_var(D, n, &st->mean_resid, &st->var_resid);
    free(D);
    mean_var(Haux, n_aux, &st->mean_h_aux, &st->var_h_aux);
    st->mean_cv = st->mean_resid + beta * st->mean_h_aux;
    st->var_est = st->var_resid / (double)n + beta * beta * st->var_h_aux / (double)n_aux;
    st->ci95_cv = 1.96 * sqrt(st->var_est);
    st->ci95_plain = 1.96 * sqrt(st->var_plain / (double)n);
}
