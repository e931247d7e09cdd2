/*
 * oracle.c -- plain serial FP64 CPU oracle (test infrastructure only; see oracle.h).
 *
 * Follows Section 3.1 of He, Liu, Wu, Zheng and Zhu step by step:
 *   problem      Eq. (3):  f(w) = lambda w' Sigma w - w' mu on W = {w >= 0, 1'w <= 1}
 *   estimator    Eq. (4)-(5): Rbar = mean of the N samples, centred covariance with N-1
 *   algorithm    Algorithm 1: resample every M iterations, gradient, linear subproblem over W,
 *                step 2/(kM+m+2), update w + gamma (s - w), return the last iterate.
 * The risk coefficient lambda reads Eq. (3) (lambda = 1/2) and Eq. (4) (lambda = 1) as one
 * family; the gradient of the sample objective is 2 lambda Sigma_hat w - Rbar.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
 * SC'11): ten rounds of two 32x32->64 multiplications and xors on a 4-word counter, with a
 * 2-word key bumped by two Weyl constants between rounds.
 * ------------------------------------------------------------------------------------------- */
static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u; /* golden ratio */
static const uint32_t PHILOX_W1 = 0xBB67AE85u; /* sqrt(3) - 1 */

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)x0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += PHILOX_W0;
        k1 += PHILOX_W1;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

double or_uniform(uint32_t x)
{
    /* odd multiples of 2^-24 strictly inside (0,1); exact in binary32 and binary64 */
    uint32_t k = x & 0x7FFFFFu;
    return ((double)(2u * k + 1u)) * ldexp(1.0, -24);
}

/* Normal number q of a stream: Philox block q/4 with counter (block, epoch, rep, domain|inst);
 * words (x0,x1) give the Box-Muller pair (z0, z1), words (x2,x3) give (z2, z3). */
void or_normals(uint64_t seed, uint32_t domain, uint32_t instance, uint64_t rep,
                uint64_t epoch, uint64_t q0, uint64_t n, double *out)
{
    const double two_pi = 6.283185307179586476925286766559;
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (uint64_t k = 0; k < n; ++k) {
        uint64_t q = q0 + k;
        uint32_t ctr[4] = {(uint32_t)(q / 4), (uint32_t)epoch, (uint32_t)rep,
                           (domain << 24) | (instance & 0xFFFFFFu)};
        uint32_t x[4];
        or_philox4x32_10(ctr, key, x);
        int pair = (int)((q % 4) / 2);
        double u1 = or_uniform(x[2 * pair]);
        double u2 = or_uniform(x[2 * pair + 1]);
        double radius = sqrt(-2.0 * log(u1));
        out[k] = (q % 2 == 0) ? radius * cos(two_pi * u2) : radius * sin(two_pi * u2);
    }
}

/* ---------------------------------------------------------------------------------------------
 * Sampling: N i.i.d. returns R_i = mu + L y_i (Section 3.1, R ~ N(mu, Sigma) with Sigma = L L').
 * Gaussian noise: y_i = z_i. Student-t noise: y_i = z_i sqrt((nu-2)/chi2_nu,i), the elliptical
 * t scaled to unit covariance, chi2 from nu extra normals per sample (normals N d + nu i + k).
 * ------------------------------------------------------------------------------------------- */
static void draw_returns(const or_problem *p, uint64_t rep, uint64_t epoch, double *Rmat,
                         double *noise /* N*d: y_i, the unit-covariance noise of each return */,
                         double *zraw /* NULL or N*d: the Gaussian numerators z_i */)
{
    const int d = p->d, N = p->N;
    const uint64_t n_main = (uint64_t)N * (uint64_t)d;
    const uint64_t n_extra = (p->noise == OR_NOISE_T) ? (uint64_t)N * (uint64_t)p->nu : 0;
    double *z = (double *)malloc(sizeof(double) * (size_t)(n_main + n_extra));
    double *y = (double *)malloc(sizeof(double) * (size_t)d);
    or_normals(p->seed, OR_DOMAIN_PATH, p->instance, rep, epoch, 0, n_main + n_extra, z);
    for (int i = 0; i < N; ++i) {
        double scale = 1.0;
        if (p->noise == OR_NOISE_T) {
            double chi2 = 0.0;
            for (int k = 0; k < p->nu; ++k) {
                double e = z[n_main + (uint64_t)p->nu * (uint64_t)i + (uint64_t)k];
                chi2 += e * e;
            }
            scale = sqrt((double)(p->nu - 2) / chi2);
        }
        for (int j = 0; j < d; ++j) y[j] = scale * z[(uint64_t)i * d + j];
        if (zraw)
            for (int j = 0; j < d; ++j) zraw[(size_t)i * d + j] = z[(uint64_t)i * d + j];
        for (int j = 0; j < d; ++j) {
            double acc = 0.0;
            for (int k = 0; k <= j; ++k) acc += p->chol[j * d + k] * y[k];
            noise[(size_t)i * d + j] = y[j];
            Rmat[(size_t)i * d + j] = p->mu[j] + acc;
        }
    }
    free(y);
    free(z);
}

/* Eq. (5) and Eq. (4): Rbar, D_i = R_i - Rbar, Sigma_hat w = (1/(N-1)) sum_i D_i (D_i' w). */
static void sample_statistics(const or_problem *p, const double *Rmat, const double *w,
                              double *rbar, double *sigma_w)
{
    const int d = p->d, N = p->N;
    for (int j = 0; j < d; ++j) {
        double acc = 0.0;
        for (int i = 0; i < N; ++i) acc += Rmat[(size_t)i * d + j];
        rbar[j] = acc / (double)N;
    }
    for (int j = 0; j < d; ++j) sigma_w[j] = 0.0;
    for (int i = 0; i < N; ++i) {
        double proj = 0.0;
        for (int j = 0; j < d; ++j) proj += (Rmat[(size_t)i * d + j] - rbar[j]) * w[j];
        for (int j = 0; j < d; ++j) sigma_w[j] += (Rmat[(size_t)i * d + j] - rbar[j]) * proj;
    }
    for (int j = 0; j < d; ++j) sigma_w[j] /= (double)(N - 1);
}

void or_draw_returns(const or_problem *p, uint64_t rep, uint64_t epoch, double *Rmat)
{
    double *noise = (double *)malloc(sizeof(double) * (size_t)p->N * p->d);
    draw_returns(p, rep, epoch, Rmat, noise, NULL);
    free(noise);
}

void or_sample_gradient(const or_problem *p, uint64_t rep, uint64_t epoch, const double *w,
                        double *grad, double *rbar, double *sigma_w)
{
    const int d = p->d, N = p->N;
    double *Rmat = (double *)malloc(sizeof(double) * (size_t)N * d);
    double *noise = (double *)malloc(sizeof(double) * (size_t)N * d);
    draw_returns(p, rep, epoch, Rmat, noise, NULL);
    sample_statistics(p, Rmat, w, rbar, sigma_w);
    for (int j = 0; j < d; ++j) grad[j] = 2.0 * p->lambda * sigma_w[j] - rbar[j];
    free(noise);
    free(Rmat);
}

double or_objective(const or_problem *p, const double *w)
{
    const int d = p->d;
    double quad = 0.0, lin = 0.0;
    for (int k = 0; k < d; ++k) {          /* (L' w)_k = sum_{j >= k} L_jk w_j */
        double v = 0.0;
        for (int j = k; j < d; ++j) v += p->chol[j * d + k] * w[j];
        quad += v * v;
    }
    for (int j = 0; j < d; ++j) lin += p->mu[j] * w[j];
    return p->lambda * quad - lin;
}

/* The epoch's reference decision for the control-variate features (see cv.c): the vertex the
 * linear subproblem picks for the fixed gradient cv_ref perturbed by this epoch's sample-mean noise,
 * cv_ref_j - L_jj zbar_j (lowest index among equal minima, the origin when the minimum is >= 0), and
 * the gap between its value and the next best. For a diagonal L this is cv_ref - L zbar; for a
 * dense factor each noise coordinate is read against its own diagonal entry, which keeps the
 * decisions' law in product form. */
static int cv_reference_decision(const or_problem *p, const double *z, double *zbar, double *vals,
                                 double *margin)
{
    const int d = p->d, N = p->N;
    for (int j = 0; j < d; ++j) {
        double s = 0.0;
        for (int i = 0; i < N; ++i) s += z[(size_t)i * d + j];
        zbar[j] = s / (double)N;
    }
    vals[0] = 0.0;                                   /* the origin */
    for (int j = 0; j < d; ++j) vals[j + 1] = p->cv_ref[j] - p->chol[j * d + j] * zbar[j];
    int best = 1;
    for (int c = 2; c <= d; ++c)
        if (vals[c] < vals[best]) best = c;
    const int pick = (vals[best] < 0.0) ? best : 0;
    double second = INFINITY;
    for (int c = 0; c <= d; ++c)
        if (c != pick && vals[c] < second) second = vals[c];
    *margin = second - vals[pick];
    return pick;
}

/* Rounding bound of a system that evaluates the sample gradient of Eq. (4)-(5) at w with unit
 * roundoff uroff (0: no bound), every sum taken in absolute values. It follows the gradient through
 * the noise coordinates y of R_i = mu + L y_i, which covers both evaluation orders a system may use:
 * return space (Sigma_hat w from the centred R_i) and noise space (L applied to sums of y, with
 * v = L'w); for a diagonal L the two coincide. The factor 8 (N + d + 8) is the accumulation depth
 * of the longest sum times a safety factor. vabs, habs: d doubles of work space; pabs: N. */
static double gradient_rounding_bound(const or_problem *p, const double *noise, const double *w, const double *g,
                                      double uroff, double *vabs, double *pabs, double *habs)
{
    const int d = p->d, N = p->N;
    if (!(uroff > 0.0)) return 0.0;
    const double kappa = 8.0 * (double)(N + d + 8);
    double amax = 0.0;
    double wabs = 0.0;
    for (int j = 0; j < d; ++j) wabs += fabs(w[j]);
    for (int m = 0; m < d; ++m) {            /* |L|' |w| */
        double acc = 0.0;
        for (int l = m; l < d; ++l) acc += fabs(p->chol[l * d + m]) * fabs(w[l]);
        vabs[m] = acc;
    }
    for (int i = 0; i < N; ++i) {            /* |y_i|' |L|' |w| */
        double acc = 0.0;
        for (int m = 0; m < d; ++m) acc += fabs(noise[(size_t)i * d + m]) * vabs[m];
        pabs[i] = acc;
    }
    for (int k = 0; k < d; ++k) {
        double quad = 0.0, lin = 0.0;
        for (int i = 0; i < N; ++i) {
            quad += fabs(noise[(size_t)i * d + k]) * pabs[i];
            lin += fabs(noise[(size_t)i * d + k]);
        }
        habs[k] = 2.0 * p->lambda * quad / (double)(N - 1) + lin / (double)N;
    }
    for (int j = 0; j < d; ++j) {
        double acc = 0.0;
        for (int k = 0; k <= j; ++k) acc += fabs(p->chol[j * d + k]) * habs[k];
        double aj = acc + fabs(p->mu[j]) + fabs(g[j]);
        if (aj > amax) amax = aj;
    }
    return kappa * uroff * amax * (1.0 + wabs);
}

void or_sample_gradient_bound(const or_problem *p, uint64_t rep, uint64_t epoch, const double *w, double uroff,
                              double *grad, double *bound)
{
    const int d = p->d, N = p->N;
    double *Rmat = (double *)malloc(sizeof(double) * (size_t)N * d);
    double *noise = (double *)malloc(sizeof(double) * (size_t)N * d);
    double *rbar = (double *)malloc(sizeof(double) * (size_t)d);
    double *sw = (double *)malloc(sizeof(double) * (size_t)d);
    double *vabs = (double *)malloc(sizeof(double) * (size_t)d);
    double *habs = (double *)malloc(sizeof(double) * (size_t)d);
    double *pabs = (double *)malloc(sizeof(double) * (size_t)N);
    draw_returns(p, rep, epoch, Rmat, noise, NULL);
    sample_statistics(p, Rmat, w, rbar, sw);
    for (int j = 0; j < d; ++j) grad[j] = 2.0 * p->lambda * sw[j] - rbar[j];
    *bound = gradient_rounding_bound(p, noise, w, grad, uroff, vabs, pabs, habs);
    free(pabs);
    free(habs);
    free(vabs);
    free(sw);
    free(rbar);
    free(noise);
    free(Rmat);
}

/* ---------------------------------------------------------------------------------------------
 * Algorithm 1, one replication.
 * ------------------------------------------------------------------------------------------- */
int or_path(const or_problem *p, uint64_t rep, uint64_t T, const uint8_t *replay, double uroff,
            or_path_out *out, uint8_t *decisions)
{
    const int d = p->d, M = p->M;
    if (d < 1 || d > OR_MAX_D || p->N < 2 || M < 1 || T < 1 || p->n_ckpt < 0 ||
        p->n_ckpt > OR_MAX_CKPT || !(p->lambda > 0.0))
        return -1;
    if (p->noise == OR_NOISE_T && p->nu < 3) return -1;
    /* with a schedule, epoch k draws N_k samples: buffers hold the largest */
    int N = p->N;
    const uint64_t n_epochs = (T + (uint64_t)M - 1) / (uint64_t)M;
    if (p->n_sched) {
        N = 0;
        for (uint64_t k = 0; k < n_epochs; ++k) {
            if (p->n_sched[k] < 2) return -1;
            if (p->n_sched[k] > N) N = p->n_sched[k];
        }
    }
    or_problem pe = *p;      /* the problem as epoch k sees it: N = N_k */

    double *Rmat = (double *)malloc(sizeof(double) * (size_t)N * d);
    double *noise = (double *)malloc(sizeof(double) * (size_t)N * d);
    double *w = (double *)malloc(sizeof(double) * (size_t)d);
    double *g = (double *)malloc(sizeof(double) * (size_t)d);
    double *rbar = (double *)malloc(sizeof(double) * (size_t)d);
    double *sw = (double *)malloc(sizeof(double) * (size_t)d);
    double *vals = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    double *vabs = (double *)malloc(sizeof(double) * (size_t)d);
    double *habs = (double *)malloc(sizeof(double) * (size_t)d);
    double *pabs = (double *)malloc(sizeof(double) * (size_t)N);
    double *zraw = (double *)malloc(sizeof(double) * (size_t)N * d);
    double *zbar = (double *)malloc(sizeof(double) * (size_t)d);
    double *rvals = (double *)malloc(sizeof(double) * (size_t)(d + 1));
    int ref_pick = 0;
    double ref_margin = INFINITY;

    memset(out, 0, sizeof(*out));
    out->tau = out->tau_lo = out->tau_hi = OR_TAU_NONE;
    out->first_mismatch = -1;
    out->min_margin = INFINITY;
    for (int j = 0; j < d; ++j) w[j] = p->w0 ? p->w0[j] : 0.0;   /* initialize w_0 */

    int ck = 0;
    for (uint64_t t = 0; t < T; ++t) {
        const uint64_t epoch = t / (uint64_t)M;        /* k = t div M, m = t mod M */
        if (t % (uint64_t)M == 0) {                    /* resample */
            if (p->n_sched) pe.N = p->n_sched[epoch];
            draw_returns(&pe, rep, epoch, Rmat, noise, zraw);
            if (p->cv_ref) ref_pick = cv_reference_decision(&pe, zraw, zbar, rvals, &ref_margin);
        }
        if (p->cv_ref) {                       /* weights (t+1)^2 and (t+1) on this epoch's pick */
            const double wt = (double)(t + 1) * (double)(t + 1);
            out->cv_count[ref_pick] += wt;
            out->cv_count1[ref_pick] += (double)(t + 1);
            if (ref_margin < OR_CV_AMBIGUOUS) out->cv_amb += wt;
        }

        /* gradient of the sample objective at w_m */
        sample_statistics(&pe, Rmat, w, rbar, sw);
        for (int j = 0; j < d; ++j) g[j] = 2.0 * p->lambda * sw[j] - rbar[j];

        /* linear subproblem over W: its vertices are the origin and e_1..e_d, so the minimiser
         * is e_j for the smallest g_j when that value is negative, else the origin; equal minima
         * go to the lowest index and a zero minimum to the origin. */
        int jmin = 0;
        for (int j = 1; j < d; ++j)
            if (g[j] < g[jmin]) jmin = j;
        int a = (g[jmin] < 0.0) ? jmin + 1 : 0;
        vals[0] = 0.0;
        for (int j = 0; j < d; ++j) vals[j + 1] = g[j];
        double best = vals[a], second = INFINITY;
        for (int c = 0; c <= d; ++c)
            if (c != a && vals[c] < second) second = vals[c];
        double margin = second - best;
        if (margin < out->min_margin) out->min_margin = margin;

        const double bound = gradient_rounding_bound(&pe, noise, w, g, uroff, vabs, pabs, habs);
        int ambiguous = (margin <= 2.0 * bound);
        if (ambiguous) out->n_ambiguous++;
        if (replay && replay[t] != (uint8_t)a) {
            int r = replay[t];
            if (ambiguous && r <= d && vals[r] <= best + 2.0 * bound) {
                a = r;
                out->n_replayed++;
            } else {
                out->n_mismatch++;
                if (out->first_mismatch < 0) out->first_mismatch = (int64_t)t;
            }
        }
        if (decisions) decisions[t] = (uint8_t)a;

        /* Frank-Wolfe gap g'(w - s) and its first passage below eps */
        double gw = 0.0, wabs = 0.0;
        for (int j = 0; j < d; ++j) { gw += g[j] * w[j]; wabs += fabs(w[j]); }
        double gap = gw - (g[jmin] < 0.0 ? g[jmin] : 0.0);
        double gap_bound = bound * (1.0 + wabs);
        if (out->tau == OR_TAU_NONE && gap <= p->gap_eps) out->tau = (uint32_t)t;
        if (out->tau_lo == OR_TAU_NONE && gap <= p->gap_eps + gap_bound) out->tau_lo = (uint32_t)t;
        if (out->tau_hi == OR_TAU_NONE && gap <= p->gap_eps - gap_bound) out->tau_hi = (uint32_t)t;

        /* step size 2/(kM+m+2) and the update w + gamma (s - w) */
        double gamma = 2.0 / ((double)t + 2.0);
        for (int j = 0; j < d; ++j) {
            double s = (a == j + 1) ? 1.0 : 0.0;
            w[j] = w[j] + gamma * (s - w[j]);
        }
        out->cnt[a] += 1;
        if (a > 0) out->wsum[a - 1] += t + 1;

        while (ck < p->n_ckpt && (uint64_t)p->ckpt[ck] == t + 1) {
            out->f_ckpt[ck] = or_objective(p, w);
            ++ck;
        }
    }
    out->y = or_objective(p, w);   /* return w: the outcome is f at the last iterate */

    double tt = (double)T * (double)(T + 1);
    for (int j = 0; j < d; ++j) {
        double closed = 2.0 * (double)out->wsum[j] / tt;
        double e = fabs(w[j] - closed);
        if (e > out->identity_err) out->identity_err = e;
    }
    free(rvals); free(zbar); free(zraw);
    free(pabs); free(habs); free(vabs);
    free(vals); free(sw); free(rbar); free(g); free(w); free(noise); free(Rmat);
    return 0;
}

int or_run_range(const or_problem *p, uint64_t r0, uint64_t r1, uint64_t T, or_path_out *out)
{
    for (uint64_t r = r0; r < r1; ++r) {
        int rc = or_path(p, r, T, NULL, 0.0, &out[r - r0], NULL);
        if (rc) return rc;
    }
    return 0;
}

/* ---------------------------------------------------------------------------------------------
 * Cross-path statistics: Neumaier-compensated sums, two-pass variance.
 * ------------------------------------------------------------------------------------------- */
typedef struct { double s, c; } nsum;

static void nsum_add(nsum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double nsum_get(const nsum *a) { return a->s + a->c; }

void or_reduce(const or_problem *p, uint64_t T, const or_path_out *paths, uint64_t n,
               or_stats *st)
{
    memset(st, 0, sizeof(*st));
    st->R = n;
    st->T = T;
    if (n == 0) return;
    nsum s = {0, 0};
    st->ymin = INFINITY;
    st->ymax = -INFINITY;
    for (uint64_t r = 0; r < n; ++r) {
        nsum_add(&s, paths[r].y);
        if (paths[r].y < st->ymin) st->ymin = paths[r].y;
        if (paths[r].y > st->ymax) st->ymax = paths[r].y;
    }
    st->mean = nsum_get(&s) / (double)n;
    nsum q = {0, 0};
    for (uint64_t r = 0; r < n; ++r) {
        double e = paths[r].y - st->mean;
        nsum_add(&q, e * e);
    }
    st->var = n > 1 ? nsum_get(&q) / (double)(n - 1) : 0.0;
    st->ci95 = 1.96 * sqrt(st->var / (double)n);

    for (int c = 0; c < p->n_ckpt; ++c) {
        nsum fs = {0, 0}, rs = {0, 0};
        uint64_t nr = 0;
        for (uint64_t r = 0; r < n; ++r) {
            double f = paths[r].f_ckpt[c];
            nsum_add(&fs, f);
            if (f != 0.0) {
                double e = (f - paths[r].y) / f;     /* RSE of Table 2: ((y_t - y*)/y_t)^2 */
                nsum_add(&rs, e * e);
                ++nr;
            }
        }
        st->f_mean[c] = nsum_get(&fs) / (double)n;
        st->rse_undef[c] = n - nr;
        st->rse_mean[c] = nr ? nsum_get(&rs) / (double)nr : 0.0;
        nsum fq = {0, 0}, rq = {0, 0};
        for (uint64_t r = 0; r < n; ++r) {
            double f = paths[r].f_ckpt[c];
            double e = f - st->f_mean[c];
            nsum_add(&fq, e * e);
            if (f != 0.0) {
                double x = (f - paths[r].y) / f;
                double u = x * x - st->rse_mean[c];
                nsum_add(&rq, u * u);
            }
        }
        st->f_sd[c] = n > 1 ? sqrt(nsum_get(&fq) / (double)(n - 1)) : 0.0;
        st->rse_sd[c] = nr > 1 ? sqrt(nsum_get(&rq) / (double)(nr - 1)) : 0.0;
    }
    uint64_t tau_sum = 0;
    for (uint64_t r = 0; r < n; ++r) {
        for (int j = 0; j <= p->d; ++j) st->decision_total[j] += paths[r].cnt[j];
        if (paths[r].tau != OR_TAU_NONE) {
            st->tau_count++;
            tau_sum += paths[r].tau;
        }
    }
    st->tau_mean = st->tau_count ? (double)tau_sum / (double)st->tau_count : 0.0;
}
