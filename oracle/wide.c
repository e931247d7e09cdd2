/*
 * wide.c -- the oracle for Algorithm 1 at the paper's own experimental shape (test infrastructure
 * only; see oracle.h).
 *
 * Section 4.1 runs Algorithm 1 on one replication of an instance with many assets (d from 5e2 to
 * 1e5, N = 25 or 50 samples per gradient, K = 1500 iterations, mu_j ~ U(-1,1), sigma_j ~
 * U(0, 0.025), Sigma diagonal). This file repeats or_path for that shape: Sigma = diag(sigma^2)
 * given as the vector sigma instead of a d x d factor, per-path arrays sized by the caller, and
 * 32-bit decisions. The method, the noise streams and the order of the steps are those of
 * or_path in oracle.c: returns R_i = mu + sigma .* z_i with z_i the standard normals
 * i d + j of the (replication, epoch) stream, the sample mean Eq. (5), the centred sample
 * covariance Eq. (4) applied to w, the gradient 2 lambda Sigma_hat w - Rbar, the vertex search
 * over W, the step 2/(t+2) and the update w + gamma (s - w). With a schedule n_sched, epoch k
 * draws N_k = n_sched[k] returns (the comment of Algorithm 1's resampling step) and its statistics
 * divide by N_k and N_k - 1.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* The returns R_i = mu + sigma .* z_i of one (replication, epoch), N x d row-major, and the
 * standard normals z behind them. */
static int wide_n(const or_wide_problem *p, uint64_t epoch) { return p->n_sched ? p->n_sched[epoch] : p->N; }

static void wide_returns(const or_wide_problem *p, int N, uint64_t rep, uint64_t epoch, double *Rmat, double *z)
{
    const int64_t d = p->d;
    or_normals(p->seed, OR_DOMAIN_PATH, p->instance, rep, epoch, 0, (uint64_t)N * (uint64_t)d, z);
    for (int i = 0; i < N; ++i)
        for (int64_t j = 0; j < d; ++j) Rmat[(size_t)i * d + j] = p->mu[j] + p->sigma[j] * z[(size_t)i * d + j];
}

/* Eq. (5) and Eq. (4): Rbar and Sigma_hat w = (1/(N-1)) sum_i D_i (D_i' w), D_i = R_i - Rbar; the
 * gradient 2 lambda Sigma_hat w - Rbar. */
static void wide_statistics(const or_wide_problem *p, int N, const double *Rmat, const double *w, double *rbar,
                            double *sw, double *g)
{
    const int64_t d = p->d;
    for (int64_t j = 0; j < d; ++j) {
        double acc = 0.0;
        for (int i = 0; i < N; ++i) acc += Rmat[(size_t)i * d + j];
        rbar[j] = acc / (double)N;
        sw[j] = 0.0;
    }
    for (int i = 0; i < N; ++i) {
        double proj = 0.0;
        for (int64_t j = 0; j < d; ++j) proj += (Rmat[(size_t)i * d + j] - rbar[j]) * w[j];
        for (int64_t j = 0; j < d; ++j) sw[j] += (Rmat[(size_t)i * d + j] - rbar[j]) * proj;
    }
    for (int64_t j = 0; j < d; ++j) {
        sw[j] /= (double)(N - 1);
        g[j] = 2.0 * p->lambda * sw[j] - rbar[j];
    }
}

/* Eq. (3) with Sigma = diag(sigma^2): lambda sum_j sigma_j^2 w_j^2 - mu'w. */
double or_wide_objective(const or_wide_problem *p, const double *w)
{
    double quad = 0.0, lin = 0.0;
    for (int64_t j = 0; j < p->d; ++j) {
        const double v = p->sigma[j] * w[j];
        quad += v * v;
        lin += p->mu[j] * w[j];
    }
    return p->lambda * quad - lin;
}

/* Rounding bound of a system that evaluates the gradient with unit roundoff uroff: every sum taken
 * in absolute values through the noise coordinates (as or_path does with L = diag(sigma)), times
 * an accumulation depth N + ceil(log2 d) + 16 -- sums over the N samples run in order, sums over
 * the d assets as trees -- and a safety factor of 8. */
static double wide_bound(const or_wide_problem *p, int N, const double *z, const double *w, const double *g,
                         double uroff, double *vabs, double *pabs)
{
    const int64_t d = p->d;
    double wabs = 0.0, amax = 0.0;
    for (int64_t m = 0; m < d; ++m) {
        vabs[m] = fabs(p->sigma[m]) * fabs(w[m]);
        wabs += fabs(w[m]);
    }
    for (int i = 0; i < N; ++i) {
        double acc = 0.0;
        for (int64_t m = 0; m < d; ++m) acc += fabs(z[(size_t)i * d + m]) * vabs[m];
        pabs[i] = acc;
    }
    for (int64_t k = 0; k < d; ++k) {
        double quad = 0.0, lin = 0.0;
        for (int i = 0; i < N; ++i) {
            quad += fabs(z[(size_t)i * d + k]) * pabs[i];
            lin += fabs(z[(size_t)i * d + k]);
        }
        const double h = 2.0 * p->lambda * quad / (double)(N - 1) + lin / (double)N;
        const double a = fabs(p->sigma[k]) * h + fabs(p->mu[k]) + fabs(g[k]);
        if (a > amax) amax = a;
    }
    int lg = 0;
    while (((int64_t)1 << lg) < d) ++lg;
    const double depth = 8.0 * (double)(N + lg + 16);
    return depth * uroff * amax * (1.0 + wabs);
}

void or_wide_gradient(const or_wide_problem *p, uint64_t rep, uint64_t epoch, const double *w, double *g,
                      double uroff, double *bound)
{
    const int64_t d = p->d;
    const int N = wide_n(p, epoch);
    double *Rmat = (double *)malloc(sizeof(double) * (size_t)N * d);
    double *z = (double *)malloc(sizeof(double) * (size_t)N * d);
    double *rbar = (double *)malloc(sizeof(double) * (size_t)d);
    double *sw = (double *)malloc(sizeof(double) * (size_t)d);
    double *vabs = (double *)malloc(sizeof(double) * (size_t)d);
    double *pabs = (double *)malloc(sizeof(double) * (size_t)N);
    wide_returns(p, N, rep, epoch, Rmat, z);
    wide_statistics(p, N, Rmat, w, rbar, sw, g);
    if (bound) *bound = uroff > 0.0 ? wide_bound(p, N, z, w, g, uroff, vabs, pabs) : 0.0;
    free(pabs); free(vabs); free(sw); free(rbar); free(z); free(Rmat);
}

int or_wide_path(const or_wide_problem *p, uint64_t rep, uint64_t T, const uint32_t *replay, double uroff,
                 or_wide_out *out, uint32_t *decisions)
{
    const int64_t d = p->d;
    const int M = p->M;
    if (d < 1 || M < 1 || T < 1 || T > 0xFFFFFFFEull || p->n_ckpt < 0 || p->n_ckpt > OR_MAX_CKPT ||
        !(p->lambda > 0.0) || !out->cnt || !out->wsum)
        return -1;
    int Nmax = 0;                        /* the largest sample size of the run's epochs */
    for (uint64_t e = 0; e * (uint64_t)M < T; ++e) {
        const int Ne = wide_n(p, e);
        if (Ne < 2) return -1;
        if (Ne > Nmax) Nmax = Ne;
    }
    int N = p->N;

    double *Rmat = (double *)malloc(sizeof(double) * (size_t)Nmax * d);
    double *z = (double *)malloc(sizeof(double) * (size_t)Nmax * d);
    double *w = (double *)malloc(sizeof(double) * (size_t)d);
    double *g = (double *)malloc(sizeof(double) * (size_t)d);
    double *rbar = (double *)malloc(sizeof(double) * (size_t)d);
    double *sw = (double *)malloc(sizeof(double) * (size_t)d);
    double *vabs = (double *)malloc(sizeof(double) * (size_t)d);
    double *pabs = (double *)malloc(sizeof(double) * (size_t)Nmax);

    uint32_t *cnt = out->cnt;
    uint64_t *wsum = out->wsum;
    memset(out, 0, sizeof(*out));
    out->cnt = cnt;
    out->wsum = wsum;
    memset(cnt, 0, sizeof(uint32_t) * (size_t)(d + 1));
    memset(wsum, 0, sizeof(uint64_t) * (size_t)d);
    out->tau = out->tau_lo = out->tau_hi = OR_TAU_NONE;
    out->first_mismatch = -1;
    out->min_margin = INFINITY;
    for (int64_t j = 0; j < d; ++j) w[j] = p->w0 ? p->w0[j] : 0.0;   /* w_0 */

    int ck = 0;
    for (uint64_t t = 0; t < T; ++t) {
        const uint64_t epoch = t / (uint64_t)M;
        if (t % (uint64_t)M == 0) {                                     /* resample N_k returns */
            N = wide_n(p, epoch);
            wide_returns(p, N, rep, epoch, Rmat, z);
        }
        wide_statistics(p, N, Rmat, w, rbar, sw, g);

        /* the vertex search over W: e_j for the smallest g_j when it is negative, else the origin;
         * equal minima go to the lowest index */
        int64_t jmin = 0;
        for (int64_t j = 1; j < d; ++j)
            if (g[j] < g[jmin]) jmin = j;
        uint32_t a = (g[jmin] < 0.0) ? (uint32_t)(jmin + 1) : 0u;
        const double best = (a == 0) ? 0.0 : g[a - 1];
        double second = (a == 0) ? INFINITY : 0.0;   /* the origin's value is 0 */
        for (int64_t j = 0; j < d; ++j)
            if ((uint32_t)(j + 1) != a && g[j] < second) second = g[j];
        const double margin = second - best;
        if (margin < out->min_margin) out->min_margin = margin;

        const double bound = uroff > 0.0 ? wide_bound(p, N, z, w, g, uroff, vabs, pabs) : 0.0;
        const int ambiguous = margin <= 2.0 * bound;
        if (ambiguous) out->n_ambiguous++;
        if (replay && replay[t] != a) {
            const uint32_t r = replay[t];
            const double rv = (r == 0) ? 0.0 : (r <= (uint64_t)d ? g[r - 1] : INFINITY);
            if (ambiguous && r <= (uint64_t)d && rv <= best + 2.0 * bound) {
                a = r;
                out->n_replayed++;
            } else {
                out->n_mismatch++;
                if (out->first_mismatch < 0) out->first_mismatch = (int64_t)t;
            }
        }
        if (decisions) decisions[t] = a;

        /* Frank-Wolfe gap g'(w - s) and its first passage below eps */
        double gw = 0.0, wabs = 0.0;
        for (int64_t j = 0; j < d; ++j) {
            gw += g[j] * w[j];
            wabs += fabs(w[j]);
        }
        const double gap = gw - (g[jmin] < 0.0 ? g[jmin] : 0.0);
        const double gap_bound = bound * (1.0 + wabs);
        if (out->tau == OR_TAU_NONE && gap <= p->gap_eps) out->tau = (uint32_t)t;
        if (out->tau_lo == OR_TAU_NONE && gap <= p->gap_eps + gap_bound) out->tau_lo = (uint32_t)t;
        if (out->tau_hi == OR_TAU_NONE && gap <= p->gap_eps - gap_bound) out->tau_hi = (uint32_t)t;

        /* step 2/(t+2), update w + gamma (s - w) */
        const double gamma = 2.0 / ((double)t + 2.0);
        for (int64_t j = 0; j < d; ++j) {
            const double s = (a == (uint32_t)(j + 1)) ? 1.0 : 0.0;
            w[j] = w[j] + gamma * (s - w[j]);
        }
        cnt[a] += 1;
        if (a > 0) wsum[a - 1] += t + 1;

        while (ck < p->n_ckpt && (uint64_t)p->ckpt[ck] == t + 1) {
            out->f_ckpt[ck] = or_wide_objective(p, w);
            ++ck;
        }
    }
    out->y = or_wide_objective(p, w);

    const double tt = (double)T * (double)(T + 1);
    for (int64_t j = 0; j < d; ++j) {
        const double e = fabs(w[j] - 2.0 * (double)wsum[j] / tt);
        if (e > out->identity_err) out->identity_err = e;
    }
    free(pabs); free(vabs); free(sw); free(rbar); free(g); free(w); free(z); free(Rmat);
    return 0;
}
