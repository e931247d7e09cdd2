/*
 * newsvendor.c -- the oracle for Algorithm 2 (Section 3.2, Task 2: the multi-product constrained
 * newsvendor solved by stochastic Frank-Wolfe). Test infrastructure only; see oracle.h.
 *
 * Products j = 1..n with demand xi_j ~ N(mu_j, sigma_j^2), unit cost k_j, holding cost h_j and
 * selling value v_j. Cost Eq. (6): f_j(x) = k x + h E(x - xi)^+ + v E(xi - x)^+; problem Eq. (7):
 * minimise sum_j f_j(x_j) over X = {A x <= C, x >= 0}, here with one resource row c'x <= C (c > 0),
 * whose vertices are the origin and (C / c_j) e_j. Gradient Eq. (8): f_j'(x) = k - v + (h + v) Phi_j(x),
 * estimated by Eq. (9) from S demand samples per product: k - v + (h + v) #{s : d_j^(s) <= x_j} / S.
 * Algorithm 2: resample every M iterations, gradient, the vertex minimising s'g (the smallest
 * g_j / c_j when negative, else the origin; lowest index among equal values), step 2/(t+2), update
 * x + gamma (s - x). The demand samples are d_j^(s) = mu_j + sigma_j z with z the standard normal
 * s n + j of the (replication, epoch) stream in domain 4.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* E(x - xi)^+ and E(xi - x)^+ for xi ~ N(mu, sigma^2): with z = (x - mu)/sigma, sigma (z Phi(z) + phi(z))
 * and sigma (phi(z) - z (1 - Phi(z))); sigma = 0 gives (x - mu)^+ and (mu - x)^+. */
static void nv_expected_over_under(double x, double mu, double sigma, double *over, double *under)
{
    if (!(sigma > 0.0)) {
        *over = x > mu ? x - mu : 0.0;
        *under = mu > x ? mu - x : 0.0;
        return;
    }
    const double z = (x - mu) / sigma;
    const double pdf = 0.39894228040143267794 * exp(-0.5 * z * z);   /* 1/sqrt(2 pi) */
    const double cdf = 0.5 * erfc(-z / sqrt(2.0));
    const double upper = 0.5 * erfc(z / sqrt(2.0));   /* 1 - Phi(z) without cancellation */
    *over = sigma * (z * cdf + pdf);
    *under = sigma * (pdf - z * upper);
}

double or_nv_cost(const or_nv_problem *p, const double *x)
{
    double total = 0.0;
    for (int64_t j = 0; j < p->n; ++j) {
        double over, under;
        nv_expected_over_under(x[j], p->mu[j], p->sigma[j], &over, &under);
        total += p->k[j] * x[j] + p->h[j] * over + p->v[j] * under;
    }
    return total;
}

/* Eq. (9) at x for the demand samples d (S x n row-major): the count of samples <= x_j and the gradient. */
static void nv_gradient(const or_nv_problem *p, const double *d, const double *x, uint32_t *count, double *g)
{
    const int64_t n = p->n;
    const int S = p->S;
    for (int64_t j = 0; j < n; ++j) {
        uint32_t c = 0;
        for (int s = 0; s < S; ++s) c += (d[(size_t)s * n + j] <= x[j]) ? 1u : 0u;
        count[j] = c;
        g[j] = p->k[j] - p->v[j] + (p->h[j] + p->v[j]) * (double)c / (double)S;
    }
}

static void nv_demands(const or_nv_problem *p, uint64_t rep, uint64_t epoch, double *z, double *d)
{
    const int64_t n = p->n;
    const int S = p->S;
    or_normals(p->seed, OR_DOMAIN_NEWSVENDOR, p->instance, rep, epoch, 0, (uint64_t)S * (uint64_t)n, z);
    for (int s = 0; s < S; ++s)
        for (int64_t j = 0; j < n; ++j) d[(size_t)s * n + j] = p->mu[j] + p->sigma[j] * z[(size_t)s * n + j];
}

/* Uncertainty of g_j for a system that draws the normals and forms x in binary32 (unit roundoff u):
 * a sample whose normal lies within delta_j of the threshold (x_j - mu_j)/sigma_j may fall on either
 * side, which moves the count by one; plus the rounding of g_j itself. In units of g_j / c_j. */
static double nv_uncertainty(const or_nv_problem *p, const double *z, const double *x, int64_t j, double u)
{
    if (!(u > 0.0)) return 0.0;
    const int64_t n = p->n;
    double e = 8.0 * u * (fabs(p->k[j] - p->v[j]) + fabs(p->h[j] + p->v[j]));
    if (p->sigma[j] > 0.0) {
        const double thr = (x[j] - p->mu[j]) / p->sigma[j];
        const double delta = 256.0 * u * (1.0 + fabs(thr) + (fabs(x[j]) + fabs(p->mu[j])) / p->sigma[j]);
        int amb = 0;
        for (int s = 0; s < p->S; ++s)
            if (fabs(z[(size_t)s * n + j] - thr) <= delta) ++amb;
        e += fabs(p->h[j] + p->v[j]) * (double)amb / (double)p->S;
    }
    return e / p->c[j];
}

void or_nv_gradient_bound(const or_nv_problem *p, uint64_t rep, uint64_t epoch, const double *x, double u,
                          double *e)
{
    const size_t m = (size_t)p->S * (size_t)p->n;
    double *z = (double *)malloc(sizeof(double) * m);
    double *d = (double *)malloc(sizeof(double) * m);
    nv_demands(p, rep, epoch, z, d);
    /* nv_uncertainty is in units of g_j / c_j: multiply back (c is 1 where the caller has no row) */
    for (int64_t j = 0; j < p->n; ++j) e[j] = nv_uncertainty(p, z, x, j, u) * p->c[j];
    free(d);
    free(z);
}

void or_nv_gradient(const or_nv_problem *p, uint64_t rep, uint64_t epoch, const double *x, double *g,
                    uint32_t *count)
{
    const size_t m = (size_t)p->S * (size_t)p->n;
    double *z = (double *)malloc(sizeof(double) * m);
    double *d = (double *)malloc(sizeof(double) * m);
    uint32_t *cnt = count ? count : (uint32_t *)malloc(sizeof(uint32_t) * (size_t)p->n);
    nv_demands(p, rep, epoch, z, d);
    nv_gradient(p, d, x, cnt, g);
    if (!count) free(cnt);
    free(d);
    free(z);
}

int or_nv_path(const or_nv_problem *p, uint64_t rep, uint64_t T, const uint32_t *replay, double uroff,
               or_nv_out *out, uint32_t *decisions)
{
    const int64_t n = p->n;
    const int S = p->S, M = p->M;
    if (n < 1 || S < 1 || M < 1 || T < 1 || T > 0xFFFFFFFEull || p->n_ckpt < 0 || p->n_ckpt > OR_MAX_CKPT ||
        !(p->C > 0.0) || !out->cnt || !out->wsum)
        return -1;
    for (int64_t j = 0; j < n; ++j)
        if (!(p->c[j] > 0.0)) return -1;

    const size_t m = (size_t)S * (size_t)n;
    double *z = (double *)malloc(sizeof(double) * m);
    double *d = (double *)malloc(sizeof(double) * m);
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double *g = (double *)malloc(sizeof(double) * (size_t)n);
    double *r = (double *)malloc(sizeof(double) * (size_t)n);
    double *e = (double *)malloc(sizeof(double) * (size_t)n);
    uint32_t *count = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);

    uint32_t *cnt = out->cnt;
    uint64_t *wsum = out->wsum;
    memset(out, 0, sizeof(*out));
    out->cnt = cnt;
    out->wsum = wsum;
    memset(cnt, 0, sizeof(uint32_t) * (size_t)(n + 1));
    memset(wsum, 0, sizeof(uint64_t) * (size_t)n);
    out->tau = out->tau_lo = out->tau_hi = OR_TAU_NONE;
    out->first_mismatch = -1;
    out->min_margin = INFINITY;
    for (int64_t j = 0; j < n; ++j) x[j] = p->x0 ? p->x0[j] : 0.0;

    int ck = 0;
    for (uint64_t t = 0; t < T; ++t) {
        const uint64_t epoch = t / (uint64_t)M;
        if (t % (uint64_t)M == 0) nv_demands(p, rep, epoch, z, d);   /* resample */
        nv_gradient(p, d, x, count, g);

        /* the vertex minimising s'g over X: (C/c_j) e_j for the smallest ratio g_j / c_j when it is
         * negative, else the origin; equal ratios go to the lowest index */
        int64_t jmin = 0;
        for (int64_t j = 0; j < n; ++j) {
            r[j] = g[j] / p->c[j];
            if (r[j] < r[jmin]) jmin = j;
        }
        uint32_t a = (r[jmin] < 0.0) ? (uint32_t)(jmin + 1) : 0u;
        const double best = (a == 0) ? 0.0 : r[a - 1];
        double second = (a == 0) ? INFINITY : 0.0;
        for (int64_t j = 0; j < n; ++j)
            if ((uint32_t)(j + 1) != a && r[j] < second) second = r[j];
        const double margin = second - best;
        if (margin < out->min_margin) out->min_margin = margin;

        /* ambiguity: the interval of some other vertex's value reaches that of the chosen one */
        int ambiguous = 0;
        double ea = 0.0;
        if (uroff > 0.0) {
            for (int64_t j = 0; j < n; ++j) e[j] = nv_uncertainty(p, z, x, j, uroff);
            ea = (a == 0) ? 0.0 : e[a - 1];
            for (int64_t j = 0; j < n && !ambiguous; ++j)
                if ((uint32_t)(j + 1) != a && r[j] - e[j] <= best + ea) ambiguous = 1;
            if (a != 0 && 0.0 <= best + ea) ambiguous = 1;       /* the origin's value is exactly 0 */
        }
        if (ambiguous) out->n_ambiguous++;
        if (replay && replay[t] != a) {
            const uint32_t q = replay[t];
            int ok = 0;
            if (ambiguous && q <= (uint64_t)n) {
                const double lower = (q == 0) ? 0.0 : r[q - 1] - e[q - 1];
                ok = lower <= best + ea;
            }
            if (ok) {
                a = q;
                out->n_replayed++;
            } else {
                out->n_mismatch++;
                if (out->first_mismatch < 0) out->first_mismatch = (int64_t)t;
            }
        }
        if (decisions) decisions[t] = a;

        /* Frank-Wolfe gap g'(x - s) and its first passage below eps */
        double gx = 0.0, gx_abs = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            gx += g[j] * x[j];
            gx_abs += fabs(g[j] * x[j]);
        }
        const double smin = (r[jmin] < 0.0) ? p->C * r[jmin] : 0.0;
        const double gap = gx - smin;
        double gap_bound = 0.0;
        if (uroff > 0.0) {
            double emax = 0.0, xs = 0.0;
            for (int64_t j = 0; j < n; ++j) {
                if (e[j] * p->c[j] > emax) emax = e[j] * p->c[j];
                xs += fabs(x[j]);
            }
            gap_bound = emax * xs + p->C * (ea + 8.0 * uroff * fabs(best)) + 64.0 * uroff * gx_abs;
        }
        if (out->tau == OR_TAU_NONE && gap <= p->gap_eps) out->tau = (uint32_t)t;
        if (out->tau_lo == OR_TAU_NONE && gap <= p->gap_eps + gap_bound) out->tau_lo = (uint32_t)t;
        if (out->tau_hi == OR_TAU_NONE && gap <= p->gap_eps - gap_bound) out->tau_hi = (uint32_t)t;

        /* step 2/(t+2) and the update x + gamma (s - x) */
        const double gamma = 2.0 / ((double)t + 2.0);
        for (int64_t j = 0; j < n; ++j) {
            const double s = (a == (uint32_t)(j + 1)) ? p->C / p->c[j] : 0.0;
            x[j] = x[j] + gamma * (s - x[j]);
        }
        cnt[a] += 1;
        if (a > 0) wsum[a - 1] += t + 1;

        while (ck < p->n_ckpt && (uint64_t)p->ckpt[ck] == t + 1) {
            out->f_ckpt[ck] = or_nv_cost(p, x);
            ++ck;
        }
    }
    out->y = or_nv_cost(p, x);

    const double tt = (double)T * (double)(T + 1);
    for (int64_t j = 0; j < n; ++j) {
        const double closed = (p->C / p->c[j]) * 2.0 * (double)wsum[j] / tt;
        const double err = fabs(x[j] - closed) / (p->C / p->c[j]);
        if (err > out->identity_err) out->identity_err = err;
    }
    free(count); free(e); free(r); free(g); free(x); free(d); free(z);
    return 0;
}
