/*
 * sqn.c -- the oracle for Algorithms 3-4 (Section 3.3, Task 3: stochastic quasi-Newton for binary
 * classification). Test infrastructure only; see oracle.h.
 *
 * Loss Eq. (10)-(11): F(w) = -(1/N) sum_i z_i log c(w; x_i) + (1 - z_i) log(1 - c(w; x_i)),
 * c(w; x) = 1 / (1 + exp(-x'w)). Mini-batch gradient Eq. (12) over b sampled rows (the gradient of
 * the loss term -[z log c + (1 - z) log(1 - c)] is (c - z) x), sub-sampled Hessian Eq. (13) over b_H
 * rows applied to a vector: (1/b_H) sum_i c (1 - c) (x_i's) x_i. Algorithm 3: alpha_k = beta / k;
 * gradient steps for k <= 2L, then steps along -H_t g; every L iterations the average of the last L
 * iterates closes a window, and from the second window on a correction pair
 * s_t = wbar_t - wbar_{t-1}, y_t = Hessian(wbar_t) s_t is stored (the M most recent are kept).
 * Algorithm 4: H = (s_t'y_t)/(y_t'y_t) I, then the BFGS update over the stored pairs, oldest first,
 * H <- (I - rho s y') H (I - rho y s') + rho s s' with rho = 1/(y's), formed explicitly (n x n).
 * Sampled rows: index floor(u N / 2^32) for the 32-bit Philox words u of counter
 * (q/4, k, replication, domain | instance), q = 0, 1, ...; domain 5 for the gradient samples of
 * iteration k, domain 6 for the Hessian samples of the pair closed at iteration k.
 * With pairs_fp32 the stored pairs are rounded to binary32: s, then y = Hessian(wbar_t) applied to
 * the rounded s, then y itself; everything else stays binary64.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

void or_sqn_indices(const or_sqn_problem *p, uint64_t rep, uint64_t k, uint32_t domain, uint32_t count,
                    uint32_t *idx)
{
    const uint32_t key[2] = {(uint32_t)p->seed, (uint32_t)(p->seed >> 32)};
    for (uint32_t q = 0; q < count; ++q) {
        const uint32_t ctr[4] = {q / 4, (uint32_t)k, (uint32_t)rep, (domain << 24) | (p->instance & 0xFFFFFFu)};
        uint32_t x[4];
        or_philox4x32_10(ctr, key, x);
        idx[q] = (uint32_t)(((uint64_t)x[q % 4] * (uint64_t)p->N) >> 32);
    }
}

static double sigmoid(double a) { return 1.0 / (1.0 + exp(-a)); }

static double row_dot(const or_sqn_problem *p, uint64_t i, const double *w)
{
    const uint8_t *x = p->X + i * (uint64_t)p->n;
    double a = 0.0;
    for (int64_t j = 0; j < p->n; ++j)
        if (x[j]) a += w[j];
    return a;
}

double or_sqn_loss(const or_sqn_problem *p, const double *w)
{
    double total = 0.0;
    for (int64_t i = 0; i < p->N; ++i) {
        const double a = row_dot(p, (uint64_t)i, w);
        /* -[z log c + (1 - z) log(1 - c)] = log(1 + e^{-a}) + (1 - z) a, evaluated without overflow */
        const double softplus = a > 0.0 ? log1p(exp(-a)) : log1p(exp(a)) - a;
        total += softplus + (p->z[i] ? 0.0 : a);
    }
    return total / (double)p->N;
}

/* Eq. (12): (1/b) sum over the sampled rows of (c(w; x_i) - z_i) x_i */
void or_sqn_gradient(const or_sqn_problem *p, const uint32_t *idx, uint32_t b, const double *w, double *g)
{
    for (int64_t j = 0; j < p->n; ++j) g[j] = 0.0;
    for (uint32_t s = 0; s < b; ++s) {
        const uint64_t i = idx[s];
        const double r = sigmoid(row_dot(p, i, w)) - (double)p->z[i];
        const uint8_t *x = p->X + i * (uint64_t)p->n;
        for (int64_t j = 0; j < p->n; ++j)
            if (x[j]) g[j] += r;
    }
    for (int64_t j = 0; j < p->n; ++j) g[j] /= (double)b;
}

/* Eq. (13) applied to v: (1/b_H) sum over the sampled rows of c (1 - c) (x_i'v) x_i, c at w */
void or_sqn_hessian_vector(const or_sqn_problem *p, const uint32_t *idx, uint32_t bh, const double *w,
                           const double *v, double *out)
{
    for (int64_t j = 0; j < p->n; ++j) out[j] = 0.0;
    for (uint32_t s = 0; s < bh; ++s) {
        const uint64_t i = idx[s];
        const double c = sigmoid(row_dot(p, i, w));
        const double coef = c * (1.0 - c) * row_dot(p, i, v);
        const uint8_t *x = p->X + i * (uint64_t)p->n;
        for (int64_t j = 0; j < p->n; ++j)
            if (x[j]) out[j] += coef;
    }
    for (int64_t j = 0; j < p->n; ++j) out[j] /= (double)bh;
}

/* Algorithm 4 over pairs (S, Y) [m][n], oldest first; H is n x n row-major. The update
 * (I - rho s y') H (I - rho y s') + rho s s' is applied in its expanded form
 * H - rho (s (Hy)' + (Hy) s') + (rho^2 y'Hy + rho) s s' (H symmetric), O(n^2) per pair. */
void or_sqn_hessian_approx(int64_t n, int m, const double *S, const double *Y, double *H)
{
    const double *st = S + (size_t)(m - 1) * n, *yt = Y + (size_t)(m - 1) * n;
    double sy = 0.0, yy = 0.0;
    for (int64_t a = 0; a < n; ++a) {
        sy += st[a] * yt[a];
        yy += yt[a] * yt[a];
    }
    const double gamma = sy / yy;
    for (int64_t a = 0; a < n; ++a)
        for (int64_t c = 0; c < n; ++c) H[a * n + c] = (a == c) ? gamma : 0.0;
    double *Hy = (double *)malloc(sizeof(double) * (size_t)n);
    for (int j = 0; j < m; ++j) {
        const double *s = S + (size_t)j * n, *y = Y + (size_t)j * n;
        double ys = 0.0;
        for (int64_t a = 0; a < n; ++a) ys += y[a] * s[a];
        const double rho = 1.0 / ys;
        double yHy = 0.0;
        for (int64_t a = 0; a < n; ++a) {
            double acc = 0.0;
            for (int64_t c = 0; c < n; ++c) acc += H[a * n + c] * y[c];
            Hy[a] = acc;
            yHy += y[a] * acc;
        }
        const double k2 = rho * rho * yHy + rho;
        for (int64_t a = 0; a < n; ++a)
            for (int64_t c = 0; c < n; ++c)
                H[a * n + c] += -rho * (s[a] * Hy[c] + Hy[a] * s[c]) + k2 * s[a] * s[c];
    }
    free(Hy);
}

int or_sqn_run(const or_sqn_problem *p, uint64_t rep, uint64_t K, or_sqn_out *out)
{
    const int64_t n = p->n;
    if (n < 1 || p->N < 1 || p->L < 1 || p->M < 1 || p->b < 1 || p->bH < 1 || !(p->beta > 0.0) || K < 1 ||
        p->n_ckpt < 0 || p->n_ckpt > OR_MAX_CKPT || !out->w)
        return -1;
    double *w = out->w;
    double *acc = (double *)calloc((size_t)n, sizeof(double));      /* running sum of iterates */
    double *wbar_prev = (double *)calloc((size_t)n, sizeof(double));
    double *wbar = (double *)malloc(sizeof(double) * (size_t)n);
    double *g = (double *)malloc(sizeof(double) * (size_t)n);
    double *dir = (double *)malloc(sizeof(double) * (size_t)n);
    double *S = (double *)malloc(sizeof(double) * (size_t)p->M * n);  /* stored pairs, oldest first */
    double *Y = (double *)malloc(sizeof(double) * (size_t)p->M * n);
    double *H = (double *)malloc(sizeof(double) * (size_t)n * n);
    uint32_t *idx = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(p->b > p->bH ? p->b : p->bH));
    int m = 0;              /* pairs stored */
    int64_t t = -1;         /* windows closed minus one: the t of Algorithm 3 */
    int H_ready = 0;
    memset(out->F_ckpt, 0, sizeof(out->F_ckpt));
    out->pairs = 0;
    for (int64_t j = 0; j < n; ++j) w[j] = 0.0;                     /* w^1 = 0 */

    int ck = 0;
    for (uint64_t k = 1; k <= K; ++k) {
        or_sqn_indices(p, rep, k, OR_DOMAIN_SQN_GRAD, (uint32_t)p->b, idx);
        or_sqn_gradient(p, idx, (uint32_t)p->b, w, g);
        for (int64_t j = 0; j < n; ++j) acc[j] += w[j];
        const double alpha = p->beta / (double)k;
        if (k <= 2 * (uint64_t)p->L) {
            for (int64_t j = 0; j < n; ++j) w[j] -= alpha * g[j];
        } else {
            if (!H_ready) {
                or_sqn_hessian_approx(n, m, S, Y, H);
                H_ready = 1;
            }
            for (int64_t a = 0; a < n; ++a) {
                double s = 0.0;
                for (int64_t c = 0; c < n; ++c) s += H[a * n + c] * g[c];
                dir[a] = s;
            }
            for (int64_t j = 0; j < n; ++j) w[j] -= alpha * dir[j];
        }
        if (k % (uint64_t)p->L == 0) {
            ++t;
            for (int64_t j = 0; j < n; ++j) wbar[j] = acc[j] / (double)p->L;
            if (t > 0) {
                if (m == p->M) {                      /* drop the oldest pair */
                    memmove(S, S + n, sizeof(double) * (size_t)(p->M - 1) * n);
                    memmove(Y, Y + n, sizeof(double) * (size_t)(p->M - 1) * n);
                    --m;
                }
                double *s = S + (size_t)m * n, *y = Y + (size_t)m * n;
                for (int64_t j = 0; j < n; ++j) {
                    s[j] = wbar[j] - wbar_prev[j];
                    if (p->pairs_fp32) s[j] = (double)(float)s[j];
                }
                or_sqn_indices(p, rep, k, OR_DOMAIN_SQN_HESS, (uint32_t)p->bH, idx);
                or_sqn_hessian_vector(p, idx, (uint32_t)p->bH, wbar, s, y);
                if (p->pairs_fp32)
                    for (int64_t j = 0; j < n; ++j) y[j] = (double)(float)y[j];
                ++m;
                ++out->pairs;
                H_ready = 0;
            }
            memcpy(wbar_prev, wbar, sizeof(double) * (size_t)n);
            memset(acc, 0, sizeof(double) * (size_t)n);
        }
        while (ck < p->n_ckpt && (uint64_t)p->ckpt[ck] == k) {
            out->F_ckpt[ck] = or_sqn_loss(p, w);
            ++ck;
        }
    }
    out->F = or_sqn_loss(p, w);
    free(idx); free(H); free(Y); free(S); free(dir); free(g); free(wbar); free(wbar_prev); free(acc);
    return 0;
}
