// host_core.cpp -- device-free host logic of the C ABI: parameter validation, instance
// coefficients, the tile plan of batched runs, and the final FP64 statistics (double-double
// arithmetic on the reduced sums). Plain C++; no HIP runtime calls.
#include "host_core.hpp"

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <numeric>

namespace fw {
namespace host {

int fail(char *err, int code, const char *fmt, ...)
{
    if (err) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(err, kErrLen, fmt, ap);
        va_end(ap);
    }
    return code;
}

bool finite(double x) { return std::isfinite(x); }

int validate(char *err, const sim_params *p, uint64_t R, uint64_t T)
{
    if (!p) return fail(err, SIM_EINVAL, "params is NULL");
    if (p->abi_version != SIM_ABI_VERSION)
        return fail(err, SIM_EINVAL, "abi_version %u != %u", p->abi_version, SIM_ABI_VERSION);
    if (p->d < 1 || p->d > SIM_MAX_D) return fail(err, SIM_EINVAL, "d=%u outside [1, 64]", p->d);
    if (R < 1 || R > 0xFFFFFFFFull) return fail(err, SIM_EINVAL, "R=%llu outside [1, 2^32)", (unsigned long long)R);
    if (T < 1 || T > 0xFFFFFFFEull) return fail(err, SIM_EINVAL, "T=%llu outside [1, 2^32-2]", (unsigned long long)T);
    if (!p->mu) return fail(err, SIM_EINVAL, "mu is NULL");
    for (uint32_t j = 0; j < p->d; ++j)
        if (!finite(p->mu[j])) return fail(err, SIM_EINVAL, "mu[%u] not finite", j);
    if (p->chol) {
        const uint32_t d = p->d;
        for (uint32_t j = 0; j < d; ++j)
            for (uint32_t k = 0; k < d; ++k) {
                const double x = p->chol[j * d + k];
                if (!finite(x)) return fail(err, SIM_EINVAL, "chol[%u][%u] not finite", j, k);
                if (k > j && x != 0.0) return fail(err, SIM_EINVAL, "chol[%u][%u] above the diagonal is not 0", j, k);
            }
        if (d != 32 && d != 64)
            return fail(err, SIM_EUNSUPPORTED, "dense Cholesky factors need d = 32 or 64 (d=%u)", d);
        if (p->state_precision != SIM_FP32)
            return fail(err, SIM_EUNSUPPORTED, "dense Cholesky factors run in FP32 state only");
        if (T > kMaxDenseT)
            return fail(err, SIM_EUNSUPPORTED, "dense Cholesky factors need T <= %llu", (unsigned long long)kMaxDenseT);
    } else {
        if (!p->sigma) return fail(err, SIM_EINVAL, "sigma is NULL");
        for (uint32_t j = 0; j < p->d; ++j)
            if (!finite(p->sigma[j]) || p->sigma[j] < 0.0)
                return fail(err, SIM_EINVAL, "sigma[%u] must be finite and >= 0", j);
        // one lane per replication holds the state of at most 32 (FP32) or 16 (FP64) assets
        const uint32_t dmax = p->state_precision == SIM_FP64 ? 16u : 32u;
        if (p->d > dmax)
            return fail(err, SIM_EUNSUPPORTED, "diagonal Sigma with d=%u: the per-lane kernels hold d <= %u in this "
                        "precision (sim_run_wide takes many assets on a few replications)", p->d, dmax);
    }
    if (!(p->risk_coef > 0.0) || !finite(p->risk_coef))
        return fail(err, SIM_EINVAL, "risk_coef must be finite and > 0");
    if (p->w0) {
        double s = 0.0;
        for (uint32_t j = 0; j < p->d; ++j) {
            if (!finite(p->w0[j]) || p->w0[j] < 0.0) return fail(err, SIM_EINVAL, "w0[%u] outside W", j);
            s += p->w0[j];
        }
        if (s > 1.0 + 1e-12) return fail(err, SIM_EINVAL, "w0 sums to %g > 1", s);
    }
    if (p->n_samples < 2) return fail(err, SIM_EINVAL, "n_samples must be >= 2 (Eq. (4) divides by N-1)");
    if (p->n_samples > (1u << 24)) return fail(err, SIM_EINVAL, "n_samples above 2^24");
    if (p->n_schedule) {
        // per-epoch sample sizes N_k (the remark on Algorithm 1's resampling step): the per-lane
        // kernels with a diagonal Sigma, without control-variate features
        if (p->chol) return fail(err, SIM_EUNSUPPORTED, "n_schedule with a dense factor");
        if (p->flags & SIM_CV_FEATURES) return fail(err, SIM_EUNSUPPORTED, "n_schedule with control-variate features");
        if (p->resample_every < 1) return fail(err, SIM_EINVAL, "resample_every must be >= 1");
        const uint64_t epochs = (T + p->resample_every - 1) / p->resample_every;
        if (epochs > (1u << 24)) return fail(err, SIM_EINVAL, "n_schedule: more than 2^24 epochs");
        for (uint64_t e = 0; e < epochs; ++e) {
            const uint32_t n = p->n_schedule[e];
            if (n < 2 || n > (1u << 24))
                return fail(err, SIM_EINVAL, "n_schedule[%llu] = %u outside [2, 2^24]", (unsigned long long)e, n);
            if ((uint64_t)n * (p->d + (p->noise == SIM_NOISE_T ? p->nu : 0u)) > 0xFFFFFFF0ull)
                return fail(err, SIM_EINVAL, "n_schedule[%llu]: N (d + nu) normals per epoch above 2^32 - 16",
                            (unsigned long long)e);
        }
    }
    // a replication's normals of one epoch are numbered in 32 bits: N d Gaussian numerators, then
    // N nu chi-square normals for t noise
    if ((uint64_t)p->n_samples * (p->d + (p->noise == SIM_NOISE_T ? p->nu : 0u)) > 0xFFFFFFF0ull)
        return fail(err, SIM_EINVAL, "N (d + nu) normals per epoch above 2^32 - 16");
    if (p->resample_every < 1) return fail(err, SIM_EINVAL, "resample_every must be >= 1");
    if (p->noise != SIM_NOISE_GAUSS && p->noise != SIM_NOISE_T) return fail(err, SIM_EINVAL, "unknown noise");
    if (p->noise == SIM_NOISE_T && (p->nu < 3 || p->nu > 1024))
        return fail(err, SIM_EINVAL, "nu must be an integer in [3, 1024]");
    if (p->state_precision != SIM_FP32 && p->state_precision != SIM_FP64)
        return fail(err, SIM_EINVAL, "unknown state_precision");
    if (p->n_checkpoints > SIM_MAX_CKPT) return fail(err, SIM_EINVAL, "more than 8 checkpoints");
    for (uint32_t k = 0; k < p->n_checkpoints; ++k) {
        if (p->checkpoints[k] < 1 || p->checkpoints[k] > T)
            return fail(err, SIM_EINVAL, "checkpoint %u outside [1, T]", k);
        if (k && p->checkpoints[k] <= p->checkpoints[k - 1])
            return fail(err, SIM_EINVAL, "checkpoints must increase strictly");
    }
    if (!finite(p->gap_eps) || p->gap_eps < 0.0) return fail(err, SIM_EINVAL, "gap_eps must be finite and >= 0");
    if (p->flags & ~(uint32_t)(SIM_KEEP_PATHS | SIM_DECISION_LOG | SIM_CV_FEATURES))
        return fail(err, SIM_EINVAL, "unknown flag bits");
    if (p->flags & SIM_CV_FEATURES) {
        if (p->state_precision != SIM_FP32)
            return fail(err, SIM_EUNSUPPORTED, "control-variate features need FP32 state");
        if (p->chol) {
            if (T > kMaxDenseFeatT)
                return fail(err, SIM_EUNSUPPORTED, "control-variate features with a dense factor need T <= %llu",
                            (unsigned long long)kMaxDenseFeatT);
        } else {
            if (p->d > 32) return fail(err, SIM_EUNSUPPORTED, "control-variate features need d <= 32");
            if (T > kMaxNarrowT)
                return fail(err, SIM_EUNSUPPORTED, "control-variate features need T <= %llu",
                            (unsigned long long)kMaxNarrowT);
        }
        if (!p->cv_ref) return fail(err, SIM_EINVAL, "control-variate features need cv_ref");
        for (uint32_t j = 0; j < p->d; ++j) {
            if (!finite(p->cv_ref[j])) return fail(err, SIM_EINVAL, "cv_ref[%u] not finite", j);
            if (!(cv_scale(p, j) > 0.0))
                return fail(err, SIM_EUNSUPPORTED, "control-variate features need every sigma_j (or L_jj) > 0");
        }
    }
    if (p->instance_id >= (1u << 24)) return fail(err, SIM_EINVAL, "instance_id must be < 2^24");
    if (p->flags & SIM_DECISION_LOG) {
        if (p->log_rep_count < 1 || p->log_rep_count > 65536)
            return fail(err, SIM_EINVAL, "log_rep_count must be in [1, 65536]");
        if (p->log_rep_begin >= R || p->log_rep_count > R - p->log_rep_begin)
            return fail(err, SIM_EINVAL, "logged replications exceed R");
        if (T * p->log_rep_count > (1ull << 34)) return fail(err, SIM_EINVAL, "decision log above 16 GiB");
    }
    return SIM_OK;
}

int validate_wide(char *err, const sim_params *p, uint64_t R, uint64_t T)
{
    if (!p) return fail(err, SIM_EINVAL, "params is NULL");
    if (p->abi_version != SIM_ABI_VERSION)
        return fail(err, SIM_EINVAL, "abi_version %u != %u", p->abi_version, SIM_ABI_VERSION);
    if (p->d < 4 || p->d > SIM_WIDE_MAX_D || p->d % 4 != 0)
        return fail(err, SIM_EINVAL, "d=%u: the wide path needs a multiple of 4 in [4, %u]", p->d, SIM_WIDE_MAX_D);
    if (R < 1 || R > SIM_WIDE_MAX_R)
        return fail(err, SIM_EINVAL, "R=%llu outside [1, %u]", (unsigned long long)R, SIM_WIDE_MAX_R);
    if (T < 1 || T > 0xFFFFFFFEull) return fail(err, SIM_EINVAL, "T=%llu outside [1, 2^32-2]", (unsigned long long)T);
    if (R * T > (1ull << 30)) return fail(err, SIM_EINVAL, "R T above 2^30 (the decision record)");
    if (p->chol) return fail(err, SIM_EUNSUPPORTED, "the wide path takes a diagonal Sigma (chol must be NULL)");
    if (!p->mu || !p->sigma) return fail(err, SIM_EINVAL, "mu and sigma are required");
    for (uint32_t j = 0; j < p->d; ++j) {
        if (!finite(p->mu[j])) return fail(err, SIM_EINVAL, "mu[%u] not finite", j);
        if (!finite(p->sigma[j]) || p->sigma[j] < 0.0) return fail(err, SIM_EINVAL, "sigma[%u] must be finite and >= 0", j);
    }
    if (!(p->risk_coef > 0.0) || !finite(p->risk_coef))
        return fail(err, SIM_EINVAL, "risk_coef must be finite and > 0");
    if (p->w0) {
        double s = 0.0;
        for (uint32_t j = 0; j < p->d; ++j) {
            if (!finite(p->w0[j]) || p->w0[j] < 0.0) return fail(err, SIM_EINVAL, "w0[%u] outside W", j);
            s += p->w0[j];
        }
        if (s > 1.0 + 1e-12) return fail(err, SIM_EINVAL, "w0 sums to %g > 1", s);
    }
    if (p->n_samples < 2 || p->n_samples > SIM_WIDE_MAX_N)
        return fail(err, SIM_EINVAL, "n_samples must be in [2, %u]", SIM_WIDE_MAX_N);
    if (p->resample_every < 1) return fail(err, SIM_EINVAL, "resample_every must be >= 1");
    if (p->n_schedule) {
        const uint64_t epochs = (T + p->resample_every - 1) / p->resample_every;
        for (uint64_t e = 0; e < epochs; ++e)
            if (p->n_schedule[e] < 2 || p->n_schedule[e] > SIM_WIDE_MAX_N)
                return fail(err, SIM_EINVAL, "n_schedule[%llu] = %u outside [2, %u]", (unsigned long long)e,
                            p->n_schedule[e], SIM_WIDE_MAX_N);
    }
    if (p->noise != SIM_NOISE_GAUSS) return fail(err, SIM_EUNSUPPORTED, "the wide path draws Gaussian noise only");
    if (p->state_precision != SIM_FP32) return fail(err, SIM_EUNSUPPORTED, "the wide path runs in FP32 state");
    if (p->n_checkpoints > SIM_MAX_CKPT) return fail(err, SIM_EINVAL, "more than 8 checkpoints");
    for (uint32_t k = 0; k < p->n_checkpoints; ++k) {
        if (p->checkpoints[k] < 1 || p->checkpoints[k] > T)
            return fail(err, SIM_EINVAL, "checkpoint %u outside [1, T]", k);
        if (k && p->checkpoints[k] <= p->checkpoints[k - 1])
            return fail(err, SIM_EINVAL, "checkpoints must increase strictly");
    }
    if (!finite(p->gap_eps) || p->gap_eps < 0.0) return fail(err, SIM_EINVAL, "gap_eps must be finite and >= 0");
    if (p->flags & ~(uint32_t)(SIM_KEEP_PATHS | SIM_DECISION_LOG))
        return fail(err, SIM_EINVAL, "the wide path takes no flag but SIM_KEEP_PATHS and SIM_DECISION_LOG");
    if (p->instance_id >= (1u << 24)) return fail(err, SIM_EINVAL, "instance_id must be < 2^24");
    return SIM_OK;
}

// The checks shared by both forms of Algorithm 2; `one_row`: the single resource row c'x <= C.
static int validate_nv_common(char *err, const sim_nv_params *p, uint64_t R, uint64_t T, bool one_row)
{
    if (!p) return fail(err, SIM_EINVAL, "params is NULL");
    if (p->abi_version != SIM_ABI_VERSION)
        return fail(err, SIM_EINVAL, "abi_version %u != %u", p->abi_version, SIM_ABI_VERSION);
    if (p->n < 4 || p->n > SIM_NV_MAX_N || p->n % 4 != 0)
        return fail(err, SIM_EINVAL, "n=%u: products must be a multiple of 4 in [4, %u]", p->n, SIM_NV_MAX_N);
    if (R < 1 || R > SIM_WIDE_MAX_R)
        return fail(err, SIM_EINVAL, "R=%llu outside [1, %u]", (unsigned long long)R, SIM_WIDE_MAX_R);
    if (T < 1 || T > 0xFFFFFFFEull) return fail(err, SIM_EINVAL, "T=%llu outside [1, 2^32-2]", (unsigned long long)T);
    if (R * T > (1ull << 30)) return fail(err, SIM_EINVAL, "R T above 2^30 (the decision record)");
    if (!p->mu || !p->sigma || !p->k || !p->h || !p->v || (one_row && !p->c))
        return fail(err, SIM_EINVAL, one_row ? "mu, sigma, k, h, v and c are required" : "mu, sigma, k, h and v are required");
    if (one_row && (!finite(p->C) || !(p->C > 0.0))) return fail(err, SIM_EINVAL, "C must be finite and > 0");
    for (uint32_t j = 0; j < p->n; ++j) {
        if (!finite(p->mu[j]) || !finite(p->k[j]) || !finite(p->h[j]) || !finite(p->v[j]))
            return fail(err, SIM_EINVAL, "product %u: mu, k, h, v must be finite", j);
        if (!finite(p->sigma[j]) || p->sigma[j] < 0.0) return fail(err, SIM_EINVAL, "sigma[%u] must be finite and >= 0", j);
        if (one_row && (!finite(p->c[j]) || !(p->c[j] > 0.0))) return fail(err, SIM_EINVAL, "c[%u] must be finite and > 0", j);
    }
    if (p->x0) {
        double used = 0.0;
        for (uint32_t j = 0; j < p->n; ++j) {
            if (!finite(p->x0[j]) || p->x0[j] < 0.0) return fail(err, SIM_EINVAL, "x0[%u] outside X", j);
            if (one_row) used += p->c[j] * p->x0[j];
        }
        if (one_row && used > p->C * (1.0 + 1e-12)) return fail(err, SIM_EINVAL, "x0 uses %g > C", used);
    }
    if (p->n_samples < 1 || p->n_samples > SIM_NV_MAX_S)
        return fail(err, SIM_EINVAL, "n_samples must be in [1, %u]", SIM_NV_MAX_S);
    if (p->resample_every < 1) return fail(err, SIM_EINVAL, "resample_every must be >= 1");
    if (p->n_checkpoints > SIM_MAX_CKPT) return fail(err, SIM_EINVAL, "more than 8 checkpoints");
    for (uint32_t k = 0; k < p->n_checkpoints; ++k) {
        if (p->checkpoints[k] < 1 || p->checkpoints[k] > T)
            return fail(err, SIM_EINVAL, "checkpoint %u outside [1, T]", k);
        if (k && p->checkpoints[k] <= p->checkpoints[k - 1])
            return fail(err, SIM_EINVAL, "checkpoints must increase strictly");
    }
    if (!finite(p->gap_eps) || p->gap_eps < 0.0) return fail(err, SIM_EINVAL, "gap_eps must be finite and >= 0");
    if (p->instance_id >= (1u << 24)) return fail(err, SIM_EINVAL, "instance_id must be < 2^24");
    return SIM_OK;
}

int validate_newsvendor(char *err, const sim_nv_params *p, uint64_t R, uint64_t T)
{
    return validate_nv_common(err, p, R, T, true);
}

int validate_newsvendor_lp(char *err, const sim_nv_params *p, const sim_nv_constraints *con, uint64_t R, uint64_t T)
{
    if (int rc = validate_nv_common(err, p, R, T, false)) return rc;
    if (!con) return fail(err, SIM_EINVAL, "constraints are NULL");
    const uint32_t M = con->n_resources, n = p->n;
    if (M < 1 || M > SIM_NV_MAX_RES) return fail(err, SIM_EINVAL, "n_resources=%u outside [1, %u]", M, SIM_NV_MAX_RES);
    if (n > SIM_NV_LP_MAX_N) return fail(err, SIM_EUNSUPPORTED, "n=%u above %u on the general-constraint path", n, SIM_NV_LP_MAX_N);
    if (R * T > (1ull << 24)) return fail(err, SIM_EINVAL, "R T above 2^24 (the vertex record)");
    if (!con->A || !con->C) return fail(err, SIM_EINVAL, "A and C are required");
    for (uint32_t i = 0; i < M; ++i)
        if (!finite(con->C[i]) || !(con->C[i] > 0.0)) return fail(err, SIM_EINVAL, "C[%u] must be finite and > 0", i);
    for (uint32_t j = 0; j < n; ++j) {
        bool pos = false;
        for (uint32_t i = 0; i < M; ++i) {
            const double a = con->A[static_cast<size_t>(i) * n + j];
            if (!finite(a) || a < 0.0) return fail(err, SIM_EINVAL, "A[%u][%u] must be finite and >= 0", i, j);
            pos = pos || a > 0.0;
        }
        if (!pos) return fail(err, SIM_EINVAL, "product %u uses no resource: X would be unbounded", j);
    }
    if (p->x0)
        for (uint32_t i = 0; i < M; ++i) {
            double used = 0.0;
            for (uint32_t j = 0; j < n; ++j) used += con->A[static_cast<size_t>(i) * n + j] * p->x0[j];
            if (used > con->C[i] * (1.0 + 1e-12)) return fail(err, SIM_EINVAL, "x0 uses %g > C[%u] of resource %u", used, i, i);
        }
    return SIM_OK;
}

int validate_sqn(char *err, const sim_sqn_params *p, uint64_t N, uint32_t n, uint64_t R, uint64_t K)
{
    if (!p) return fail(err, SIM_EINVAL, "params is NULL");
    if (p->abi_version != SIM_ABI_VERSION)
        return fail(err, SIM_EINVAL, "abi_version %u != %u", p->abi_version, SIM_ABI_VERSION);
    if (n < 1 || n > SIM_SQN_MAX_N) return fail(err, SIM_EINVAL, "n=%u outside [1, %u]", n, SIM_SQN_MAX_N);
    if (N < 1 || N >= (1ull << 31)) return fail(err, SIM_EINVAL, "N=%llu outside [1, 2^31)", (unsigned long long)N);
    if (R < 1 || R > SIM_SQN_MAX_R)
        return fail(err, SIM_EINVAL, "R=%llu outside [1, %u]", (unsigned long long)R, SIM_SQN_MAX_R);
    if (K < 1 || K > 0xFFFFFFFFull) return fail(err, SIM_EINVAL, "K=%llu outside [1, 2^32-1]", (unsigned long long)K);
    if (p->L < 1) return fail(err, SIM_EINVAL, "L must be >= 1");
    if (p->M < 1 || p->M > SIM_SQN_MAX_M) return fail(err, SIM_EINVAL, "M=%u outside [1, %u]", p->M, SIM_SQN_MAX_M);
    if (p->b < 1 || p->b > SIM_SQN_MAX_B) return fail(err, SIM_EINVAL, "b=%u outside [1, %u]", p->b, SIM_SQN_MAX_B);
    if (p->b_H < 1 || p->b_H > SIM_SQN_MAX_B)
        return fail(err, SIM_EINVAL, "b_H=%u outside [1, %u]", p->b_H, SIM_SQN_MAX_B);
    if (!finite(p->beta) || !(p->beta > 0.0)) return fail(err, SIM_EINVAL, "beta must be finite and > 0");
    if (p->n_checkpoints > SIM_MAX_CKPT) return fail(err, SIM_EINVAL, "more than 8 checkpoints");
    for (uint32_t k = 0; k < p->n_checkpoints; ++k) {
        if (p->checkpoints[k] < 1 || p->checkpoints[k] > K)
            return fail(err, SIM_EINVAL, "checkpoint %u outside [1, K]", k);
        if (k && p->checkpoints[k] <= p->checkpoints[k - 1])
            return fail(err, SIM_EINVAL, "checkpoints must increase strictly");
    }
    if (p->instance_id >= (1u << 24)) return fail(err, SIM_EINVAL, "instance_id must be < 2^24");
    if (p->pairs_fp32 > 1) return fail(err, SIM_EINVAL, "pairs_fp32 must be 0 or 1");
    return SIM_OK;
}

void fill_schedule(const sim_params *p, uint64_t T, std::vector<unsigned char> &buf, SchedLayout &L)
{
    const uint64_t E = (T + p->resample_every - 1) / p->resample_every;
    const uint32_t d = p->d;
    auto up = [](uint64_t x) { return (x + 255) / 256 * 256; };
    L.epochs = E;
    L.off_n = 0;
    L.off_inv_f = up(L.off_n + 4 * E);
    L.off_inv_d = up(L.off_inv_f + 4 * E);
    L.off_c_f = up(L.off_inv_d + 8 * E);
    L.off_c_d = up(L.off_c_f + 4 * E * 2 * d);
    L.bytes = up(L.off_c_d + 8 * E * 2 * d);
    buf.assign(L.bytes, 0);
    uint32_t *n = reinterpret_cast<uint32_t *>(buf.data() + L.off_n);
    float *inv_f = reinterpret_cast<float *>(buf.data() + L.off_inv_f);
    double *inv_d = reinterpret_cast<double *>(buf.data() + L.off_inv_d);
    float *cf = reinterpret_cast<float *>(buf.data() + L.off_c_f);
    double *cd = reinterpret_cast<double *>(buf.data() + L.off_c_d);
    const double kappa = fw::kBoxMullerScale;
    for (uint64_t e = 0; e < E; ++e) {
        // the coefficients of fill_desc with N = N_k, rounded the same way
        const double N = (double)p->n_schedule[e];
        n[e] = p->n_schedule[e];
        inv_f[e] = (float)(1.0 / N);
        inv_d[e] = 1.0 / N;
        for (uint32_t j = 0; j < d; ++j) {
            const double sg = p->sigma[j], sz = kappa * sg;
            cf[e * 2 * d + j] = (float)(sz / N);
            cf[e * 2 * d + d + j] = (float)(2.0 * p->risk_coef * sz / (N - 1.0));
            cd[e * 2 * d + j] = sg / N;
            cd[e * 2 * d + d + j] = 2.0 * p->risk_coef * sg / (N - 1.0);
        }
    }
}

void fill_desc(InstanceDesc &D, const sim_params *p, uint64_t R, uint64_t T, uint64_t seed)
{
    std::memset(&D, 0, sizeof(D));
    D.d = p->d;
    D.N = p->n_samples;
    D.M = p->resample_every;
    D.noise = p->noise;
    D.nu = p->nu;
    D.n_ckpt = p->n_checkpoints;
    D.flags = p->flags;
    D.instance = p->instance_id;
    D.R = R;
    D.T = T;
    D.seed = seed;
    D.log_begin = (p->flags & SIM_DECISION_LOG) ? p->log_rep_begin : 0;
    D.log_count = (p->flags & SIM_DECISION_LOG) ? p->log_rep_count : 0;
    for (uint32_t k = 0; k < p->n_checkpoints; ++k) D.ckpt[k] = p->checkpoints[k];
    D.lambda = p->risk_coef;
    D.gap_eps = p->gap_eps;
    D.has_w0 = p->w0 ? 1u : 0u;
    const double N = (double)p->n_samples;
    const double kappa = fw::kBoxMullerScale;
    const double tnu = (p->noise == SIM_NOISE_T) ? std::sqrt((double)p->nu - 2.0) : 1.0;
    D.tscale_d = tnu;
    D.inv_n_d = 1.0 / N;
    D.tscale_f = (float)(tnu / kappa);
    D.inv_n_f = (float)(1.0 / N);
    if (p->flags & SIM_CV_FEATURES) {
        const CvLaw law = cv_law(p, T);
        for (uint32_t j = 0; j < p->d; ++j) {
            D.cv_b[j] = (float)p->cv_ref[j];
            D.cv_s[j] = (float)(cv_scale(p, j) * kappa / N);
        }
        for (uint32_t c = 0; c <= p->d; ++c) {
            D.cv_mean[c] = law.mean[c];
            D.cv_inv[c] = law.inv[c];
        }
        D.cv_mean1 = law.mean1;
        D.cv_inv1 = law.inv1;
        D.cv_top = law.top;
    }
    for (uint32_t j = 0; j < p->d; ++j) {
        // with a dense L the per-asset scale is the marginal standard deviation |row j of L|
        double sg = 0.0;
        if (p->chol) {
            for (uint32_t k = 0; k <= j; ++k) sg += p->chol[j * p->d + k] * p->chol[j * p->d + k];
            sg = std::sqrt(sg);
        } else {
            sg = p->sigma[j];
        }
        const double mu = p->mu[j], w0 = p->w0 ? p->w0[j] : 0.0;
        D.mu_d[j] = mu;
        D.sig_d[j] = sg;
        D.w0_d[j] = w0;
        D.c1_d[j] = sg / N;
        D.c2_d[j] = 2.0 * p->risk_coef * sg / (N - 1.0);
        const double sz = kappa * sg;
        D.mu_f[j] = (float)mu;
        D.sz_f[j] = (float)sz;
        D.isz_f[j] = sz > 0.0 ? (float)(1.0 / sz) : 0.0f;
        D.w0_f[j] = (float)w0;
        D.c1_f[j] = (float)(sz / N);
        D.c2_f[j] = (float)(2.0 * p->risk_coef * sz / (N - 1.0));
    }
}

// ---- double-double arithmetic for the final statistics ----------------------------------------
struct DD {
    double h, l;
};
DD two_sum(double a, double b)
{
    double s = a + b, bb = s - a;
    return {s, (a - (s - bb)) + (b - bb)};
}
DD dd_add(DD a, DD b)
{
    DD s = two_sum(a.h, b.h);
    double e = s.l + a.l + b.l;
    double h = s.h + e;
    return {h, e - (h - s.h)};
}
DD dd_neg(DD a) { return {-a.h, -a.l}; }
DD dd_mul(DD a, DD b)
{
    double p = a.h * b.h;
    double e = std::fma(a.h, b.h, -p) + (a.h * b.l + a.l * b.h);
    double h = p + e;
    return {h, e - (h - p)};
}
DD dd_div_d(DD a, double b)
{
    double q1 = a.h / b;
    DD p = dd_mul({q1, 0.0}, {b, 0.0});
    DD r = dd_add(a, dd_neg(p));
    double q2 = r.h / b;
    DD q = two_sum(q1, q2);
    return q;
}

struct Moments {
    double mean, var, n;
};
Moments moments(const double *f)
{
    const DD S{f[0], f[1]}, Q{f[2], f[3]};
    const double n = f[4];
    Moments m{0.0, 0.0, n};
    if (n <= 0.0) return m;
    DD mean = dd_div_d(S, n);
    m.mean = mean.h + mean.l;
    if (n > 1.0) {
        DD ss = dd_div_d(dd_mul(S, S), n);
        DD num = dd_add(Q, dd_neg(ss));
        DD var = dd_div_d(num, n - 1.0);
        m.var = var.h + var.l;
        if (m.var < 0.0) m.var = 0.0;
    }
    return m;
}

// min over W of lambda sum sigma_j^2 w_j^2 - mu'w (KKT water-filling), diagonal Sigma with every
// sigma_j > 0: w_j(nu) = max(0, (mu_j - nu) / (2 lambda sigma_j^2)) with nu >= 0 chosen so that
// sum_j w_j <= 1 holds with complementary slackness. NaN when some sigma_j is zero.
namespace {

double normal_cdf(double x) { return 0.5 * std::erfc(-x / std::sqrt(2.0)); }

// Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on P_n (three-term recurrence)
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    const double pi = 3.14159265358979323846;
    for (int i = 0; i < (n + 1) / 2; ++i) {
        double z = std::cos(pi * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= n; ++k) {
                const double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = pk;
            }
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            const double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-16) break;
        }
        double p0 = 1.0, p1 = z;
        for (int k = 2; k <= n; ++k) {
            const double pk = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
            p0 = p1;
            p1 = pk;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[i] = -z;
        x[n - 1 - i] = z;
        w[i] = w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

}  // namespace

void cv_pick_probs(uint32_t d, const double *b, const double *s, double *p)
{
    // origin: every b_k - s_k Z_k >= 0; vertex a: b_a - s_a z < 0 and below every other value,
    // integrated over z > b_a / s_a with 16-point Gauss-Legendre panels of width <= 1/8
    static std::vector<double> gx, gw;
    if (gx.empty()) gauss_legendre(16, gx, gw);
    double p0 = 1.0;
    for (uint32_t k = 0; k < d; ++k) p0 *= normal_cdf(b[k] / s[k]);
    p[0] = p0;
    const double inv_sqrt_2pi = 0.39894228040143267793994605993438;
    for (uint32_t a = 0; a < d; ++a) {
        const double lo = std::max(b[a] / s[a], -13.0), hi = 13.0;
        double acc = 0.0;
        if (lo < hi) {
            const int panels = (int)std::ceil((hi - lo) * 8.0);
            const double h = (hi - lo) / panels;
            for (int q = 0; q < panels; ++q) {
                const double c = lo + (q + 0.5) * h;
                for (int i = 0; i < 16; ++i) {
                    const double z = c + 0.5 * h * gx[i];
                    double f = inv_sqrt_2pi * std::exp(-0.5 * z * z);
                    for (uint32_t k = 0; k < d; ++k)
                        if (k != a) f *= normal_cdf((b[k] - b[a] + s[a] * z) / s[k]);
                    acc += 0.5 * h * gw[i] * f;
                }
            }
        }
        p[a + 1] = acc;
    }
}

double cv_scale(const sim_params *p, uint32_t j) { return p->chol ? p->chol[j * p->d + j] : p->sigma[j]; }

CvLaw cv_law(const sim_params *p, uint64_t T)
{
    CvLaw L;
    const uint32_t d = p->d, M = p->resample_every;
    std::vector<double> s(d);
    for (uint32_t j = 0; j < d; ++j) s[j] = cv_scale(p, j) / std::sqrt((double)p->n_samples);
    cv_pick_probs(d, p->cv_ref, s.data(), L.p);
    // per epoch e: W2_e, W1_e = sums of (t+1)^2 and (t+1) over its iterations;
    // S2 = sum W2_e, S4 = sum W2_e^2, S1 = sum W1_e, S11 = sum W1_e^2
    L.S2 = L.S4 = L.S1 = L.S11 = 0.0;
    L.epochs = 0;
    for (uint64_t t0 = 0; t0 < T; t0 += M, ++L.epochs) {
        const uint64_t t1 = std::min<uint64_t>(t0 + M, T);
        const double w2 = (double)(t1 * (t1 + 1) * (2 * t1 + 1) / 6 - t0 * (t0 + 1) * (2 * t0 + 1) / 6);
        const double w1 = (double)(t1 * (t1 + 1) / 2 - t0 * (t0 + 1) / 2);
        L.S2 += w2;
        L.S4 += w2 * w2;
        L.S1 += w1;
        L.S11 += w1 * w1;
    }
    auto inv_sd = [](double S, double p) { return 1.0 / std::sqrt(S * std::max(p * (1.0 - p), 1e-4)); };
    double cum = 0.0;
    L.top = 0;
    for (uint32_t c = 0; c <= d; ++c) {
        L.mean[c] = L.p[c] * L.S2;
        L.inv[c] = inv_sd(L.S4, L.p[c]);
        cum += L.p[c];
        L.cum[c] = cum;
        if (L.p[c] > L.p[L.top]) L.top = c;
    }
    L.cum[d] = 2.0;   // every uniform falls below the last bound
    L.mean1 = L.p[L.top] * L.S1;
    L.inv1 = inv_sd(L.S11, L.p[L.top]);
    return L;
}

int dense_asset_of(int p, int k) { return (k >> 2) * 16 + 4 * p + (k & 3); }

void dense_operands(const double *L, uint32_t d, float *Ag, float *Av, double *L64)
{
    const double kappa = fw::kBoxMullerScale;
    const uint32_t K = d / 4;
    for (uint32_t mt = 0; mt < d / 16; ++mt)
        for (uint32_t kk = 0; kk < K; ++kk)
            for (uint32_t lane = 0; lane < 64; ++lane) {
                const uint32_t row = 16 * mt + (lane & 15);
                const uint32_t col = (uint32_t)dense_asset_of((int)(lane >> 4), (int)kk);
                const size_t at = ((size_t)mt * K + kk) * 64 + lane;
                Ag[at] = (float)(kappa * L[row * d + col]);   // g = L h
                Av[at] = (float)(kappa * L[col * d + row]);   // v = L'w
            }
    for (uint32_t i = 0; i < d * d; ++i) L64[i] = L[i];
}

double kkt_fstar(const double *mu, const double *sigma, uint32_t d, double lambda)
{
    for (uint32_t j = 0; j < d; ++j)
        if (!(sigma[j] > 0.0)) return NAN;
    auto w_of = [&](double nu, uint32_t j) {
        const double w = (mu[j] - nu) / (2.0 * lambda * sigma[j] * sigma[j]);
        return w > 0.0 ? w : 0.0;
    };
    auto total = [&](double nu) {
        double s = 0.0;
        for (uint32_t j = 0; j < d; ++j) s += w_of(nu, j);
        return s;
    };
    double nu = 0.0;
    if (total(0.0) > 1.0) {
        double lo = 0.0, hi = 0.0;
        for (uint32_t j = 0; j < d; ++j) hi = mu[j] > hi ? mu[j] : hi;
        for (int it = 0; it < 200; ++it) {
            const double mid = 0.5 * (lo + hi);
            if (total(mid) > 1.0) lo = mid;
            else hi = mid;
        }
        nu = hi;
    }
    double f = 0.0;
    for (uint32_t j = 0; j < d; ++j) {
        const double w = w_of(nu, j);
        f += lambda * sigma[j] * sigma[j] * w * w - mu[j] * w;
    }
    return f;
}

void fill_stats(sim_stats_out *out, const double *F, uint32_t nc, const uint64_t *ckpts, double ymin,
                double ymax, const uint64_t *dec, uint32_t d, uint64_t tau_count, uint64_t tau_sum, uint64_t R,
                uint64_t T, double fstar, double ms, double path_steps)
{
    std::memset(out, 0, sizeof(*out));
    out->R = R;
    out->T = T;
    Moments y = moments(F);
    out->mean = y.mean;
    out->var = y.var;
    out->ci95_halfwidth = 1.96 * std::sqrt(y.var / (double)R);
    out->min = ymin;
    out->max = ymax;
    out->f_star = fstar;
    out->n_checkpoints = nc;
    for (uint32_t k = 0; k < nc; ++k) {
        out->checkpoints[k] = ckpts[k];
        Moments f = moments(F + (1 + k) * fw::kStreamFields);
        Moments e = moments(F + (1 + nc + k) * fw::kStreamFields);
        out->f_mean[k] = f.mean;
        out->f_sd[k] = std::sqrt(f.var);
        out->rse_mean[k] = e.mean;
        out->rse_sd[k] = std::sqrt(e.var);
        out->rse_undefined[k] = R - (uint64_t)e.n;
    }
    for (uint32_t j = 0; j <= d; ++j) out->decision_total[j] = dec[j];
    out->tau_count = tau_count;
    out->tau_mean = tau_count ? (double)tau_sum / (double)tau_count : 0.0;
    out->kernel_ms = ms;
    out->path_steps_per_s = ms > 0.0 ? path_steps / (ms * 1e-3) : 0.0;
}


namespace {

uint32_t reps_per_tile(uint32_t P) { return 64u / P; }

uint32_t log2u(uint32_t x)
{
    uint32_t k = 0;
    while ((1u << k) < x) ++k;
    return k;
}

}  // namespace

uint32_t asset_lanes(uint32_t d)
{
    uint32_t Pa = 1;
    while (Pa * 8u < d) Pa *= 2;
    return Pa;
}

uint32_t chunk_of(uint32_t N, uint32_t d, uint32_t Ps, bool t_noise)
{
    const uint32_t align = t_noise ? 4u : ((d & 3u) == 0 ? 1u : ((d & 1u) == 0 ? 2u : 4u));
    uint32_t c = (N + Ps - 1) / Ps;
    return (c + align - 1) / align * align;
}

// Work of one lane of one tile per run, in VALU instructions: ~80 per Philox block drawn (four
// normals), ~40 per sample read back (eight products and sums, butterfly steps), ~20 chi-square
// normals' worth per t sample, ~150 per iteration for the gradient, subproblem and update, and
// 32 per stage of the butterfly over the sample lanes.
double lane_cost(const sim_params &p, uint64_t T, uint32_t P)
{
    const bool t_noise = p.noise == SIM_NOISE_T;
    const uint32_t d = p.d, Pa = asset_lanes(d), Ps = P / Pa;
    const uint32_t G = (d & 3u) == 0 ? 1u : ((d & 1u) == 0 ? 2u : 4u);
    const double rounds = (double)chunk_of(p.n_samples, d, Ps, t_noise) / G;
    const double blocks = std::ceil((double)(G * d / 4) / Pa);
    const double per_round = 80.0 * blocks + G * (40.0 + 4.0 * log2u(Pa) + (t_noise ? 20.0 * p.nu : 0.0));
    return (double)T * (rounds * per_round + 150.0 + 32.0 * log2u(Ps));
}

// Every bound the tile kernels read from the plan, checked on the finished tables before any
// upload: the tile range of each class launch, the lanes per replication and replications per
// wavefront, the replication range of each tile, the slot permutation and its per-instance
// ranges, the signature width (33 bits) and the numbering of each lane's normals.
static int check_plan(char *err, uint32_t n_inst, const sim_params *p, const uint64_t *R, const uint64_t *T,
                      const BatchPlan &P)
{
    const uint64_t n = P.n_tiles;
    if (P.tiles.size() != n) return fail(err, SIM_EINVAL, "plan: tile table size");
    if (P.slot_begin.size() != (size_t)n_inst + 1 || P.slot_begin[0] != 0 || P.slot_begin[n_inst] != n)
        return fail(err, SIM_EINVAL, "plan: slot ranges do not cover the tiles");
    for (uint32_t i = 0; i < n_inst; ++i) {
        if (P.slot_begin[i] > P.slot_begin[i + 1]) return fail(err, SIM_EINVAL, "plan: slot ranges decrease");
        if (T[i] > kMaxBatchT)
            return fail(err, SIM_EUNSUPPORTED, "instance %u: T=%llu above %llu in a batch (33-bit signature)", i,
                        (unsigned long long)T[i], (unsigned long long)kMaxBatchT);
        if (P.desc[i].R != R[i] || P.desc[i].T != T[i] || P.desc[i].d != p[i].d || P.desc[i].N != p[i].n_samples)
            return fail(err, SIM_EINVAL, "plan: descriptor %u disagrees with the parameters", i);
    }
    std::vector<uint8_t> seen(n, 0);
    std::vector<uint64_t> reps(n_inst, 0);
    for (uint64_t q = 0; q < n; ++q) {
        const Tile &tl = P.tiles[q];
        if (tl.inst >= n_inst) return fail(err, SIM_EINVAL, "plan: tile %llu names instance %u", (unsigned long long)q, tl.inst);
        const sim_params &pi = p[tl.inst];
        const uint32_t L = tl.P;
        if (L < 1 || L > 64 || (L & (L - 1))) return fail(err, SIM_EINVAL, "plan: tile %llu has %u lanes per replication", (unsigned long long)q, L);
        if (tl.Pa != asset_lanes(pi.d) || L % tl.Pa)
            return fail(err, SIM_EINVAL, "plan: tile %llu splits %u assets over %u lanes", (unsigned long long)q, pi.d, tl.Pa);
        if (tl.nrep < 1 || tl.nrep * L > 64) return fail(err, SIM_EINVAL, "plan: tile %llu holds %u replications", (unsigned long long)q, tl.nrep);
        if ((uint64_t)tl.rep0 + tl.nrep > R[tl.inst]) return fail(err, SIM_EINVAL, "plan: tile %llu exceeds R", (unsigned long long)q);
        if (tl.slot >= n || seen[tl.slot] || tl.slot < P.slot_begin[tl.inst] || tl.slot >= P.slot_begin[tl.inst + 1])
            return fail(err, SIM_EINVAL, "plan: tile %llu has slot %u", (unsigned long long)q, tl.slot);
        seen[tl.slot] = 1;
        const bool tn = pi.noise == SIM_NOISE_T;
        if (pi.d > 8u * tl.Pa || pi.d > 32u) return fail(err, SIM_EINVAL, "plan: tile %llu holds d=%u", (unsigned long long)q, pi.d);
        const uint32_t Ps = L / tl.Pa;
        const uint64_t chunk = chunk_of(pi.n_samples, pi.d, Ps, tn);
        if (chunk * Ps < pi.n_samples) return fail(err, SIM_EINVAL, "plan: tile %llu leaves samples out", (unsigned long long)q);
        // highest normal a lane draws: its chunk's numerators with the overrun of its last round
        // (at most 32 Pa normals) and the second block of a pair, and the chi-square normals of
        // the same samples
        const uint64_t top = (uint64_t)pi.n_samples * pi.d + (tn ? (chunk * Ps + 32 * tl.Pa + 1) * pi.nu : 0) +
                             chunk * Ps * pi.d + 32 * tl.Pa + 4 * (2 * tl.Pa + 1);
        if (top > 0xFFFFFFFFull) return fail(err, SIM_EINVAL, "plan: tile %llu numbers normals past 2^32", (unsigned long long)q);
        reps[tl.inst] += tl.nrep;
    }
    for (uint32_t i = 0; i < n_inst; ++i)
        if (reps[i] != R[i]) return fail(err, SIM_EINVAL, "plan: instance %u covers %llu of %llu replications", i,
                                         (unsigned long long)reps[i], (unsigned long long)R[i]);
    return SIM_OK;
}

static int plan_batch_impl(char *err, uint32_t n_inst, const sim_params *p, const uint64_t *R, const uint64_t *T,
                           uint64_t seed, const sim_batch_config *cfg, uint32_t n_cu, BatchPlan &out)
{
    if (n_inst < 1 || n_inst > 65536 || !p || !R || !T)
        return fail(err, SIM_EINVAL, "need 1 <= n_inst <= 65536 and non-NULL p, R, T");
    if (n_cu < 1) return fail(err, SIM_EINVAL, "n_cu must be >= 1");
    for (uint32_t i = 0; i < n_inst; ++i) {
        int rc = validate(err, &p[i], R[i], T[i]);
        if (rc) return rc;
        if (p[i].n_schedule) return fail(err, SIM_EUNSUPPORTED, "instance %u: n_schedule in a batch", i);
        if (p[i].state_precision != SIM_FP32)
            return fail(err, SIM_EUNSUPPORTED, "instance %u: batched runs use FP32 state", i);
        if (p[i].d > 32) return fail(err, SIM_EUNSUPPORTED, "instance %u: d > 32 in a batch", i);
        if (T[i] > kMaxBatchT)
            return fail(err, SIM_EUNSUPPORTED, "instance %u: T above %llu in a batch (33-bit signature)", i,
                        (unsigned long long)kMaxBatchT);
        if (p[i].chol) return fail(err, SIM_EUNSUPPORTED, "instance %u: batched runs take diagonal Sigma", i);
        if (p[i].flags & SIM_CV_FEATURES)
            return fail(err, SIM_EUNSUPPORTED, "instance %u: batched runs do not write features", i);
        if (cfg && cfg->lanes_per_rep) {
            const uint32_t P = cfg->lanes_per_rep[i];
            if (P != 0 && (P > 64 || (P & (P - 1)) != 0))
                return fail(err, SIM_EINVAL, "instance %u: lanes_per_rep must be 0 or a power of two <= 64", i);
        }
    }
    if (cfg && (!(cfg->heavy_factor >= 0.0) || !std::isfinite(cfg->heavy_factor)))
        return fail(err, SIM_EINVAL, "heavy_factor must be finite and >= 0");
    if (cfg && (cfg->flags & ~(uint32_t)(SIM_KEEP_PATHS | SIM_BATCH_GRAPH)))
        return fail(err, SIM_EINVAL, "unknown batch flag bits");
    if (cfg && cfg->reserved) return fail(err, SIM_EINVAL, "reserved field must be 0");

    // lanes per replication: the asset lanes d needs, times the smallest power of two of sample
    // lanes whose per-lane work fits theta x the balanced run time
    const double n_simd = 4.0 * n_cu;
    const double theta = (cfg && cfg->heavy_factor > 0.0) ? cfg->heavy_factor : 0.5;
    out.P.assign(n_inst, 1u);
    for (uint32_t i = 0; i < n_inst; ++i) out.P[i] = asset_lanes(p[i].d);
    for (int pass = 0; pass < 3; ++pass) {
        double total = 0.0;
        for (uint32_t i = 0; i < n_inst; ++i) {
            const uint64_t tiles = (R[i] + reps_per_tile(out.P[i]) - 1) / reps_per_tile(out.P[i]);
            total += tiles * lane_cost(p[i], T[i], out.P[i]);
        }
        const double target = theta * total / n_simd;
        for (uint32_t i = 0; i < n_inst; ++i) {
            uint32_t P = asset_lanes(p[i].d);
            while (P < 64 && lane_cost(p[i], T[i], P) > target) P *= 2;
            out.P[i] = P;
        }
    }
    if (cfg && cfg->lanes_per_rep)
        for (uint32_t i = 0; i < n_inst; ++i)
            if (cfg->lanes_per_rep[i]) {
                if (cfg->lanes_per_rep[i] < asset_lanes(p[i].d))
                    return fail(err, SIM_EINVAL, "instance %u: lanes_per_rep %u below the %u lanes its d=%u assets need",
                                i, cfg->lanes_per_rep[i], asset_lanes(p[i].d), p[i].d);
                out.P[i] = cfg->lanes_per_rep[i];
            }

    out.tiles_of.assign(n_inst, 0u);
    out.slot_begin.assign(n_inst + 1, 0u);
    out.path_base.assign(n_inst, 0);
    out.cnt_base.assign(n_inst, 0);
    out.wsum_base.assign(n_inst, 0);
    out.dlog_base.assign(n_inst, 0);
    uint64_t n_tiles = 0, total_R = 0, cntb = 0, wsb = 0, dlb = 0, steps = 0;
    uint32_t max_ckpt = 1;
    for (uint32_t i = 0; i < n_inst; ++i) {
        const uint32_t rpt = reps_per_tile(out.P[i]);
        const uint64_t nt = (R[i] + rpt - 1) / rpt;
        if (n_tiles + nt > 0xFFFFFFFFull) return fail(err, SIM_EINVAL, "more than 2^32 - 1 tiles");
        out.tiles_of[i] = (uint32_t)nt;
        out.slot_begin[i] = (uint32_t)n_tiles;
        n_tiles += nt;
        out.path_base[i] = total_R;
        out.cnt_base[i] = cntb;
        out.wsum_base[i] = wsb;
        out.dlog_base[i] = dlb;
        cntb += (uint64_t)(p[i].d + 1) * R[i];
        wsb += (uint64_t)p[i].d * R[i];
        if (p[i].flags & SIM_DECISION_LOG) dlb += T[i] * p[i].log_rep_count;
        total_R += R[i];
        steps += R[i] * T[i];
        max_ckpt = std::max(max_ckpt, p[i].n_checkpoints);
    }
    out.slot_begin[n_inst] = (uint32_t)n_tiles;
    out.n_tiles = (uint32_t)n_tiles;
    out.total_R = total_R;
    out.total_steps = steps;
    out.cnt_total = cntb;
    out.wsum_total = wsb;
    out.dlog_total = dlb;
    out.max_ckpt = max_ckpt;

    out.desc.assign(n_inst, InstanceDesc{});
    out.fstar.assign(n_inst, NAN);
    for (uint32_t i = 0; i < n_inst; ++i) {
        InstanceDesc &D = out.desc[i];
        fill_desc(D, &p[i], R[i], T[i], seed);
        D.path_base = out.path_base[i];
        D.cnt_base = out.cnt_base[i];
        D.wsum_base = out.wsum_base[i];
        D.dlog_base = out.dlog_base[i];
        out.fstar[i] = kkt_fstar(p[i].mu, p[i].sigma, p[i].d, p[i].risk_coef);
    }

    // tiles in instance-major replication order get consecutive slots; hand them out longest first
    std::vector<Tile> tiles(n_tiles);
    std::vector<double> cost(n_tiles);
    uint64_t k = 0;
    for (uint32_t i = 0; i < n_inst; ++i) {
        const uint32_t rpt = reps_per_tile(out.P[i]);
        const double c = lane_cost(p[i], T[i], out.P[i]);
        for (uint32_t t = 0; t < out.tiles_of[i]; ++t, ++k) {
            Tile &tl = tiles[k];
            tl.inst = i;
            tl.rep0 = t * rpt;
            tl.slot = (uint32_t)k;
            tl.nrep = (uint16_t)std::min<uint64_t>(rpt, R[i] - (uint64_t)t * rpt);
            tl.P = (uint8_t)out.P[i];
            tl.Pa = (uint8_t)asset_lanes(p[i].d);
            cost[k] = c;
        }
    }
    // the one-wavefront form (a replication per wavefront, an asset per lane) when every instance
    // asks for 64 lanes per replication, has Gaussian noise and its N d normals fit the staging area
    out.wave_mode = n_tiles > 0;
    for (uint32_t i = 0; i < n_inst; ++i)
        if (out.P[i] != 64 || p[i].noise != SIM_NOISE_GAUSS ||
            (uint64_t)p[i].n_samples * p[i].d + 3 > kBatchStageFloats)
            out.wave_mode = false;
    std::vector<uint32_t> order(n_tiles);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return cost[a] > cost[b]; });
    out.tiles.resize(n_tiles);
    for (uint64_t q = 0; q < n_tiles; ++q) out.tiles[q] = tiles[order[q]];
    return check_plan(err, n_inst, p, R, T, out);
}

int plan_batch(char *err, uint32_t n_inst, const sim_params *p, const uint64_t *R, const uint64_t *T,
               uint64_t seed, const sim_batch_config *cfg, uint32_t n_cu, BatchPlan &out)
{
    // the plan's tables grow with the number of tiles (up to 2^32 - 1): a failed host allocation is
    // an error code, never an exception through the C interface
    try {
        return plan_batch_impl(err, n_inst, p, R, T, seed, cfg, n_cu, out);
    } catch (const std::bad_alloc &) {
        return fail(err, SIM_ENOMEM, "host memory for the batch plan");
    }
}

}  // namespace host
}  // namespace fw
