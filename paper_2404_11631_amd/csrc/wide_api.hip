// wide_api.hip -- host side of the wide path (sim_run_wide): validation, device buffers, the
// per-iteration launch sequence, and the statistics and per-path records of the last wide run.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "engine.hpp"
#include "wide.hpp"

using namespace fw::host;

namespace {

int ensure_events(sim_ctx *ctx, WideState &w)
{
    if (!w.ev0) HIP_TRY(ctx, hipEventCreate(&w.ev0));
    if (!w.ev1) HIP_TRY(ctx, hipEventCreate(&w.ev1));
    return SIM_OK;
}

// The largest sample size over the run's epochs.
uint32_t wide_nmax(const sim_params *p, uint64_t T)
{
    uint32_t n = p->n_samples;
    if (p->n_schedule) {
        const uint64_t epochs = (T + p->resample_every - 1) / p->resample_every;
        for (uint64_t e = 0; e < epochs; ++e) n = std::max(n, p->n_schedule[e]);
    }
    return n;
}

// Device arguments over the context's wide buffers for problem p.
fw::WideArgs wide_args(WideState &w, const sim_params *p, uint64_t R, uint64_t T, uint64_t seed)
{
    fw::WideArgs A{};
    const uint32_t d = p->d;
    A.d = d;
    A.nq = d / 4;
    A.N = wide_nmax(p, T);
    A.nwg = w.nwg;
    A.R = static_cast<uint32_t>(R);
    A.k0 = static_cast<uint32_t>(seed);
    A.k1 = static_cast<uint32_t>(seed >> 32);
    A.dom = p->instance_id & 0xFFFFFFu;
    A.gap_eps = static_cast<float>(p->gap_eps);
    A.lambda = p->risk_coef;
    const float *af = static_cast<const float *>(w.asset_f.ptr);
    A.mu_f = af;
    A.sz_f = af + d;
    A.c1_f = af + 2 * static_cast<size_t>(d);
    A.c2_f = af + 3 * static_cast<size_t>(d);
    A.w0_f = af + 4 * static_cast<size_t>(d);
    const double *ad = static_cast<const double *>(w.asset_d.ptr);
    A.mu_d = ad;
    A.sig_d = ad + d;
    A.S = static_cast<uint64_t *>(w.S.ptr);
    A.cnt = static_cast<uint32_t *>(w.cnt.ptr);
    A.tau = static_cast<uint32_t *>(w.tau.ptr);
    A.dec = static_cast<uint32_t *>(w.dec.ptr);
    A.T = T;
    A.s1 = static_cast<float *>(w.s1.ptr);
    A.part_dot = static_cast<float *>(w.part_dot.ptr);
    A.part_qn = static_cast<float *>(w.part_qn.ptr);
    A.dot = static_cast<float *>(w.dot.ptr);
    A.qn = static_cast<float *>(w.qn.ptr);
    A.wg_g = static_cast<float *>(w.wg_g.ptr);
    A.wg_j = static_cast<uint32_t *>(w.wg_j.ptr);
    A.wg_gw = static_cast<float *>(w.wg_gw.ptr);
    A.fval = static_cast<double *>(w.fval.ptr);
    A.stats = static_cast<double *>(w.stats.ptr);
    A.origin_total = static_cast<uint64_t *>(w.origin.ptr);
    return A;
}

}  // namespace

extern "C" {

int sim_validate_wide(const sim_params *p, uint64_t R, uint64_t T, char *msg, size_t len)
{
    char err[kErrLen] = {0};
    const int rc = validate_wide(err, p, R, T);
    if (msg && len) std::snprintf(msg, len, "%s", rc ? err : "");
    return rc;
}

int sim_run_wide(sim_ctx *ctx, const sim_params *p, uint64_t R, uint64_t T, uint64_t seed)
{
    if (!ctx) return SIM_EINVAL;
    if (int rc = validate_wide(ctx->err, p, R, T)) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    WideState &w = ctx->wide;
    w.have = false;
    if (int rc = ensure_events(ctx, w)) return rc;
    const uint32_t d = p->d, N = p->n_samples, nc = p->n_checkpoints;
    const uint32_t Nmax = wide_nmax(p, T);
    const uint32_t nq = d / 4;
    w.nwg = (nq + fw::kWideQuads - 1) / fw::kWideQuads;
    const size_t D = d;

    // per-asset coefficients (FP32 in units of the scaled normals, FP64 for the objective)
    const double kappa = fw::kBoxMullerScale;
    std::vector<float> af;
    std::vector<double> ad;
    try {
        af.resize(5 * D);
        ad.resize(2 * D);
    } catch (const std::bad_alloc &) {
        return set_err(ctx, SIM_ENOMEM, "host staging of the asset coefficients");
    }
    for (size_t j = 0; j < D; ++j) {
        const double sz = kappa * p->sigma[j];
        af[j] = static_cast<float>(p->mu[j]);
        af[D + j] = static_cast<float>(sz);
        af[2 * D + j] = static_cast<float>(sz / N);
        af[3 * D + j] = static_cast<float>(2.0 * p->risk_coef * sz / (N - 1.0));
        af[4 * D + j] = p->w0 ? static_cast<float>(p->w0[j]) : 0.0f;
        ad[j] = p->mu[j];
        ad[D + j] = p->sigma[j];
    }
    int rc;
    if ((rc = ensure(ctx, w.asset_f, sizeof(float) * af.size())) || (rc = ensure(ctx, w.asset_d, sizeof(double) * ad.size())) ||
        (rc = ensure(ctx, w.S, sizeof(uint64_t) * R * D)) || (rc = ensure(ctx, w.cnt, sizeof(uint32_t) * R * (D + 1))) ||
        (rc = ensure(ctx, w.tau, sizeof(uint32_t) * R)) || (rc = ensure(ctx, w.dec, sizeof(uint32_t) * R * T)) ||
        (rc = ensure(ctx, w.s1, sizeof(float) * R * D)) ||
        (rc = ensure(ctx, w.part_dot, sizeof(float) * R * Nmax * w.nwg)) ||
        (rc = ensure(ctx, w.part_qn, sizeof(float) * R * w.nwg)) || (rc = ensure(ctx, w.dot, sizeof(float) * R * Nmax)) ||
        (rc = ensure(ctx, w.qn, sizeof(float) * R)) || (rc = ensure(ctx, w.wg_g, sizeof(float) * 2 * R * w.nwg)) ||
        (rc = ensure(ctx, w.wg_j, sizeof(uint32_t) * 2 * R * w.nwg)) ||
        (rc = ensure(ctx, w.wg_gw, sizeof(float) * 2 * R * w.nwg)) ||
        (rc = ensure(ctx, w.fval, sizeof(double) * R * (nc + 1))) ||
        (rc = ensure(ctx, w.stats, sizeof(double) * (fw::kMaxStreams * fw::kStreamFields + 2))) ||
        (rc = ensure(ctx, w.origin, sizeof(uint64_t))))
        return rc;
    hipStream_t st = ctx->stream;
    HIP_TRY(ctx, hipMemcpyAsync(w.asset_f.ptr, af.data(), sizeof(float) * af.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipMemcpyAsync(w.asset_d.ptr, ad.data(), sizeof(double) * ad.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipMemsetAsync(w.S.ptr, 0, sizeof(uint64_t) * R * D, st));
    HIP_TRY(ctx, hipMemsetAsync(w.cnt.ptr, 0, sizeof(uint32_t) * R * (D + 1), st));
    HIP_TRY(ctx, hipMemsetAsync(w.tau.ptr, 0xFF, sizeof(uint32_t) * R, st));
    // the host vectors must outlive the copies
    HIP_TRY(ctx, hipStreamSynchronize(st));

    const fw::WideArgs A = wide_args(w, p, R, T, seed);
    HIP_TRY(ctx, hipEventRecord(w.ev0, st));
    // The step of iteration t runs inside the next iteration's sample launch unless an objective
    // evaluation needs the updated signature first or t is the last iteration.
    const int lrc = fw::wide_sequence(
        N, p->n_schedule, p->resample_every, T, p->w0 != nullptr, nc, p->checkpoints,
        [&](uint64_t t, uint32_t e, const fw::WideEpoch &E, float cw, bool from_w0, bool fold_prev) {
            return fw::launch_wide_iteration(A, t, e, E, cw, from_w0, fold_prev, st)
                       ? set_err(ctx, SIM_EDEVICE, "wide launch failed at t=%llu", (unsigned long long)t)
                       : 0;
        },
        [&](uint64_t t) {
            return fw::launch_wide_step(A, t, st)
                       ? set_err(ctx, SIM_EDEVICE, "wide step launch failed at t=%llu", (unsigned long long)t)
                       : 0;
        },
        [&](double c, uint32_t slot) {
            return fw::launch_wide_objective(A, c, slot, st) ? set_err(ctx, SIM_EDEVICE, "wide objective launch failed") : 0;
        });
    if (lrc) return lrc;
    if (fw::launch_wide_objective(A, 2.0 / (static_cast<double>(T) * static_cast<double>(T + 1)), nc, st) ||
        fw::launch_wide_finalize(A, nc, st))
        return set_err(ctx, SIM_EDEVICE, "wide finalize launch failed");
    HIP_TRY(ctx, hipEventRecord(w.ev1, st));

    w.params = *p;
    w.params.mu = w.params.sigma = w.params.chol = w.params.w0 = w.params.cv_ref = nullptr;
    w.params.n_schedule = nullptr;
    w.R = R;
    w.T = T;
    w.fstar = kkt_fstar(p->mu, p->sigma, d, p->risk_coef);
    w.have = true;
    return SIM_OK;
}

int sim_wide_stats(sim_ctx *ctx, sim_stats_out *out)
{
    if (!ctx || !out) return SIM_EINVAL;
    WideState &w = ctx->wide;
    if (!w.have) return set_err(ctx, SIM_ESTATE, "no wide run yet");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipEventSynchronize(w.ev1));
    const uint32_t nc = w.params.n_checkpoints, n_streams = 1 + 2 * nc;
    double F[fw::kMaxStreams * fw::kStreamFields + 2];
    uint64_t origin = 0;
    std::vector<uint32_t> tau(w.R);
    HIP_TRY(ctx, hipMemcpy(F, w.stats.ptr, sizeof(double) * (n_streams * fw::kStreamFields + 2), hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(&origin, w.origin.ptr, sizeof(uint64_t), hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(tau.data(), w.tau.ptr, sizeof(uint32_t) * w.R, hipMemcpyDeviceToHost));
    float ms = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, w.ev0, w.ev1));
    uint64_t tc = 0, ts = 0;
    for (uint32_t x : tau)
        if (x != SIM_TAU_NONE) {
            ++tc;
            ts += x;
        }
    fill_stats(out, F, nc, w.params.checkpoints, F[n_streams * fw::kStreamFields], F[n_streams * fw::kStreamFields + 1],
               &origin, 0, tc, ts, w.R, w.T, w.fstar, ms, static_cast<double>(w.R) * static_cast<double>(w.T));
    return SIM_OK;
}

int sim_wide_paths(sim_ctx *ctx, sim_wide_view *out)
{
    if (!ctx || !out) return SIM_EINVAL;
    WideState &w = ctx->wide;
    if (!w.have) return set_err(ctx, SIM_ESTATE, "no wide run yet");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipEventSynchronize(w.ev1));
    std::memset(out, 0, sizeof(*out));
    out->R = w.R;
    out->T = w.T;
    out->d = w.params.d;
    out->n_checkpoints = w.params.n_checkpoints;
    const double *fv = static_cast<const double *>(w.fval.ptr);
    out->y = fv + static_cast<size_t>(w.params.n_checkpoints) * w.R;
    out->f_ckpt = w.params.n_checkpoints ? fv : nullptr;
    out->cnt = static_cast<const uint32_t *>(w.cnt.ptr);
    out->wsum = static_cast<const uint64_t *>(w.S.ptr);
    out->tau = static_cast<const uint32_t *>(w.tau.ptr);
    out->decisions = static_cast<const uint32_t *>(w.dec.ptr);
    return SIM_OK;
}

}  // extern "C"
