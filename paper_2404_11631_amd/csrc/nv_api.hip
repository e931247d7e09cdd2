// nv_api.hip -- host side of Algorithm 2 (sim_run_newsvendor): validation, device buffers, the
// per-iteration launch sequence, and the statistics and records of the last newsvendor run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "engine.hpp"
#include "newsvendor.hpp"

using namespace fw::host;

namespace {

fw::NvArgs nv_args(NvState &w, const sim_nv_params *p, uint64_t R, uint64_t T, uint64_t seed)
{
    fw::NvArgs A{};
    const uint32_t n = p->n;
    const size_t N = n;
    A.n = n;
    A.nq = n / 4;
    A.S = p->n_samples;
    A.nwg = w.nwg;
    A.P = w.P;
    A.R = static_cast<uint32_t>(R);
    A.k0 = static_cast<uint32_t>(seed);
    A.k1 = static_cast<uint32_t>(seed >> 32);
    A.dom = (fw::kNvDomain << 24) | (p->instance_id & 0xFFFFFFu);
    A.C = static_cast<float>(p->C);
    A.gap_eps = static_cast<float>(p->gap_eps);
    const float *f = static_cast<const float *>(w.prod_f.ptr);
    A.mu_f = f;
    A.isk_f = f + N;
    A.a_f = f + 2 * N;
    A.b_f = f + 3 * N;
    A.ic_f = f + 4 * N;
    A.xs_f = f + 5 * N;
    A.x0_f = f + 6 * N;
    const double *d = static_cast<const double *>(w.prod_d.ptr);
    A.mu_d = d;
    A.sig_d = d + N;
    A.k_d = d + 2 * N;
    A.h_d = d + 3 * N;
    A.v_d = d + 4 * N;
    A.xs_d = d + 5 * N;
    A.S_sig = static_cast<uint64_t *>(w.S.ptr);
    A.cnt = static_cast<uint32_t *>(w.cnt.ptr);
    A.tau = static_cast<uint32_t *>(w.tau.ptr);
    A.dec = static_cast<uint32_t *>(w.dec.ptr);
    A.T = T;
    A.wg_r = static_cast<float *>(w.wg_r.ptr);
    A.wg_j = static_cast<uint32_t *>(w.wg_j.ptr);
    A.wg_gx = static_cast<float *>(w.wg_gx.ptr);
    A.cost_part = static_cast<double *>(w.cost_part.ptr);
    A.fval = static_cast<double *>(w.fval.ptr);
    A.stats = static_cast<double *>(w.stats.ptr);
    A.origin_total = static_cast<uint64_t *>(w.origin.ptr);
    return A;
}

}  // namespace

extern "C" {

int sim_validate_newsvendor(const sim_nv_params *p, uint64_t R, uint64_t T, char *msg, size_t len)
{
    char err[kErrLen] = {0};
    const int rc = validate_newsvendor(err, p, R, T);
    if (msg && len) std::snprintf(msg, len, "%s", rc ? err : "");
    return rc;
}

int sim_run_newsvendor(sim_ctx *ctx, const sim_nv_params *p, uint64_t R, uint64_t T, uint64_t seed)
{
    if (!ctx) return SIM_EINVAL;
    if (int rc = validate_newsvendor(ctx->err, p, R, T)) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    NvState &w = ctx->nv;
    w.have = false;
    if (!w.ev0) HIP_TRY(ctx, hipEventCreate(&w.ev0));
    if (!w.ev1) HIP_TRY(ctx, hipEventCreate(&w.ev1));
    const uint32_t n = p->n, nc = p->n_checkpoints;
    const uint32_t nq = n / 4;
    w.P = fw::nv_lanes_per_quad(nq, R, p->n_samples);
    const uint32_t quads_per_wg = fw::kNvBlock / w.P;
    w.nwg = (nq + quads_per_wg - 1) / quads_per_wg;
    const size_t N = n;

    // per product: binary32 coefficients (the normals carry the factor 1/sqrt(2 ln 2)), binary64 for Eq. (6)
    const double kappa = fw::kBoxMullerScale;
    std::vector<float> pf;
    std::vector<double> pd;
    try {
        pf.resize(7 * N);
        pd.resize(6 * N);
    } catch (const std::bad_alloc &) {
        return set_err(ctx, SIM_ENOMEM, "host staging of the product coefficients");
    }
    for (size_t j = 0; j < N; ++j) {
        const double xs = p->C / p->c[j];
        pf[j] = static_cast<float>(p->mu[j]);
        pf[N + j] = p->sigma[j] > 0.0 ? static_cast<float>(1.0 / (kappa * p->sigma[j])) : INFINITY;
        pf[2 * N + j] = static_cast<float>(p->k[j] - p->v[j]);
        pf[3 * N + j] = static_cast<float>((p->h[j] + p->v[j]) / p->n_samples);
        pf[4 * N + j] = static_cast<float>(1.0 / p->c[j]);
        pf[5 * N + j] = static_cast<float>(xs);
        pf[6 * N + j] = p->x0 ? static_cast<float>(p->x0[j]) : 0.0f;
        pd[j] = p->mu[j];
        pd[N + j] = p->sigma[j];
        pd[2 * N + j] = p->k[j];
        pd[3 * N + j] = p->h[j];
        pd[4 * N + j] = p->v[j];
        pd[5 * N + j] = xs;
    }
    int rc;
    if ((rc = ensure(ctx, w.prod_f, sizeof(float) * pf.size())) || (rc = ensure(ctx, w.prod_d, sizeof(double) * pd.size())) ||
        (rc = ensure(ctx, w.S, sizeof(uint64_t) * R * N)) || (rc = ensure(ctx, w.cnt, sizeof(uint32_t) * R * (N + 1))) ||
        (rc = ensure(ctx, w.tau, sizeof(uint32_t) * R)) || (rc = ensure(ctx, w.dec, sizeof(uint32_t) * R * T)) ||
        (rc = ensure(ctx, w.wg_r, sizeof(float) * 2 * R * w.nwg)) ||
        (rc = ensure(ctx, w.wg_j, sizeof(uint32_t) * 2 * R * w.nwg)) ||
        (rc = ensure(ctx, w.wg_gx, sizeof(float) * 2 * R * w.nwg)) || (rc = ensure(ctx, w.fval, sizeof(double) * R * (nc + 1))) ||
        (rc = ensure(ctx, w.stats, sizeof(double) * (fw::kMaxStreams * fw::kStreamFields + 2))) ||
        (rc = ensure(ctx, w.origin, sizeof(uint64_t))) ||
        (rc = ensure(ctx, w.cost_part, sizeof(double) * 2 * R * ((N + fw::kNvCostChunk - 1) / fw::kNvCostChunk))))
        return rc;
    hipStream_t st = ctx->stream;
    HIP_TRY(ctx, hipMemcpyAsync(w.prod_f.ptr, pf.data(), sizeof(float) * pf.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipMemcpyAsync(w.prod_d.ptr, pd.data(), sizeof(double) * pd.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipMemsetAsync(w.S.ptr, 0, sizeof(uint64_t) * R * N, st));
    HIP_TRY(ctx, hipMemsetAsync(w.cnt.ptr, 0, sizeof(uint32_t) * R * (N + 1), st));
    HIP_TRY(ctx, hipMemsetAsync(w.tau.ptr, 0xFF, sizeof(uint32_t) * R, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));   // the host vectors must outlive the copies

    const fw::NvArgs A = nv_args(w, p, R, T, seed);
    const uint64_t M = p->resample_every;
    HIP_TRY(ctx, hipEventRecord(w.ev0, st));
    // The step of iteration t runs inside the next iteration's sample launch unless a cost
    // evaluation needs the updated signature first or t is the last iteration.
    uint32_t ck = 0;
    bool pending = false;
    for (uint64_t t = 0; t < T; ++t) {
        const float cw = t == 0 ? 0.0f : static_cast<float>(2.0 / (static_cast<double>(t) * static_cast<double>(t + 1)));
        if (fw::launch_nv_sample(A, t, static_cast<uint32_t>(t / M), cw, t == 0 && p->x0 != nullptr, pending, st))
            return set_err(ctx, SIM_EDEVICE, "newsvendor sample launch failed at t=%llu", (unsigned long long)t);
        const bool cost_next = ck < nc && p->checkpoints[ck] == t + 1;
        pending = !(cost_next || t + 1 == T);
        if (!pending && fw::launch_nv_step(A, t, st))
            return set_err(ctx, SIM_EDEVICE, "newsvendor step launch failed at t=%llu", (unsigned long long)t);
        while (ck < nc && p->checkpoints[ck] == t + 1) {
            const double c = 2.0 / (static_cast<double>(t + 1) * static_cast<double>(t + 2));
            if (fw::launch_nv_cost(A, c, ck, st)) return set_err(ctx, SIM_EDEVICE, "newsvendor cost launch failed");
            ++ck;
        }
    }
    if (fw::launch_nv_cost(A, 2.0 / (static_cast<double>(T) * static_cast<double>(T + 1)), nc, st) ||
        fw::launch_nv_finalize(A, nc, st))
        return set_err(ctx, SIM_EDEVICE, "newsvendor finalize launch failed");
    HIP_TRY(ctx, hipEventRecord(w.ev1, st));

    w.params = *p;
    w.params.mu = w.params.sigma = w.params.k = w.params.h = w.params.v = w.params.c = w.params.x0 = nullptr;
    w.R = R;
    w.T = T;
    w.have = true;
    return SIM_OK;
}

int sim_nv_stats(sim_ctx *ctx, sim_stats_out *out)
{
    if (!ctx || !out) return SIM_EINVAL;
    NvState &w = ctx->nv;
    if (!w.have) return set_err(ctx, SIM_ESTATE, "no newsvendor run yet");
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
               &origin, 0, tc, ts, w.R, w.T, NAN, ms, static_cast<double>(w.R) * static_cast<double>(w.T));
    return SIM_OK;
}

int sim_nv_paths(sim_ctx *ctx, sim_wide_view *out)
{
    if (!ctx || !out) return SIM_EINVAL;
    NvState &w = ctx->nv;
    if (!w.have) return set_err(ctx, SIM_ESTATE, "no newsvendor run yet");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipEventSynchronize(w.ev1));
    std::memset(out, 0, sizeof(*out));
    out->R = w.R;
    out->T = w.T;
    out->d = w.params.n;
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

// ---- Algorithm 2 over X = {A x <= C, x >= 0} -------------------------------------------------

int sim_validate_newsvendor_lp(const sim_nv_params *p, const sim_nv_constraints *con, uint64_t R, uint64_t T, char *msg,
                               size_t len)
{
    char err[kErrLen] = {0};
    const int rc = validate_newsvendor_lp(err, p, con, R, T);
    if (msg && len) std::snprintf(msg, len, "%s", rc ? err : "");
    return rc;
}

int sim_run_newsvendor_lp(sim_ctx *ctx, const sim_nv_params *p, const sim_nv_constraints *con, uint64_t R, uint64_t T,
                          uint64_t seed)
{
    if (!ctx) return SIM_EINVAL;
    if (int rc = validate_newsvendor_lp(ctx->err, p, con, R, T)) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    NvLpState &w = ctx->nvlp;
    w.have = false;
    if (!w.ev0) HIP_TRY(ctx, hipEventCreate(&w.ev0));
    if (!w.ev1) HIP_TRY(ctx, hipEventCreate(&w.ev1));
    const uint32_t n = p->n, nc = p->n_checkpoints, M = con->n_resources;
    const size_t N = n;
    w.P = fw::nv_lanes_per_quad(n / 4, R, p->n_samples);
    w.nwg = (n / 4 + fw::kNvBlock / w.P - 1) / (fw::kNvBlock / w.P);

    // per product, binary64: mean, threshold scale, k - v, h + v, sigma, k, h, v, x_0
    const double kappa = fw::kBoxMullerScale;
    std::vector<double> pd;
    try {
        pd.resize(9 * N);
    } catch (const std::bad_alloc &) {
        return set_err(ctx, SIM_ENOMEM, "host staging of the product coefficients");
    }
    double gscale = 0.0;
    for (size_t j = 0; j < N; ++j) {
        pd[j] = p->mu[j];
        pd[N + j] = p->sigma[j] > 0.0 ? 1.0 / (kappa * p->sigma[j]) : INFINITY;
        pd[2 * N + j] = p->k[j] - p->v[j];
        pd[3 * N + j] = p->h[j] + p->v[j];
        pd[4 * N + j] = p->sigma[j];
        pd[5 * N + j] = p->k[j];
        pd[6 * N + j] = p->h[j];
        pd[7 * N + j] = p->v[j];
        pd[8 * N + j] = p->x0 ? p->x0[j] : 0.0;
        gscale = std::max(gscale, std::fabs(p->k[j] - p->v[j]) + std::fabs(p->h[j] + p->v[j]));
    }
    const size_t ncost = (N + fw::kNvCostChunk - 1) / fw::kNvCostChunk;
    int rc;
    if ((rc = ensure(ctx, w.prod_d, sizeof(double) * pd.size())) || (rc = ensure(ctx, w.Am, sizeof(double) * M * N)) ||
        (rc = ensure(ctx, w.Cv, sizeof(double) * M)) || (rc = ensure(ctx, w.x, sizeof(double) * R * N)) ||
        (rc = ensure(ctx, w.g, sizeof(double) * R * N)) ||
        (rc = ensure(ctx, w.rec_basis, sizeof(uint32_t) * R * T * M)) ||
        (rc = ensure(ctx, w.rec_value, sizeof(double) * R * T * M)) ||
        (rc = ensure(ctx, w.rec_piv, sizeof(uint32_t) * R * T)) || (rc = ensure(ctx, w.tau, sizeof(uint32_t) * R)) ||
        (rc = ensure(ctx, w.origin, sizeof(uint32_t) * R)) || (rc = ensure(ctx, w.cost_part, sizeof(double) * 2 * R * ncost)) ||
        (rc = ensure(ctx, w.fval, sizeof(double) * R * (nc + 1))) ||
        (rc = ensure(ctx, w.stats, sizeof(double) * (fw::kMaxStreams * fw::kStreamFields + 2))) ||
        (rc = ensure(ctx, w.origin_total, sizeof(uint64_t))))
        return rc;
    hipStream_t st = ctx->stream;
    HIP_TRY(ctx, hipMemcpyAsync(w.prod_d.ptr, pd.data(), sizeof(double) * pd.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipMemcpyAsync(w.Am.ptr, con->A, sizeof(double) * M * N, hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipMemcpyAsync(w.Cv.ptr, con->C, sizeof(double) * M, hipMemcpyHostToDevice, st));
    for (uint64_t r = 0; r < R; ++r)       // every replication starts at x_0
        HIP_TRY(ctx, hipMemcpyAsync(static_cast<double *>(w.x.ptr) + r * N, pd.data() + 8 * N, sizeof(double) * N,
                                    hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipMemsetAsync(w.tau.ptr, 0xFF, sizeof(uint32_t) * R, st));
    HIP_TRY(ctx, hipMemsetAsync(w.origin.ptr, 0, sizeof(uint32_t) * R, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));   // the host vectors must outlive the copies

    fw::NvLpArgs A{};
    A.n = n;
    A.nq = n / 4;
    A.S = p->n_samples;
    A.nwg = w.nwg;
    A.P = w.P;
    A.R = static_cast<uint32_t>(R);
    A.M = M;
    A.k0 = static_cast<uint32_t>(seed);
    A.k1 = static_cast<uint32_t>(seed >> 32);
    A.dom = (fw::kNvDomain << 24) | (p->instance_id & 0xFFFFFFu);
    A.max_pivots = SIM_NV_LP_MAX_PIVOTS;
    A.gap_eps = p->gap_eps;
    A.eps_r = 1e-12 * (1.0 + gscale);
    A.eps_d = 1e-12;
    const double *d = static_cast<const double *>(w.prod_d.ptr);
    A.mu_d = d;
    A.isk_d = d + N;
    A.km_d = d + 2 * N;
    A.hv_d = d + 3 * N;
    A.sig_d = d + 4 * N;
    A.k_d = d + 5 * N;
    A.h_d = d + 6 * N;
    A.v_d = d + 7 * N;
    A.x0_d = d + 8 * N;
    A.Am = static_cast<const double *>(w.Am.ptr);
    A.Cv = static_cast<const double *>(w.Cv.ptr);
    A.x = static_cast<double *>(w.x.ptr);
    A.g = static_cast<double *>(w.g.ptr);
    A.rec_basis = static_cast<uint32_t *>(w.rec_basis.ptr);
    A.rec_value = static_cast<double *>(w.rec_value.ptr);
    A.rec_piv = static_cast<uint32_t *>(w.rec_piv.ptr);
    A.tau = static_cast<uint32_t *>(w.tau.ptr);
    A.origin = static_cast<uint32_t *>(w.origin.ptr);
    A.T = T;
    A.cost_part = static_cast<double *>(w.cost_part.ptr);
    A.fval = static_cast<double *>(w.fval.ptr);
    A.stats = static_cast<double *>(w.stats.ptr);
    A.origin_total = static_cast<uint64_t *>(w.origin_total.ptr);

    HIP_TRY(ctx, hipEventRecord(w.ev0, st));
    // The update of iteration t runs at the start of the next iteration's gradient launch unless a
    // cost evaluation needs x_{t+1} first or t is the last iteration.
    const int lrc = fw::nv_lp_sequence(
        p->resample_every, T, nc, p->checkpoints,
        [&](uint64_t t, uint32_t epoch, bool fold_prev) {
            return fw::launch_nv_lp_gradient(A, t, epoch, fold_prev, st)
                       ? set_err(ctx, SIM_EDEVICE, "newsvendor gradient launch failed at t=%llu", (unsigned long long)t)
                       : 0;
        },
        [&](uint64_t t) {
            return fw::launch_nv_lp_subproblem(A, t, st)
                       ? set_err(ctx, SIM_EDEVICE, "newsvendor subproblem launch failed at t=%llu", (unsigned long long)t)
                       : 0;
        },
        [&](uint64_t t) {
            return fw::launch_nv_lp_update(A, t, st)
                       ? set_err(ctx, SIM_EDEVICE, "newsvendor update launch failed at t=%llu", (unsigned long long)t)
                       : 0;
        },
        [&](uint32_t slot) {
            return fw::launch_nv_lp_cost(A, slot, st) ? set_err(ctx, SIM_EDEVICE, "newsvendor cost launch failed") : 0;
        });
    if (lrc) return lrc;
    if (fw::launch_nv_lp_cost(A, nc, st) || fw::launch_nv_lp_finalize(A, nc, st))
        return set_err(ctx, SIM_EDEVICE, "newsvendor finalize launch failed");
    HIP_TRY(ctx, hipEventRecord(w.ev1, st));

    w.params = *p;
    w.params.mu = w.params.sigma = w.params.k = w.params.h = w.params.v = w.params.c = w.params.x0 = nullptr;
    w.M = M;
    w.R = R;
    w.T = T;
    w.have = true;
    return SIM_OK;
}

int sim_nv_lp_stats(sim_ctx *ctx, sim_stats_out *out)
{
    if (!ctx || !out) return SIM_EINVAL;
    NvLpState &w = ctx->nvlp;
    if (!w.have) return set_err(ctx, SIM_ESTATE, "no general-constraint newsvendor run yet");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipEventSynchronize(w.ev1));
    const uint32_t nc = w.params.n_checkpoints, n_streams = 1 + 2 * nc;
    double F[fw::kMaxStreams * fw::kStreamFields + 2];
    uint64_t origin = 0;
    std::vector<uint32_t> tau(w.R);
    HIP_TRY(ctx, hipMemcpy(F, w.stats.ptr, sizeof(double) * (n_streams * fw::kStreamFields + 2), hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(&origin, w.origin_total.ptr, sizeof(uint64_t), hipMemcpyDeviceToHost));
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
               &origin, 0, tc, ts, w.R, w.T, NAN, ms, static_cast<double>(w.R) * static_cast<double>(w.T));
    return SIM_OK;
}

int sim_nv_lp_paths(sim_ctx *ctx, sim_nv_lp_view *out)
{
    if (!ctx || !out) return SIM_EINVAL;
    NvLpState &w = ctx->nvlp;
    if (!w.have) return set_err(ctx, SIM_ESTATE, "no general-constraint newsvendor run yet");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipEventSynchronize(w.ev1));
    std::memset(out, 0, sizeof(*out));
    out->R = w.R;
    out->T = w.T;
    out->n = w.params.n;
    out->n_resources = w.M;
    out->n_checkpoints = w.params.n_checkpoints;
    const double *fv = static_cast<const double *>(w.fval.ptr);
    out->y = fv + static_cast<size_t>(w.params.n_checkpoints) * w.R;
    out->f_ckpt = w.params.n_checkpoints ? fv : nullptr;
    out->x = static_cast<const double *>(w.x.ptr);
    out->tau = static_cast<const uint32_t *>(w.tau.ptr);
    out->basis = static_cast<const uint32_t *>(w.rec_basis.ptr);
    out->value = static_cast<const double *>(w.rec_value.ptr);
    out->pivots = static_cast<const uint32_t *>(w.rec_piv.ptr);
    return SIM_OK;
}

}  // extern "C"
