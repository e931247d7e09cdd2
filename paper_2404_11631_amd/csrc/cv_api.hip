// cv_api.hip -- host side of the control variate declared in include/sim.h: surrogate training
// on pairs from the simulation, the held-out fit of beta, the estimator (paths, surrogate, draws
// from the features' law, FP64 moments), and the surrogate primitives the tests drive.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <vector>

#include "engine.hpp"

using namespace fw::host;

namespace {

constexpr uint64_t kAuxChunk = 1ull << 22;
constexpr uint64_t kRefPilot = 1ull << 14;   // replications of the run that fixes the reference gradient
constexpr uint32_t kMomentBlocks = 512;

// host double-double accumulation of chunk sums
struct Acc {
    double h = 0.0, l = 0.0;
    void add(double bh, double bl)
    {
        const double s = h + bh, bb = s - h;
        double e = (h - (s - bb)) + (bh - bb);
        e += l + bl;
        h = s + e;
        l = e - (h - s);
    }
    double value() const { return h + l; }
};

// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): per-epoch permutation constants
uint64_t splitmix64(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

fw::MlpDev mlp_dev(CvState &cv)
{
    fw::MlpDev m = fw::mlp_layout(cv.F);
    m.theta = (float *)cv.theta.ptr;
    m.w1a = (uint16_t *)cv.w1a.ptr;
    m.w2a = (uint16_t *)cv.w2a.ptr;
    m.w2t = (uint16_t *)cv.w2t.ptr;
    return m;
}

size_t w1a_bytes(int F) { return sizeof(uint16_t) * 2 * ((F + 15) / 16) * 64 * 8; }
constexpr size_t kW2aBytes = sizeof(uint16_t) * 2 * 4 * 64 * 8;

int ensure_mlp(sim_ctx *ctx, int F)
{
    CvState &cv = ctx->cv;
    if (F < 3 || F > 66) return set_err(ctx, SIM_EINVAL, "surrogate inputs F=%d outside [3, 66]", F);
    if (cv.F != F) {
        cv.have_mlp = false;
        cv.have_fit = false;
    }
    const fw::MlpDev m = fw::mlp_layout(F);
    int rc;
    if ((rc = ensure(ctx, cv.theta, sizeof(float) * m.P))) return rc;
    if ((rc = ensure(ctx, cv.mom1, sizeof(float) * m.P))) return rc;
    if ((rc = ensure(ctx, cv.mom2, sizeof(float) * m.P))) return rc;
    if ((rc = ensure(ctx, cv.w1a, w1a_bytes(F)))) return rc;
    if ((rc = ensure(ctx, cv.w2a, kW2aBytes))) return rc;
    if ((rc = ensure(ctx, cv.w2t, kW2aBytes))) return rc;
    cv.F = F;
    return SIM_OK;
}

// operand copies from the master weights (padding columns of W1 stay zero), moments cleared
int refresh_after_upload(sim_ctx *ctx)
{
    CvState &cv = ctx->cv;
    const fw::MlpDev m = mlp_dev(cv);
    HIP_TRY(ctx, hipMemsetAsync(cv.w1a.ptr, 0, w1a_bytes(cv.F), ctx->stream));
    if (fw::launch_mlp_copies(m, ctx->stream)) return set_err(ctx, SIM_EDEVICE, "surrogate copy launch failed");
    HIP_TRY(ctx, hipMemsetAsync(cv.mom1.ptr, 0, sizeof(float) * m.P, ctx->stream));
    HIP_TRY(ctx, hipMemsetAsync(cv.mom2.ptr, 0, sizeof(float) * m.P, ctx->stream));
    cv.n_steps = 0;
    return SIM_OK;
}

// FP64 moments of (A - sa, B - sb) over n pairs; A or B may be NULL (then 0). out: 5 sums
int moments(sim_ctx *ctx, const double *A, const float *B, uint64_t n, double sa, double sb, double out[5])
{
    CvState &cv = ctx->cv;
    int rc;
    if ((rc = ensure(ctx, cv.mpart, sizeof(double) * 10 * kMomentBlocks))) return rc;
    if ((rc = ensure(ctx, cv.mout, sizeof(double) * 10))) return rc;
    if ((rc = ensure(ctx, cv.mdone, 64))) return rc;
    std::fill(out, out + 5, 0.0);
    if (n == 0) return SIM_OK;
    const uint32_t nb = (uint32_t)std::min<uint64_t>(kMomentBlocks, (n + 255) / 256);
    HIP_TRY(ctx, hipMemsetAsync(cv.mdone.ptr, 0, 4, ctx->stream));
    if (fw::launch_cv_moments(A, B, n, sa, sb, (double *)cv.mpart.ptr, nb, (double *)cv.mout.ptr,
                              (uint32_t *)cv.mdone.ptr, ctx->stream))
        return set_err(ctx, SIM_EDEVICE, "moment launch failed");
    double h[10];
    HIP_TRY(ctx, hipMemcpyAsync(h, cv.mout.ptr, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
    for (int s = 0; s < 5; ++s) out[s] = h[2 * s] + h[2 * s + 1];
    return SIM_OK;
}

struct MeanVar {
    double mean, var;
};
MeanVar mean_var(double s, double s2, double shift, uint64_t n)
{
    const double m = s / (double)n;
    return {shift + m, n > 1 ? (s2 - s * m) / (double)(n - 1) : 0.0};
}

fw::AuxLaw aux_law(const sim_params *p, uint64_t T, uint64_t seed)
{
    const CvLaw L = cv_law(p, T);
    fw::AuxLaw law{};
    law.seed = seed;
    law.instance = p->instance_id;
    law.d = (int)p->d;
    law.T = T;
    law.M = p->resample_every;
    law.top = L.top;
    law.mean1 = L.mean1;
    law.inv1 = L.inv1;
    for (uint32_t c = 0; c <= p->d; ++c) {
        law.cum[c] = L.cum[c];
        law.mean[c] = L.mean[c];
        law.inv[c] = L.inv[c];
    }
    return law;
}

int ensure_events(sim_ctx *ctx)
{
    CvState &cv = ctx->cv;
    if (!cv.ev0) HIP_TRY(ctx, hipEventCreate(&cv.ev0));
    if (!cv.ev1) HIP_TRY(ctx, hipEventCreate(&cv.ev1));
    if (!cv.ev_a) HIP_TRY(ctx, hipEventCreate(&cv.ev_a));
    if (!cv.ev_b) HIP_TRY(ctx, hipEventCreate(&cv.ev_b));
    return SIM_OK;
}

float elapsed(hipEvent_t a, hipEvent_t b)
{
    float ms = 0.0f;
    (void)hipEventElapsedTime(&ms, a, b);
    return ms;
}

}  // namespace

extern "C" {

int sim_cv_law(const sim_params *p, uint64_t T, double *probs, double *S2, double *S4, char *msg, size_t len)
{
    char err[kErrLen] = {0};
    if (!p || !probs) return SIM_EINVAL;
    sim_params q = *p;
    q.flags = SIM_CV_FEATURES;
    const int rc = validate(err, &q, 1, T);
    if (msg && len) std::snprintf(msg, len, "%s", rc ? err : "");
    if (rc) return rc;
    const CvLaw L = cv_law(&q, T);
    for (uint32_t c = 0; c <= q.d; ++c) probs[c] = L.p[c];
    if (S2) *S2 = L.S2;
    if (S4) *S4 = L.S4;
    return SIM_OK;
}

int sim_mlp_set_params(sim_ctx *ctx, uint32_t F, const float *theta)
{
    if (!ctx || !theta) return SIM_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    int rc = ensure_mlp(ctx, (int)F);
    if (rc) return rc;
    CvState &cv = ctx->cv;
    const fw::MlpDev m = mlp_dev(cv);
    HIP_TRY(ctx, ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize());
    HIP_TRY(ctx, hipMemcpy(cv.theta.ptr, theta, sizeof(float) * m.P, hipMemcpyHostToDevice));
    if ((rc = refresh_after_upload(ctx))) return rc;
    HIP_TRY(ctx, ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize());
    cv.have_mlp = true;
    cv.have_fit = false;
    return SIM_OK;
}

int sim_mlp_get_params(sim_ctx *ctx, uint32_t F, float *theta)
{
    if (!ctx || !theta) return SIM_EINVAL;
    CvState &cv = ctx->cv;
    if (!cv.have_mlp) return set_err(ctx, SIM_ESTATE, "no surrogate parameters yet");
    if ((int)F != cv.F) return set_err(ctx, SIM_EINVAL, "F=%u but the surrogate has %d inputs", F, cv.F);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize());
    HIP_TRY(ctx, hipMemcpy(theta, cv.theta.ptr, sizeof(float) * fw::mlp_layout(cv.F).P, hipMemcpyDeviceToHost));
    return SIM_OK;
}

int sim_mlp_forward(sim_ctx *ctx, const float *x, uint64_t n, float *out)
{
    if (!ctx || (n && (!x || !out))) return SIM_EINVAL;
    CvState &cv = ctx->cv;
    if (!cv.have_mlp) return set_err(ctx, SIM_ESTATE, "no surrogate parameters yet");
    if (n > (1ull << 31)) return set_err(ctx, SIM_EINVAL, "n above 2^31");
    if (n == 0) return SIM_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    int rc;
    if ((rc = ensure(ctx, cv.xio, sizeof(float) * cv.F * n))) return rc;
    if ((rc = ensure(ctx, cv.hout, sizeof(float) * n))) return rc;
    HIP_TRY(ctx, ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize());
    HIP_TRY(ctx, hipMemcpy(cv.xio.ptr, x, sizeof(float) * cv.F * n, hipMemcpyHostToDevice));
    if (fw::launch_mlp_forward(mlp_dev(cv), (const float *)cv.xio.ptr, n, n, 0.0f, 1.0f, (float *)cv.hout.ptr,
                               ctx->stream))
        return set_err(ctx, SIM_EDEVICE, "surrogate forward launch failed");
    HIP_TRY(ctx, hipMemcpyAsync(out, cv.hout.ptr, sizeof(float) * n, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize());
    return SIM_OK;
}

int sim_mlp_grad(sim_ctx *ctx, const float *x, const float *y, uint64_t n, float *grad, double *loss)
{
    if (!ctx || !x || !y || !grad || n == 0) return SIM_EINVAL;
    CvState &cv = ctx->cv;
    if (!cv.have_mlp) return set_err(ctx, SIM_ESTATE, "no surrogate parameters yet");
    if (n > (1u << 20)) return set_err(ctx, SIM_EINVAL, "n above 2^20");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    const fw::MlpDev m = mlp_dev(cv);
    const uint64_t nparts = (n + 127) / 128;
    int rc;
    if ((rc = ensure(ctx, cv.xio, sizeof(float) * cv.F * n))) return rc;
    if ((rc = ensure(ctx, cv.yio, sizeof(float) * n))) return rc;
    if ((rc = ensure(ctx, cv.part, sizeof(float) * (m.P + 1) * nparts))) return rc;
    if ((rc = ensure(ctx, cv.grad, sizeof(float) * (m.P + 1)))) return rc;
    HIP_TRY(ctx, ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize());
    HIP_TRY(ctx, hipMemcpy(cv.xio.ptr, x, sizeof(float) * cv.F * n, hipMemcpyHostToDevice));
    HIP_TRY(ctx, hipMemcpy(cv.yio.ptr, y, sizeof(float) * n, hipMemcpyHostToDevice));
    if (fw::launch_mlp_grad(m, (const float *)cv.xio.ptr, n, (const float *)cv.yio.ptr, 0, n, 1, 0, n,
                            1.0f / (float)n, (float *)cv.part.ptr, ctx->stream))
        return set_err(ctx, SIM_EDEVICE, "surrogate gradient launch failed");
    const fw::AdamStep none{};
    if (fw::launch_mlp_reduce(m, (const float *)cv.part.ptr, (uint32_t)nparts, 0, none, nullptr, nullptr,
                              (float *)cv.grad.ptr, nullptr, ctx->stream))
        return set_err(ctx, SIM_EDEVICE, "surrogate reduction launch failed");
    std::vector<float> g(m.P + 1);
    HIP_TRY(ctx, hipMemcpyAsync(g.data(), cv.grad.ptr, sizeof(float) * (m.P + 1), hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize());
    std::memcpy(grad, g.data(), sizeof(float) * m.P);
    if (loss) *loss = (double)g[m.P] / (double)n;
    return SIM_OK;
}

int sim_cv_aux_draws(sim_ctx *ctx, const sim_params *p, uint64_t T, uint64_t seed, uint64_t k0, uint64_t n,
                     float *x)
{
    if (!ctx || !p || (n && !x)) return SIM_EINVAL;
    sim_params q = *p;
    q.flags = SIM_CV_FEATURES;
    int rc = validate(ctx->err, &q, 1, T);
    if (rc) return rc;
    if (k0 + n > (1ull << 32)) return set_err(ctx, SIM_EINVAL, "draw index beyond 2^32");
    if (n == 0) return SIM_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    CvState &cv = ctx->cv;
    const uint32_t F = p->d + 2;
    if ((rc = ensure(ctx, cv.xaux, sizeof(float) * F * n))) return rc;
    if (fw::launch_cv_aux(aux_law(&q, T, seed), k0, n, (float *)cv.xaux.ptr, n, ctx->stream))
        return set_err(ctx, SIM_EDEVICE, "aux launch failed");
    HIP_TRY(ctx, hipMemcpyAsync(x, cv.xaux.ptr, sizeof(float) * F * n, hipMemcpyDeviceToHost, ctx->stream));
    HIP_TRY(ctx, ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize());
    return SIM_OK;
}

int sim_cv_fit(sim_ctx *ctx, const sim_params *p, uint64_t T, uint64_t seed, const sim_cv_opts *o,
               sim_cv_fit_out *out)
{
    if (!ctx || !p || !o || !out) return SIM_EINVAL;
    if (o->n_runs < 1 || o->epochs < 1) return set_err(ctx, SIM_EINVAL, "n_runs and epochs must be >= 1");
    if (o->batch < 128 || o->batch > 65536 || o->batch % 128)
        return set_err(ctx, SIM_EINVAL, "batch must be a multiple of 128 in [128, 65536]");
    if (o->R_train < o->batch) return set_err(ctx, SIM_EINVAL, "R_train below the batch");
    if (o->R_pilot < 2) return set_err(ctx, SIM_EINVAL, "R_pilot must be >= 2");
    if (!(o->lr > 0.0) || !std::isfinite(o->lr)) return set_err(ctx, SIM_EINVAL, "lr must be finite and > 0");
    if (o->reinit > 1) return set_err(ctx, SIM_EINVAL, "reinit must be 0 or 1");
    const uint64_t n = (uint64_t)o->n_runs * o->R_train;
    if (n > (1ull << 31)) return set_err(ctx, SIM_EINVAL, "more than 2^31 training pairs");
    // the features' reference gradient: 2 lambda Sigma wbar - mu, wbar the mean of w_T over a plain
    // pilot run with its own seed
    sim_params qp = *p;
    qp.flags = SIM_KEEP_PATHS;
    qp.n_checkpoints = 0;
    qp.cv_ref = nullptr;
    int rc = validate(ctx->err, &qp, kRefPilot, T);
    if (rc) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    CvState &cv = ctx->cv;
    {
        if ((rc = run_impl(ctx, &qp, kRefPilot, T, seed + o->n_runs + 1, 0u))) return rc;
        std::vector<uint64_t> ws((size_t)p->d * kRefPilot);
        HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));
        HIP_TRY(ctx, hipMemcpy(ws.data(), ctx->wsum.ptr, sizeof(uint64_t) * ws.size(), hipMemcpyDeviceToHost));
        const double c = 2.0 / ((double)T * (double)(T + 1));
        const uint32_t d = p->d;
        std::vector<double> wbar(d), v(d, 0.0);
        for (uint32_t j = 0; j < d; ++j) {
            double acc = 0.0;
            for (uint64_t r = 0; r < kRefPilot; ++r) acc += (double)ws[j * kRefPilot + r];
            wbar[j] = c * acc / (double)kRefPilot;
        }
        if (p->chol) {
            // Sigma wbar = L (L' wbar)
            for (uint32_t k = 0; k < d; ++k)
                for (uint32_t j = k; j < d; ++j) v[k] += p->chol[j * d + k] * wbar[j];
            for (uint32_t j = 0; j < d; ++j) {
                double sw = 0.0;
                for (uint32_t k = 0; k <= j; ++k) sw += p->chol[j * d + k] * v[k];
                cv.ref[j] = 2.0 * p->risk_coef * sw - p->mu[j];
            }
        } else {
            for (uint32_t j = 0; j < d; ++j)
                cv.ref[j] = 2.0 * p->risk_coef * p->sigma[j] * p->sigma[j] * wbar[j] - p->mu[j];
        }
    }
    sim_params q = *p;
    q.flags = SIM_CV_FEATURES;
    q.cv_ref = cv.ref;
    if ((rc = validate(ctx->err, &q, std::max<uint64_t>(o->R_train, o->R_pilot), T))) return rc;
    const int F = (int)q.d + 2;
    if ((rc = ensure_mlp(ctx, F))) return rc;
    if ((rc = ensure_events(ctx))) return rc;
    const fw::MlpDev m = mlp_dev(cv);
    std::memset(out, 0, sizeof(*out));
    for (uint32_t j = 0; j < q.d; ++j) out->ref[j] = cv.ref[j];

    // training pairs
    if ((rc = ensure(ctx, cv.xtrain, sizeof(float) * F * n))) return rc;
    if ((rc = ensure(ctx, cv.ytrain, sizeof(double) * n))) return rc;
    if ((rc = ensure(ctx, cv.ttrain, sizeof(float) * n))) return rc;
    hipEvent_t t0, t1, t2, t3;
    HIP_TRY(ctx, hipEventCreate(&t0));
    HIP_TRY(ctx, hipEventCreate(&t1));
    HIP_TRY(ctx, hipEventCreate(&t2));
    HIP_TRY(ctx, hipEventCreate(&t3));
    struct Ev {
        hipEvent_t *e[4];
        ~Ev()
        {
            for (auto x : e) (void)hipEventDestroy(*x);
        }
    } ev_guard{{&t0, &t1, &t2, &t3}};
    HIP_TRY(ctx, hipEventRecord(t0, ctx->stream));
    for (uint32_t k = 0; k < o->n_runs; ++k) {
        if ((rc = run_impl(ctx, &q, o->R_train, T, seed + k, fw::kFlagYOnly))) return rc;
        HIP_TRY(ctx, hipMemcpy2DAsync((float *)cv.xtrain.ptr + k * o->R_train, sizeof(float) * n, ctx->feat.ptr,
                                      sizeof(float) * o->R_train, sizeof(float) * o->R_train, F,
                                      hipMemcpyDeviceToDevice, ctx->stream));
        HIP_TRY(ctx, hipMemcpyAsync((double *)cv.ytrain.ptr + k * o->R_train, ctx->y.ptr, sizeof(double) * o->R_train,
                                    hipMemcpyDeviceToDevice, ctx->stream));
    }
    HIP_TRY(ctx, hipEventRecord(t1, ctx->stream));
    double mo[5];
    if ((rc = moments(ctx, (const double *)cv.ytrain.ptr, nullptr, n, 0.0, 0.0, mo))) return rc;
    const MeanVar yv = mean_var(mo[0], mo[2], 0.0, n);
    cv.y_mean = yv.mean;
    cv.y_sd = yv.var > 0.0 ? std::sqrt(yv.var) : 1.0;
    if (fw::launch_cv_target((const double *)cv.ytrain.ptr, n, cv.y_mean, 1.0 / cv.y_sd, (float *)cv.ttrain.ptr,
                             ctx->stream))
        return set_err(ctx, SIM_EDEVICE, "target launch failed");

    // weights
    if (o->reinit || !cv.have_mlp) {
        if (fw::launch_mlp_init(m, seed, q.instance_id, ctx->stream))
            return set_err(ctx, SIM_EDEVICE, "surrogate init launch failed");
        if ((rc = refresh_after_upload(ctx))) return rc;
        cv.have_mlp = true;
    }

    // Adam over minibatches of a fresh affine permutation a q + c (mod n) per epoch
    const uint64_t spe = n / o->batch;
    const uint32_t nparts = o->batch / 128;
    if ((rc = ensure(ctx, cv.part, sizeof(float) * (m.P + 1) * nparts))) return rc;
    if ((rc = ensure(ctx, cv.loss_hist, sizeof(float) * spe * o->epochs))) return rc;
    for (uint32_t e = 0; e < o->epochs; ++e) {
        const uint64_t r0 = splitmix64(seed ^ (0x5DEECE66Dull * (e + 1)));
        uint64_t a = n > 1 ? 1 + r0 % (n - 1) : 1;
        while (std::gcd(a, n) != 1) a = (a + 1) % n;
        const uint64_t c = splitmix64(r0) % n;
        for (uint64_t s = 0; s < spe; ++s) {
            if (fw::launch_mlp_grad(m, (const float *)cv.xtrain.ptr, n, (const float *)cv.ttrain.ptr, s * o->batch,
                                    o->batch, a, c, n, 1.0f / (float)o->batch, (float *)cv.part.ptr, ctx->stream))
                return set_err(ctx, SIM_EDEVICE, "surrogate gradient launch failed");
            const double t = (double)(++cv.n_steps);
            fw::AdamStep st{(float)o->lr, 0.9f, 0.999f, 1e-8f, (float)(1.0 / (1.0 - std::pow(0.9, t))),
                            (float)(1.0 / (1.0 - std::pow(0.999, t)))};
            if (fw::launch_mlp_reduce(m, (const float *)cv.part.ptr, nparts, 1, st, (float *)cv.mom1.ptr,
                                      (float *)cv.mom2.ptr, nullptr, (float *)cv.loss_hist.ptr + e * spe + s,
                                      ctx->stream))
                return set_err(ctx, SIM_EDEVICE, "surrogate update launch failed");
        }
    }
    HIP_TRY(ctx, hipEventRecord(t2, ctx->stream));

    // beta on a held-out pilot
    if ((rc = run_impl(ctx, &q, o->R_pilot, T, seed + o->n_runs, fw::kFlagYOnly))) return rc;
    if ((rc = ensure(ctx, cv.hout, sizeof(float) * o->R_pilot))) return rc;
    if (fw::launch_mlp_forward(m, (const float *)ctx->feat.ptr, o->R_pilot, o->R_pilot, (float)cv.y_mean,
                               (float)cv.y_sd, (float *)cv.hout.ptr, ctx->stream))
        return set_err(ctx, SIM_EDEVICE, "surrogate forward launch failed");
    HIP_TRY(ctx, hipEventRecord(t3, ctx->stream));
    if ((rc = moments(ctx, (const double *)ctx->y.ptr, (const float *)cv.hout.ptr, o->R_pilot, cv.y_mean, cv.y_mean,
                      mo)))
        return rc;
    const uint64_t np = o->R_pilot;
    const MeanVar py = mean_var(mo[0], mo[2], cv.y_mean, np), ph = mean_var(mo[1], mo[3], cv.y_mean, np);
    const double cov = (mo[4] - mo[0] * mo[1] / (double)np) / (double)(np - 1);
    cv.beta = ph.var > 0.0 ? cov / ph.var : 0.0;
    cv.rho2 = (ph.var > 0.0 && py.var > 0.0) ? cov * cov / (ph.var * py.var) : 0.0;
    cv.n_train = n;
    cv.have_fit = true;

    std::vector<float> lh(spe * o->epochs);
    HIP_TRY(ctx, hipMemcpy(lh.data(), cv.loss_hist.ptr, sizeof(float) * lh.size(), hipMemcpyDeviceToHost));
    double l0 = 0.0, l1 = 0.0;
    for (uint64_t s = 0; s < spe; ++s) {
        l0 += lh[s];
        l1 += lh[(o->epochs - 1) * spe + s];
    }
    out->n_train = n;
    out->steps = spe * o->epochs;
    out->y_mean = cv.y_mean;
    out->y_sd = cv.y_sd;
    out->loss_first_epoch = l0 / ((double)spe * o->batch);
    out->loss_last_epoch = l1 / ((double)spe * o->batch);
    out->beta = cv.beta;
    out->rho2 = cv.rho2;
    out->pilot_var_y = py.var;
    out->sim_ms = elapsed(t0, t1);
    out->train_ms = elapsed(t1, t2);
    out->pilot_ms = elapsed(t2, t3);
    return SIM_OK;
}

int sim_run_cv(sim_ctx *ctx, const sim_params *p, uint64_t R, uint64_t T, uint64_t seed, uint64_t R_aux,
               sim_cv_stats_out *out)
{
    if (!ctx || !p || !out) return SIM_EINVAL;
    CvState &cv = ctx->cv;
    if (!cv.have_fit) return set_err(ctx, SIM_ESTATE, "no fitted surrogate (sim_cv_fit)");
    if (R < 2 || R_aux < 2) return set_err(ctx, SIM_EINVAL, "R and R_aux must be >= 2");
    if (R_aux > (1ull << 32)) return set_err(ctx, SIM_EINVAL, "R_aux above 2^32");
    sim_params q = *p;
    q.flags = SIM_CV_FEATURES;
    q.cv_ref = cv.ref;
    if ((int)q.d + 2 != cv.F) return set_err(ctx, SIM_EINVAL, "the surrogate was fitted for d=%d", cv.F - 2);
    int rc = validate(ctx->err, &q, R, T);
    if (rc) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    if ((rc = ensure_events(ctx))) return rc;
    const fw::MlpDev m = mlp_dev(cv);
    std::memset(out, 0, sizeof(*out));

    HIP_TRY(ctx, hipEventRecord(cv.ev0, ctx->stream));
    if ((rc = run_impl(ctx, &q, R, T, seed, fw::kFlagYOnly))) return rc;
    const hipEvent_t path_start = ctx->ev_start, path_stop = ctx->ev_stop;
    if ((rc = ensure(ctx, cv.hout, sizeof(float) * R))) return rc;
    if (fw::launch_mlp_forward(m, (const float *)ctx->feat.ptr, R, R, (float)cv.y_mean, (float)cv.y_sd,
                               (float *)cv.hout.ptr, ctx->stream))
        return set_err(ctx, SIM_EDEVICE, "surrogate forward launch failed");
    double mo[5];
    if ((rc = moments(ctx, (const double *)ctx->y.ptr, (const float *)cv.hout.ptr, R, cv.y_mean, cv.y_mean, mo)))
        return rc;

    const fw::AuxLaw law = aux_law(&q, T, seed);
    const uint64_t chunk = std::min<uint64_t>(R_aux, kAuxChunk);
    if ((rc = ensure(ctx, cv.xaux, sizeof(float) * cv.F * chunk))) return rc;
    if ((rc = ensure(ctx, cv.haux, sizeof(float) * chunk))) return rc;
    Acc sb, sb2;
    float aux_ms = 0.0f;
    for (uint64_t k0 = 0; k0 < R_aux; k0 += chunk) {
        const uint64_t nk = std::min(chunk, R_aux - k0);
        HIP_TRY(ctx, hipEventRecord(cv.ev_a, ctx->stream));
        if (fw::launch_cv_aux(law, k0, nk, (float *)cv.xaux.ptr, nk, ctx->stream))
            return set_err(ctx, SIM_EDEVICE, "aux launch failed");
        if (fw::launch_mlp_forward(m, (const float *)cv.xaux.ptr, nk, nk, (float)cv.y_mean, (float)cv.y_sd,
                                   (float *)cv.haux.ptr, ctx->stream))
            return set_err(ctx, SIM_EDEVICE, "surrogate forward launch failed");
        HIP_TRY(ctx, hipEventRecord(cv.ev_b, ctx->stream));
        double ma[5];
        if ((rc = moments(ctx, nullptr, (const float *)cv.haux.ptr, nk, 0.0, cv.y_mean, ma))) return rc;
        aux_ms += elapsed(cv.ev_a, cv.ev_b);
        sb.add(ma[1], 0.0);
        sb2.add(ma[3], 0.0);
        cv.n_aux_last = nk;
    }
    HIP_TRY(ctx, hipEventRecord(cv.ev1, ctx->stream));
    HIP_TRY(ctx, hipStreamSynchronize(ctx->stream));

    const MeanVar y = mean_var(mo[0], mo[2], cv.y_mean, R), hv = mean_var(mo[1], mo[3], cv.y_mean, R);
    const double cov = (mo[4] - mo[0] * mo[1] / (double)R) / (double)(R - 1);
    const MeanVar ha = mean_var(sb.value(), sb2.value(), cv.y_mean, R_aux);
    const double b = cv.beta;
    out->R = R;
    out->R_aux = R_aux;
    out->beta = b;
    out->mean_plain = y.mean;
    out->var_plain = y.var;
    out->ci95_plain = 1.96 * std::sqrt(y.var / (double)R);
    out->mean_resid = y.mean - b * hv.mean;
    out->var_resid = y.var - 2.0 * b * cov + b * b * hv.var;
    out->mean_h_aux = ha.mean;
    out->var_h_aux = ha.var;
    out->mean_cv = out->mean_resid + b * ha.mean;
    out->var_est = out->var_resid / (double)R + b * b * ha.var / (double)R_aux;
    out->ci95_cv = 1.96 * std::sqrt(out->var_est);
    out->rho2 = (hv.var > 0.0 && y.var > 0.0) ? cov * cov / (hv.var * y.var) : 0.0;
    out->kernel_ms = elapsed(cv.ev0, cv.ev1);
    out->paths_ms = elapsed(path_start, path_stop);
    out->aux_ms = aux_ms;
    cv.R = R;
    return SIM_OK;
}

int sim_cv_paths(sim_ctx *ctx, sim_cv_view *out)
{
    if (!ctx || !out) return SIM_EINVAL;
    CvState &cv = ctx->cv;
    if (!cv.R) return set_err(ctx, SIM_ESTATE, "no control-variate run yet");
    std::memset(out, 0, sizeof(*out));
    out->R = cv.R;
    out->n_aux = cv.n_aux_last;
    out->F = (uint32_t)cv.F;
    out->y = (const double *)ctx->y.ptr;
    out->h = (const float *)cv.hout.ptr;
    out->x = (const float *)ctx->feat.ptr;
    out->x_aux = (const float *)cv.xaux.ptr;
    out->h_aux = (const float *)cv.haux.ptr;
    return SIM_OK;
}

}  // extern "C"
