// sim_api.hip -- host engine behind the C ABI declared in include/sim.h: validation, instance
// coefficients, device buffers, launch, and the final FP64 statistics.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "../../include/sim.h"
#include "sim_types.hpp"

namespace fw {
int launch_fw_paths(const InstanceDesc &host_desc, const InstanceDesc *dev_desc, const RunBuffers &B,
                    bool fp64, hipStream_t stream, int *kernel_width);
}

using fw::InstanceDesc;
using fw::RunBuffers;

struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

struct sim_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    char err[512] = {0};
    InstanceDesc *desc_host = nullptr;    // pinned staging for the async upload
    InstanceDesc *desc_dev = nullptr;
    DevBuf y, fck, cnt, wsum, tau, dlog, part_f, part_i, done, final_f, final_i;
    RunBuffers bufs{};
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    bool have_run = false;
    sim_params last{};
    double last_mu[SIM_MAX_D], last_sigma[SIM_MAX_D];
    bool last_diag = true;
    uint64_t R = 0, T = 0;
    int kernel_width = 0;
};

namespace {

int set_err(sim_ctx *ctx, int code, const char *fmt, ...)
{
    if (ctx) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(ctx->err, sizeof(ctx->err), fmt, ap);
        va_end(ap);
    }
    return code;
}

#define HIP_TRY(ctx, call)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return set_err((ctx), SIM_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));   \
    } while (0)

int ensure(sim_ctx *ctx, DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    if (b.bytes >= bytes) return SIM_OK;
    if (b.ptr) {
        HIP_TRY(ctx, hipFree(b.ptr));
        b.ptr = nullptr;
        b.bytes = 0;
    }
    hipError_t e = hipMalloc(&b.ptr, bytes);
    if (e != hipSuccess) {
        b.ptr = nullptr;
        return set_err(ctx, SIM_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    b.bytes = bytes;
    return SIM_OK;
}

void free_buf(DevBuf &b)
{
    if (b.ptr) (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
}

bool finite(double x) { return std::isfinite(x); }

int validate(sim_ctx *ctx, const sim_params *p, uint64_t R, uint64_t T)
{
    if (!p) return set_err(ctx, SIM_EINVAL, "params is NULL");
    if (p->abi_version != SIM_ABI_VERSION)
        return set_err(ctx, SIM_EINVAL, "abi_version %u != %u", p->abi_version, SIM_ABI_VERSION);
    if (p->d < 1 || p->d > SIM_MAX_D) return set_err(ctx, SIM_EINVAL, "d=%u outside [1, 64]", p->d);
    if (R < 1 || R > 0xFFFFFFFFull) return set_err(ctx, SIM_EINVAL, "R=%llu outside [1, 2^32)", (unsigned long long)R);
    if (T < 1 || T > 0xFFFFFFFEull) return set_err(ctx, SIM_EINVAL, "T=%llu outside [1, 2^32-2]", (unsigned long long)T);
    if (!p->mu) return set_err(ctx, SIM_EINVAL, "mu is NULL");
    if (p->chol) return set_err(ctx, SIM_EUNSUPPORTED, "dense Cholesky factors are not supported by sim_run");
    if (!p->sigma) return set_err(ctx, SIM_EINVAL, "sigma is NULL");
    for (uint32_t j = 0; j < p->d; ++j) {
        if (!finite(p->mu[j])) return set_err(ctx, SIM_EINVAL, "mu[%u] not finite", j);
        if (!finite(p->sigma[j]) || p->sigma[j] < 0.0)
            return set_err(ctx, SIM_EINVAL, "sigma[%u] must be finite and >= 0", j);
    }
    if (!(p->risk_coef > 0.0) || !finite(p->risk_coef))
        return set_err(ctx, SIM_EINVAL, "risk_coef must be finite and > 0");
    if (p->w0) {
        double s = 0.0;
        for (uint32_t j = 0; j < p->d; ++j) {
            if (!finite(p->w0[j]) || p->w0[j] < 0.0) return set_err(ctx, SIM_EINVAL, "w0[%u] outside W", j);
            s += p->w0[j];
        }
        if (s > 1.0 + 1e-12) return set_err(ctx, SIM_EINVAL, "w0 sums to %g > 1", s);
    }
    if (p->n_samples < 2) return set_err(ctx, SIM_EINVAL, "n_samples must be >= 2 (Eq. (4) divides by N-1)");
    if (p->n_samples > (1u << 24)) return set_err(ctx, SIM_EINVAL, "n_samples above 2^24");
    if (p->resample_every < 1) return set_err(ctx, SIM_EINVAL, "resample_every must be >= 1");
    if (p->noise != SIM_NOISE_GAUSS && p->noise != SIM_NOISE_T) return set_err(ctx, SIM_EINVAL, "unknown noise");
    if (p->noise == SIM_NOISE_T && (p->nu < 3 || p->nu > 1024))
        return set_err(ctx, SIM_EINVAL, "nu must be an integer in [3, 1024]");
    if (p->state_precision != SIM_FP32 && p->state_precision != SIM_FP64)
        return set_err(ctx, SIM_EINVAL, "unknown state_precision");
    if (p->n_checkpoints > SIM_MAX_CKPT) return set_err(ctx, SIM_EINVAL, "more than 8 checkpoints");
    for (uint32_t k = 0; k < p->n_checkpoints; ++k) {
        if (p->checkpoints[k] < 1 || p->checkpoints[k] > T)
            return set_err(ctx, SIM_EINVAL, "checkpoint %u outside [1, T]", k);
        if (k && p->checkpoints[k] <= p->checkpoints[k - 1])
            return set_err(ctx, SIM_EINVAL, "checkpoints must increase strictly");
    }
    if (!finite(p->gap_eps) || p->gap_eps < 0.0) return set_err(ctx, SIM_EINVAL, "gap_eps must be finite and >= 0");
    if (p->flags & ~(uint32_t)(SIM_KEEP_PATHS | SIM_DECISION_LOG)) return set_err(ctx, SIM_EINVAL, "unknown flag bits");
    if (p->instance_id >= (1u << 24)) return set_err(ctx, SIM_EINVAL, "instance_id must be < 2^24");
    if (p->flags & SIM_DECISION_LOG) {
        if (p->log_rep_count < 1 || p->log_rep_count > 65536)
            return set_err(ctx, SIM_EINVAL, "log_rep_count must be in [1, 65536]");
        if (p->log_rep_begin >= R || p->log_rep_count > R - p->log_rep_begin)
            return set_err(ctx, SIM_EINVAL, "logged replications exceed R");
        if (T * p->log_rep_count > (1ull << 34)) return set_err(ctx, SIM_EINVAL, "decision log above 16 GiB");
    }
    return SIM_OK;
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
    for (uint32_t j = 0; j < p->d; ++j) {
        const double mu = p->mu[j], sg = p->sigma[j], w0 = p->w0 ? p->w0[j] : 0.0;
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

}  // namespace

extern "C" {

const char *sim_strerror(int code)
{
    switch (code) {
    case SIM_OK: return "ok";
    case SIM_EINVAL: return "invalid argument";
    case SIM_ENOMEM: return "out of memory";
    case SIM_EDEVICE: return "HIP device error";
    case SIM_ESTATE: return "call out of order";
    case SIM_EUNSUPPORTED: return "unsupported combination";
    default: return "unknown error";
    }
}

int sim_last_error(sim_ctx *ctx, char *buf, size_t len)
{
    if (!ctx || !buf || len == 0) return SIM_EINVAL;
    std::snprintf(buf, len, "%s", ctx->err);
    return SIM_OK;
}

int sim_create(int device, void *hip_stream, sim_ctx **out)
{
    if (!out) return SIM_EINVAL;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return SIM_EDEVICE;
    if (device < 0 || device >= n) return SIM_EINVAL;
    sim_ctx *ctx = new (std::nothrow) sim_ctx();
    if (!ctx) return SIM_ENOMEM;
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    int rc = SIM_OK;
    auto fail = [&](int code) {
        sim_destroy(ctx);
        return code;
    };
    if (hipSetDevice(device) != hipSuccess) return fail(SIM_EDEVICE);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return fail(SIM_EDEVICE);
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return fail(SIM_EUNSUPPORTED);
    if (hipHostMalloc((void **)&ctx->desc_host, sizeof(InstanceDesc), hipHostMallocDefault) != hipSuccess)
        return fail(SIM_ENOMEM);
    if (hipMalloc((void **)&ctx->desc_dev, sizeof(InstanceDesc)) != hipSuccess) return fail(SIM_ENOMEM);
    if (hipEventCreate(&ctx->ev_start) != hipSuccess || hipEventCreate(&ctx->ev_stop) != hipSuccess)
        return fail(SIM_EDEVICE);
    rc = ensure(ctx, ctx->done, 64);
    if (rc) return fail(rc);
    if (hipMemset(ctx->done.ptr, 0, 64) != hipSuccess) return fail(SIM_EDEVICE);
    if (hipDeviceSynchronize() != hipSuccess) return fail(SIM_EDEVICE);
    *out = ctx;
    return SIM_OK;
}

int sim_validate(const sim_params *p, uint64_t R, uint64_t T, char *msg, size_t len)
{
    sim_ctx scratch_ctx;
    const int rc = validate(&scratch_ctx, p, R, T);
    if (msg && len) std::snprintf(msg, len, "%s", rc ? scratch_ctx.err : "");
    return rc;
}

int sim_set_stream(sim_ctx *ctx, void *hip_stream)
{
    if (!ctx) return SIM_EINVAL;
    ctx->stream = (hipStream_t)hip_stream;
    return SIM_OK;
}

void sim_destroy(sim_ctx *ctx)
{
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    else (void)hipDeviceSynchronize();
    for (DevBuf *b : {&ctx->y, &ctx->fck, &ctx->cnt, &ctx->wsum, &ctx->tau, &ctx->dlog, &ctx->part_f,
                      &ctx->part_i, &ctx->done, &ctx->final_f, &ctx->final_i})
        free_buf(*b);
    if (ctx->desc_dev) (void)hipFree(ctx->desc_dev);
    if (ctx->desc_host) (void)hipHostFree(ctx->desc_host);
    if (ctx->ev_start) (void)hipEventDestroy(ctx->ev_start);
    if (ctx->ev_stop) (void)hipEventDestroy(ctx->ev_stop);
    delete ctx;
}

int sim_run(sim_ctx *ctx, const sim_params *p, uint64_t R, uint64_t T, uint64_t seed)
{
    if (!ctx) return SIM_EINVAL;
    int rc = validate(ctx, p, R, T);
    if (rc) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    // the previous run may still read the staging descriptor
    HIP_TRY(ctx, ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize());

    const uint32_t d = p->d;
    const bool keep = (p->flags & SIM_KEEP_PATHS) != 0;
    const bool log = (p->flags & SIM_DECISION_LOG) != 0;
    const uint32_t nblocks = (uint32_t)((R + fw::kBlock - 1) / fw::kBlock);
    const uint32_t n_streams = 1 + 2 * p->n_checkpoints;
    if ((rc = ensure(ctx, ctx->fck, sizeof(double) * (size_t)R * (p->n_checkpoints ? p->n_checkpoints : 1)))) return rc;
    if ((rc = ensure(ctx, ctx->part_f, sizeof(double) * ((size_t)n_streams * fw::kStreamFields + 2) * nblocks))) return rc;
    if ((rc = ensure(ctx, ctx->part_i, sizeof(uint64_t) * (size_t)(d + 3) * nblocks))) return rc;
    if ((rc = ensure(ctx, ctx->final_f, sizeof(double) * ((size_t)fw::kMaxStreams * fw::kStreamFields + 2)))) return rc;
    if ((rc = ensure(ctx, ctx->final_i, sizeof(uint64_t) * (fw::kMaxD + 3)))) return rc;
    if (keep) {
        if ((rc = ensure(ctx, ctx->y, sizeof(double) * R))) return rc;
        if ((rc = ensure(ctx, ctx->tau, sizeof(uint32_t) * R))) return rc;
        if ((rc = ensure(ctx, ctx->cnt, sizeof(uint32_t) * (size_t)(d + 1) * R))) return rc;
        if ((rc = ensure(ctx, ctx->wsum, sizeof(uint64_t) * (size_t)d * R))) return rc;
    }
    if (log && (rc = ensure(ctx, ctx->dlog, (size_t)T * p->log_rep_count))) return rc;

    fill_desc(*ctx->desc_host, p, R, T, seed);
    HIP_TRY(ctx, hipMemcpyAsync(ctx->desc_dev, ctx->desc_host, sizeof(InstanceDesc), hipMemcpyHostToDevice, ctx->stream));

    RunBuffers &B = ctx->bufs;
    B.y = keep ? (double *)ctx->y.ptr : nullptr;
    B.fck = (double *)ctx->fck.ptr;
    B.cnt = keep ? (uint32_t *)ctx->cnt.ptr : nullptr;
    B.wsum = keep ? (uint64_t *)ctx->wsum.ptr : nullptr;
    B.tau = keep ? (uint32_t *)ctx->tau.ptr : nullptr;
    B.dlog = log ? (uint8_t *)ctx->dlog.ptr : nullptr;
    B.part_f = (double *)ctx->part_f.ptr;
    B.part_i = (uint64_t *)ctx->part_i.ptr;
    B.done = (uint32_t *)ctx->done.ptr;
    B.final_f = (double *)ctx->final_f.ptr;
    B.final_i = (uint64_t *)ctx->final_i.ptr;
    B.nblocks = nblocks;
    B.n_streams = n_streams;

    HIP_TRY(ctx, hipEventRecord(ctx->ev_start, ctx->stream));
    int width = 0;
    rc = fw::launch_fw_paths(*ctx->desc_host, ctx->desc_dev, B, p->state_precision == SIM_FP64, ctx->stream, &width);
    if (rc == -5) return set_err(ctx, SIM_EUNSUPPORTED, "no kernel for d=%u with this precision and noise", d);
    if (rc) return set_err(ctx, SIM_EDEVICE, "kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
    HIP_TRY(ctx, hipEventRecord(ctx->ev_stop, ctx->stream));

    ctx->last = *p;
    ctx->last.mu = ctx->last.sigma = ctx->last.chol = ctx->last.w0 = nullptr;
    for (uint32_t j = 0; j < d; ++j) {
        ctx->last_mu[j] = p->mu[j];
        ctx->last_sigma[j] = p->sigma[j];
    }
    ctx->last_diag = true;
    ctx->R = R;
    ctx->T = T;
    ctx->kernel_width = width;
    ctx->have_run = true;
    return SIM_OK;
}

int sim_stats(sim_ctx *ctx, sim_stats_out *out)
{
    if (!ctx || !out) return SIM_EINVAL;
    if (!ctx->have_run) return set_err(ctx, SIM_ESTATE, "no run yet");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipEventSynchronize(ctx->ev_stop));
    const uint32_t d = ctx->last.d, nc = ctx->last.n_checkpoints;
    const uint32_t n_streams = 1 + 2 * nc;
    double F[fw::kMaxStreams * fw::kStreamFields + 2];
    uint64_t I[fw::kMaxD + 3];
    HIP_TRY(ctx, hipMemcpy(F, ctx->final_f.ptr, sizeof(double) * (n_streams * fw::kStreamFields + 2), hipMemcpyDeviceToHost));
    HIP_TRY(ctx, hipMemcpy(I, ctx->final_i.ptr, sizeof(uint64_t) * (d + 3), hipMemcpyDeviceToHost));
    float ms = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->ev_start, ctx->ev_stop));

    std::memset(out, 0, sizeof(*out));
    out->R = ctx->R;
    out->T = ctx->T;
    Moments y = moments(F);
    out->mean = y.mean;
    out->var = y.var;
    out->ci95_halfwidth = 1.96 * std::sqrt(y.var / (double)ctx->R);
    out->min = F[n_streams * fw::kStreamFields];
    out->max = F[n_streams * fw::kStreamFields + 1];
    out->f_star = ctx->last_diag ? kkt_fstar(ctx->last_mu, ctx->last_sigma, d, ctx->last.risk_coef) : NAN;
    out->n_checkpoints = nc;
    for (uint32_t k = 0; k < nc; ++k) {
        out->checkpoints[k] = ctx->last.checkpoints[k];
        Moments f = moments(F + (1 + k) * fw::kStreamFields);
        Moments e = moments(F + (1 + nc + k) * fw::kStreamFields);
        out->f_mean[k] = f.mean;
        out->f_sd[k] = std::sqrt(f.var);
        out->rse_mean[k] = e.mean;
        out->rse_sd[k] = std::sqrt(e.var);
        out->rse_undefined[k] = ctx->R - (uint64_t)e.n;
    }
    for (uint32_t j = 0; j <= d; ++j) out->decision_total[j] = I[j];
    out->tau_count = I[d + 1];
    out->tau_mean = I[d + 1] ? (double)I[d + 2] / (double)I[d + 1] : 0.0;
    out->kernel_ms = ms;
    out->path_steps_per_s = ms > 0.0f ? (double)ctx->R * (double)ctx->T / (ms * 1e-3) : 0.0;
    return SIM_OK;
}

int sim_paths(sim_ctx *ctx, sim_path_view *out)
{
    if (!ctx || !out) return SIM_EINVAL;
    if (!ctx->have_run) return set_err(ctx, SIM_ESTATE, "no run yet");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipEventSynchronize(ctx->ev_stop));
    std::memset(out, 0, sizeof(*out));
    out->R = ctx->R;
    out->T = ctx->T;
    out->d = ctx->last.d;
    out->n_checkpoints = ctx->last.n_checkpoints;
    const bool keep = (ctx->last.flags & SIM_KEEP_PATHS) != 0;
    out->y = keep ? (const double *)ctx->y.ptr : nullptr;
    out->f_ckpt = ctx->last.n_checkpoints ? (const double *)ctx->fck.ptr : nullptr;
    out->cnt = keep ? (const uint32_t *)ctx->cnt.ptr : nullptr;
    out->wsum = keep ? (const uint64_t *)ctx->wsum.ptr : nullptr;
    out->tau = keep ? (const uint32_t *)ctx->tau.ptr : nullptr;
    if (ctx->last.flags & SIM_DECISION_LOG) {
        out->decisions = (const uint8_t *)ctx->dlog.ptr;
        out->log_rep_begin = ctx->last.log_rep_begin;
        out->log_rep_count = ctx->last.log_rep_count;
    }
    return SIM_OK;
}

int sim_copy_to_host(sim_ctx *ctx, void *host_dst, const void *device_src, size_t bytes)
{
    if (!ctx || (!host_dst && bytes) || (!device_src && bytes)) return SIM_EINVAL;
    if (bytes == 0) return SIM_OK;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize());
    HIP_TRY(ctx, hipMemcpy(host_dst, device_src, bytes, hipMemcpyDeviceToHost));
    return SIM_OK;
}

}  // extern "C"
