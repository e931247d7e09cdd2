// sim_api.hip -- host engine behind the C ABI declared in include/sim.h: validation, instance
// coefficients, device buffers, launch, and the final FP64 statistics.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>

#include "engine.hpp"
#include "host_core.hpp"

namespace fw {
namespace host {

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

int ensure(sim_ctx *ctx, DevBuf &b, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    if (b.bytes >= bytes) return SIM_OK;
    if (ctx->ws_limit && ctx->ws_used - b.bytes + bytes > ctx->ws_limit)
        return set_err(ctx, SIM_ENOMEM, "the context's workspace limit of %llu bytes cannot hold a buffer of %zu bytes "
                       "(%llu in use)", (unsigned long long)ctx->ws_limit, bytes, (unsigned long long)ctx->ws_used);
    if (b.ptr) {
        HIP_TRY(ctx, hipFree(b.ptr));
        ctx->ws_used -= b.bytes;
        b.ptr = nullptr;
        b.bytes = 0;
    }
    hipError_t e = hipMalloc(&b.ptr, bytes);
    if (e != hipSuccess) {
        b.ptr = nullptr;
        return set_err(ctx, SIM_ENOMEM, "hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
    }
    b.bytes = bytes;
    ctx->ws_used += bytes;
    return SIM_OK;
}

void free_buf(DevBuf &b)
{
    if (b.ptr) (void)hipFree(b.ptr);
    b.ptr = nullptr;
    b.bytes = 0;
}

}  // namespace host
}  // namespace fw

using namespace fw::host;

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
    if (hipEventCreate(&ctx->batch.ev0) != hipSuccess || hipEventCreate(&ctx->batch.ev1) != hipSuccess)
        return fail(SIM_EDEVICE);
    rc = ensure(ctx, ctx->done, 64);
    if (rc) return fail(rc);
    if (hipMemset(ctx->done.ptr, 0, 64) != hipSuccess) return fail(SIM_EDEVICE);
    if (hipDeviceSynchronize() != hipSuccess) return fail(SIM_EDEVICE);
    *out = ctx;
    return SIM_OK;
}

int sim_create_ex(int device, void *hip_stream, uint64_t workspace_bytes, sim_ctx **out)
{
    const int rc = sim_create(device, hip_stream, out);
    if (rc) return rc;
    sim_ctx *ctx = *out;
    if (workspace_bytes && ctx->ws_used > workspace_bytes) {
        sim_destroy(ctx);
        *out = nullptr;
        return SIM_ENOMEM;
    }
    ctx->ws_limit = workspace_bytes;
    return SIM_OK;
}

int sim_param_gen(uint32_t d, int regime, uint64_t seed, double *mu, double *sigma)
{
    if (d == 0 || !mu || !sigma) return SIM_EINVAL;
    double lo_mu, hi_mu, hi_sig;
    if (regime == SIM_REGIME_UNIT) {
        lo_mu = 0.0;
        hi_mu = 1.0;
        hi_sig = 1.0;
    } else if (regime == SIM_REGIME_PAPER) {
        lo_mu = -1.0;
        hi_mu = 1.0;
        hi_sig = 0.025;
    } else {
        return SIM_EINVAL;
    }
    // SplitMix64 (Steele, Lea and Flood, 2014); the top 53 bits give a uniform on [0, 1)
    uint64_t x = seed;
    auto next = [&x]() {
        x += 0x9E3779B97F4A7C15ull;
        uint64_t z = x;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return static_cast<double>((z ^ (z >> 31)) >> 11) * 0x1.0p-53;
    };
    for (uint32_t j = 0; j < d; ++j) mu[j] = lo_mu + (hi_mu - lo_mu) * next();
    for (uint32_t j = 0; j < d; ++j) sigma[j] = hi_sig * next();
    return SIM_OK;
}

int sim_workspace_bytes(sim_ctx *ctx, uint64_t *used)
{
    if (!ctx || !used) return SIM_EINVAL;
    *used = ctx->ws_used;
    return SIM_OK;
}

int sim_validate(const sim_params *p, uint64_t R, uint64_t T, char *msg, size_t len)
{
    char err[fw::host::kErrLen] = {0};
    const int rc = validate(err, p, R, T);
    if (msg && len) std::snprintf(msg, len, "%s", rc ? err : "");
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
                      &ctx->part_i, &ctx->done, &ctx->final_f, &ctx->final_i, &ctx->dense,
                      &ctx->feat, &ctx->sched})
        free_buf(*b);
    if (ctx->dense_host) (void)hipHostFree(ctx->dense_host);
    if (ctx->desc_dev) (void)hipFree(ctx->desc_dev);
    if (ctx->desc_host) (void)hipHostFree(ctx->desc_host);
    if (ctx->ev_start) (void)hipEventDestroy(ctx->ev_start);
    if (ctx->ev_stop) (void)hipEventDestroy(ctx->ev_stop);
    BatchState &b = ctx->batch;
    for (DevBuf *x : {&b.inst, &b.tiles, &b.slots, &b.partials, &b.final_stats, &b.fck, &b.y, &b.tau, &b.cnt,
                      &b.wsum, &b.dlog})
        free_buf(*x);
    if (b.inst_host) (void)hipHostFree(b.inst_host);
    if (b.tiles_host) (void)hipHostFree(b.tiles_host);
    if (b.slots_host) (void)hipHostFree(b.slots_host);
    if (b.ev0) (void)hipEventDestroy(b.ev0);
    if (b.ev1) (void)hipEventDestroy(b.ev1);
    if (b.exec) (void)hipGraphExecDestroy(b.exec);
    if (b.capture) (void)hipStreamDestroy(b.capture);
    CvState &cv = ctx->cv;
    for (DevBuf *x : {&cv.theta, &cv.w1a, &cv.w2a, &cv.w2t, &cv.mom1, &cv.mom2, &cv.part, &cv.grad, &cv.loss_hist,
                      &cv.xtrain, &cv.ytrain, &cv.ttrain, &cv.xio, &cv.yio, &cv.hout, &cv.xaux, &cv.haux, &cv.mpart,
                      &cv.mout, &cv.mdone})
        free_buf(*x);
    for (hipEvent_t e : {cv.ev0, cv.ev1, cv.ev_a, cv.ev_b})
        if (e) (void)hipEventDestroy(e);
    NvLpState &lp = ctx->nvlp;
    for (DevBuf *x : {&lp.prod_d, &lp.Am, &lp.Cv, &lp.x, &lp.g, &lp.rec_basis, &lp.rec_value, &lp.rec_piv,
                      &lp.tau, &lp.origin, &lp.cost_part, &lp.fval, &lp.stats, &lp.origin_total})
        free_buf(*x);
    for (hipEvent_t e : {lp.ev0, lp.ev1})
        if (e) (void)hipEventDestroy(e);
    WideState &wd = ctx->wide;
    for (DevBuf *x : {&wd.asset_f, &wd.asset_d, &wd.S, &wd.cnt, &wd.tau, &wd.dec, &wd.s1, &wd.part_dot, &wd.part_qn,
                      &wd.dot, &wd.qn, &wd.wg_g, &wd.wg_j, &wd.wg_gw, &wd.fval, &wd.stats, &wd.origin})
        free_buf(*x);
    for (hipEvent_t e : {wd.ev0, wd.ev1})
        if (e) (void)hipEventDestroy(e);
    NvState &nv = ctx->nv;
    for (DevBuf *x : {&nv.prod_f, &nv.prod_d, &nv.S, &nv.cnt, &nv.tau, &nv.dec, &nv.wg_r, &nv.wg_j, &nv.wg_gx,
                      &nv.cost_part, &nv.fval, &nv.stats, &nv.origin})
        free_buf(*x);
    for (hipEvent_t e : {nv.ev0, nv.ev1})
        if (e) (void)hipEventDestroy(e);
    SqnState &sq = ctx->sqn;
    for (DevBuf *x : {&sq.X, &sq.z, &sq.S, &sq.Y, &sq.wprev, &sq.acc, &sq.wsnap, &sq.wt, &sq.H, &sq.hscratch, &sq.pairs, &sq.loss_part, &sq.fval, &sq.stats})
        free_buf(*x);
    for (hipEvent_t e : {sq.ev0, sq.ev1, sq.ev2, sq.ev3, sq.ev4})
        if (e) (void)hipEventDestroy(e);
    delete ctx;
}

}  // extern "C"

namespace fw {
namespace host {

// One run of Algorithm 1 over R replications; `internal` adds descriptor flag bits the public
// flags do not carry (kFlagYOnly).
int run_impl(sim_ctx *ctx, const sim_params *p, uint64_t R, uint64_t T, uint64_t seed, uint32_t internal,
             const RunInto *into)
{
    if (!ctx) return SIM_EINVAL;
    int rc = validate(ctx->err, p, R, T);
    if (rc) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    // the previous run may still read the staging descriptor
    HIP_TRY(ctx, ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize());

    const uint32_t d = p->d;
    const bool keep = (p->flags & SIM_KEEP_PATHS) != 0;
    const bool want_y = keep || (internal & fw::kFlagYOnly);
    const bool log = (p->flags & SIM_DECISION_LOG) != 0;
    const bool dense = p->chol != nullptr;
    const uint32_t reps_per_block = dense ? fw::kDenseRepsPerBlock : fw::kBlock;
    const uint32_t nblocks = (uint32_t)((R + reps_per_block - 1) / reps_per_block);
    const uint32_t n_streams = 1 + 2 * p->n_checkpoints;
    if ((rc = ensure(ctx, ctx->fck, sizeof(double) * (size_t)R * (p->n_checkpoints ? p->n_checkpoints : 1)))) return rc;
    if ((rc = ensure(ctx, ctx->part_f, sizeof(double) * ((size_t)n_streams * fw::kStreamFields + 2) * nblocks))) return rc;
    if ((rc = ensure(ctx, ctx->part_i, sizeof(uint64_t) * (size_t)(d + 3) * nblocks))) return rc;
    if ((rc = ensure(ctx, ctx->final_f, sizeof(double) * ((size_t)fw::kMaxStreams * fw::kStreamFields + 2)))) return rc;
    if ((rc = ensure(ctx, ctx->final_i, sizeof(uint64_t) * (fw::kMaxD + 3)))) return rc;
    if (want_y && (rc = ensure(ctx, ctx->y, sizeof(double) * R))) return rc;
    if (keep) {
        if ((rc = ensure(ctx, ctx->tau, sizeof(uint32_t) * R))) return rc;
        if ((rc = ensure(ctx, ctx->cnt, sizeof(uint32_t) * (size_t)(d + 1) * R))) return rc;
        if ((rc = ensure(ctx, ctx->wsum, sizeof(uint64_t) * (size_t)d * R))) return rc;
    }
    if (log && (rc = ensure(ctx, ctx->dlog, (size_t)T * p->log_rep_count))) return rc;
    const bool feat = (p->flags & SIM_CV_FEATURES) != 0;
    if (feat && (rc = ensure(ctx, ctx->feat, sizeof(float) * (size_t)(d + 2) * R))) return rc;

    // dense L: the two MFMA-ordered FP32 operands and L in FP64, staged through pinned memory
    const size_t dense_f = (size_t)SIM_MAX_D * SIM_MAX_D;
    const size_t dense_bytes = 2 * dense_f * sizeof(float) + dense_f * sizeof(double);
    if (dense) {
        if ((rc = ensure(ctx, ctx->dense, dense_bytes))) return rc;
        if (!ctx->dense_host && hipHostMalloc(&ctx->dense_host, dense_bytes, hipHostMallocDefault) != hipSuccess) {
            ctx->dense_host = nullptr;
            return set_err(ctx, SIM_ENOMEM, "pinned staging of %zu bytes", dense_bytes);
        }
        float *ag = (float *)ctx->dense_host;
        double *l64 = (double *)(ag + 2 * dense_f);
        dense_operands(p->chol, d, ag, ag + dense_f, l64);
        HIP_TRY(ctx, hipMemcpyAsync(ctx->dense.ptr, ctx->dense_host, dense_bytes, hipMemcpyHostToDevice, ctx->stream));
    }

    // per-epoch sample sizes: the table is uploaded from a host copy kept until the next run
    // (every run first waits for the previous one on the stream)
    SchedLayout sl;
    if (p->n_schedule) {
        try {
            fill_schedule(p, T, ctx->sched_host, sl);
        } catch (const std::bad_alloc &) {
            return set_err(ctx, SIM_ENOMEM, "host memory for the sample-size table");
        }
        if ((rc = ensure(ctx, ctx->sched, sl.bytes))) return rc;
        HIP_TRY(ctx, hipMemcpyAsync(ctx->sched.ptr, ctx->sched_host.data(), sl.bytes, hipMemcpyHostToDevice, ctx->stream));
    }

    fill_desc(*ctx->desc_host, p, R, T, seed);
    ctx->desc_host->flags |= internal;
    HIP_TRY(ctx, hipMemcpyAsync(ctx->desc_dev, ctx->desc_host, sizeof(InstanceDesc), hipMemcpyHostToDevice, ctx->stream));

    RunBuffers &B = ctx->bufs;
    B.y = want_y ? (double *)ctx->y.ptr : nullptr;
    B.fck = (into && into->fck) ? into->fck : (double *)ctx->fck.ptr;
    B.cnt = keep ? (uint32_t *)ctx->cnt.ptr : nullptr;
    B.wsum = keep ? (uint64_t *)ctx->wsum.ptr : nullptr;
    B.tau = keep ? (uint32_t *)ctx->tau.ptr : nullptr;
    B.dlog = log ? (uint8_t *)ctx->dlog.ptr : nullptr;
    B.feat = feat ? (float *)ctx->feat.ptr : nullptr;
    B.part_f = (double *)ctx->part_f.ptr;
    B.part_i = (uint64_t *)ctx->part_i.ptr;
    B.done = (uint32_t *)ctx->done.ptr;
    B.final_f = (into && into->final_f) ? into->final_f : (double *)ctx->final_f.ptr;
    B.final_i = (into && into->final_i) ? into->final_i : (uint64_t *)ctx->final_i.ptr;
    B.nblocks = nblocks;
    B.n_streams = n_streams;
    B.dense_g = dense ? (const float *)ctx->dense.ptr : nullptr;
    B.dense_v = dense ? (const float *)ctx->dense.ptr + dense_f : nullptr;
    B.dense_l64 = dense ? (const double *)((const float *)ctx->dense.ptr + 2 * dense_f) : nullptr;
    const unsigned char *sb = static_cast<const unsigned char *>(ctx->sched.ptr);
    B.sched_n = p->n_schedule ? reinterpret_cast<const uint32_t *>(sb + sl.off_n) : nullptr;
    B.sched_inv_f = p->n_schedule ? reinterpret_cast<const float *>(sb + sl.off_inv_f) : nullptr;
    B.sched_inv_d = p->n_schedule ? reinterpret_cast<const double *>(sb + sl.off_inv_d) : nullptr;
    B.sched_c_f = p->n_schedule ? reinterpret_cast<const float *>(sb + sl.off_c_f) : nullptr;
    B.sched_c_d = p->n_schedule ? reinterpret_cast<const double *>(sb + sl.off_c_d) : nullptr;

    HIP_TRY(ctx, hipEventRecord(ctx->ev_start, ctx->stream));
    int width = 0;
    if (dense) {
        rc = fw::launch_fw_dense(*ctx->desc_host, ctx->desc_dev, B, ctx->stream);
        width = 2;
    } else {
        rc = fw::launch_fw_paths(*ctx->desc_host, ctx->desc_dev, B, p->state_precision == SIM_FP64, ctx->stream, &width);
    }
    if (rc == -5) return set_err(ctx, SIM_EUNSUPPORTED, "no kernel for d=%u with this precision and noise", d);
    if (rc) return set_err(ctx, SIM_EDEVICE, "kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
    HIP_TRY(ctx, hipEventRecord(ctx->ev_stop, ctx->stream));

    ctx->last = *p;
    ctx->last.mu = ctx->last.sigma = ctx->last.chol = ctx->last.w0 = nullptr;
    ctx->last.n_schedule = nullptr;
    for (uint32_t j = 0; j < d; ++j) {
        ctx->last_mu[j] = p->mu[j];
        ctx->last_sigma[j] = dense ? 0.0 : p->sigma[j];
    }
    ctx->last_diag = !dense;
    ctx->R = R;
    ctx->T = T;
    ctx->kernel_width = width;
    ctx->have_run = true;
    ctx->last_into = into != nullptr;
    return SIM_OK;
}

}  // namespace host
}  // namespace fw

extern "C" {

int sim_run(sim_ctx *ctx, const sim_params *p, uint64_t R, uint64_t T, uint64_t seed)
{
    return run_impl(ctx, p, R, T, seed, 0u);
}

int sim_run_into(sim_ctx *ctx, const sim_params *p, uint64_t R, uint64_t T, uint64_t seed, double *f_ckpt,
                 double *stats_f, uint64_t *stats_i)
{
    if (!ctx) return SIM_EINVAL;
    if (!p || !stats_f || !stats_i) return set_err(ctx, SIM_EINVAL, "params, stats_f and stats_i are required");
    if (p->n_checkpoints && !f_ckpt) return set_err(ctx, SIM_EINVAL, "f_ckpt is required with checkpoints");
    fw::host::RunInto into;
    into.fck = p->n_checkpoints ? f_ckpt : nullptr;
    into.final_f = stats_f;
    into.final_i = stats_i;
    return run_impl(ctx, p, R, T, seed, 0u, &into);
}

int sim_stats(sim_ctx *ctx, sim_stats_out *out)
{
    if (!ctx || !out) return SIM_EINVAL;
    if (!ctx->have_run) return set_err(ctx, SIM_ESTATE, "no run yet");
    if (ctx->last_into)
        return set_err(ctx, SIM_ESTATE, "the last run wrote its statistics to caller memory (sim_stats_from_raw)");
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

    const double fstar = ctx->last_diag ? kkt_fstar(ctx->last_mu, ctx->last_sigma, d, ctx->last.risk_coef) : NAN;
    fill_stats(out, F, nc, ctx->last.checkpoints, F[n_streams * fw::kStreamFields],
               F[n_streams * fw::kStreamFields + 1], I, d, I[d + 1], I[d + 2], ctx->R, ctx->T, fstar, ms,
               (double)ctx->R * (double)ctx->T);
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
    out->f_ckpt = (ctx->last.n_checkpoints && !ctx->last_into) ? (const double *)ctx->fck.ptr : nullptr;
    out->f_ckpt_stride = ctx->R;
    out->cnt = keep ? (const uint32_t *)ctx->cnt.ptr : nullptr;
    out->wsum = keep ? (const uint64_t *)ctx->wsum.ptr : nullptr;
    out->tau = keep ? (const uint32_t *)ctx->tau.ptr : nullptr;
    if (ctx->last.flags & SIM_DECISION_LOG) {
        out->decisions = (const uint8_t *)ctx->dlog.ptr;
        out->log_rep_begin = ctx->last.log_rep_begin;
        out->log_rep_count = ctx->last.log_rep_count;
    }
    if (ctx->last.flags & SIM_CV_FEATURES) {
        out->x = (const float *)ctx->feat.ptr;
        out->n_features = ctx->last.d + 2;
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
