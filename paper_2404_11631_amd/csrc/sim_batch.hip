// sim_batch.hip -- host side of batched runs (sim_run_batch): the tile plan (host_core.cpp),
// device buffers, and the launches: one tile kernel per (d bucket, noise) class present, tiles
// longest first, then the per-instance reduction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "engine.hpp"

using namespace fw::host;

extern "C" {

int sim_plan_batch(uint32_t n_inst, const sim_params *p, const uint64_t *R, const uint64_t *T,
                   const sim_batch_config *cfg, uint32_t n_cu, uint32_t *lanes_per_rep, uint32_t *n_tiles,
                   char *msg, size_t len)
{
    char err[kErrLen] = {0};
    BatchPlan plan;
    const int rc = plan_batch(err, n_inst, p, R, T, 0, cfg, n_cu, plan);
    if (msg && len) std::snprintf(msg, len, "%s", rc ? err : "");
    if (rc) return rc;
    for (uint32_t i = 0; i < n_inst; ++i) {
        if (lanes_per_rep) lanes_per_rep[i] = plan.P[i];
        if (n_tiles) n_tiles[i] = plan.tiles_of[i];
    }
    return SIM_OK;
}

int sim_run_batch(sim_ctx *ctx, uint32_t n_inst, const sim_params *p, const uint64_t *R, const uint64_t *T,
                  uint64_t seed, const sim_batch_config *cfg)
{
    if (!ctx) return SIM_EINVAL;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipDeviceProp_t prop;
    HIP_TRY(ctx, hipGetDeviceProperties(&prop, ctx->device));
    BatchPlan plan;
    int rc = plan_batch(ctx->err, n_inst, p, R, T, seed, cfg, (uint32_t)prop.multiProcessorCount, plan);
    if (rc) return rc;
    HIP_TRY(ctx, ctx->stream ? hipStreamSynchronize(ctx->stream) : hipDeviceSynchronize());

    BatchState &b = ctx->batch;
    b.have = false;
    b.n_inst = n_inst;
    b.params.assign(p, p + n_inst);
    for (auto &q : b.params) q.mu = q.sigma = q.chol = q.w0 = nullptr;
    b.R.assign(R, R + n_inst);
    b.T.assign(T, T + n_inst);
    b.keep = cfg && (cfg->flags & SIM_KEEP_PATHS);
    b.plan = std::move(plan);
    const BatchPlan &P = b.plan;
    const uint64_t n_tiles = P.n_tiles;

    // pinned staging for the asynchronous uploads
    auto grow_host = [&](void **ptr, size_t &cap, size_t bytes) -> int {
        if (cap >= bytes) return SIM_OK;
        if (*ptr) (void)hipHostFree(*ptr);
        *ptr = nullptr;
        cap = 0;
        if (hipHostMalloc(ptr, bytes, hipHostMallocDefault) != hipSuccess)
            return set_err(ctx, SIM_ENOMEM, "pinned staging of %zu bytes", bytes);
        cap = bytes;
        return SIM_OK;
    };
    if ((rc = grow_host((void **)&b.inst_host, b.inst_host_cap, sizeof(InstanceDesc) * n_inst))) return rc;
    if ((rc = grow_host((void **)&b.tiles_host, b.tiles_host_cap, sizeof(fw::Tile) * n_tiles))) return rc;
    if ((rc = grow_host((void **)&b.slots_host, b.slots_host_cap, sizeof(uint32_t) * (n_inst + 1)))) return rc;
    std::memcpy(b.inst_host, P.desc.data(), sizeof(InstanceDesc) * n_inst);
    std::memcpy(b.tiles_host, P.tiles.data(), sizeof(fw::Tile) * n_tiles);
    std::memcpy(b.slots_host, P.slot_begin.data(), sizeof(uint32_t) * (n_inst + 1));

    // device buffers
    if ((rc = ensure(ctx, b.inst, sizeof(InstanceDesc) * n_inst))) return rc;
    if ((rc = ensure(ctx, b.tiles, sizeof(fw::Tile) * n_tiles))) return rc;
    if ((rc = ensure(ctx, b.slots, sizeof(uint32_t) * (n_inst + 1)))) return rc;
    if ((rc = ensure(ctx, b.partials, sizeof(fw::TilePartial) * n_tiles))) return rc;
    if ((rc = ensure(ctx, b.final_stats, sizeof(fw::TilePartial) * n_inst))) return rc;
    if ((rc = ensure(ctx, b.fck, sizeof(double) * P.max_ckpt * P.total_R))) return rc;
    if (b.keep) {
        if ((rc = ensure(ctx, b.y, sizeof(double) * P.total_R))) return rc;
        if ((rc = ensure(ctx, b.tau, sizeof(uint32_t) * P.total_R))) return rc;
        if ((rc = ensure(ctx, b.cnt, sizeof(uint32_t) * P.cnt_total))) return rc;
        if ((rc = ensure(ctx, b.wsum, sizeof(uint64_t) * P.wsum_total))) return rc;
    }
    if (P.dlog_total && (rc = ensure(ctx, b.dlog, P.dlog_total))) return rc;

    fw::BatchBuffers B{};
    B.inst = (const InstanceDesc *)b.inst.ptr;
    B.tiles = (const fw::Tile *)b.tiles.ptr;
    B.n_tiles = P.n_tiles;
    B.n_inst = n_inst;
    B.partials = (fw::TilePartial *)b.partials.ptr;
    B.slot_begin = (const uint32_t *)b.slots.ptr;
    B.fck = (double *)b.fck.ptr;
    B.total_R = P.total_R;
    B.y = b.keep ? (double *)b.y.ptr : nullptr;
    B.tau = b.keep ? (uint32_t *)b.tau.ptr : nullptr;
    B.cnt = b.keep ? (uint32_t *)b.cnt.ptr : nullptr;
    B.wsum = b.keep ? (uint64_t *)b.wsum.ptr : nullptr;
    B.dlog = P.dlog_total ? (uint8_t *)b.dlog.ptr : nullptr;
    B.final_stats = (fw::TilePartial *)b.final_stats.ptr;

    HIP_TRY(ctx, hipMemcpyAsync(b.inst.ptr, b.inst_host, sizeof(InstanceDesc) * n_inst, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(b.tiles.ptr, b.tiles_host, sizeof(fw::Tile) * n_tiles, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(b.slots.ptr, b.slots_host, sizeof(uint32_t) * (n_inst + 1), hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipEventRecord(b.ev0, ctx->stream));
    if (fw::launch_fw_batch(B, P.class_begin, ctx->stream))
        return set_err(ctx, SIM_EDEVICE, "batch launch failed: %s", hipGetErrorString(hipGetLastError()));
    HIP_TRY(ctx, hipEventRecord(b.ev1, ctx->stream));
    b.have = true;
    return SIM_OK;
}

int sim_batch_stats(sim_ctx *ctx, uint32_t instance, sim_stats_out *out)
{
    if (!ctx || !out) return SIM_EINVAL;
    BatchState &b = ctx->batch;
    if (!b.have) return set_err(ctx, SIM_ESTATE, "no batched run yet");
    if (instance >= b.n_inst) return set_err(ctx, SIM_EINVAL, "instance %u >= %u", instance, b.n_inst);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipEventSynchronize(b.ev1));
    fw::TilePartial tp;
    HIP_TRY(ctx, hipMemcpy(&tp, (const fw::TilePartial *)b.final_stats.ptr + instance, sizeof(tp), hipMemcpyDeviceToHost));
    float ms = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, b.ev0, b.ev1));
    const sim_params &q = b.params[instance];
    fill_stats(out, tp.f, q.n_checkpoints, q.checkpoints, tp.ymin, tp.ymax, tp.dec, q.d, tp.tau_count, tp.tau_sum,
               b.R[instance], b.T[instance], b.plan.fstar[instance], ms, (double)b.plan.total_steps);
    return SIM_OK;
}

int sim_batch_paths(sim_ctx *ctx, uint32_t instance, sim_path_view *out, uint32_t *lanes_per_rep, uint32_t *n_tiles)
{
    if (!ctx || !out) return SIM_EINVAL;
    BatchState &b = ctx->batch;
    if (!b.have) return set_err(ctx, SIM_ESTATE, "no batched run yet");
    if (instance >= b.n_inst) return set_err(ctx, SIM_EINVAL, "instance %u >= %u", instance, b.n_inst);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipEventSynchronize(b.ev1));
    const sim_params &q = b.params[instance];
    const BatchPlan &P = b.plan;
    const uint64_t base = P.path_base[instance];
    std::memset(out, 0, sizeof(*out));
    out->R = b.R[instance];
    out->T = b.T[instance];
    out->d = q.d;
    out->n_checkpoints = q.n_checkpoints;
    if (b.keep) {
        out->y = (const double *)b.y.ptr + base;
        out->tau = (const uint32_t *)b.tau.ptr + base;
        out->cnt = (const uint32_t *)b.cnt.ptr + P.cnt_base[instance];
        out->wsum = (const uint64_t *)b.wsum.ptr + P.wsum_base[instance];
    }
    out->f_ckpt = q.n_checkpoints ? (const double *)b.fck.ptr + base : nullptr;
    out->f_ckpt_stride = P.total_R;
    if (q.flags & SIM_DECISION_LOG) {
        out->decisions = (const uint8_t *)b.dlog.ptr + P.dlog_base[instance];
        out->log_rep_begin = q.log_rep_begin;
        out->log_rep_count = q.log_rep_count;
    }
    if (lanes_per_rep) *lanes_per_rep = P.P[instance];
    if (n_tiles) *n_tiles = P.tiles_of[instance];
    return SIM_OK;
}

}  // extern "C"
