// sim_batch.hip -- host side of batched runs (sim_run_batch): the tile plan (host_core.cpp),
// device buffers, and the launches: the tile kernel over every tile (longest first), then the
// per-instance reduction.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

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
    B.wave_mode = P.wave_mode ? 1u : 0u;

    HIP_TRY(ctx, hipMemcpyAsync(b.inst.ptr, b.inst_host, sizeof(InstanceDesc) * n_inst, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(b.tiles.ptr, b.tiles_host, sizeof(fw::Tile) * n_tiles, hipMemcpyHostToDevice, ctx->stream));
    HIP_TRY(ctx, hipMemcpyAsync(b.slots.ptr, b.slots_host, sizeof(uint32_t) * (n_inst + 1), hipMemcpyHostToDevice, ctx->stream));
    const bool graph = cfg && (cfg->flags & SIM_BATCH_GRAPH);
    const fw::BatchBuffers &A = b.exec_args;
    const bool same_args = A.inst == B.inst && A.tiles == B.tiles && A.n_tiles == B.n_tiles && A.n_inst == B.n_inst &&
                           A.partials == B.partials && A.slot_begin == B.slot_begin && A.fck == B.fck &&
                           A.total_R == B.total_R && A.y == B.y && A.tau == B.tau && A.cnt == B.cnt &&
                           A.wsum == B.wsum && A.dlog == B.dlog && A.final_stats == B.final_stats &&
                           A.wave_mode == B.wave_mode;
    if (graph && (!b.exec || !same_args)) {
        // capture the two kernel launches on the library's own stream (default priority)
        if (b.exec) {
            HIP_TRY(ctx, hipGraphExecDestroy(b.exec));
            b.exec = nullptr;
        }
        if (!b.capture) HIP_TRY(ctx, hipStreamCreateWithFlags(&b.capture, hipStreamNonBlocking));
        HIP_TRY(ctx, hipStreamBeginCapture(b.capture, hipStreamCaptureModeThreadLocal));
        const int lrc = fw::launch_fw_batch(B, b.capture);
        hipGraph_t g = nullptr;
        const hipError_t ec = hipStreamEndCapture(b.capture, &g);
        if (lrc || ec != hipSuccess || !g) {
            if (g) (void)hipGraphDestroy(g);
            return set_err(ctx, SIM_EDEVICE, "batch graph capture failed: %s", hipGetErrorString(ec));
        }
        const hipError_t ei = hipGraphInstantiate(&b.exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (ei != hipSuccess) {
            b.exec = nullptr;
            return set_err(ctx, SIM_EDEVICE, "batch graph instantiation failed: %s", hipGetErrorString(ei));
        }
        b.exec_args = B;
        ++b.graph_captures;
    }
    HIP_TRY(ctx, hipEventRecord(b.ev0, ctx->stream));
    if (graph) {
        HIP_TRY(ctx, hipGraphLaunch(b.exec, ctx->stream));
        ++b.graph_launches;
    } else if (fw::launch_fw_batch(B, ctx->stream)) {
        return set_err(ctx, SIM_EDEVICE, "batch launch failed: %s", hipGetErrorString(hipGetLastError()));
    }
    HIP_TRY(ctx, hipEventRecord(b.ev1, ctx->stream));
    b.have = true;
    return SIM_OK;
}

namespace {

// candidates of theta, heaviest splitting last
constexpr double kTuneThetas[] = {2.0, 1.0, 0.5, 0.25, 0.125, 0.0625, 0.03125};
constexpr uint32_t kTuneN = sizeof(kTuneThetas) / sizeof(kTuneThetas[0]);
static_assert(kTuneN <= SIM_TUNE_MAX_CAND, "candidate list exceeds sim_tune_out");

uint64_t fnv1a(uint64_t h, const void *data, size_t n)
{
    const unsigned char *b = static_cast<const unsigned char *>(data);
    for (size_t i = 0; i < n; ++i) {
        h ^= b[i];
        h *= 0x100000001B3ull;
    }
    return h;
}

// the cached theta of `key`, from a JSON-lines file written by append_cache
bool read_cache(const char *path, uint64_t key, double *theta)
{
    if (!path) return false;
    FILE *f = std::fopen(path, "r");
    if (!f) return false;
    char line[4096];
    char want[64];
    std::snprintf(want, sizeof(want), "\"key\": \"%016llx\"", (unsigned long long)key);
    bool found = false;
    while (std::fgets(line, sizeof(line), f)) {
        if (!std::strstr(line, want)) continue;
        const char *h = std::strstr(line, "\"heavy_factor\": ");
        double v = 0.0;
        if (h && std::sscanf(h + 16, "%lf", &v) == 1 && v > 0.0 && std::isfinite(v)) {
            *theta = v;
            found = true;
        }
    }
    std::fclose(f);
    return found;
}

void append_cache(const char *path, uint64_t key, const char *device, uint32_t t_scale, const sim_tune_out &o)
{
    if (!path) return;
    FILE *f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "{\"key\": \"%016llx\", \"device\": \"%s\", \"abi\": %u, \"t_scale\": %u, "
                    "\"heavy_factor\": %.17g, \"candidates\": [",
                 (unsigned long long)key, device, (unsigned)SIM_ABI_VERSION, t_scale, o.heavy_factor);
    for (uint32_t c = 0; c < o.n_candidates; ++c)
        std::fprintf(f, "%s{\"heavy_factor\": %.17g, \"ms\": %.6f}", c ? ", " : "", o.cand_theta[c], o.cand_ms[c]);
    std::fprintf(f, "]}\n");
    std::fclose(f);
}

}  // namespace

int sim_tune_batch(sim_ctx *ctx, uint32_t n_inst, const sim_params *p, const uint64_t *R, const uint64_t *T,
                   uint64_t seed, uint32_t t_scale, const char *cache_path, sim_tune_out *out)
{
    if (!ctx || !out) return SIM_EINVAL;
    if (t_scale < 1) return set_err(ctx, SIM_EINVAL, "t_scale must be >= 1");
    if (n_inst < 1 || n_inst > 65536 || !p || !R || !T)
        return set_err(ctx, SIM_EINVAL, "need 1 <= n_inst <= 65536 and non-NULL p, R, T");
    std::memset(out, 0, sizeof(*out));
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    hipDeviceProp_t prop;
    HIP_TRY(ctx, hipGetDeviceProperties(&prop, ctx->device));

    // the reduced problem: horizons divided by t_scale, no checkpoints, logs or records
    std::vector<sim_params> q(p, p + n_inst);
    std::vector<uint64_t> Ts(n_inst);
    for (uint32_t i = 0; i < n_inst; ++i) {
        q[i].n_checkpoints = 0;
        q[i].flags = 0;
        q[i].log_rep_begin = q[i].log_rep_count = 0;
        Ts[i] = std::max<uint64_t>(1, T[i] / t_scale);
    }
    // the plan of the full problem must be valid before anything is cached for it
    {
        BatchPlan check;
        const int rc = plan_batch(ctx->err, n_inst, p, R, T, seed, nullptr, (uint32_t)prop.multiProcessorCount, check);
        if (rc) return rc;
    }

    uint64_t key = 0xCBF29CE484222325ull;
    key = fnv1a(key, prop.name, std::strlen(prop.name));
    key = fnv1a(key, prop.gcnArchName, std::strlen(prop.gcnArchName));
    const uint32_t abi = SIM_ABI_VERSION;
    key = fnv1a(key, &abi, sizeof(abi));
    key = fnv1a(key, kTuneThetas, sizeof(kTuneThetas));
    key = fnv1a(key, &n_inst, sizeof(n_inst));
    for (uint32_t i = 0; i < n_inst; ++i) {
        const uint64_t f[6] = {p[i].d, p[i].n_samples, T[i], R[i], p[i].noise, p[i].noise == SIM_NOISE_T ? p[i].nu : 0u};
        key = fnv1a(key, f, sizeof(f));
    }
    out->key = key;
    double theta = 0.0;
    if (read_cache(cache_path, key, &theta)) {
        out->heavy_factor = theta;
        out->from_cache = 1;
        return SIM_OK;
    }

    double best = INFINITY;
    for (uint32_t c = 0; c < kTuneN; ++c) {
        sim_batch_config cfg{};
        cfg.heavy_factor = kTuneThetas[c];
        double ms_best = INFINITY;
        for (int rep = 0; rep < 2; ++rep) {
            const int rc = sim_run_batch(ctx, n_inst, q.data(), R, Ts.data(), seed, &cfg);
            if (rc) return rc;
            HIP_TRY(ctx, hipEventSynchronize(ctx->batch.ev1));
            float ms = 0.0f;
            HIP_TRY(ctx, hipEventElapsedTime(&ms, ctx->batch.ev0, ctx->batch.ev1));
            ms_best = std::min(ms_best, (double)ms);
        }
        out->cand_theta[c] = kTuneThetas[c];
        out->cand_ms[c] = ms_best;
        if (ms_best < best) {
            best = ms_best;
            out->heavy_factor = kTuneThetas[c];
        }
    }
    out->n_candidates = kTuneN;
    append_cache(cache_path, key, prop.name, t_scale, *out);
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
