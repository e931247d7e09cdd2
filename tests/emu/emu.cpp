// CPU emulation of the batched tile kernels (test infrastructure only): the real host planner and
// the real device source, compiled for the host against tests/emu/shim, each workgroup run as
// lockstep threads, every buffer in host memory.
#include <hip/hip_runtime.h>
thread_local Dim3emu threadIdx;
thread_local Dim3emu blockIdx;
EmuBlock *g_block = nullptr;

#include "../../paper_2404_11631_amd/csrc/fw_batch.hip"
#include "../../paper_2404_11631_amd/csrc/host_core.hpp"

#include <cstdio>
#include <vector>

using namespace fw;
using namespace fw::host;

static BatchPlan g_plan;
static std::vector<TilePartial> g_partials, g_final;
static std::vector<double> g_fck, g_y;
static std::vector<uint32_t> g_tau, g_cnt;
static std::vector<uint64_t> g_wsum;
static std::vector<uint8_t> g_dlog;
static std::vector<sim_params> g_params;
static std::vector<uint64_t> g_R, g_T;
static char g_err[512];

extern "C" int emu_run_batch(uint32_t n_inst, const sim_params *p, const uint64_t *R, const uint64_t *T,
                             uint64_t seed, const sim_batch_config *cfg, int keep)
{
    g_plan = BatchPlan{};
    const int rc = plan_batch(g_err, n_inst, p, R, T, seed, cfg, 256, g_plan);
    if (rc) return rc;
    g_params.assign(p, p + n_inst);
    g_R.assign(R, R + n_inst);
    g_T.assign(T, T + n_inst);
    BatchPlan &P = g_plan;
    g_partials.assign(P.n_tiles, TilePartial{});
    g_final.assign(n_inst, TilePartial{});
    g_fck.assign((size_t)P.max_ckpt * P.total_R, 0.0);
    g_y.assign(keep ? P.total_R : 0, 0.0);
    g_tau.assign(keep ? P.total_R : 0, 0);
    g_cnt.assign(keep ? P.cnt_total : 0, 0);
    g_wsum.assign(keep ? P.wsum_total : 0, 0);
    g_dlog.assign(P.dlog_total, 0xEE);
    BatchBuffers B{};
    B.inst = P.desc.data();
    B.tiles = P.tiles.data();
    B.n_tiles = P.n_tiles;
    B.n_inst = n_inst;
    B.partials = g_partials.data();
    B.slot_begin = P.slot_begin.data();
    B.fck = g_fck.data();
    B.total_R = P.total_R;
    B.y = keep ? g_y.data() : nullptr;
    B.tau = keep ? g_tau.data() : nullptr;
    B.cnt = keep ? g_cnt.data() : nullptr;
    B.wsum = keep ? g_wsum.data() : nullptr;
    B.dlog = P.dlog_total ? g_dlog.data() : nullptr;
    B.final_stats = g_final.data();
    B.wave_mode = P.wave_mode ? 1u : 0u;
    for (uint32_t t = 0; t < P.n_tiles; ++t)
        emu_run_block(B.wave_mode ? 128 : 64, t, [&] { if (B.wave_mode) fw_wave_kernel(B); else fw_tile_kernel(B); });
    for (uint32_t i = 0; i < n_inst; ++i) emu_run_block(256, i, [&] { fw_batch_reduce(B); });
    return 0;
}

extern "C" int emu_batch_stats(uint32_t i, sim_stats_out *out)
{
    const TilePartial &tp = g_final[i];
    const sim_params &q = g_params[i];
    fill_stats(out, tp.f, q.n_checkpoints, q.checkpoints, tp.ymin, tp.ymax, tp.dec, q.d, tp.tau_count, tp.tau_sum,
               g_R[i], g_T[i], g_plan.fstar[i], 0.0, 0.0);
    return 0;
}

extern "C" int emu_batch_paths(uint32_t i, sim_path_view *out, uint32_t *P, uint32_t *nt)
{
    const sim_params &q = g_params[i];
    const uint64_t base = g_plan.path_base[i];
    std::memset(out, 0, sizeof(*out));
    out->R = g_R[i];
    out->T = g_T[i];
    out->d = q.d;
    out->n_checkpoints = q.n_checkpoints;
    if (!g_y.empty()) {
        out->y = g_y.data() + base;
        out->tau = g_tau.data() + base;
        out->cnt = g_cnt.data() + g_plan.cnt_base[i];
        out->wsum = g_wsum.data() + g_plan.wsum_base[i];
    }
    out->f_ckpt = q.n_checkpoints ? g_fck.data() + base : nullptr;
    out->f_ckpt_stride = g_plan.total_R;
    if (q.flags & SIM_DECISION_LOG) {
        out->decisions = g_dlog.data() + g_plan.dlog_base[i];
        out->log_rep_begin = q.log_rep_begin;
        out->log_rep_count = q.log_rep_count;
    }
    *P = g_plan.P[i];
    *nt = g_plan.tiles_of[i];
    return 0;
}

// Philox4x32-10 started from a stream's row (philox_row / philox_block) against the generator run
// in full, on n counters from a SplitMix64 sequence; returns the number of differing words.
extern "C" int emu_philox_row_check(uint64_t seed, int n)
{
    uint64_t x = seed;
    auto next = [&x]() {
        x += 0x9E3779B97F4A7C15ull;
        uint64_t z = x;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    int bad = 0;
    for (int i = 0; i < n; ++i) {
        const uint64_t a = next(), b = next(), c = next();
        const uint32_t blk = (uint32_t)a, e = (uint32_t)(a >> 32), r = (uint32_t)b, s = (uint32_t)(b >> 32);
        const uint32_t k0 = (uint32_t)c, k1 = (uint32_t)(c >> 32);
        const Words4 full = philox4x32_10(blk, e, r, s, k0, k1);
        const Words4 fast = philox_block(philox_row(e, r, k0), blk, s, k0, k1);
        bad += (full.x0 != fast.x0) + (full.x1 != fast.x1) + (full.x2 != fast.x2) + (full.x3 != fast.x3);
    }
    return bad;
}

// The device generator for one counter and key, for comparison with the oracle's.
extern "C" void emu_philox(const uint32_t *ctr, const uint32_t *key, uint32_t *out)
{
    const Words4 w = philox4x32_10(ctr[0], ctr[1], ctr[2], ctr[3], key[0], key[1]);
    out[0] = w.x0;
    out[1] = w.x1;
    out[2] = w.x2;
    out[3] = w.x3;
}
