// engine.hpp -- host engine internals shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/sim.h"
#include "host_core.hpp"
#include "mlp.hpp"
#include "sim_types.hpp"

namespace fw {
int launch_fw_paths(const InstanceDesc &host_desc, const InstanceDesc *dev_desc, const RunBuffers &B,
                    bool fp64, hipStream_t stream, int *kernel_width);
int launch_fw_batch(const BatchBuffers &B, hipStream_t stream);
int launch_fw_dense(const InstanceDesc &host_desc, const InstanceDesc *dev_desc, const RunBuffers &B,
                    hipStream_t stream);
constexpr int kDenseLanesPerRep = 4;                       // dense-L kernels: four lanes per replication
constexpr int kDenseRepsPerBlock = kBlock / kDenseLanesPerRep;
}  // namespace fw

using fw::InstanceDesc;
using fw::RunBuffers;

struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
};

// State of the last batched run.
struct BatchState {
    bool have = false;
    bool keep = false;
    uint32_t n_inst = 0;
    fw::host::BatchPlan plan;
    std::vector<sim_params> params;           // pointers cleared
    std::vector<uint64_t> R, T;
    DevBuf inst, tiles, slots, partials, final_stats, fck, y, tau, cnt, wsum, dlog;
    InstanceDesc *inst_host = nullptr;        // pinned staging
    size_t inst_host_cap = 0;
    fw::Tile *tiles_host = nullptr;           // pinned staging
    size_t tiles_host_cap = 0;
    uint32_t *slots_host = nullptr;           // pinned staging
    size_t slots_host_cap = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    // SIM_BATCH_GRAPH: the captured launches, kept while the kernel arguments are unchanged
    hipStream_t capture = nullptr;
    hipGraphExec_t exec = nullptr;
    fw::BatchBuffers exec_args{};
    uint64_t graph_launches = 0, graph_captures = 0;
};

// Control-variate surrogate, its training data and the estimator's buffers.
struct CvState {
    bool have_mlp = false, have_fit = false;
    int F = 0;
    DevBuf theta, w1a, w2a, w2t, mom1, mom2, part, grad, loss_hist;
    DevBuf xtrain, ytrain, ttrain;        // training pairs: [F][n] features, Y (FP64), target (FP32)
    DevBuf xio, yio, hout;                // staging of sim_mlp_forward / sim_mlp_grad, and h(x) of a run
    DevBuf xaux, haux, mpart, mout, mdone;
    uint64_t n_train = 0, n_steps = 0, R = 0, n_aux_last = 0;
    double y_mean = 0.0, y_sd = 1.0, beta = 0.0, rho2 = 0.0;
    double ref[SIM_MAX_D] = {0};          // the features' reference gradient of the fitted surrogate
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev_a = nullptr, ev_b = nullptr;
};

// Buffers and description of the last wide run (sim_run_wide).
struct WideState {
    bool have = false;
    sim_params params{};                  // pointers cleared
    uint64_t R = 0, T = 0;
    uint32_t nwg = 0;
    double fstar = 0.0;
    DevBuf asset_f, asset_d, S, cnt, tau, dec, s1, part_dot, part_qn, dot, qn, wg_g, wg_j, wg_gw, fval,
        stats, origin;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

// Buffers and description of the last newsvendor run (sim_run_newsvendor).
struct NvState {
    bool have = false;
    sim_nv_params params{};               // pointers cleared
    uint64_t R = 0, T = 0;
    uint32_t nwg = 0, P = 1;              // sample workgroups; lanes per quad
    DevBuf prod_f, prod_d, S, cnt, tau, dec, wg_r, wg_j, wg_gx, cost_part, fval, stats, origin;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

// Buffers and description of the last general-constraint newsvendor run (sim_run_newsvendor_lp).
struct NvLpState {
    bool have = false;
    sim_nv_params params{};               // pointers cleared
    uint32_t M = 0, nwg = 0, P = 1;       // resource rows; gradient workgroups; lanes per quad
    uint64_t R = 0, T = 0;
    DevBuf prod_d, Am, Cv, x, g, rec_basis, rec_value, rec_piv, tau, origin, cost_part, fval, stats, origin_total;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

// Data set and buffers of the last stochastic quasi-Newton run (sim_sqn_load, sim_run_sqn).
struct SqnState {
    bool have_data = false, have = false;
    uint64_t N = 0;
    uint32_t n = 0, ld = 0, xw = 0;       // features; vector stride; bitmap words per row
    sim_sqn_params params{};
    uint64_t R = 0, K = 0;
    uint32_t nblk = 0;
    DevBuf X, z, S, Y, wprev, acc, wsnap, wt, pairs, loss_part, fval, stats;
    DevBuf H, hscratch;                   // sim_sqn_hessian: the n x n matrix and its work space
    DevBuf sw, sg, sxpart, sdpart, shpart, sypart, ssmall;   // sim_run_sqn_split: iterate, gradient, partial sums, small matrices
    hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr, ev3 = nullptr, ev4 = nullptr;
};

struct sim_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    char err[512] = {0};
    InstanceDesc *desc_host = nullptr;    // pinned staging for the async upload
    InstanceDesc *desc_dev = nullptr;
    DevBuf y, fck, cnt, wsum, tau, dlog, part_f, part_i, done, final_f, final_i;
    DevBuf dense;                         // dense-L operands: Ag, Av (FP32), L (FP64)
    DevBuf feat;                          // control-variate features [(d+2)][R]
    DevBuf sched;                         // per-epoch sample-size table (sim_params.n_schedule)
    std::vector<unsigned char> sched_host; // its host copy, kept until the next run
    void *dense_host = nullptr;           // pinned staging of the same
    RunBuffers bufs{};
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    bool have_run = false;
    sim_params last{};
    double last_mu[SIM_MAX_D], last_sigma[SIM_MAX_D];
    bool last_diag = true;
    uint64_t R = 0, T = 0;
    int kernel_width = 0;
    uint64_t ws_limit = 0;                // sim_create_ex: cap on the bytes of the context's buffers (0: none)
    uint64_t ws_used = 0;                 // bytes the context's buffers hold now
    bool last_into = false;               // the last sim_run wrote its statistics to caller memory
    BatchState batch;
    CvState cv;
    WideState wide;
    NvState nv;
    NvLpState nvlp;
    SqnState sqn;
};


namespace fw {
namespace host {
// Caller device memory for a run's outputs (sim_run_into); NULL members use the context's buffers.
struct RunInto {
    double *fck = nullptr, *final_f = nullptr;
    uint64_t *final_i = nullptr;
};
int run_impl(sim_ctx *ctx, const sim_params *p, uint64_t R, uint64_t T, uint64_t seed, uint32_t internal,
             const RunInto *into = nullptr);
int set_err(sim_ctx *ctx, int code, const char *fmt, ...);
int ensure(sim_ctx *ctx, DevBuf &b, size_t bytes);
void free_buf(DevBuf &b);
}  // namespace host
}  // namespace fw

#define HIP_TRY(ctx, call)                                                                       \
    do {                                                                                         \
        hipError_t e_ = (call);                                                                  \
        if (e_ != hipSuccess)                                                                    \
            return fw::host::set_err((ctx), SIM_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)
