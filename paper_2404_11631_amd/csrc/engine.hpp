// engine.hpp -- host engine internals shared by the C-ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/sim.h"
#include "host_core.hpp"
#include "sim_types.hpp"

namespace fw {
int launch_fw_paths(const InstanceDesc &host_desc, const InstanceDesc *dev_desc, const RunBuffers &B,
                    bool fp64, hipStream_t stream, int *kernel_width);
int launch_fw_batch(const BatchBuffers &B, const uint32_t *class_begin, hipStream_t stream);
int launch_fw_dense(const InstanceDesc &host_desc, const InstanceDesc *dev_desc, const RunBuffers &B,
                    hipStream_t stream);
constexpr int kDenseRepsPerBlock = kBlock / 2;   // dense-L kernels: two lanes per replication
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
};

struct sim_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    char err[512] = {0};
    InstanceDesc *desc_host = nullptr;    // pinned staging for the async upload
    InstanceDesc *desc_dev = nullptr;
    DevBuf y, fck, cnt, wsum, tau, dlog, part_f, part_i, done, final_f, final_i;
    DevBuf dense;                         // dense-L operands: Ag, Av (FP32), L (FP64)
    void *dense_host = nullptr;           // pinned staging of the same
    RunBuffers bufs{};
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    bool have_run = false;
    sim_params last{};
    double last_mu[SIM_MAX_D], last_sigma[SIM_MAX_D];
    bool last_diag = true;
    uint64_t R = 0, T = 0;
    int kernel_width = 0;
    BatchState batch;
};


namespace fw {
namespace host {
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
