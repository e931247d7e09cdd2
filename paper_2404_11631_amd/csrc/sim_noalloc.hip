// sim_noalloc.hip -- sim_run's fused one-lane-per-replication path (Algorithm 1, Section 3.1, with
// its cross-path reduction) for callers that cannot allocate device memory.
//
// Every intermediate of the fused kernel (the instance descriptor, the per-workgroup partial sums
// and the finishing counter) lives in one file-scope device array per GPU, `scratch`, sized for
// R <= SIM_NOALLOC_MAX_R. Host code never passes the array's name to a kernel: its device address
// is taken once per device with hipGetSymbolAddress and kept. The descriptor reaches the device as
// kernel arguments of a small copy kernel (two halves by value), which also clears the finishing
// counter, so a call issues only kernel launches: no allocation, no memset, no host buffer that
// must outlive the call.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>

#include "engine.hpp"

namespace {

constexpr size_t kDescBytes = (sizeof(fw::InstanceDesc) + 255) / 256 * 256;
constexpr uint32_t kMaxBlocks = (SIM_NOALLOC_MAX_R + fw::kBlock - 1) / fw::kBlock;
constexpr size_t kPartFBytes = sizeof(double) * ((size_t)fw::kMaxStreams * fw::kStreamFields + 2) * kMaxBlocks;
constexpr size_t kPartIBytes = sizeof(uint64_t) * (size_t)(32 + 3) * kMaxBlocks;
// layout: descriptor | finishing counter (256 bytes) | partial sums (FP64) | partial counts (u64)
constexpr size_t kOffDone = kDescBytes;
constexpr size_t kOffPartF = kOffDone + 256;
constexpr size_t kOffPartI = kOffPartF + (kPartFBytes + 255) / 256 * 256;
constexpr size_t kScratchBytes = kOffPartI + (kPartIBytes + 255) / 256 * 256;
static_assert(kScratchBytes <= SIM_NOALLOC_SCRATCH_BYTES, "scratch layout exceeds the stated maximum");

static __device__ __align__(256) unsigned char scratch[SIM_NOALLOC_SCRATCH_BYTES];

// half of the descriptor's bytes, passed by value
constexpr size_t kHalf = (sizeof(fw::InstanceDesc) + 1) / 2;
struct DescHalf {
    unsigned char b[kHalf];
};

__global__ __launch_bounds__(256) void noalloc_stage(unsigned char *base, DescHalf h, uint32_t offset,
                                                     uint32_t n, int clear)
{
    for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) base[offset + i] = h.b[i];
    if (clear && threadIdx.x == 0) *reinterpret_cast<uint32_t *>(base + kOffDone) = 0u;
}

constexpr int kMaxDevices = 64;
std::mutex g_mu;
unsigned char *g_ptr[kMaxDevices] = {nullptr};

int scratch_of(int device, unsigned char **out, char *err, size_t len)
{
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            std::snprintf(err, len, "hipGetSymbolAddress(scratch) on device %d: %s", device, hipGetErrorString(e));
            return SIM_EDEVICE;
        }
        g_ptr[device] = static_cast<unsigned char *>(p);
    }
    *out = g_ptr[device];
    return SIM_OK;
}

thread_local char t_err[fw::host::kErrLen];

int noalloc_fail(int code, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(t_err, sizeof(t_err), fmt, ap);
    va_end(ap);
    return code;
}

}  // namespace

extern "C" {

int sim_run_noalloc(int device, void *hip_stream, const sim_params *p, uint64_t R, uint64_t T, uint64_t seed,
                    double *f_ckpt, double *stats_f, uint64_t *stats_i)
{
    t_err[0] = '\0';
    const int rc = fw::host::validate(t_err, p, R, T);
    if (rc) return rc;
    if (R > SIM_NOALLOC_MAX_R)
        return noalloc_fail(SIM_EINVAL, "R=%llu above the no-allocation limit %u", (unsigned long long)R,
                            (unsigned)SIM_NOALLOC_MAX_R);
    if (p->chol) return noalloc_fail(SIM_EUNSUPPORTED, "the no-allocation path takes a diagonal Sigma");
    if (p->state_precision != SIM_FP32) return noalloc_fail(SIM_EUNSUPPORTED, "the no-allocation path runs FP32 state");
    if (p->flags) return noalloc_fail(SIM_EUNSUPPORTED, "the no-allocation path keeps no per-path records, logs or features");
    if (p->n_schedule) return noalloc_fail(SIM_EUNSUPPORTED, "the no-allocation path takes one sample size");
    if (!stats_f || !stats_i) return noalloc_fail(SIM_EINVAL, "stats_f and stats_i are required");
    if (p->n_checkpoints && !f_ckpt) return noalloc_fail(SIM_EINVAL, "f_ckpt is required with checkpoints");
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n || device >= kMaxDevices)
        return noalloc_fail(SIM_EINVAL, "device %d not present", device);
    if (hipSetDevice(device) != hipSuccess) return noalloc_fail(SIM_EDEVICE, "hipSetDevice(%d) failed", device);
    unsigned char *base = nullptr;
    int src = scratch_of(device, &base, t_err, sizeof(t_err));
    if (src) return src;

    fw::InstanceDesc desc;
    std::memset(&desc, 0, sizeof(desc));
    fw::host::fill_desc(desc, p, R, T, seed);
    const hipStream_t stream = static_cast<hipStream_t>(hip_stream);
    const unsigned char *raw = reinterpret_cast<const unsigned char *>(&desc);
    for (int half = 0; half < 2; ++half) {
        DescHalf h;
        std::memset(&h, 0, sizeof(h));
        const size_t off = half * kHalf;
        const size_t len = half == 0 ? kHalf : sizeof(desc) - kHalf;
        std::memcpy(h.b, raw + off, len);
        hipLaunchKernelGGL(noalloc_stage, dim3(1), dim3(256), 0, stream, base, h, (uint32_t)off, (uint32_t)len,
                           half == 0 ? 1 : 0);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return noalloc_fail(SIM_EDEVICE, "descriptor staging: %s", hipGetErrorString(e));
    }

    const uint32_t nblocks = (uint32_t)((R + fw::kBlock - 1) / fw::kBlock);
    fw::RunBuffers B{};
    B.fck = f_ckpt;
    B.part_f = reinterpret_cast<double *>(base + kOffPartF);
    B.part_i = reinterpret_cast<uint64_t *>(base + kOffPartI);
    B.done = reinterpret_cast<uint32_t *>(base + kOffDone);
    B.final_f = stats_f;
    B.final_i = stats_i;
    B.nblocks = nblocks;
    B.n_streams = 1 + 2 * p->n_checkpoints;
    const int lrc = fw::launch_fw_paths(desc, reinterpret_cast<const fw::InstanceDesc *>(base), B, false, stream, nullptr);
    if (lrc == -5) return noalloc_fail(SIM_EUNSUPPORTED, "no kernel for d=%u", p->d);
    if (lrc) return noalloc_fail(SIM_EDEVICE, "kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
    return SIM_OK;
}

int sim_noalloc_last_error(char *buf, size_t len)
{
    if (!buf || !len) return SIM_EINVAL;
    std::snprintf(buf, len, "%s", t_err);
    return SIM_OK;
}

int sim_stats_from_raw(const sim_params *p, uint64_t R, uint64_t T, const double *stats_f, const uint64_t *stats_i,
                       sim_stats_out *out)
{
    if (!p || !stats_f || !stats_i || !out) return SIM_EINVAL;
    char err[fw::host::kErrLen];
    const int rc = fw::host::validate(err, p, R, T);
    if (rc) return rc;
    const uint32_t d = p->d, nc = p->n_checkpoints, ns = 1 + 2 * nc;
    const double fstar = p->chol ? NAN : fw::host::kkt_fstar(p->mu, p->sigma, d, p->risk_coef);
    fw::host::fill_stats(out, stats_f, nc, p->checkpoints, stats_f[ns * fw::kStreamFields],
                         stats_f[ns * fw::kStreamFields + 1], stats_i, d, stats_i[d + 1], stats_i[d + 2], R, T, fstar,
                         0.0, (double)R * (double)T);
    return SIM_OK;
}

}  // extern "C"
