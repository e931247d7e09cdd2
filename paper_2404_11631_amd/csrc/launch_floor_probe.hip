// launch_floor_probe.hip -- the cost of one dependent kernel launch on gfx950: a chain of 3,000
// kernels that do almost nothing, on one stream, launched one by one and replayed from a captured
// HIP graph, timed with HIP events; with 4 workgroups (the wide path's smallest grid) and with 782
// (its grid at 1e5 assets). Supports the launch-chain roofline of the wide and newsvendor paths.
#include <hip/hip_runtime.h>
#include <cstdio>

#define CK(x)                                                                                      \
    do {                                                                                           \
        hipError_t e_ = (x);                                                                       \
        if (e_ != hipSuccess) {                                                                    \
            std::printf("%s failed: %s\n", #x, hipGetErrorString(e_));                             \
            return 1;                                                                              \
        }                                                                                          \
    } while (0)

constexpr int kWords = 1 << 20;   // every index below is reduced modulo this buffer size

__global__ void touch_one(float *p, int k)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) p[k & (kWords - 1)] += 1.0f;
}
__global__ void touch_all(float *p, int k)
{
    p[(blockIdx.x * blockDim.x + threadIdx.x) & (kWords - 1)] += static_cast<float>(k);
}

int main()
{
    float *p = nullptr;
    CK(hipMalloc(&p, sizeof(float) * kWords));
    CK(hipMemset(p, 0, sizeof(float) * kWords));
    hipStream_t s;
    CK(hipStreamCreate(&s));
    hipEvent_t a, b;
    CK(hipEventCreate(&a));
    CK(hipEventCreate(&b));
    const int n = 3000;
    for (int grid : {4, 782}) {
        auto chain = [&] {
            for (int k = 0; k < n; ++k) {
                if (grid == 4) hipLaunchKernelGGL(touch_one, dim3(grid), dim3(256), 0, s, p, k);
                else hipLaunchKernelGGL(touch_all, dim3(grid), dim3(256), 0, s, p, k);
            }
        };
        for (int rep = 0; rep < 3; ++rep) {
            CK(hipEventRecord(a, s));
            chain();
            CK(hipEventRecord(b, s));
            CK(hipEventSynchronize(b));
            float ms = 0.0f;
            CK(hipEventElapsedTime(&ms, a, b));
            hipGraph_t g;
            hipGraphExec_t ge;
            CK(hipStreamBeginCapture(s, hipStreamCaptureModeGlobal));
            chain();
            CK(hipStreamEndCapture(s, &g));
            CK(hipGraphInstantiate(&ge, g, nullptr, nullptr, 0));
            CK(hipGraphLaunch(ge, s));
            CK(hipStreamSynchronize(s));
            CK(hipEventRecord(a, s));
            CK(hipGraphLaunch(ge, s));
            CK(hipEventRecord(b, s));
            CK(hipEventSynchronize(b));
            float gms = 0.0f;
            CK(hipEventElapsedTime(&gms, a, b));
            std::printf("%d workgroups: launched %.2f us per kernel, graph %.2f us per kernel\n", grid, 1e3 * ms / n,
                        1e3 * gms / n);
            CK(hipGraphExecDestroy(ge));
            CK(hipGraphDestroy(g));
        }
    }
    CK(hipFree(p));
    return 0;
}
