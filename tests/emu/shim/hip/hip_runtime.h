// CPU emulation of the HIP device API subset the batched tile kernels use (test infrastructure:
// runs one workgroup as lockstep threads so the kernel logic can be checked against the oracle
// without a GPU).
#pragma once
#include <atomic>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <functional>
#include <memory>
#include <thread>
#include <vector>

#define __device__
#define __host__
#define __global__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __HIP_MEMORY_SCOPE_AGENT 0

struct Dim3emu { unsigned x, y, z; };
struct float4 { float x, y, z, w; };
inline float4 make_float4(float x, float y, float z, float w) { return float4{x, y, z, w}; }
struct uint4 { unsigned x, y, z, w; };
struct double2 { double x, y; };
struct ulonglong2 { unsigned long long x, y; };
template <class T> inline T atomicAdd(T *p, T v) { return std::atomic_ref<T>(*p).fetch_add(v); }
inline double2 make_double2(double x, double y) { return double2{x, y}; }
inline unsigned __umulhi(unsigned a, unsigned b) { return static_cast<unsigned>((static_cast<unsigned long long>(a) * b) >> 32); }
extern thread_local Dim3emu threadIdx;
extern thread_local Dim3emu blockIdx;
inline thread_local Dim3emu blockDim{1, 1, 1};   // set for each emulated thread of a block
typedef int hipError_t;
typedef void *hipStream_t;
#define hipSuccess 0
inline hipError_t hipGetLastError() { return 0; }
struct dim3 { unsigned x, y, z; dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {} };
#define hipLaunchKernelGGL(...) ((void)0)
template <class F> hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *b, F, int, int) { *b = 4; return 0; }

// lockstep exchange for shuffles: every thread of the block calls the shuffle at the same point
struct EmuBlock {
    int nthreads;
    std::barrier<> *bar;                  // the workgroup (__syncthreads)
    std::vector<uint64_t> slot;
    std::vector<std::barrier<> *> wave;   // one per wavefront of 64 threads (shuffles)
    std::vector<std::barrier<> *> half;   // one per half wavefront (width-32 shuffles)
};
extern EmuBlock *g_block;

// Every lane of the group a shuffle spans takes part in it: the wavefront, or the half wavefront for
// width-32 shuffles (kernels whose half wavefronts follow control flow of their own).
template <class T> inline T emu_exchange(T v, int src, int width = 64)
{
    uint64_t bits = 0;
    std::memcpy(&bits, &v, sizeof(T));
    std::barrier<> *b = width == 32 ? g_block->half[threadIdx.x / 32] : g_block->wave[threadIdx.x / 64];
    g_block->slot[threadIdx.x] = bits;
    b->arrive_and_wait();
    uint64_t got = g_block->slot[src];
    b->arrive_and_wait();
    T out;
    std::memcpy(&out, &got, sizeof(T));
    return out;
}
template <class T> inline T __shfl(T v, int src, int width = 64)
{
    int base = threadIdx.x / width * width;
    return emu_exchange(v, base + (src % width), width);
}
template <class T> inline T __shfl_xor(T v, unsigned m, int width = 64)
{
    int lane = threadIdx.x % width, base = threadIdx.x - lane;
    return emu_exchange(v, base + ((lane ^ m) % width), width);
}
template <class T> inline T __shfl_down(T v, unsigned off, int width = 64)
{
    int lane = threadIdx.x % width, base = threadIdx.x - lane;
    int src = lane + (int)off < width ? lane + (int)off : lane;
    return emu_exchange(v, base + src, width);
}
inline void __syncthreads() { g_block->bar->arrive_and_wait(); }
// threads are not lockstep here: the wave barrier synchronizes the wavefront's 64 threads
inline void __builtin_amdgcn_wave_barrier() { g_block->wave[threadIdx.x / 64]->arrive_and_wait(); }
// DPP: quad_perm (dpp_ctrl < 0x100), lane 4q + i reads lane 4q + ((ctrl >> 2i) & 3); row_mirror
// (0x140), lane i of a 16-lane row reads lane 15 - i; row_half_mirror (0x141), lane i of an 8-lane
// half row reads lane 7 - i
inline int __builtin_amdgcn_mov_dpp(int v, int ctrl, int, int, bool)
{
    const int lane = threadIdx.x % 64, base = threadIdx.x - lane;
    int src;
    if (ctrl == 0x140) src = (lane & ~15) | (15 - (lane & 15));
    else if (ctrl == 0x141) src = (lane & ~7) | (7 - (lane & 7));
    else src = (lane & ~3) | ((ctrl >> (2 * (lane & 3))) & 3);
    return emu_exchange(v, base + src, 32);   // within a half wavefront: a half may call it alone
}
// v_permlane16_swap with both operands x: the pair (x[lane & ~16], x[lane | 16])
struct EmuPair32 {
    uint32_t v[2];
    uint32_t operator[](int i) const { return v[i]; }
};
inline EmuPair32 __builtin_amdgcn_permlane16_swap(uint32_t x, uint32_t, bool, bool)
{
    const int lane = threadIdx.x % 64, base = threadIdx.x - lane;
    const uint32_t lo = (uint32_t)emu_exchange((int)x, base + (lane & ~16), 32);
    const uint32_t hi = (uint32_t)emu_exchange((int)x, base + (lane | 16), 32);
    return EmuPair32{{lo, hi}};
}
// v_permlane32_swap with both operands x: the pair (x[lane & ~32], x[lane | 32])
inline EmuPair32 __builtin_amdgcn_permlane32_swap(uint32_t x, uint32_t, bool, bool)
{
    const int lane = threadIdx.x % 64, base = threadIdx.x - lane;
    const uint32_t lo = (uint32_t)emu_exchange((int)x, base + (lane & ~32));
    const uint32_t hi = (uint32_t)emu_exchange((int)x, base + (lane | 32));
    return EmuPair32{{lo, hi}};
}
inline float __int_as_float(int x) { float f; std::memcpy(&f, &x, 4); return f; }
inline int __float_as_int(float f) { int x; std::memcpy(&x, &f, 4); return x; }
inline void __threadfence() { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline void __builtin_amdgcn_fence(int, const char *) { std::atomic_thread_fence(std::memory_order_seq_cst); }
template <class T> inline T __hip_atomic_fetch_add(T *p, T v, int, int)
{
    return std::atomic_ref<T>(*p).fetch_add(v);
}
template <class T> inline void __hip_atomic_store(T *p, T v, int, int) { std::atomic_ref<T>(*p).store(v); }
template <class T> inline T __hip_atomic_load(T *p, int, int) { return std::atomic_ref<T>(*p).load(); }
inline float __uint_as_float(uint32_t x) { float f; std::memcpy(&f, &x, 4); return f; }
inline long long __double_as_longlong(double d) { long long x; std::memcpy(&x, &d, 8); return x; }
inline double __longlong_as_double(long long x) { double d; std::memcpy(&d, &x, 8); return d; }
inline uint32_t __float_as_uint(float f) { uint32_t x; std::memcpy(&x, &f, 4); return x; }
inline float __builtin_amdgcn_sqrtf(float x) { return std::sqrt(x); }
inline float __builtin_amdgcn_logf(float x) { return std::log2(x); }
inline float __builtin_amdgcn_cosf(float x) { return (float)std::cos(6.283185307179586 * x); }
inline float __builtin_amdgcn_sinf(float x) { return (float)std::sin(6.283185307179586 * x); }
inline float __builtin_amdgcn_rsqf(float x) { return 1.0f / std::sqrt(x); }
// three-input bitwise function given by its 8-entry truth table, row index 4 a + 2 b + c
// register pinning is an optimiser hint on the device; nothing to do on the host
#define FW_PIN_VGPR(x) ((void)(x))

inline uint32_t __builtin_amdgcn_bitop3_b32(uint32_t a, uint32_t b, uint32_t c, uint32_t lut)
{
    uint32_t r = 0;
    for (int i = 0; i < 8; ++i)
        if ((lut >> i) & 1u) r |= ((i & 4) ? a : ~a) & ((i & 2) ? b : ~b) & ((i & 1) ? c : ~c);
    return r;
}
inline void sincospi(double x, double *s, double *c) { *s = std::sin(M_PI * x); *c = std::cos(M_PI * x); }
using std::fma; using std::fmin; using std::fmax; using std::sqrt; using std::log; using std::min;
// binary64 operations rounded on their own (the host compiles these without contraction)
inline double __dadd_rn(double a, double b) { volatile double r = a + b; return r; }
inline double __dsub_rn(double a, double b) { volatile double r = a - b; return r; }
inline double __dmul_rn(double a, double b) { volatile double r = a * b; return r; }
inline double __ddiv_rn(double a, double b) { volatile double r = a / b; return r; }
inline float fmaf(float a, float b, float c) { return std::fma(a, b, c); }

// runs kernel body f on a block of n threads in lockstep
inline void emu_run_block(int n, unsigned bx, const std::function<void()> &f, unsigned by = 0)
{
    std::barrier<> bar(n);
    std::vector<std::unique_ptr<std::barrier<>>> waves;
    EmuBlock blk{n, &bar, std::vector<uint64_t>(n), {}};
    for (int w = 0; w < (n + 63) / 64; ++w) {
        waves.emplace_back(new std::barrier<>(std::min(64, n - 64 * w)));
        blk.wave.push_back(waves.back().get());
    }
    for (int h = 0; h < (n + 31) / 32; ++h) {
        waves.emplace_back(new std::barrier<>(std::min(32, n - 32 * h)));
        blk.half.push_back(waves.back().get());
    }
    g_block = &blk;
    std::vector<std::thread> th;
    for (int i = 0; i < n; ++i)
        th.emplace_back([&, i] { threadIdx = {(unsigned)i, 0, 0}; blockIdx = {bx, by, 0}; blockDim = {(unsigned)n, 1, 1}; f(); });
    for (auto &t : th) t.join();
    g_block = nullptr;
}
