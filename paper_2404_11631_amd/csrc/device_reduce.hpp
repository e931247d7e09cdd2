// device_reduce.hpp -- deterministic reductions shared by the path kernels: double-double
// (TwoSum) accumulation and fixed-order wavefront / workgroup trees.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sim_types.hpp"

namespace fw {

__device__ __forceinline__ void dd_add(double &h, double &l, double bh, double bl)
{
    const double s = h + bh;
    const double bb = s - h;
    double e = (h - (s - bb)) + (bh - bb);
    e += l + bl;
    const double hs = s + e;
    l = e - (hs - s);
    h = hs;
}

// Workgroup sum of a double-double; the result is valid in thread 0. Fixed tree: shuffle-down
// within each wavefront, then the four wavefront partials in order.
__device__ __forceinline__ void block_sum_dd(double &h, double &l, double *sm)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double oh = __shfl_down(h, off, 64);
        const double ol = __shfl_down(l, off, 64);
        dd_add(h, l, oh, ol);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) {
        sm[2 * wave] = h;
        sm[2 * wave + 1] = l;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        h = sm[0];
        l = sm[1];
        for (int k = 1; k < kBlock / 64; ++k) dd_add(h, l, sm[2 * k], sm[2 * k + 1]);
    }
    __syncthreads();
}

__device__ __forceinline__ uint64_t block_sum_u64(uint64_t x, uint64_t *sm)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_down(x, off, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sm[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 1; k < kBlock / 64; ++k) x += sm[k];
    __syncthreads();
    return x;
}

template <bool IS_MAX>
__device__ __forceinline__ double block_extreme(double x, double *sm)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_down(x, off, 64);
        x = IS_MAX ? fmax(x, o) : fmin(x, o);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    if (lane == 0) sm[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0)
        for (int k = 1; k < kBlock / 64; ++k) x = IS_MAX ? fmax(x, sm[k]) : fmin(x, sm[k]);
    __syncthreads();
    return x;
}

__device__ __forceinline__ void store_agent(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_agent(uint64_t *p, uint64_t v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double load_agent(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t load_agent(const uint64_t *p)
{
    return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wavefront (64-lane) sums and extremes, valid in lane 0: fixed shuffle-down tree.
__device__ __forceinline__ void wave_sum_dd(double &h, double &l)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double oh = __shfl_down(h, off, 64);
        const double ol = __shfl_down(l, off, 64);
        dd_add(h, l, oh, ol);
    }
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_down(x, off, 64);
    return x;
}

template <bool IS_MAX>
__device__ __forceinline__ double wave_extreme(double x)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        const double o = __shfl_down(x, off, 64);
        x = IS_MAX ? fmax(x, o) : fmin(x, o);
    }
    return x;
}

}  // namespace fw
