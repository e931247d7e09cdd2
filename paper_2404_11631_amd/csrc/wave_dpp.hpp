// wave_dpp.hpp -- sums and (value, index) minima over 32 or 64 lanes of a wavefront on gfx950's
// DPP lane moves and lane swaps, without the LDS crossbar a shuffle goes through.
//
// The exchanges: lane ^ 1 and lane ^ 2 (quad permutes), the other quad of each 8 lanes (half-row
// mirror), the other 8 of each 16 (row mirror), the other 16 of each 32 (v_permlane16_swap) and the
// other 32 (v_permlane32_swap). Each step combines a lane's value with its partner's, and the
// combination is symmetric (a sum, or the smaller value with the lower index among equal values),
// so every lane of a group ends with the same bits. Every lane of the wavefront must take part.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fw {

template <int CTRL>
__device__ __forceinline__ float dpp_move(float x)
{
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, true));
}

template <int CTRL>
__device__ __forceinline__ uint32_t dpp_move(uint32_t x)
{
    return static_cast<uint32_t>(__builtin_amdgcn_mov_dpp(static_cast<int>(x), CTRL, 0xF, 0xF, true));
}

// binary64 values move as their two 32-bit halves
template <int CTRL>
__device__ __forceinline__ double dpp_move(double x)
{
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(x));
    const uint32_t lo = dpp_move<CTRL>(static_cast<uint32_t>(b)), hi = dpp_move<CTRL>(static_cast<uint32_t>(b >> 32));
    return __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(hi) << 32) | lo));
}

// the values of lane & ~16 and lane | 16 (16-lane swap), or lane & ~32 and lane | 32 (32-lane swap)
template <bool WIDE>
__device__ __forceinline__ void lane_swap(double x, double &first, double &second)
{
    const uint64_t b = static_cast<uint64_t>(__double_as_longlong(x));
    const uint32_t lo = static_cast<uint32_t>(b), hi = static_cast<uint32_t>(b >> 32);
    uint32_t l0, l1, h0, h1;
    if constexpr (WIDE) {
        const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        l0 = l[0], l1 = l[1], h0 = h[0], h1 = h[1];
    } else {
        const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        l0 = l[0], l1 = l[1], h0 = h[0], h1 = h[1];
    }
    first = __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(h0) << 32) | l0));
    second = __longlong_as_double(static_cast<long long>((static_cast<uint64_t>(h1) << 32) | l1));
}

// lanes in groups of 16 hold their group's sum
__device__ __forceinline__ float dpp_sum16(float x)
{
    x += dpp_move<0xB1>(x);
    x += dpp_move<0x4E>(x);
    x += dpp_move<0x141>(x);
    x += dpp_move<0x140>(x);
    return x;
}

// the sum over each half wavefront (32 lanes)
__device__ __forceinline__ float dpp_sum32(float x)
{
    x = dpp_sum16(x);
    const auto h = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(h[0]) + __uint_as_float(h[1]);
}

// the sum over the wavefront (64 lanes)
__device__ __forceinline__ float dpp_sum64(float x)
{
    x = dpp_sum32(x);
    const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(h[0]) + __uint_as_float(h[1]);
}

// integer sums over aligned groups of P consecutive lanes (P a power of two, 1 to 16, the same in
// every lane): after the two quad steps a quad's lanes agree, so the half-row mirror adds the other
// quad of 8 lanes and the row mirror the other 8 of 16
__device__ __forceinline__ uint32_t dpp_sum_lanes(uint32_t x, uint32_t P)
{
    if (P >= 2u) x += dpp_move<0xB1>(x);
    if (P >= 4u) x += dpp_move<0x4E>(x);
    if (P >= 8u) x += dpp_move<0x141>(x);
    if (P >= 16u) x += dpp_move<0x140>(x);
    return x;
}

__device__ __forceinline__ void argmin_take(float &g, uint32_t &j, float og, uint32_t oj)
{
    if (og < g || (og == g && oj < j)) {
        g = og;
        j = oj;
    }
}

template <int CTRL>
__device__ __forceinline__ void argmin_dpp(float &g, uint32_t &j)
{
    argmin_take(g, j, dpp_move<CTRL>(g), dpp_move<CTRL>(j));
}

// (value, index) minimum over each half wavefront, lowest index among equal values
__device__ __forceinline__ void dpp_argmin32(float &g, uint32_t &j)
{
    argmin_dpp<0xB1>(g, j);
    argmin_dpp<0x4E>(g, j);
    argmin_dpp<0x141>(g, j);
    argmin_dpp<0x140>(g, j);
    const auto hg = __builtin_amdgcn_permlane16_swap(__float_as_uint(g), __float_as_uint(g), false, false);
    const auto hj = __builtin_amdgcn_permlane16_swap(j, j, false, false);
    const bool upper = (threadIdx.x & 16u) != 0u;   // the partner's value is the other row's
    argmin_take(g, j, __uint_as_float(upper ? hg[0] : hg[1]), upper ? hj[0] : hj[1]);
}

// the same over the wavefront (64 lanes)
__device__ __forceinline__ void dpp_argmin64(float &g, uint32_t &j)
{
    dpp_argmin32(g, j);
    const auto hg = __builtin_amdgcn_permlane32_swap(__float_as_uint(g), __float_as_uint(g), false, false);
    const auto hj = __builtin_amdgcn_permlane32_swap(j, j, false, false);
    const bool upper = (threadIdx.x & 32u) != 0u;
    argmin_take(g, j, __uint_as_float(upper ? hg[0] : hg[1]), upper ? hj[0] : hj[1]);
}

// binary64 sum over the wavefront, rounded to nearest at every step
__device__ __forceinline__ double dpp_sum64(double x)
{
    x = __dadd_rn(x, dpp_move<0xB1>(x));
    x = __dadd_rn(x, dpp_move<0x4E>(x));
    x = __dadd_rn(x, dpp_move<0x141>(x));
    x = __dadd_rn(x, dpp_move<0x140>(x));
    double a, b;
    lane_swap<false>(x, a, b);
    x = __dadd_rn(a, b);
    lane_swap<true>(x, a, b);
    return __dadd_rn(a, b);
}

__device__ __forceinline__ void argmin_take(double &g, uint32_t &j, double og, uint32_t oj)
{
    if (og < g || (og == g && oj < j)) {
        g = og;
        j = oj;
    }
}

// binary64 (value, index) minimum over the wavefront, lowest index among equal values
__device__ __forceinline__ void dpp_argmin64(double &g, uint32_t &j)
{
    argmin_take(g, j, dpp_move<0xB1>(g), dpp_move<0xB1>(j));
    argmin_take(g, j, dpp_move<0x4E>(g), dpp_move<0x4E>(j));
    argmin_take(g, j, dpp_move<0x141>(g), dpp_move<0x141>(j));
    argmin_take(g, j, dpp_move<0x140>(g), dpp_move<0x140>(j));
    double a, b;
    lane_swap<false>(g, a, b);
    auto hj = __builtin_amdgcn_permlane16_swap(j, j, false, false);
    bool upper = (threadIdx.x & 16u) != 0u;
    argmin_take(g, j, upper ? a : b, upper ? hj[0] : hj[1]);
    lane_swap<true>(g, a, b);
    hj = __builtin_amdgcn_permlane32_swap(j, j, false, false);
    upper = (threadIdx.x & 32u) != 0u;
    argmin_take(g, j, upper ? a : b, upper ? hj[0] : hj[1]);
}

}  // namespace fw
