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

}  // namespace fw
