// device_rng.hpp -- counter-based noise for the path kernels (gfx950).
//
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two 32x32->64 products of
// counter words 0 and 2 with the round multipliers, xored into the other words with the key; the
// key advances by the two Weyl increments between rounds.
//
// Uniforms: u = (2 (x mod 2^23) + 1) 2^-24, built by inserting the low 23 bits of x into the
// mantissa of 1.0 and subtracting 1 - 2^-24 (exact by Sterbenz), so binary32 and binary64 see the
// same value.
//
// Box-Muller: (u1, u2) -> sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2). The binary32 path evaluates
// the hardware log2, sqrt, sin and cos (angles in revolutions) and returns the pair divided by
// sqrt(2 ln 2); callers fold that constant into the per-asset scale. The binary64 path uses the
// device math library with sincospi.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "sim_types.hpp"

// Makes a value opaque to the optimiser without emitting an instruction, so that it stays in a
// vector register instead of being recomputed where it is used.
#ifndef FW_PIN_VGPR
#define FW_PIN_VGPR(x) asm volatile("" : "+v"(x))
#endif

namespace fw {

struct Words4 {
    uint32_t x0, x1, x2, x3;
};

__device__ __forceinline__ Words4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                                uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        // three-input xors in one v_bitop3_b32 each (truth table 0x96: odd parity)
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p0 >> 32), c3, k1, 0x96);
        c1 = static_cast<uint32_t>(p1);
        c3 = static_cast<uint32_t>(p0);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words4{c0, c1, c2, c3};
}

// The same generator over counters (b, e, r, s) of which only the block word b changes along a
// stream: round 1's product of word 2 (= r) and round 2's product of word 0 depend on (e, r) and
// the key alone, so a stream computes them once and each block starts from them.
struct PhiloxRow {
    uint32_t w1;     // word 1 after round 1: low half of M1 r
    uint32_t p_hi;   // round 2 product of word 0 (hi(M1 r) ^ e ^ k0) with M0: high half
    uint32_t p_lo;   //                                                      low half
};

__device__ __forceinline__ PhiloxRow philox_row(uint32_t e, uint32_t r, uint32_t k0)
{
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * r;
    const uint32_t x = static_cast<uint32_t>(p1 >> 32) ^ e ^ k0;
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * x;
    PhiloxRow row{static_cast<uint32_t>(p1), static_cast<uint32_t>(p0 >> 32), static_cast<uint32_t>(p0)};
    // keep the row live in registers: left to itself the compiler recomputes the two products
    // in every block
    FW_PIN_VGPR(row.w1);
    FW_PIN_VGPR(row.p_hi);
    FW_PIN_VGPR(row.p_lo);
    return row;
}

// Philox4x32-10 of counter (b, e, r, s) from the row of (e, r); equal to philox4x32_10(b, e, r, s).
__device__ __forceinline__ Words4 philox_block(const PhiloxRow &row, uint32_t b, uint32_t s, uint32_t k0,
                                               uint32_t k1)
{
    // round 1, block word only
    const uint64_t q = static_cast<uint64_t>(0xD2511F53u) * b;
    const uint32_t a2 = static_cast<uint32_t>(q >> 32) ^ s ^ k1;
    const uint32_t a3 = static_cast<uint32_t>(q);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
    // round 2: word 0's product comes from the row
    const uint64_t q2 = static_cast<uint64_t>(0xCD9E8D57u) * a2;
    uint32_t c0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(q2 >> 32), row.w1, k0, 0x96);
    uint32_t c2 = __builtin_amdgcn_bitop3_b32(row.p_hi, a3, k1, 0x96);
    uint32_t c1 = static_cast<uint32_t>(q2);
    uint32_t c3 = row.p_lo;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
#pragma unroll
    for (int round = 2; round < 10; ++round) {
        const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
        const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
        const uint32_t n0 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p1 >> 32), c1, k0, 0x96);
        const uint32_t n2 = __builtin_amdgcn_bitop3_b32(static_cast<uint32_t>(p0 >> 32), c3, k1, 0x96);
        c1 = static_cast<uint32_t>(p1);
        c3 = static_cast<uint32_t>(p0);
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Words4{c0, c1, c2, c3};
}

// (2 (x mod 2^23) + 1) 2^-24 in binary32, exactly
__device__ __forceinline__ float uniform_open01(uint32_t x)
{
    return __uint_as_float((x & 0x007FFFFFu) | 0x3F800000u) - 0x1.fffffep-1f;
}

struct Pair32 {
    float c, s;
};

// (z0, z1) / sqrt(2 ln 2) with z0 = sqrt(-2 ln u1) cos(2 pi u2), z1 = ... sin(2 pi u2)
__device__ __forceinline__ Pair32 box_muller_scaled(uint32_t xa, uint32_t xb)
{
    const float u1 = uniform_open01(xa);
    const float u2 = uniform_open01(xb);
    const float rad = __builtin_amdgcn_sqrtf(-__builtin_amdgcn_logf(u1));   // sqrt(-log2 u1)
    return Pair32{rad * __builtin_amdgcn_cosf(u2), rad * __builtin_amdgcn_sinf(u2)};
}

struct Pair64 {
    double c, s;
};

__device__ __forceinline__ Pair64 box_muller64(uint32_t xa, uint32_t xb)
{
    const double u1 = static_cast<double>(uniform_open01(xa));
    const double u2 = static_cast<double>(uniform_open01(xb));
    const double rad = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    return Pair64{rad * c, rad * s};
}

// Four normals (z_{4b}, ..., z_{4b+3}) of one Philox block, in the precision of the path.
template <typename Real>
struct Block4 {
    Real z[4];
};

template <typename Real>
__device__ __forceinline__ Block4<Real> normals_block(uint32_t block, uint32_t epoch, uint32_t rep,
                                                      uint32_t domain_instance, uint32_t k0,
                                                      uint32_t k1);

template <>
__device__ __forceinline__ Block4<float> normals_block<float>(uint32_t block, uint32_t epoch,
                                                              uint32_t rep, uint32_t dom,
                                                              uint32_t k0, uint32_t k1)
{
    const Words4 x = philox4x32_10(block, epoch, rep, dom, k0, k1);
    const Pair32 a = box_muller_scaled(x.x0, x.x1);
    const Pair32 b = box_muller_scaled(x.x2, x.x3);
    return Block4<float>{{a.c, a.s, b.c, b.s}};
}

// Block b of the stream of row (e, r), binary32.
__device__ __forceinline__ Block4<float> normals_block_row(const PhiloxRow &row, uint32_t block, uint32_t dom,
                                                           uint32_t k0, uint32_t k1)
{
    const Words4 x = philox_block(row, block, dom, k0, k1);
    const Pair32 a = box_muller_scaled(x.x0, x.x1);
    const Pair32 b = box_muller_scaled(x.x2, x.x3);
    return Block4<float>{{a.c, a.s, b.c, b.s}};
}

template <>
__device__ __forceinline__ Block4<double> normals_block<double>(uint32_t block, uint32_t epoch,
                                                                uint32_t rep, uint32_t dom,
                                                                uint32_t k0, uint32_t k1)
{
    const Words4 x = philox4x32_10(block, epoch, rep, dom, k0, k1);
    const Pair64 a = box_muller64(x.x0, x.x1);
    const Pair64 b = box_muller64(x.x2, x.x3);
    return Block4<double>{{a.c, a.s, b.c, b.s}};
}

// Sequential reader of normals q0, q0+1, ... of one stream. The position inside the current
// block is the same in every lane of a wavefront (all lanes walk the same index sequence), so the
// refill branch is uniform.
template <typename Real>
struct NormalCursor {
    Real buf[4];
    uint32_t next_block;
    uint32_t pos;

    __device__ __forceinline__ void seek(uint32_t q0, uint32_t epoch, uint32_t rep, uint32_t dom,
                                         uint32_t k0, uint32_t k1)
    {
        next_block = q0 >> 2;
        pos = q0 & 3u;
        refill(epoch, rep, dom, k0, k1);
    }
    __device__ __forceinline__ void refill(uint32_t epoch, uint32_t rep, uint32_t dom, uint32_t k0,
                                           uint32_t k1)
    {
        const Block4<Real> b = normals_block<Real>(next_block, epoch, rep, dom, k0, k1);
        buf[0] = b.z[0];
        buf[1] = b.z[1];
        buf[2] = b.z[2];
        buf[3] = b.z[3];
        ++next_block;
    }
    __device__ __forceinline__ Real next(uint32_t epoch, uint32_t rep, uint32_t dom, uint32_t k0,
                                         uint32_t k1)
    {
        if (pos == 4u) {
            refill(epoch, rep, dom, k0, k1);
            pos = 0u;
        }
        const uint32_t p = pos++;
        return p == 0u ? buf[0] : (p == 1u ? buf[1] : (p == 2u ? buf[2] : buf[3]));
    }
};

}  // namespace fw
