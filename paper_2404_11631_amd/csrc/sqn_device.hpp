// sqn_device.hpp -- device helpers of the stochastic quasi-Newton kernels (Algorithms 3-4,
// Section 3.3): the logistic function, the sampled rows of an iteration, the sum of a vector over
// a word of feature bits, and four-entry loads and stores of iterates and stored pairs.
#pragma once

#include <hip/hip_runtime.h>

#include "device_rng.hpp"
#include "sqn.hpp"

namespace fw {
namespace {

__device__ __forceinline__ double sigmoid(double a) { return 1.0 / (1.0 + exp(-a)); }

// The b (or b_H) rows of iteration k: floor(u N / 2^32) for the words u of counter (q/4, k, rep,
// domain | instance). The caller synchronises before the rows are read.
__device__ __forceinline__ void draw_rows(const SqnArgs &A, uint32_t rep, uint64_t k, uint32_t dom, uint32_t count,
                                          uint32_t *idx)
{
    const uint32_t nb = (count + 3) / 4;
    for (uint32_t q = threadIdx.x; q < nb; q += blockDim.x) {
        const Words4 x = philox4x32_10(q, static_cast<uint32_t>(k), rep, (dom << 24) | A.inst, A.k0, A.k1);
        const uint32_t u[4] = {x.x0, x.x1, x.x2, x.x3};
#pragma unroll
        for (int c = 0; c < 4; ++c)
            if (4 * q + c < count) idx[4 * q + c] = __umulhi(u[c], A.N);
    }
}

// v summed over the set bits of a 32-feature word starting at feature j0, lowest bit first.
__device__ __forceinline__ double word_dot(uint32_t bits, const double *v, uint32_t j0)
{
    double a = 0.0;
    while (bits) {
        a += v[j0 + __builtin_ctz(bits)];
        bits &= bits - 1;
    }
    return a;
}

__device__ __forceinline__ void load4(const double *p, double (&v)[4])
{
    const double2 a = reinterpret_cast<const double2 *>(p)[0];
    const double2 b = reinterpret_cast<const double2 *>(p)[1];
    v[0] = a.x;
    v[1] = a.y;
    v[2] = b.x;
    v[3] = b.y;
}

__device__ __forceinline__ void store4(double *p, const double (&v)[4])
{
    reinterpret_cast<double2 *>(p)[0] = make_double2(v[0], v[1]);
    reinterpret_cast<double2 *>(p)[1] = make_double2(v[2], v[3]);
}

// the same for pairs stored in binary32: one 16-byte access, rounded to nearest on the way out
__device__ __forceinline__ void load4(const float *p, double (&v)[4])
{
    const float4 a = *reinterpret_cast<const float4 *>(p);
    v[0] = a.x;
    v[1] = a.y;
    v[2] = a.z;
    v[3] = a.w;
}

__device__ __forceinline__ void store4(float *p, const double (&v)[4])
{
    *reinterpret_cast<float4 *>(p) = make_float4(static_cast<float>(v[0]), static_cast<float>(v[1]),
                                                 static_cast<float>(v[2]), static_cast<float>(v[3]));
}

}  // namespace
}  // namespace fw
