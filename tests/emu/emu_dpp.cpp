// CPU emulation of the wavefront reductions in csrc/wave_dpp.hpp (test infrastructure only): each
// DPP / lane-swap reduction against the xor shuffle butterfly (lane ^ 1, ^ 2, ..., ^ 32) over the
// same 64 lane values, compared bit for bit. The shim models each DPP control and lane swap by its
// documented lane mapping.
#include <hip/hip_runtime.h>
thread_local Dim3emu threadIdx;
thread_local Dim3emu blockIdx;
EmuBlock *g_block = nullptr;

#include "../../paper_2404_11631_amd/csrc/wave_dpp.hpp"

#include <atomic>
#include <cstring>

using namespace fw;

namespace {

template <typename T>
T xor_sum(T x, int width)
{
    for (int m = 1; m < width; m <<= 1) x = x + __shfl_xor(x, m, 64);
    return x;
}

template <typename T>
void xor_argmin(T &g, uint32_t &j, int width)
{
    for (int m = 1; m < width; m <<= 1) {
        const T og = __shfl_xor(g, m, 64);
        const uint32_t oj = __shfl_xor(j, m, 64);
        if (og < g || (og == g && oj < j)) {
            g = og;
            j = oj;
        }
    }
}

template <typename T>
bool same_bits(T a, T b) { return std::memcmp(&a, &b, sizeof(T)) == 0; }

}  // namespace

// One case: 64 float values xf, 64 double values xd, 64 indices jx, 64 counts cx. Returns the
// number of lanes whose DPP result differs from the butterfly's in any of the checks.
extern "C" int emu_dpp_case(const float *xf, const double *xd, const uint32_t *jx, const uint32_t *cx)
{
    std::atomic<int> bad{0};
    emu_run_block(64, 0, [&] {
        const uint32_t l = threadIdx.x;
        int b = 0;
        b += !same_bits(dpp_sum32(xf[l]), xor_sum(xf[l], 32));
        b += !same_bits(dpp_sum64(xf[l]), xor_sum(xf[l], 64));
        b += !same_bits(dpp_sum64(xd[l]), xor_sum(xd[l], 64));
        {
            float g = xf[l], h = xf[l];
            uint32_t j = jx[l], k = jx[l];
            dpp_argmin32(g, j);
            xor_argmin(h, k, 32);
            b += !same_bits(g, h) || j != k;
        }
        {
            float g = xf[l], h = xf[l];
            uint32_t j = jx[l], k = jx[l];
            dpp_argmin64(g, j);
            xor_argmin(h, k, 64);
            b += !same_bits(g, h) || j != k;
        }
        {
            double g = xd[l], h = xd[l];
            uint32_t j = jx[l], k = jx[l];
            dpp_argmin64(g, j);
            xor_argmin(h, k, 64);
            b += !same_bits(g, h) || j != k;
        }
        for (uint32_t P = 1; P <= 16; P <<= 1) b += dpp_sum_lanes(cx[l], P) != xor_sum(cx[l], static_cast<int>(P));
        bad += b;
    });
    return bad.load();
}
