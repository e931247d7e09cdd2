// CPU emulation of the split SQN kernels (test infrastructure only): the real device source and
// the real launch sequence (sqn_split_sequence), compiled for the host against tests/emu/shim, each
// workgroup run as lockstep threads, one after another (highest index first: no workgroup may rely
// on another of its launch), every buffer in host memory. The data set is packed into the bitmap
// the way sim_sqn_load packs it.
#include <hip/hip_runtime.h>
thread_local Dim3emu threadIdx;
thread_local Dim3emu blockIdx;
EmuBlock *g_block = nullptr;

#include "../../paper_2404_11631_amd/csrc/fw_sqn_split.hip"
#include "../../paper_2404_11631_amd/csrc/host_core.hpp"

#include <vector>

using namespace fw;

namespace {

struct SqnEmu {
    std::vector<uint32_t> X, pairs;
    std::vector<uint8_t> z;
    std::vector<double> S, Y, wprev, acc, wsnap, w, g, xpart, dpart, hpart, ypart, small;
    std::vector<float> Sf, Yf;
    uint32_t n = 0, ld = 0, nc = 0;
    uint64_t R = 0;
} e;

char g_err[512];

template <typename PT>
int run(SqnSplit &P, uint64_t K)
{
    const uint32_t W = P.W, R = P.A.R;
    auto grid = [&](uint32_t nx, const std::function<void()> &body) {
        for (uint32_t r = 0; r < R; ++r)
            for (uint32_t b = nx; b-- > 0;) emu_run_block(kSplitThreads, b, body, r);
    };
    return sqn_split_sequence(K, P.A.L, P.A.M, P.A.n_ckpt, P.A.ckpt, [&](SqnSplitKernel kind, const SqnSplitStep &st) {
        switch (kind) {
        case SqnSplitKernel::Start: grid(W, [&] { sqn_split_start(P, st); }); break;
        case SqnSplitKernel::Grad: grid(W, [&] { sqn_split_grad<PT>(P, st); }); break;
        case SqnSplitKernel::Dir: grid(W, [&] { sqn_split_dir<PT>(P, st); }); break;
        case SqnSplitKernel::Win1: grid(W, [&] { sqn_split_win1<PT>(P, st); }); break;
        case SqnSplitKernel::Win2: grid(W, [&] { sqn_split_win2<PT>(P, st); }); break;
        case SqnSplitKernel::Small: grid(1, [&] { sqn_split_small(P, st); }); break;
        }
        return 0;
    });
}

}  // namespace

extern "C" int emu_run_sqn_split(const uint8_t *X, const uint8_t *z, uint64_t N, uint32_t n, const sim_sqn_params *p,
                                 uint64_t R, uint64_t K, uint64_t seed)
{
    if (int rc = fw::host::validate_sqn(g_err, p, N, n, R, K)) return rc;
    if (R > kSplitMaxR) return SIM_EINVAL;
    e = SqnEmu{};
    const uint32_t xw = ((n + 31) / 32 + 3) / 4 * 4, ld = (n + 3) / 4 * 4, nc = p->n_checkpoints;
    e.n = n;
    e.ld = ld;
    e.nc = nc;
    e.R = R;
    e.X.assign(static_cast<size_t>(N) * xw, 0u);
    for (uint64_t i = 0; i < N; ++i)
        for (uint32_t j = 0; j < n; ++j) e.X[i * xw + (j >> 5)] |= static_cast<uint32_t>(X[i * n + j]) << (j & 31);
    e.z.assign(z, z + N);
    const size_t RL = static_cast<size_t>(R) * ld;
    if (p->pairs_fp32) {
        e.Sf.assign(RL * p->M, NAN);
        e.Yf.assign(RL * p->M, NAN);
    } else {
        e.S.assign(RL * p->M, NAN);
        e.Y.assign(RL * p->M, NAN);
    }
    e.wprev.assign(RL, NAN);
    e.acc.assign(RL, NAN);
    e.wsnap.assign((nc + 1) * RL, NAN);
    e.pairs.assign(R, 0xEEEEEEEEu);

    SqnSplit P{};
    SqnArgs &A = P.A;
    A.n = n;
    A.ld = ld;
    A.nq = ld / 4;
    A.N = static_cast<uint32_t>(N);
    A.L = p->L;
    A.M = p->M;
    A.b = p->b;
    A.bH = p->b_H;
    A.k0 = static_cast<uint32_t>(seed);
    A.k1 = static_cast<uint32_t>(seed >> 32);
    A.inst = p->instance_id & 0xFFFFFFu;
    A.R = static_cast<uint32_t>(R);
    A.n_ckpt = nc;
    A.xw = xw;
    A.K = K;
    A.beta = p->beta;
    for (uint32_t c = 0; c < nc; ++c) A.ckpt[c] = p->checkpoints[c];
    A.X = e.X.data();
    A.z = e.z.data();
    A.S = p->pairs_fp32 ? static_cast<void *>(e.Sf.data()) : static_cast<void *>(e.S.data());
    A.Y = p->pairs_fp32 ? static_cast<void *>(e.Yf.data()) : static_cast<void *>(e.Y.data());
    A.pairs_fp32 = p->pairs_fp32 ? 1u : 0u;
    A.wprev = e.wprev.data();
    A.acc = e.acc.data();
    A.wsnap = e.wsnap.data();
    A.pairs = e.pairs.data();
    P.W = sqn_split_slices(A.nq);
    const size_t W = P.W;
    e.w.assign(RL, NAN);
    e.g.assign(RL, NAN);
    e.xpart.assign(2 * R * A.b * W, NAN);
    e.dpart.assign(R * 2 * A.M * W, NAN);
    e.hpart.assign(R * 2 * A.bH * W, NAN);
    e.ypart.assign(R * 3 * A.M * W, NAN);
    e.small.assign(R * kSqnSmall, NAN);
    P.w = e.w.data();
    P.g = e.g.data();
    P.xpart = e.xpart.data();
    P.dpart = e.dpart.data();
    P.hpart = e.hpart.data();
    P.ypart = e.ypart.data();
    P.small = e.small.data();
    return p->pairs_fp32 ? run<float>(P, K) : run<double>(P, K);
}

// The last emulated run's iterates: w [n_checkpoints + 1][R][n] (the checkpoints, then w^{K+1}) and
// the pair counts [R].
extern "C" void emu_sqn_split_out(double *w, uint32_t *pairs)
{
    for (size_t c = 0; c <= e.nc; ++c)
        for (size_t r = 0; r < e.R; ++r)
            std::copy(e.wsnap.begin() + (c * e.R + r) * e.ld, e.wsnap.begin() + (c * e.R + r) * e.ld + e.n,
                      w + (c * e.R + r) * e.n);
    std::copy(e.pairs.begin(), e.pairs.end(), pairs);
}

extern "C" const char *emu_sqn_split_error() { return g_err; }
