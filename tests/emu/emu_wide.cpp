// CPU emulation of the wide path's kernels (test infrastructure only): the real device source and
// the real launch sequence (wide_sequence), compiled for the host against tests/emu/shim, each
// workgroup run as lockstep threads, one after another (highest index first: no workgroup may rely
// on another of its launch), every buffer in host memory. The per-asset
// coefficients are prepared as sim_run_wide prepares them.
#include <hip/hip_runtime.h>
thread_local Dim3emu threadIdx;
thread_local Dim3emu blockIdx;
EmuBlock *g_block = nullptr;

#include "../../paper_2404_11631_amd/csrc/fw_wide.hip"
#include "../../paper_2404_11631_amd/csrc/host_core.hpp"

#include <vector>

using namespace fw;

namespace {

struct WideEmu {
    std::vector<float> af, s1, part_dot, part_qn, dot, qn, wg_g, wg_gw;
    std::vector<double> ad, fval;
    std::vector<uint64_t> S;
    std::vector<uint32_t> cnt, tau, dec, wg_j;
    uint32_t d = 0, nc = 0;
    uint64_t R = 0, T = 0;
} g;

char g_err[512];

}  // namespace

extern "C" int emu_run_wide(const sim_params *p, uint64_t R, uint64_t T, uint64_t seed)
{
    if (int rc = fw::host::validate_wide(g_err, p, R, T)) return rc;
    const uint32_t d = p->d, N = p->n_samples, nc = p->n_checkpoints;
    uint32_t Nmax = N;
    if (p->n_schedule)
        for (uint64_t e = 0; e * p->resample_every < T; ++e) Nmax = std::max(Nmax, p->n_schedule[e]);
    const uint32_t nq = d / 4, nwg = (nq + kWideQuads - 1) / kWideQuads;
    const size_t D = d;
    g = WideEmu{};
    g.d = d;
    g.nc = nc;
    g.R = R;
    g.T = T;
    g.af.resize(5 * D);
    g.ad.resize(2 * D);
    for (size_t j = 0; j < D; ++j) {
        const double sz = kBoxMullerScale * p->sigma[j];
        g.af[j] = static_cast<float>(p->mu[j]);
        g.af[D + j] = static_cast<float>(sz);
        g.af[2 * D + j] = static_cast<float>(sz / N);
        g.af[3 * D + j] = static_cast<float>(2.0 * p->risk_coef * sz / (N - 1.0));
        g.af[4 * D + j] = p->w0 ? static_cast<float>(p->w0[j]) : 0.0f;
        g.ad[j] = p->mu[j];
        g.ad[D + j] = p->sigma[j];
    }
    g.S.assign(R * D, 0);
    g.cnt.assign(R * (D + 1), 0);
    g.tau.assign(R, kTauNone);
    g.dec.assign(R * T, 0xEEEEEEEEu);
    g.s1.assign(R * D, NAN);
    g.part_dot.assign(R * Nmax * nwg, NAN);
    g.part_qn.assign(R * nwg, NAN);
    g.dot.assign(R * Nmax, NAN);
    g.qn.assign(R, NAN);
    g.wg_g.assign(2 * R * nwg, NAN);
    g.wg_gw.assign(2 * R * nwg, NAN);
    g.wg_j.assign(2 * R * nwg, 0xEEEEEEEEu);
    g.fval.assign(R * (nc + 1), NAN);

    WideArgs A{};
    A.d = d;
    A.nq = nq;
    A.N = Nmax;
    A.nwg = nwg;
    A.R = static_cast<uint32_t>(R);
    A.k0 = static_cast<uint32_t>(seed);
    A.k1 = static_cast<uint32_t>(seed >> 32);
    A.dom = p->instance_id & 0xFFFFFFu;
    A.gap_eps = static_cast<float>(p->gap_eps);
    A.lambda = p->risk_coef;
    A.mu_f = g.af.data();
    A.sz_f = g.af.data() + D;
    A.c1_f = g.af.data() + 2 * D;
    A.c2_f = g.af.data() + 3 * D;
    A.w0_f = g.af.data() + 4 * D;
    A.mu_d = g.ad.data();
    A.sig_d = g.ad.data() + D;
    A.S = g.S.data();
    A.cnt = g.cnt.data();
    A.tau = g.tau.data();
    A.dec = g.dec.data();
    A.T = T;
    A.s1 = g.s1.data();
    A.part_dot = g.part_dot.data();
    A.part_qn = g.part_qn.data();
    A.dot = g.dot.data();
    A.qn = g.qn.data();
    A.wg_g = g.wg_g.data();
    A.wg_j = g.wg_j.data();
    A.wg_gw = g.wg_gw.data();
    A.fval = g.fval.data();

    auto grid = [&](uint32_t nx, const std::function<void()> &body) {
        for (uint32_t r = 0; r < R; ++r)
            for (uint32_t b = nx; b-- > 0;) emu_run_block(kWideBlock, b, body, r);
    };
    const int rc = wide_sequence(
        N, p->n_schedule, p->resample_every, T, p->w0 != nullptr, nc, p->checkpoints,
        [&](uint64_t t, uint32_t e, const WideEpoch &E, float cw, bool from_w0, bool fold_prev) {
            const int64_t prev = fold_prev ? static_cast<int64_t>(t) - 1 : -1;
            grid(nwg, [&] { wide_sample_kernel(A, e, E.n, cw, from_w0 ? 1 : 0, prev, E.par); });
            grid(E.n + 1, [&] { wide_dot_kernel(A, E.n); });
            grid(nwg, [&] { wide_gradient_kernel(A, e, E, cw, from_w0 ? 1 : 0); });
            return 0;
        },
        [&](uint64_t t) {
            for (uint32_t r = 0; r < R; ++r)
                emu_run_block(kWideBlock, r, [&] { wide_step_kernel(A, t, static_cast<uint32_t>(t & 1)); });
            return 0;
        },
        [&](double c, uint32_t slot) {
            for (uint32_t r = 0; r < R; ++r) emu_run_block(kWideBlock, r, [&] { wide_objective_kernel(A, c, slot); });
            return 0;
        });
    if (rc) return rc;
    const double cT = 2.0 / (static_cast<double>(T) * static_cast<double>(T + 1));
    for (uint32_t r = 0; r < R; ++r) emu_run_block(kWideBlock, r, [&] { wide_objective_kernel(A, cT, nc); });
    return 0;
}

// Per-path records of the last emulated run, in sim_wide_paths' layouts.
extern "C" void emu_wide_paths(double *y, double *f_ckpt, uint32_t *cnt, uint64_t *wsum, uint32_t *tau, uint32_t *dec)
{
    std::copy(g.fval.begin() + g.nc * g.R, g.fval.end(), y);
    std::copy(g.fval.begin(), g.fval.begin() + g.nc * g.R, f_ckpt);
    std::copy(g.cnt.begin(), g.cnt.end(), cnt);
    std::copy(g.S.begin(), g.S.end(), wsum);
    std::copy(g.tau.begin(), g.tau.end(), tau);
    std::copy(g.dec.begin(), g.dec.end(), dec);
}

extern "C" const char *emu_wide_error() { return g_err; }
