// CPU emulation of Algorithm 2's general-constraint kernels (test infrastructure only): the real
// device source and the real launch sequence (nv_lp_sequence), compiled for the host against
// tests/emu/shim, each workgroup run as lockstep threads, one after another (highest index first:
// no workgroup may rely on another of its launch), every buffer in host memory. The per-product
// coefficients are prepared as sim_run_newsvendor_lp prepares them.
#include <hip/hip_runtime.h>
thread_local Dim3emu threadIdx;
thread_local Dim3emu blockIdx;
EmuBlock *g_block = nullptr;

#include "../../paper_2404_11631_amd/csrc/fw_newsvendor.hip"
#include "../../paper_2404_11631_amd/csrc/host_core.hpp"

#include <algorithm>
#include <vector>

using namespace fw;

namespace {

struct NvLpEmu {
    std::vector<double> pd, Am, Cv, x, g, rec_value, cost_part, fval, stats;
    std::vector<uint32_t> rec_basis, rec_piv, tau, origin;
    uint64_t origin_total = 0;
    uint32_t n = 0, M = 0, nc = 0;
    uint64_t R = 0, T = 0;
} e;

char g_err[512];

}  // namespace

extern "C" int emu_run_nv_lp(const sim_nv_params *p, const sim_nv_constraints *con, uint64_t R, uint64_t T,
                             uint64_t seed)
{
    if (int rc = fw::host::validate_newsvendor_lp(g_err, p, con, R, T)) return rc;
    const uint32_t n = p->n, M = con->n_resources, nc = p->n_checkpoints;
    const size_t N = n;
    e = NvLpEmu{};
    e.n = n;
    e.M = M;
    e.nc = nc;
    e.R = R;
    e.T = T;
    e.pd.resize(9 * N);
    double gscale = 0.0;
    for (size_t j = 0; j < N; ++j) {
        e.pd[j] = p->mu[j];
        e.pd[N + j] = p->sigma[j] > 0.0 ? 1.0 / (kBoxMullerScale * p->sigma[j]) : INFINITY;
        e.pd[2 * N + j] = p->k[j] - p->v[j];
        e.pd[3 * N + j] = p->h[j] + p->v[j];
        e.pd[4 * N + j] = p->sigma[j];
        e.pd[5 * N + j] = p->k[j];
        e.pd[6 * N + j] = p->h[j];
        e.pd[7 * N + j] = p->v[j];
        e.pd[8 * N + j] = p->x0 ? p->x0[j] : 0.0;
        gscale = std::max(gscale, std::fabs(p->k[j] - p->v[j]) + std::fabs(p->h[j] + p->v[j]));
    }
    e.Am.assign(con->A, con->A + static_cast<size_t>(M) * N);
    e.Cv.assign(con->C, con->C + M);
    e.x.resize(R * N);
    for (uint64_t r = 0; r < R; ++r) std::copy(e.pd.begin() + 8 * N, e.pd.begin() + 9 * N, e.x.begin() + r * N);
    e.g.assign(R * N, NAN);
    e.rec_basis.assign(R * T * M, 0xEEEEEEEEu);
    e.rec_value.assign(R * T * M, NAN);
    e.rec_piv.assign(R * T, 0xEEEEEEEEu);
    e.tau.assign(R, kTauNone);
    e.origin.assign(R, 0);
    const size_t ncost = (N + kNvCostChunk - 1) / kNvCostChunk;
    e.cost_part.assign(2 * R * ncost, NAN);
    e.fval.assign(R * (nc + 1), NAN);
    e.stats.assign(kMaxStreams * kStreamFields + 2, NAN);

    NvLpArgs A{};
    A.n = n;
    A.nq = n / 4;
    A.S = p->n_samples;
    A.P = nv_lanes_per_quad(n / 4, R, p->n_samples);
    A.nwg = (n / 4 + kNvBlock / A.P - 1) / (kNvBlock / A.P);
    A.R = static_cast<uint32_t>(R);
    A.M = M;
    A.k0 = static_cast<uint32_t>(seed);
    A.k1 = static_cast<uint32_t>(seed >> 32);
    A.dom = (kNvDomain << 24) | (p->instance_id & 0xFFFFFFu);
    A.max_pivots = SIM_NV_LP_MAX_PIVOTS;
    A.gap_eps = p->gap_eps;
    A.eps_r = 1e-12 * (1.0 + gscale);
    A.eps_d = 1e-12;
    const double *d = e.pd.data();
    A.mu_d = d;
    A.isk_d = d + N;
    A.km_d = d + 2 * N;
    A.hv_d = d + 3 * N;
    A.sig_d = d + 4 * N;
    A.k_d = d + 5 * N;
    A.h_d = d + 6 * N;
    A.v_d = d + 7 * N;
    A.x0_d = d + 8 * N;
    A.Am = e.Am.data();
    A.Cv = e.Cv.data();
    A.x = e.x.data();
    A.g = e.g.data();
    A.rec_basis = e.rec_basis.data();
    A.rec_value = e.rec_value.data();
    A.rec_piv = e.rec_piv.data();
    A.tau = e.tau.data();
    A.origin = e.origin.data();
    A.T = T;
    A.cost_part = e.cost_part.data();
    A.fval = e.fval.data();
    A.stats = e.stats.data();
    A.origin_total = &e.origin_total;

    auto grid = [&](uint32_t nx, uint32_t ny, int threads, const std::function<void()> &body) {
        for (uint32_t y = 0; y < ny; ++y)
            for (uint32_t b = nx; b-- > 0;) emu_run_block(threads, b, body, y);
    };
    const uint32_t ncost32 = static_cast<uint32_t>(ncost);
    auto cost = [&](uint32_t slot) {
        grid(ncost32, A.R, kBlock, [&] { nv_lp_cost_kernel(A); });
        grid(A.R, 1, kBlock, [&] { nv_lp_cost_sum_kernel(A, slot); });
        return 0;
    };
    const int rc = nv_lp_sequence(
        p->resample_every, T, nc, p->checkpoints,
        [&](uint64_t t, uint32_t epoch, bool fold_prev) {
            grid(A.nwg, A.R, kNvBlock, [&] { nv_lp_gradient_kernel(A, t, epoch, fold_prev ? 1 : 0); });
            return 0;
        },
        [&](uint64_t t) {
            if (A.n <= kNvLpSmallN)
                grid(A.R, 1, kNvLpBlockSmall, [&] { nv_lp_subproblem_kernel<kNvLpBlockSmall>(A, t); });
            else
                grid(A.R, 1, kNvLpBlockLarge, [&] { nv_lp_subproblem_kernel<kNvLpBlockLarge>(A, t); });
            return 0;
        },
        [&](uint64_t t) {
            grid((n + kNvBlock - 1) / kNvBlock, A.R, kNvBlock, [&] { nv_lp_update_kernel(A, t); });
            return 0;
        },
        cost);
    if (rc) return rc;
    cost(nc);
    grid(1, 1, 64, [&] { nv_lp_finalize_kernel(A, nc); });
    return 0;
}

// Records of the last emulated run in sim_nv_lp_view's layouts.
extern "C" void emu_nv_lp_paths(double *y, double *f_ckpt, double *x, uint32_t *tau, uint32_t *basis, double *value,
                                uint32_t *pivots)
{
    std::copy(e.fval.begin() + e.nc * e.R, e.fval.begin() + (e.nc + 1) * e.R, y);
    std::copy(e.fval.begin(), e.fval.begin() + e.nc * e.R, f_ckpt);
    std::copy(e.x.begin(), e.x.end(), x);
    std::copy(e.tau.begin(), e.tau.end(), tau);
    std::copy(e.rec_basis.begin(), e.rec_basis.end(), basis);
    std::copy(e.rec_value.begin(), e.rec_value.end(), value);
    std::copy(e.rec_piv.begin(), e.rec_piv.end(), pivots);
}

extern "C" const char *emu_nv_lp_error() { return g_err; }
