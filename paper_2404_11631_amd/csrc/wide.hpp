// wide.hpp -- Algorithm 1 at the paper's experimental shape (Section 4.1: d up to 1e5 assets,
// N = 25-50 samples per gradient, K = 1500 iterations, one or a few replications): the device
// arguments shared by the kernels (fw_wide.hip) and the host driver (wide_api.hip).
#pragma once

#include <stdint.h>

namespace fw {

constexpr int kWideBlock = 256;                 // threads per workgroup
constexpr int kWideChunks = 8;                  // sample chunks per workgroup (i = c, c + 8, ...)
constexpr int kWideQuads = kWideBlock / kWideChunks;   // asset quads per workgroup (128 assets)
constexpr uint32_t kWideMaxR = 64;
constexpr uint32_t kWideMaxN = 1024;
constexpr uint64_t kWideMaxD = 1ull << 22;

struct WideArgs {
    // instance: d assets in nq = d/4 quads, nwg workgroups per replication
    uint32_t d, nq, N, nwg, R;                  // N: the largest sample size of the run (buffer stride)
    uint32_t k0, k1, dom;                       // Philox key, stream domain (path noise)
    float gap_eps;
    double lambda;
    // per asset; sz = sqrt(2 ln 2) sigma, c1 = sz / N0, c2 = 2 lambda sz / (N0 - 1) for the base size N0
    const float *mu_f, *sz_f, *c1_f, *c2_f, *w0_f;
    const double *mu_d, *sig_d;
    // state of each replication r
    uint64_t *S;                                // [R][d] signature: sum of (t+1) over steps choosing e_j
    uint32_t *cnt;                              // [R][d+1] decision counts, origin first
    uint32_t *tau;                              // [R] first step with FW gap <= eps
    uint32_t *dec;                              // [R][T] decisions (0 origin, j+1 vertex e_j)
    uint64_t T;
    // per-step scratch
    float *s1;                                  // [R][d] sum of the step's normals per asset
    float *part_dot;                            // [R][N][nwg] workgroup partials of z_i'v
    float *part_qn;                             // [R][nwg] workgroup partials of s1'v
    float *dot;                                 // [R][N] z_i'v
    float *qn;                                  // [R] s1'v
    // two buffers by iteration parity: a sample launch may read the previous iteration's partials
    float *wg_g;                                // [2][R][nwg] workgroup minimum of the gradient
    uint32_t *wg_j;                             // [2][R][nwg] its asset
    float *wg_gw;                               // [2][R][nwg] workgroup partial of g'w
    // outcomes
    double *fval;                               // [n_ckpt + 1][R] f(w_c) per checkpoint, then f(w_T)
    double *stats;                              // kMaxStreams x kStreamFields + 2 (min, max of Y)
    uint64_t *origin_total;                     // [1] decisions for the origin over all replications
};

// The sample size of one epoch: N_k returns, 1/N_k, and the factors N0/N_k and (N0-1)/(N_k-1) that
// turn the base coefficients c1, c2 into those of N_k (exactly 1 when N_k = N0).
struct WideEpoch {
    uint32_t n;
    float inv_n, sc1, sc2;
    uint32_t par;                               // buffer of the iteration's workgroup partials (t & 1)
};

// The launches of a run of T iterations (resample every M; N samples, or n_schedule[epoch]): for each
// t, iter(t, epoch, E, cw, from_w0, fold_prev) (w_t = cw S, w_0 at t = 0 when from_w0; fold_prev: the
// sample launch first takes the step of iteration t - 1); step(t) where that step cannot wait for
// the next iteration (an objective evaluation follows, or t is the last iteration); objective(c, slot)
// at w = c S for every checkpoint equal to t + 1. Each callback returns 0 or an error, which ends the
// sequence and is returned.
template <class Iter, class Step, class Objective>
int wide_sequence(uint32_t N, const uint32_t *n_schedule, uint64_t M, uint64_t T, bool has_w0, uint32_t n_ckpt,
                  const uint64_t *checkpoints, Iter iter, Step step, Objective objective)
{
    uint32_t ck = 0;
    bool pending = false;
    for (uint64_t t = 0; t < T; ++t) {
        const float cw = t == 0 ? 0.0f : static_cast<float>(2.0 / (static_cast<double>(t) * static_cast<double>(t + 1)));
        const uint64_t e = t / M;
        const uint32_t Ne = n_schedule ? n_schedule[e] : N;
        const WideEpoch E{Ne, static_cast<float>(1.0 / Ne), static_cast<float>(static_cast<double>(N) / Ne),
                          static_cast<float>((N - 1.0) / (Ne - 1.0)), static_cast<uint32_t>(t & 1)};
        if (int rc = iter(t, static_cast<uint32_t>(e), E, cw, t == 0 && has_w0, pending)) return rc;
        const bool objective_next = ck < n_ckpt && checkpoints[ck] == t + 1;
        pending = !(objective_next || t + 1 == T);
        if (!pending)
            if (int rc = step(t)) return rc;
        while (ck < n_ckpt && checkpoints[ck] == t + 1) {
            if (int rc = objective(2.0 / (static_cast<double>(t + 1) * static_cast<double>(t + 2)), ck)) return rc;
            ++ck;
        }
    }
    return 0;
}

// One iteration without its step (sample, dot, gradient): w_t = cw S (or w_0 at t = 0 when from_w0),
// epoch = t div M of size E; with fold_prev the sample launch first takes the step of iteration t - 1.
int launch_wide_iteration(const WideArgs &A, uint64_t t, uint32_t epoch, const WideEpoch &E, float cw, bool from_w0,
                          bool fold_prev, hipStream_t s);
// The step of iteration t on its own.
int launch_wide_step(const WideArgs &A, uint64_t t, hipStream_t s);
// f(w) at w = c S into fval[slot][r].
int launch_wide_objective(const WideArgs &A, double c, uint32_t slot, hipStream_t s);
// Cross-replication statistics of Y and of the n_ckpt checkpoints into stats.
int launch_wide_finalize(const WideArgs &A, uint32_t n_ckpt, hipStream_t s);

}  // namespace fw
