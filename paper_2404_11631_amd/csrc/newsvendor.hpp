// newsvendor.hpp -- Algorithm 2 (Section 3.2, Task 2): the multi-product newsvendor by stochastic
// Frank-Wolfe. Device arguments shared by the kernels (fw_newsvendor.hip) and the host driver
// (nv_api.hip).
#pragma once

#include <stdint.h>

namespace fw {

constexpr int kNvBlock = 256;                   // threads per workgroup: kNvBlock / P quads of products
constexpr uint32_t kNvMaxLanes = 16;            // lanes per quad at most

// Lanes per quad for n/4 quads and R replications: the smallest power of two that gives ~65536
// threads (a wavefront per SIMD on every compute unit), at most kNvMaxLanes and at most S.
inline uint32_t nv_lanes_per_quad(uint32_t nq, uint64_t R, uint32_t S)
{
    uint32_t P = 1;
    while (P < kNvMaxLanes && 2 * P <= S && static_cast<uint64_t>(nq) * R * P < 65536u) P *= 2;
    return P;
}
constexpr uint32_t kNvMaxR = 64;
constexpr uint32_t kNvMaxS = 1024;
constexpr uint64_t kNvMaxN = 1ull << 24;
constexpr uint32_t kNvDomain = 4u;              // Philox stream domain of the demand samples
constexpr uint32_t kNvCostChunk = 4096;         // products per workgroup of the cost evaluation

struct NvArgs {
    uint32_t n, nq, S, nwg, R;                  // products, quads, samples per product, workgroups
    uint32_t P;                                 // lanes per quad (a power of two <= kNvMaxLanes), splitting its samples
    uint32_t k0, k1, dom;                       // Philox key; counter word 3 (domain 4 | instance)
    float C, gap_eps;
    // per product, binary32: threshold scale 1/(sqrt(2 ln 2) sigma), k - v, (h + v)/S, 1/c, C/c, x_0
    const float *mu_f, *isk_f, *a_f, *b_f, *ic_f, *xs_f, *x0_f;
    // per product, binary64, for the cost Eq. (6)
    const double *mu_d, *sig_d, *k_d, *h_d, *v_d, *xs_d;
    // state of each replication
    uint64_t *S_sig;                            // [R][n] sum of (t+1) over steps choosing vertex j
    uint32_t *cnt;                              // [R][n+1] decision counts, origin first
    uint32_t *tau;                              // [R]
    uint32_t *dec;                              // [R][T]
    uint64_t T;
    // per-iteration scratch
    // two buffers by iteration parity: a sample launch may read the previous iteration's partials
    float *wg_r;                                // [2][R][nwg] smallest g_j / c_j of the workgroup
    uint32_t *wg_j;                             // [2][R][nwg] its product
    float *wg_gx;                               // [2][R][nwg] the workgroup's part of g'x
    // outcomes
    double *cost_part;                          // [R][ceil(n / kNvCostChunk)][2] double-double partials
    double *fval;                               // [n_ckpt + 1][R]
    double *stats;                              // kMaxStreams x kStreamFields + 2
    uint64_t *origin_total;
};

// Iteration t's samples and workgroup partials; with fold_prev it first takes the step of iteration
// t - 1 (whose partials the previous launch left in the other buffer).
int launch_nv_sample(const NvArgs &A, uint64_t t, uint32_t epoch, float cw, bool from_x0, bool fold_prev, hipStream_t s);
// The step of iteration t on its own.
int launch_nv_step(const NvArgs &A, uint64_t t, hipStream_t s);
int launch_nv_cost(const NvArgs &A, double c, uint32_t slot, hipStream_t s);
int launch_nv_finalize(const NvArgs &A, uint32_t n_ckpt, hipStream_t s);

// ---- Algorithm 2 over X = {A x <= C, x >= 0} with M resource rows (Eq. (7)) --------------------
// threads of the subproblem workgroup (one per replication): few products leave a pricing pass
// short, and then four wavefronts' barriers cost less than sixteen's
constexpr int kNvLpBlockSmall = 256;
constexpr int kNvLpBlockLarge = 1024;
constexpr uint32_t kNvLpSmallN = 2048;          // products up to which the small workgroup runs
constexpr uint32_t kNvLpMaxM = 8;

struct NvLpArgs {
    uint32_t n, nq, S, nwg, R, M;
    uint32_t P;                                 // lanes per quad in the gradient launch (nv_lanes_per_quad)
    uint32_t k0, k1, dom;                       // Philox key; counter word 3 (domain 4 | instance)
    uint32_t max_pivots;
    double gap_eps;
    double eps_r, eps_d;                        // reduced-cost and pivot-element tolerances
    // per product, binary64
    const double *mu_d, *isk_d;                 // mean; 1/(sqrt(2 ln 2) sigma) (infinite for sigma = 0)
    const double *km_d, *hv_d;                  // k - v; h + v
    const double *sig_d, *k_d, *h_d, *v_d;      // for the cost Eq. (6)
    const double *x0_d;                         // starting point (zeros for the origin)
    const double *Am;                           // [M][n] resource use
    const double *Cv;                           // [M] resource levels
    // state of each replication
    double *x;                                  // [R][n] the iterate
    double *g;                                  // [R][n] the iteration's gradient Eq. (9)
    uint32_t *rec_basis;                        // [R][T][M] each iteration's basis
    double *rec_value;                          // [R][T][M] and its basic variables
    uint32_t *rec_piv;                          // [R][T] pivots taken (max_pivots + 1: not solved)
    uint32_t *tau;                              // [R]
    uint32_t *origin;                           // [R] iterations whose vertex is the origin
    uint64_t T;
    // outcomes
    double *cost_part;                          // [R][ceil(n / kNvCostChunk)][2]
    double *fval;                               // [n_ckpt + 1][R]
    double *stats;                              // kMaxStreams x kStreamFields + 2
    uint64_t *origin_total;
};

// The launches of a run of T iterations (resample every M): for each t, gradient(t, epoch, fold_prev)
// and subproblem(t); update(t) where the update cannot wait for the next gradient launch (a cost
// evaluation follows, or t is the last iteration); cost(slot) for every checkpoint equal to t + 1.
// Each callback returns 0 or an error, which ends the sequence and is returned.
template <class Gradient, class Subproblem, class Update, class Cost>
int nv_lp_sequence(uint64_t M, uint64_t T, uint32_t n_ckpt, const uint64_t *checkpoints, Gradient gradient,
                   Subproblem subproblem, Update update, Cost cost)
{
    uint32_t ck = 0;
    bool pending = false;
    for (uint64_t t = 0; t < T; ++t) {
        if (int rc = gradient(t, static_cast<uint32_t>(t / M), pending)) return rc;
        if (int rc = subproblem(t)) return rc;
        const bool cost_next = ck < n_ckpt && checkpoints[ck] == t + 1;
        pending = !(cost_next || t + 1 == T);
        if (!pending)
            if (int rc = update(t)) return rc;
        while (ck < n_ckpt && checkpoints[ck] == t + 1) {
            if (int rc = cost(ck)) return rc;
            ++ck;
        }
    }
    return 0;
}

// Iteration t's gradient at x_t; with fold_prev it first moves x to x_t = x_{t-1} + gamma (s - x_{t-1})
// with the vertex the previous subproblem launch recorded.
int launch_nv_lp_gradient(const NvLpArgs &A, uint64_t t, uint32_t epoch, bool fold_prev, hipStream_t s);
// Iteration t's linear subproblem, its records and the Frank-Wolfe gap.
int launch_nv_lp_subproblem(const NvLpArgs &A, uint64_t t, hipStream_t s);
// The update of iteration t on its own (before a cost evaluation and after the last iteration).
int launch_nv_lp_update(const NvLpArgs &A, uint64_t t, hipStream_t s);
int launch_nv_lp_cost(const NvLpArgs &A, uint32_t slot, hipStream_t s);
int launch_nv_lp_finalize(const NvLpArgs &A, uint32_t n_ckpt, hipStream_t s);

}  // namespace fw
