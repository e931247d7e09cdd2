// newsvendor.hpp -- Algorithm 2 (Section 3.2, Task 2): the multi-product newsvendor by stochastic
// Frank-Wolfe. Device arguments shared by the kernels (fw_newsvendor.hip) and the host driver
// (nv_api.hip).
#pragma once

#include <stdint.h>

namespace fw {

constexpr int kNvBlock = 256;                   // threads per workgroup, one quad of products each
constexpr uint32_t kNvMaxR = 64;
constexpr uint32_t kNvMaxS = 1024;
constexpr uint64_t kNvMaxN = 1ull << 24;
constexpr uint32_t kNvDomain = 4u;              // Philox stream domain of the demand samples
constexpr uint32_t kNvCostChunk = 4096;         // products per workgroup of the cost evaluation

struct NvArgs {
    uint32_t n, nq, S, nwg, R;                  // products, quads, samples per product, workgroups
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

}  // namespace fw
