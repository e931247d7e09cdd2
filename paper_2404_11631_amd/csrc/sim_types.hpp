// sim_types.hpp -- device-resident instance description, run buffers and reduction layout shared
// by the host engine and the path kernels.
#pragma once

#include <stdint.h>

namespace fw {

constexpr int kMaxD = 64;
constexpr int kMaxCkpt = 8;
constexpr uint32_t kTauNone = 0xFFFFFFFFu;
constexpr int kBlock = 256;                      // replications per workgroup (4 wavefronts)
constexpr int kMaxStreams = 1 + 2 * kMaxCkpt;    // Y, f(w_c), RSE_c
constexpr int kStreamFields = 5;                 // sum hi, sum lo, squares hi, squares lo, count
constexpr uint64_t kMaxNarrowT = 92681;          // largest T with T(T+1)/2 < 2^32
constexpr uint64_t kMaxBatchT = 131071;          // largest T with T(T+1)/2 < 2^33 (batched tiles)
// sqrt(2 ln 2): binary32 Box-Muller pairs are produced divided by this constant
constexpr double kBoxMullerScale = 1.1774100225154746910115693264597;

// One instance of problem Eq. (3) with the coefficients the path kernels use, precomputed on the
// host. Binary32 paths work with normals divided by sqrt(2 ln 2), so their per-asset scale carries
// that constant (see device_rng.hpp).
struct InstanceDesc {
    uint32_t d, N, M, noise, nu, n_ckpt, flags, instance;
    uint64_t R, T, seed;
    uint64_t log_begin, log_count;
    uint64_t ckpt[kMaxCkpt];
    double lambda, gap_eps;
    uint32_t has_w0, pad_;
    // binary64: objective and gradient coefficients
    double mu_d[kMaxD], sig_d[kMaxD], w0_d[kMaxD];
    double c1_d[kMaxD];      // sigma / N                (sample mean term, Eq. (5))
    double c2_d[kMaxD];      // 2 lambda sigma / (N-1)   (covariance term, Eq. (4))
    double tscale_d;         // sqrt(nu - 2)
    double inv_n_d;
    // binary32, normals scaled by 1/sqrt(2 ln 2)
    float mu_f[kMaxD], sz_f[kMaxD], isz_f[kMaxD], w0_f[kMaxD];
    float c1_f[kMaxD], c2_f[kMaxD];
    float tscale_f;          // sqrt(nu - 2) / sqrt(2 ln 2)
    float inv_n_f;
    // batched runs: offsets of this instance in the concatenated per-path arrays
    uint64_t path_base;      // into Y, tau, f(w_c) (per checkpoint stride = total R)
    uint64_t cnt_base;       // into counts   ([d+1][R] block of this instance)
    uint64_t wsum_base;      // into signatures ([d][R] block of this instance)
    uint64_t dlog_base;      // into the decision log ([T][log_count] block)
    // control-variate features (flag 4): reference decisions and their law
    float cv_b[kMaxD];           // reference gradient b
    float cv_s[kMaxD];           // sigma_j sqrt(2 ln 2) / N: times the binary32 sum s1_j gives sigma_j zbar_j
    double cv_mean[kMaxD + 1];   // p_c S2, category c (0 origin, j+1 vertex e_j)
    double cv_inv[kMaxD + 1];    // 1 / sqrt(S4 max(p_c (1 - p_c), 1e-4))
    double cv_mean1, cv_inv1;    // the same for the (t+1)-weighted count of category cv_top
    uint32_t cv_top, cv_pad_;
};

// One wavefront's unit of work in a batched run: `nrep` replications of one instance starting at
// rep0, with P lanes per replication: Pa of them split the assets (8 per lane at most), P / Pa
// split the samples. Tiles are stored longest first; `slot` is the tile's place in
// instance-major replication order, which fixes the reduction order.
struct Tile {
    uint32_t inst;
    uint32_t rep0;
    uint32_t slot;
    uint16_t nrep;
    uint8_t P;
    uint8_t Pa;
};

// Per-tile partial record of a batched run (one wavefront's replications of one instance).
constexpr int kTileStreams = 1 + 2 * kMaxCkpt;
struct TilePartial {
    double f[kTileStreams * kStreamFields];   // per stream: sum hi, sum lo, sq hi, sq lo, count
    double ymin, ymax;
    uint64_t dec[33];                         // decision totals, origin first (d <= 32)
    uint64_t tau_count, tau_sum;
};

struct BatchBuffers {
    const InstanceDesc *inst;
    const Tile *tiles;
    uint32_t n_tiles;
    uint32_t n_inst;
    TilePartial *partials;    // [n_tiles] by slot
    const uint32_t *slot_begin;   // [n_inst + 1] slot range of each instance
    double *fck;              // [max_ckpt][total R]
    uint64_t total_R;
    double *y;                // KEEP_PATHS: [total R]
    uint32_t *tau;            // KEEP_PATHS: [total R]
    uint32_t *cnt;            // KEEP_PATHS: concatenated [d_i+1][R_i]
    uint64_t *wsum;           // KEEP_PATHS: concatenated [d_i][R_i]
    uint8_t *dlog;            // DECISION_LOG: concatenated [T_i][log_count_i]
    TilePartial *final_stats; // [n_inst] reduced per instance
    uint32_t wave_mode;       // 1: every tile is one replication on a wavefront (fw_wave_kernel)
};

// LDS staging of a batched tile's normals (floats per wavefront). A replication qualifies for the
// one-wavefront form when its N d normals (rounded up to a Philox block) fit in it.
constexpr uint32_t kBatchStageFloats = 2112;

// Descriptor flag bits: 1 keep per-path records, 2 decision log, 4 control-variate features,
// 8 outcomes Y only (set by the library for its own control-variate runs).
constexpr uint32_t kFlagYOnly = 8u;

// Per-run device buffers. Structure of arrays, replication index fastest.
struct RunBuffers {
    double *y;            // [R]              (KEEP_PATHS or outcomes only)
    double *fck;          // [n_ckpt][R]      always: the epilogue reads it back for RSE
    uint32_t *cnt;        // [(d+1)][R]       (KEEP_PATHS)
    uint64_t *wsum;       // [d][R]           (KEEP_PATHS)
    uint32_t *tau;        // [R]              (KEEP_PATHS)
    uint8_t *dlog;        // [T][log_count]   (DECISION_LOG)
    double *part_f;       // [n_streams * 5 + 2][nblocks]
    uint64_t *part_i;     // [(d+1) + 2][nblocks]
    uint32_t *done;       // workgroups finished; reset to 0 by the last one
    double *final_f;      // [n_streams * 5 + 2]
    uint64_t *final_i;    // [(d+1) + 2]
    uint32_t nblocks;
    uint32_t n_streams;
    // dense correlated returns: sqrt(2 ln 2) L and its transpose, columns permuted and laid out in
    // the order the matrix-core instruction consumes them, and L itself in FP64 (row-major)
    float *feat;          // [(d+2)][R]       (CV_FEATURES)
    const float *dense_g;
    const float *dense_v;
    const double *dense_l64;
    // per-epoch sample sizes (NULL without a schedule): N_k, 1/N_k, and [E][2 d] rows c1 | c2
    const uint32_t *sched_n;
    const float *sched_inv_f;
    const double *sched_inv_d;
    const float *sched_c_f;
    const double *sched_c_d;
};

}  // namespace fw
