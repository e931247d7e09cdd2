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
};

// Per-run device buffers. Structure of arrays, replication index fastest.
struct RunBuffers {
    double *y;            // [R]              (KEEP_PATHS)
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
};

}  // namespace fw
