// sqn.hpp -- Algorithms 3-4 (Section 3.3, Task 3): stochastic quasi-Newton for the logistic loss
// Eq. (10)-(11). Device arguments shared by the kernels (fw_sqn.hip) and the host driver
// (sqn_api.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fw {

constexpr uint32_t kSqnDomGrad = 5u;        // Philox domain of the gradient rows of iteration k
constexpr uint32_t kSqnDomHess = 6u;        // Philox domain of the Hessian rows of the pair closed at k
constexpr int kSqnMaxM = 32;                // stored pairs
constexpr int kSqnMaxB = 1024;              // b and b_H
constexpr uint32_t kSqnMaxN = 8192;         // features (two quads per thread at 1024 threads)
constexpr int kSqnChunk = 8;                // values per workgroup reduction
constexpr int kSqnLossBlock = 256;          // threads of the loss kernel
constexpr uint32_t kSqnLossRows = 512;      // rows per workgroup of the loss kernels
constexpr uint32_t kSqnManySnap = 64;       // stored iterates from which the loss runs a lane per iterate
constexpr uint32_t kSqnHessianPitch = 65;   // LDS pitch (doubles) of the product kernel's k-major blocks
constexpr uint32_t kSqnComputeUnits = 256;  // compute units of the MI355X
constexpr uint32_t kSqnLdsPerCu = 160 * 1024;   // LDS bytes per compute unit

struct SqnArgs {
    uint32_t n, ld, nq;                     // features; row stride (a multiple of 4); quads ld / 4
    uint32_t N;                             // rows of the data set
    uint32_t L, M, b, bH;
    uint32_t k0, k1, inst;                  // Philox key (seed lo, hi); stream instance
    uint32_t R, n_ckpt;
    uint32_t G;                             // lanes per row in the row dot products (a power of two)
    uint32_t GV;                            // lanes per stored vector in the vector dot products
    uint64_t K;
    double beta;
    uint64_t ckpt[8];
    const uint32_t *X;                      // [N][xw] feature bits, bit j % 32 of word j / 32; zero padded
    uint32_t xw;                            // words per row, a multiple of 4
    const uint8_t *z;                       // [N] labels in {0, 1}
    void *S, *Y;                            // [R][M][ld] the stored pairs (double, or float with pairs_fp32)
    uint32_t pairs_fp32;
    double *wprev;                          // [R][ld] the previous window's average
    double *acc;                            // [R][ld] the current window's sum of iterates
    double *wsnap;                          // [n_ckpt + 1][R][ld] w after each checkpoint; the last is w^{K+1}
    double *wt;                             // [ld][(n_ckpt + 1) R] the same, feature-major (many iterates)
    uint32_t *pairs;                        // [R] correction pairs computed
    double *loss_part;                      // [n_ckpt + 1][R][nblk][2] double-double partial sums
    uint32_t nblk;                          // loss workgroups per snapshot
    double *fval;                           // [n_ckpt + 1][R] F at the checkpoints, then F(w^{K+1})
    double *stats;                          // kMaxStreams x kStreamFields + 2
};

int launch_sqn_run(const SqnArgs &A, hipStream_t s);
int launch_sqn_loss(const SqnArgs &A, hipStream_t s);
// Algorithm 4's H_t (n x n, row stride ldh, a multiple of 16) of replication rep from its m newest
// pairs (the oldest at ring slot head). scratch holds at least sqn_hessian_scratch(n) doubles.
int launch_sqn_hessian(const SqnArgs &A, uint32_t rep, uint32_t head, uint32_t m, double *scratch, double *H,
                       uint32_t ldh, hipStream_t s);
inline uint32_t sqn_hessian_ld(uint32_t n) { return (n + 15) / 16 * 16; }
inline size_t sqn_hessian_scratch(uint32_t n) { return 6 * kSqnMaxM * kSqnMaxM + 4 + 2 * static_cast<size_t>(n) * 2 * kSqnMaxM; }

}  // namespace fw
