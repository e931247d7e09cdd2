// sqn_split.hpp -- Algorithms 3-4 (Section 3.3) with one replication spread over many workgroups:
// the device arguments of fw_sqn_split.hip and the launch sequence, shared by the library
// (sqn_api.hip) and the CPU emulation of the kernels.
//
// Each workgroup (four wavefronts) owns a slice of 64 feature quads of w, of the gradient, of the
// window sum and of the stored pairs; everything that needs the whole vector (the rows' dot
// products x_i'w, S'g and Y'g, the new pair's dot products) is summed over slices in a later launch,
// slice by slice in order, from per-slice partial sums in HBM. An iteration k is:
//   grad   the rows' dot products of iteration k (partials written by the previous launch), the
//          residuals, the gradient slice, the window sum; for k <= 2L the step and the next
//          iteration's partial row dot products, else the gradient and the partial S'g, Y'g;
//   dir    (k > 2L) S'g, Y'g, the compact representation's coefficients, the direction, the step,
//          the next iteration's partial row dot products;
// and at the end of a window (k a multiple of L):
//   win1   the window average, s into the ring, and (from the second window on) the partial dot
//          products of the b_H Hessian rows with the average and with s;
//   win2   y (Eq. (13) applied to s) into the ring and the partial dot products of the new pair with
//          the stored ones;
//   small  one workgroup per replication: S'Y and Y'Y extended by the new pair (the oldest dropped
//          when the ring was full), gamma, R^-1 and C rebuilt.
// The ring's fill and head, the pair count and the snapshot slots follow from k alone, so the
// host passes them to each launch.
#pragma once

#include <stdint.h>

#include "sim.h"
#include "sqn.hpp"

namespace fw {

constexpr uint32_t kSplitQuads = 64;                    // quads per slice
constexpr uint32_t kSplitWaves = 4;                     // wavefronts per workgroup (one slice)
constexpr uint32_t kSplitThreads = kSplitQuads * kSplitWaves;
constexpr uint32_t kSplitMaxSlices = kSqnMaxN / 4 / kSplitQuads;   // 32
constexpr uint32_t kSplitMaxR = SIM_SQN_SPLIT_MAX_R;    // replications per split run
constexpr size_t kSqnSmall = 4 * static_cast<size_t>(kSqnMaxM) * kSqnMaxM + 8;   // per replication

struct SqnSplit {
    SqnArgs A;
    uint32_t W;                 // slices per replication
    double *w;                  // [R][ld] the iterate
    double *g;                  // [R][ld] the gradient of the current iteration (k > 2L)
    double *xpart;              // [2][R][b][W] partial x_i'w, by the parity of the iteration
    double *dpart;              // [R][2 M][W] partial s_i'g (2i) and y_i'g (2i + 1), oldest pair first
    double *hpart;              // [R][2][b_H][W] partial x_i'wbar, then x_i's
    double *ypart;              // [R][3 M][W] partial s_i'y (3i), s'y_i (3i + 1), y_i'y (3i + 2)
    double *small;              // [R][kSqnSmall] S'Y, Y'Y, R^-1, C (kSqnMaxM^2 each), then gamma
};

struct SqnSplitStep {
    uint64_t k;                 // the iteration
    uint32_t m, head;           // pairs held and the oldest's ring slot, before this window's pair
    int32_t snap, snap_last;    // wsnap slots that receive w^{k+1}, or -1
    uint32_t next;              // 1: also the partial row dot products of iteration k + 1
    uint32_t pair;              // window: 1 when it closes a pair
    uint32_t slot;              // window: ring slot of the new pair
    uint32_t full;              // window: the ring held M pairs
    uint32_t m_new, head_new;   // window: after the new pair
    uint32_t pairs;             // window: pairs formed so far, this one included
};

enum class SqnSplitKernel { Start, Grad, Dir, Win1, Win2, Small };

inline uint32_t sqn_split_slices(uint32_t nq) { return (nq + kSplitQuads - 1) / kSplitQuads; }

// The launches of a run of K iterations, in order: launch(kind, step) returns 0 or an error.
template <class Launch>
int sqn_split_sequence(uint64_t K, uint32_t L, uint32_t M, uint32_t n_ckpt, const uint64_t *ckpt, Launch launch)
{
    SqnSplitStep st{};
    st.snap = st.snap_last = -1;
    st.k = 1;
    if (int rc = launch(SqnSplitKernel::Start, st)) return rc;
    uint32_t m = 0, head = 0, pairs = 0, ck = 0;
    int64_t t = -1;
    for (uint64_t k = 1; k <= K; ++k) {
        st = SqnSplitStep{};
        st.k = k;
        st.m = m;
        st.head = head;
        st.snap = (ck < n_ckpt && ckpt[ck] == k) ? static_cast<int32_t>(ck++) : -1;
        st.snap_last = (k == K) ? static_cast<int32_t>(n_ckpt) : -1;
        st.next = k < K ? 1u : 0u;
        if (k <= 2ull * L) {
            if (int rc = launch(SqnSplitKernel::Grad, st)) return rc;
        } else {
            if (int rc = launch(SqnSplitKernel::Grad, st)) return rc;
            if (int rc = launch(SqnSplitKernel::Dir, st)) return rc;
        }
        if (k % L == 0) {
            ++t;
            st.pair = t > 0 ? 1u : 0u;
            st.full = m == M ? 1u : 0u;
            st.slot = st.full ? head : (head + m) % M;
            st.m_new = st.full ? m : m + 1;
            st.head_new = st.full ? (head + 1) % M : head;
            st.pairs = pairs + st.pair;
            if (int rc = launch(SqnSplitKernel::Win1, st)) return rc;
            if (st.pair) {
                if (int rc = launch(SqnSplitKernel::Win2, st)) return rc;
                if (int rc = launch(SqnSplitKernel::Small, st)) return rc;
                m = st.m_new;
                head = st.head_new;
                pairs = st.pairs;
            }
        }
    }
    return 0;
}

int launch_sqn_split(const SqnSplit &P, SqnSplitKernel kind, const SqnSplitStep &st, hipStream_t s);

}  // namespace fw
