// fw_dense.hip -- Algorithm 1 (Section 3.1) with correlated returns R_i = mu + L y_i (dense
// lower-triangular L, Sigma = L L'), Gaussian or elliptical-t noise, d in {32, 64}, FP32 state.
//
// Mapping: four lanes per replication. Lane (r, p) of a wavefront (r = lane mod 16, p = lane / 16)
// owns the d/4 assets a(p, k) = 16 (k div 4) + 4p + (k mod 4), k < d/4 -- every fourth block of four
// -- so each lane draws exactly the Philox blocks of its own assets (block i d/4 + 4m + p holds
// assets 16m + 4p .. 16m + 4p + 3 of sample i), accumulates s1 = sum_i y_i and s2 = sum_i y_i
// (y_i'v) for its assets without any cross-lane sum, and needs two xor exchanges (16, 32) per sample
// for the dot product.
//
// In noise coordinates the sample statistics factor through L (Eq. (4)-(5)):
//   Rbar = mu + L s1 / N,   (N-1) Sigma_hat w = L (s2 - s1 (s1'v) / N),   v = L'w,
// so the gradient is g = L h - mu with h = 2 lambda/(N-1) (s2 - s1 (s1'v)/N) - s1/N. The two
// d x d products per iteration (v = L'w and g = L h) are, over the 16 replications of a wavefront,
// (d x d) x (d x 16) products on v_mfma_f32_16x16x4f32: the B operand of step kk is register kk
// of every lane (K index 4kk + p), the result lands in the same per-lane asset layout, and the
// A operand (L or L' with its columns permuted once on the host) is read from global memory (L2
// resident: every wavefront reads the same d^2 values) in the order the instruction consumes it.
// Binary32 normals are scaled by 1/sqrt(2 ln 2); the host folds that constant into the FP32
// copies of L. With t noise y_i = a_i z_i enters as s1 += a_i z_i, s2 += a_i^2 (z_i'v) z_i.
#include <hip/hip_runtime.h>

#include "device_reduce.hpp"
#include "device_rng.hpp"
#include "engine.hpp"
#include "sim_types.hpp"

namespace fw {

typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kRepsPerWave = 64 / kDenseLanesPerRep;
constexpr int kRB = kDenseRepsPerBlock;   // replications per workgroup

__device__ __forceinline__ int dense_asset(int p, int k) { return (k >> 2) * 16 + 4 * p + (k & 3); }

// Sum over the four lanes of a replication (lanes r, r+16, r+32, r+48).
template <typename V>
__device__ __forceinline__ V rep_sum(V x)
{
    x += __shfl_xor(x, 16, 64);
    x += __shfl_xor(x, 32, 64);
    return x;
}

// Binary32 form on the gfx950 lane-swap instructions, without a trip through LDS: swapping the
// upper 32 lanes of one copy of x with the lower 32 of another leaves (x_lo, x_lo) and
// (x_hi, x_hi), whose sum is x + x[lane ^ 32] in every lane; the 16-lane swap does the same for
// lane ^ 16. Addition is commutative, so all four lanes hold the same bits.
template <>
__device__ __forceinline__ float rep_sum<float>(float x)
{
    const auto h = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    x = __uint_as_float(h[0]) + __uint_as_float(h[1]);
    const auto q = __builtin_amdgcn_permlane16_swap(__float_as_uint(x), __float_as_uint(x), false, false);
    return __uint_as_float(q[0]) + __uint_as_float(q[1]);
}

// out = A x B over the 16 replications of this wavefront; A (D x D) in MFMA order
// (A_mfma[(mt * D/4 + kk) * 64 + lane] = A[16 mt + lane mod 16][a(lane / 16, kk)]), read from
// global memory: every wavefront of the grid reads the same D x D values, which stay in L2.
template <int D>
__device__ __forceinline__ void dense_product(const float *A_mfma, const float (&b)[D / 4],
                                              float (&out)[D / 4], int lane)
{
    // an opaque per-call lane offset keeps the compiler from precomputing (and holding) one
    // 64-bit address per operand: each load is base + 32-bit offset
    uint32_t off = static_cast<uint32_t>(lane);
    asm volatile("" : "+v"(off));
#pragma unroll
    for (int mt = 0; mt < D / 16; ++mt) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kk = 0; kk < D / 4; ++kk)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(A_mfma[off + (mt * (D / 4) + kk) * 64], b[kk], acc, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) out[4 * mt + q] = acc[q];
    }
}

// f(w) = lambda |L'w|^2 - mu'w at w = c S, FP64 (Eq. (3)); all four lanes of a replication return
// it. sS[asset][replication] holds the signatures of the workgroup, so each lane forms
// (L'w)_m = sum_j L_jm w_j for its own assets m. Every thread of the workgroup calls this at the
// same iterations (checkpoints and the end).
template <int D>
__device__ __forceinline__ double dense_objective(const InstanceDesc *P, const double *L64,
                                                  int p, int rep, double c, const uint32_t *sS)
{
    constexpr int H = D / 4;
    __syncthreads();
    double quad = 0.0, lin = 0.0;
#pragma unroll 1
    for (int k = 0; k < H; ++k) {
        const int m = dense_asset(p, k);
        double v = 0.0;
#pragma unroll 8
        for (int j = m; j < D; ++j) v += L64[j * D + m] * static_cast<double>(sS[j * kRB + rep]);
        v *= c;
        quad += v * v;
        lin += P->mu_d[m] * (static_cast<double>(sS[m * kRB + rep]) * c);
    }
    __syncthreads();
    quad = rep_sum(quad);
    lin = rep_sum(lin);
    return P->lambda * quad - lin;
}

// Three wavefronts per SIMD: the register budget (<= 168) that still holds the per-lane state
// (16 assets x z, s1, s2, v at d = 64) without spilling in the sample loop.
//
// FEAT writes the control-variate features of each path (sim.h): per epoch the reference decision
// for cv_ref - D zbar, D = diag(L) (each noise coordinate against its own diagonal entry, so the
// decisions stay i.i.d. with the product-form law of the diagonal case), from the sums of the
// Gaussian numerators g1 (s1 itself for Gaussian noise); the per-category sums of (t+1)^2 are kept
// in LDS in 32 bits (T <= 2343).
// The feature variant at d = 64 needs the sums g1 beside z, s1, s2 and v: two wavefronts per SIMD
// (<= 256 registers) keep it free of spills.
template <int D, int NOISE, bool FEAT>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu((FEAT && D == 64) ? 2 : 3, (FEAT && D == 64) ? 2 : 3)))
void fw_dense_kernel(const InstanceDesc *P, RunBuffers B)
{
    constexpr int H = D / 4;
    __shared__ uint32_t sS[D * kRB];          // signature S_j of each replication, [asset][replication]
    __shared__ uint16_t sC[(D + 1) * kRB];    // decision counts (T <= 65535), origin first
    __shared__ uint32_t sF[FEAT ? (D + 1) * kRB : 1];   // features: sums of (t+1)^2 per category
    __shared__ double sm_f[2 * (kBlock / 64)];
    __shared__ uint64_t sm_i[kBlock / 64];
    __shared__ uint32_t sm_last;
    const float *Ag = B.dense_g;   // sqrt(2 ln 2) L, MFMA order: g = L h
    const float *Av = B.dense_v;   // sqrt(2 ln 2) L', MFMA order: v = L'w

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int p = lane >> 4;
    const uint64_t R = P->R;
    const int rep = wave * kRepsPerWave + (lane & 15);   // replication within the workgroup
    const uint64_t r64 = static_cast<uint64_t>(blockIdx.x) * kRB + rep;
    const bool active = r64 < R;
    const uint32_t r = static_cast<uint32_t>(r64);
    const uint32_t N = P->N, M = P->M;
    const uint64_t T = P->T;
    const uint32_t k0 = static_cast<uint32_t>(P->seed), k1 = static_cast<uint32_t>(P->seed >> 32);
    const uint32_t dom = P->instance & 0xFFFFFFu;
    const uint32_t n_ckpt = P->n_ckpt;
    const bool logged = active && p == 0 && (P->flags & 2u) && (r64 - P->log_begin) < P->log_count;
    const float inv_n = P->inv_n_f;
    const float cu = static_cast<float>(2.0 * P->lambda / (static_cast<double>(N) - 1.0));

#pragma unroll
    for (int k = 0; k < H; ++k) {
        sS[dense_asset(p, k) * kRB + rep] = 0u;
        sC[(dense_asset(p, k) + 1) * kRB + rep] = 0;
    }
    if (p == 0) sC[rep] = 0;
    if constexpr (FEAT) {
#pragma unroll
        for (int k = 0; k < H; ++k) sF[(dense_asset(p, k) + 1) * kRB + rep] = 0u;
        if (p == 0) sF[rep] = 0u;
    }
    uint64_t fcnt1 = 0;                       // (t+1)-weighted count of the most probable category
    uint32_t tau = kTauNone;
    uint32_t ck = 0;
    uint64_t next_ckpt = n_ckpt ? P->ckpt[0] : 0;
    uint32_t epoch = 0, m_in_epoch = 0;

    for (uint64_t t = 0; t < T; ++t) {
        // the L operands are the same every iteration; re-read them (L2-resident) rather than keep
        // 2 D^2/64 of them live in registers across the sample loop
        asm volatile("" ::: "memory");
        const float cw = t == 0 ? 0.0f
                                : static_cast<float>(2.0 / (static_cast<double>(t) * static_cast<double>(t + 1)));
        float v[H], s1[H], s2[H];
        float g1[(FEAT && NOISE == 1) ? H : 1];   // t noise: sums of the Gaussian numerators
        {
            float w[H];
#pragma unroll
            for (int k = 0; k < H; ++k) {
                w[k] = (t == 0) ? (P->has_w0 ? P->w0_f[dense_asset(p, k)] : 0.0f)
                                : static_cast<float>(sS[dense_asset(p, k) * kRB + rep]) * cw;
                s1[k] = 0.0f;
                s2[k] = 0.0f;
                if constexpr (FEAT && NOISE == 1) g1[k] = 0.0f;
            }
            dense_product<D>(Av, w, v, lane);
        }

        // t noise: the chi-square normals of sample i are normals N D + nu i + q, q < nu. In each group
        // of 16 samples lane p draws those of samples 16g + 4p .. 16g + 4p + 3 (nu whole Philox blocks
        // from N D + nu (16g + 4p)), once for the replication instead of once per lane, and sample i
        // takes its scale from lane (i mod 16) div 4 of the replication.
        float a_own[4] = {1.0f, 1.0f, 1.0f, 1.0f};
#pragma unroll 1
        for (uint32_t i = 0; i < N; ++i) {
            if constexpr (NOISE == 1) {
                if ((i & 15u) == 0u) {
                    const uint32_t nu = P->nu;
                    NormalCursor<float> chi;
                    chi.seek(N * static_cast<uint32_t>(D) + nu * (i + 4u * static_cast<uint32_t>(p)), epoch, r, dom,
                             k0, k1);
#pragma unroll
                    for (int s4 = 0; s4 < 4; ++s4) {
                        float ss = 0.0f;
#pragma unroll 1
                        for (uint32_t q = 0; q < nu; ++q) {
                            const float e = chi.next(epoch, r, dom, k0, k1);
                            ss = fmaf(e, e, ss);
                        }
                        a_own[s4] = P->tscale_f * __builtin_amdgcn_rsqf(ss);
                    }
                }
            }
            float z[H];
#pragma unroll
            for (int m = 0; m < H / 4; ++m) {
                const Block4<float> q = normals_block<float>(i * (D / 4) + 4 * m + p, epoch, r, dom, k0, k1);
                z[4 * m + 0] = q.z[0];
                z[4 * m + 1] = q.z[1];
                z[4 * m + 2] = q.z[2];
                z[4 * m + 3] = q.z[3];
                // two Philox chains in flight at most: bounds the live temporaries
                if (m & 1) __builtin_amdgcn_sched_barrier(0);
            }
            float a = 1.0f;
            if constexpr (NOISE == 1) {
                // slot i mod 4 is a_own[0] after i mod 4 rotations (all lanes rotate in step)
                a = __shfl(a_own[0], (lane & 15) + 16 * static_cast<int>((i >> 2) & 3u), 64);
                const float a0 = a_own[0];
                a_own[0] = a_own[1];
                a_own[1] = a_own[2];
                a_own[2] = a_own[3];
                a_own[3] = a0;
            }
            float dot = 0.0f;
#pragma unroll
            for (int k = 0; k < H; ++k) dot = fmaf(z[k], v[k], dot);
            dot = rep_sum(dot);
            const float a2dot = (NOISE == 1) ? a * a * dot : dot;
#pragma unroll
            for (int k = 0; k < H; ++k) {
                if constexpr (NOISE == 1) s1[k] = fmaf(a, z[k], s1[k]);
                else s1[k] += z[k];
                s2[k] = fmaf(z[k], a2dot, s2[k]);
                if constexpr (FEAT && NOISE == 1) g1[k] += z[k];
            }
        }

        if constexpr (FEAT) {
            if (m_in_epoch == 0) {
                // the epoch's reference decision (lowest index among equal minima, the origin when the
                // minimum is >= 0), weighted by the epoch's sums of (t+1)^2 and (t+1)
                float vmin = INFINITY;
                int vj = -1;
#pragma unroll
                for (int k = 0; k < H; ++k) {
                    const int j = dense_asset(p, k);
                    const float u = (NOISE == 1) ? g1[k] : s1[k];
                    const float vv = fmaf(-P->cv_s[j], u, P->cv_b[j]);
                    if (vj < 0 || vv < vmin || (vv == vmin && j < vj)) {
                        vmin = vv;
                        vj = j;
                    }
                }
#pragma unroll
                for (int x = 16; x <= 32; x <<= 1) {
                    const float ov = __shfl_xor(vmin, x, 64);
                    const int oj = __shfl_xor(vj, x, 64);
                    if (ov < vmin || (ov == vmin && oj < vj)) {
                        vmin = ov;
                        vj = oj;
                    }
                }
                const uint32_t pick = (vmin < 0.0f) ? static_cast<uint32_t>(vj + 1) : 0u;
                const uint64_t t1 = (t + M < T) ? t + M : T;
                const uint64_t w2 = (M == 1) ? (t + 1) * (t + 1)
                                             : t1 * (t1 + 1) * (2 * t1 + 1) / 6 - t * (t + 1) * (2 * t + 1) / 6;
                const uint64_t w1 = (M == 1) ? t + 1 : t1 * (t1 + 1) / 2 - t * (t + 1) / 2;
                if (p == 0) sF[pick * kRB + rep] += static_cast<uint32_t>(w2);
                fcnt1 += (pick == P->cv_top) ? w1 : 0u;
            }
        }

        float dot1 = 0.0f;
#pragma unroll
        for (int k = 0; k < H; ++k) dot1 = fmaf(s1[k], v[k], dot1);
        dot1 = rep_sum(dot1);
        const float qn = dot1 * inv_n;
#pragma unroll
        for (int k = 0; k < H; ++k) s2[k] = cu * (s2[k] - s1[k] * qn) - s1[k] * inv_n;   // h
        float g[H];
        dense_product<D>(Ag, s2, g, lane);

        // vertex search: lowest asset index among equal minima, across the four lanes
        float gmin = 0.0f, gw = 0.0f;
        int jmin = -1;
#pragma unroll
        for (int k = 0; k < H; ++k) {
            const int j = dense_asset(p, k);
            const float gj = g[k] - P->mu_f[j];
            if (jmin < 0 || gj < gmin || (gj == gmin && j < jmin)) {
                gmin = gj;
                jmin = j;
            }
            const float wk = (t == 0) ? (P->has_w0 ? P->w0_f[j] : 0.0f) : static_cast<float>(sS[j * kRB + rep]) * cw;
            gw = fmaf(gj, wk, gw);
        }
#pragma unroll
        for (int x = 16; x <= 32; x <<= 1) {
            const float og = __shfl_xor(gmin, x, 64);
            const int oj = __shfl_xor(jmin, x, 64);
            if (og < gmin || (og == gmin && oj < jmin)) {
                gmin = og;
                jmin = oj;
            }
        }
        gw = rep_sum(gw);
        const int a = (gmin < 0.0f) ? jmin + 1 : 0;
        const float gap = gw - (gmin < 0.0f ? gmin : 0.0f);
        if (tau == kTauNone && gap <= static_cast<float>(P->gap_eps)) tau = static_cast<uint32_t>(t);
        if (logged) B.dlog[t * P->log_count + (r64 - P->log_begin)] = static_cast<uint8_t>(a);

        // the lane that owns the chosen vertex updates its signature and count
        const int ja = a - 1;
        const bool mine = (a == 0) ? (p == 0) : (((ja >> 2) & 3) == p);
        if (mine) {
            sC[a * kRB + rep] += 1;
            if (a > 0) sS[ja * kRB + rep] += static_cast<uint32_t>(t + 1);
        }
        if (t + 1 == next_ckpt) {
            const double c = 2.0 / (static_cast<double>(t + 1) * static_cast<double>(t + 2));
            const double f = dense_objective<D>(P, B.dense_l64, p, rep, c, sS);
            if (active && p == 0) B.fck[static_cast<uint64_t>(ck) * R + r64] = f;
            ++ck;
            next_ckpt = ck < n_ckpt ? P->ckpt[ck] : 0;
        }
        if (++m_in_epoch == M) {
            m_in_epoch = 0;
            ++epoch;
        }
    }
    const double y = dense_objective<D>(P, B.dense_l64, p, rep,
                                        2.0 / (static_cast<double>(T) * static_cast<double>(T + 1)), sS);
    const bool leader = active && p == 0;

    if constexpr (FEAT) {
        // x_j for vertex e_j (category j+1, written by the lane owning asset j), x_d for the origin,
        // x_{d+1} the (t+1)-weighted count of the most probable category; counts are exact in FP64
        __syncthreads();
        if (active) {
#pragma unroll 1
            for (int k = 0; k < H; ++k) {
                const int j = dense_asset(p, k);
                B.feat[static_cast<uint64_t>(j) * R + r64] = static_cast<float>(
                    (static_cast<double>(sF[(j + 1) * kRB + rep]) - P->cv_mean[j + 1]) * P->cv_inv[j + 1]);
            }
            if (p == 0) {
                B.feat[static_cast<uint64_t>(D) * R + r64] =
                    static_cast<float>((static_cast<double>(sF[rep]) - P->cv_mean[0]) * P->cv_inv[0]);
                B.feat[static_cast<uint64_t>(D + 1) * R + r64] =
                    static_cast<float>((static_cast<double>(fcnt1) - P->cv_mean1) * P->cv_inv1);
            }
        }
    }
    if (leader && (P->flags & 8u) && !(P->flags & 1u)) B.y[r64] = y;   // outcomes only
    if (active && (P->flags & 1u)) {
        if (p == 0) {
            B.y[r64] = y;
            B.tau[r64] = tau;
            B.cnt[r64] = sC[rep];
        }
#pragma unroll 1
        for (int k = 0; k < H; ++k) {
            const int j = dense_asset(p, k);
            B.cnt[static_cast<uint64_t>(j + 1) * R + r64] = sC[(j + 1) * kRB + rep];
            B.wsum[static_cast<uint64_t>(j) * R + r64] = sS[j * kRB + rep];
        }
    }

    // per-workgroup partials (one lane per replication contributes)
    const uint32_t nb = B.nblocks;
    const uint32_t n_streams = 1 + 2 * n_ckpt;
    for (uint32_t s = 0; s < n_streams; ++s) {
        double x = 0.0;
        bool valid = leader;
        if (leader) {
            if (s == 0) {
                x = y;
            } else if (s <= n_ckpt) {
                x = B.fck[static_cast<uint64_t>(s - 1) * R + r64];
            } else {
                const double f = B.fck[static_cast<uint64_t>(s - 1 - n_ckpt) * R + r64];
                valid = (f != 0.0);
                const double e = valid ? (f - y) / f : 0.0;
                x = e * e;
            }
        }
        if (!valid) x = 0.0;
        double h = x, l = 0.0;
        block_sum_dd(h, l, sm_f);
        double qh = x * x, ql = fma(x, x, -(x * x));
        block_sum_dd(qh, ql, sm_f);
        double ch = valid ? 1.0 : 0.0, cl = 0.0;
        block_sum_dd(ch, cl, sm_f);
        if (threadIdx.x == 0) {
            double *base = B.part_f + static_cast<uint64_t>(s) * kStreamFields * nb + blockIdx.x;
            store_agent(base + 0 * nb, h);
            store_agent(base + 1 * nb, l);
            store_agent(base + 2 * nb, qh);
            store_agent(base + 3 * nb, ql);
            store_agent(base + 4 * nb, ch);
        }
    }
    {
        const double ymin = block_extreme<false>(leader ? y : INFINITY, sm_f);
        const double ymax = block_extreme<true>(leader ? y : -INFINITY, sm_f);
        if (threadIdx.x == 0) {
            double *base = B.part_f + static_cast<uint64_t>(n_streams) * kStreamFields * nb + blockIdx.x;
            store_agent(base, ymin);
            store_agent(base + nb, ymax);
        }
    }
    for (int j = 0; j <= D; ++j) {
        const uint32_t cj = leader ? sC[j * kRB + rep] : 0u;
        const uint64_t tot = block_sum_u64(cj, sm_i);
        if (threadIdx.x == 0) store_agent(B.part_i + static_cast<uint64_t>(j) * nb + blockIdx.x, tot);
    }
    {
        const bool hit = leader && tau != kTauNone;
        const uint64_t tc = block_sum_u64(hit ? 1u : 0u, sm_i);
        const uint64_t ts = block_sum_u64(hit ? tau : 0u, sm_i);
        if (threadIdx.x == 0) {
            store_agent(B.part_i + static_cast<uint64_t>(D + 1) * nb + blockIdx.x, tc);
            store_agent(B.part_i + static_cast<uint64_t>(D + 2) * nb + blockIdx.x, ts);
        }
    }

    // the last workgroup to finish reduces every partial in a fixed order
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t prev = __hip_atomic_fetch_add(B.done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        sm_last = (prev == nb - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!sm_last) return;
    __threadfence();
    for (uint32_t s = 0; s < n_streams; ++s) {
        const double *base = B.part_f + static_cast<uint64_t>(s) * kStreamFields * nb;
        double h = 0.0, l = 0.0, qh = 0.0, ql = 0.0, ch = 0.0, cl = 0.0;
        for (uint32_t b = threadIdx.x; b < nb; b += kBlock) {
            dd_add(h, l, load_agent(base + 0 * nb + b), load_agent(base + 1 * nb + b));
            dd_add(qh, ql, load_agent(base + 2 * nb + b), load_agent(base + 3 * nb + b));
            dd_add(ch, cl, load_agent(base + 4 * nb + b), 0.0);
        }
        block_sum_dd(h, l, sm_f);
        block_sum_dd(qh, ql, sm_f);
        block_sum_dd(ch, cl, sm_f);
        if (threadIdx.x == 0) {
            double *o = B.final_f + static_cast<uint64_t>(s) * kStreamFields;
            o[0] = h;
            o[1] = l;
            o[2] = qh;
            o[3] = ql;
            o[4] = ch + cl;
        }
    }
    {
        const double *base = B.part_f + static_cast<uint64_t>(n_streams) * kStreamFields * nb;
        double mn = INFINITY, mx = -INFINITY;
        for (uint32_t b = threadIdx.x; b < nb; b += kBlock) {
            mn = fmin(mn, load_agent(base + b));
            mx = fmax(mx, load_agent(base + nb + b));
        }
        mn = block_extreme<false>(mn, sm_f);
        mx = block_extreme<true>(mx, sm_f);
        if (threadIdx.x == 0) {
            B.final_f[n_streams * kStreamFields] = mn;
            B.final_f[n_streams * kStreamFields + 1] = mx;
        }
    }
    for (int j = 0; j < D + 3; ++j) {
        uint64_t x = 0;
        for (uint32_t b = threadIdx.x; b < nb; b += kBlock) x += load_agent(B.part_i + static_cast<uint64_t>(j) * nb + b);
        x = block_sum_u64(x, sm_i);
        if (threadIdx.x == 0) B.final_i[j] = x;
    }
    if (threadIdx.x == 0) __hip_atomic_store(B.done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

int launch_fw_dense(const InstanceDesc &host_desc, const InstanceDesc *dev_desc, const RunBuffers &B,
                    hipStream_t stream)
{
    using K = void (*)(const InstanceDesc *, RunBuffers);
    K fn = nullptr;
    const bool feat = (host_desc.flags & 4u) != 0;
    if (host_desc.d == 64)
        fn = feat ? (host_desc.noise ? fw_dense_kernel<64, 1, true> : fw_dense_kernel<64, 0, true>)
                  : (host_desc.noise ? fw_dense_kernel<64, 1, false> : fw_dense_kernel<64, 0, false>);
    if (host_desc.d == 32)
        fn = feat ? (host_desc.noise ? fw_dense_kernel<32, 1, true> : fw_dense_kernel<32, 0, true>)
                  : (host_desc.noise ? fw_dense_kernel<32, 1, false> : fw_dense_kernel<32, 0, false>);
    if (!fn) return -5;
    hipLaunchKernelGGL(fn, dim3(B.nblocks), dim3(kBlock), 0, stream, dev_desc, B);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace fw
