// fw_paths.hip -- one lane per replication of Algorithm 1 (Section 3.1), fused with the FP64
// cross-path reduction (last workgroup finalises).
//
// Per iteration t of replication r (epoch k = t div M):
//   w_t       = w_0 at t = 0, else 2 S_j / (t (t+1)) from the integer signature S_j = sum of
//               (s+1) over the steps s < t that chose e_j (the step rule 2/(t+2) gives this
//               closed form of the recurrence w + gamma (s - w));
//   sampling  N samples R_i = mu + sigma .* z_i (Gaussian) or mu + sigma .* a_i z_i (elliptical t),
//             reduced in one pass to s1 = sum_i z_i and s2 = sum_i z_i (z_i' v), v = sigma .* w, so
//             Rbar = mu + sigma .* s1 / N                                        (Eq. (5))
//             (N-1) Sigma_hat w = sigma .* (s2 - s1 (s1' v) / N)                 (Eq. (4));
//   gradient  g = 2 lambda Sigma_hat w - Rbar;
//   decision  e_j for the lowest index attaining min_j g_j when that minimum is negative, else the
//             origin (the vertices of W);
//   gap       g'(w - s) and its first passage below eps (tau);
//   update    S_j += t+1 for the chosen e_j; checkpoint f(w_{t+1}) in FP64 from S.
// The outcome is Y = f(w_T) in FP64 from the exact signature.
//
// State stays in registers: s1, s2, v (binary32 or binary64), S (u32 while T(T+1)/2 < 2^32, else
// u64) and the decision counts. No HBM traffic per step except the optional decision log.
#include <hip/hip_runtime.h>

#include "device_reduce.hpp"
#include "device_rng.hpp"
#include "sim_types.hpp"

#include <type_traits>

namespace fw {

// ---------------------------------------------------------------------------------------------
// per-precision coefficient access
// ---------------------------------------------------------------------------------------------
template <typename Real>
struct Coef;

template <>
struct Coef<float> {
    const InstanceDesc *P;
    __device__ float mu(int j) const { return P->mu_f[j]; }
    __device__ float sz(int j) const { return P->sz_f[j]; }
    __device__ float c1(int j) const { return P->c1_f[j]; }
    __device__ float c2(int j) const { return P->c2_f[j]; }
    __device__ float w0(int j) const { return P->w0_f[j]; }
    __device__ float inv_n() const { return P->inv_n_f; }
    __device__ float tscale() const { return P->tscale_f; }
    __device__ static float rsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
};

template <>
struct Coef<double> {
    const InstanceDesc *P;
    __device__ double mu(int j) const { return P->mu_d[j]; }
    __device__ double sz(int j) const { return P->sig_d[j]; }
    __device__ double c1(int j) const { return P->c1_d[j]; }
    __device__ double c2(int j) const { return P->c2_d[j]; }
    __device__ double w0(int j) const { return P->w0_d[j]; }
    __device__ double inv_n() const { return P->inv_n_d; }
    __device__ double tscale() const { return P->tscale_d; }
    __device__ static double rsqrt(double x) { return 1.0 / sqrt(x); }
};

// Block `block` of the noise stream (epoch, r): binary32 starts from the stream's Philox row,
// binary64 runs the whole generator.
template <typename Real>
__device__ __forceinline__ Block4<Real> block_of_row(const PhiloxRow &row, uint32_t block, uint32_t epoch,
                                                     uint32_t r, uint32_t dom, uint32_t k0, uint32_t k1)
{
    if constexpr (std::is_same<Real, float>::value)
        return normals_block_row(row, block, dom, k0, k1);
    else
        return normals_block<Real>(block, epoch, r, dom, k0, k1);
}

constexpr int gcd_const(int a, int b) { return b == 0 ? a : gcd_const(b, a % b); }

// f(w) = lambda sum_j sigma_j^2 w_j^2 - mu' w at w = c S (Eq. (3), diagonal Sigma), in FP64
template <int D, bool EXACT, typename WS>
__device__ __forceinline__ double objective_from_signature(const InstanceDesc *__restrict__ P,
                                                           const WS (&S)[D], double c)
{
    const int d = EXACT ? D : static_cast<int>(P->d);
    double quad = 0.0, lin = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        if (j < d) {
            const double w = static_cast<double>(S[j]) * c;
            const double sw = P->sig_d[j] * w;
            quad = fma(sw, sw, quad);
            lin = fma(P->mu_d[j], w, lin);
        }
    }
    return fma(P->lambda, quad, -lin);
}

struct LaneResult {
    double y;
    uint32_t tau;
};

// One replication of Algorithm 1; returns Y and tau, leaves decision counts in cnt.
template <int D, bool EXACT, typename Real, int NOISE, typename WS, bool FEAT, bool SCHED>
__device__ __forceinline__ void run_path(const InstanceDesc *__restrict__ P, const RunBuffers &B,
                                         uint32_t r, uint32_t (&cnt)[D + 1], WS (&S)[D],
                                         LaneResult &res, uint64_t *feat_cnt)
{
    const Coef<Real> C{P};
    const int d = EXACT ? D : static_cast<int>(P->d);
    uint32_t N = P->N;
    const uint32_t M = P->M;
    // per-epoch sample sizes: N_k, 1/N_k and the coefficient rows of the current epoch
    const Real *c1s = nullptr;
    const Real *c2s = nullptr;
    Real inv_ns = Real(0);
    auto set_epoch = [&](uint32_t e) {
        if constexpr (SCHED) {
            N = B.sched_n[e];
            if constexpr (std::is_same<Real, float>::value) {
                inv_ns = B.sched_inv_f[e];
                c1s = B.sched_c_f + static_cast<uint64_t>(e) * 2 * d;
            } else {
                inv_ns = B.sched_inv_d[e];
                c1s = B.sched_c_d + static_cast<uint64_t>(e) * 2 * d;
            }
            c2s = c1s + d;
        }
    };
    set_epoch(0);
    const uint64_t T = P->T;
    const uint32_t k0 = static_cast<uint32_t>(P->seed), k1 = static_cast<uint32_t>(P->seed >> 32);
    const uint32_t dom = P->instance & 0xFFFFFFu;   // domain 0: path noise
    const uint64_t R = P->R;
    const bool logged = (P->flags & 2u) && (static_cast<uint64_t>(r) - P->log_begin) < P->log_count;
    const uint32_t n_ckpt = P->n_ckpt;

#pragma unroll
    for (int j = 0; j < D; ++j) S[j] = 0;
#pragma unroll
    for (int j = 0; j <= D; ++j) cnt[j] = 0;
    uint32_t tau = kTauNone;
    uint32_t ck = 0;
    uint64_t next_ckpt = n_ckpt ? P->ckpt[0] : 0;
    uint32_t epoch = 0, m_in_epoch = 0;   // t = epoch * M + m_in_epoch
    // control-variate summaries: per category (0 origin, j+1 vertex e_j) the integer sum of (t+1)^2
    // over iterations whose epoch's reference decision is that category, in this thread's column
    // of LDS (feat_cnt[c * kBlock]); the (t+1)-weighted count of the most probable category
    uint64_t fcnt1 = 0;
    const uint32_t ftop = FEAT ? P->cv_top : 0u;
    if constexpr (FEAT) {
#pragma unroll
        for (int c = 0; c <= D; ++c) feat_cnt[c * kBlock] = 0;
    }

    for (uint64_t t = 0; t < T; ++t) {
        // iterate w_t (scale factor of the signature) and v = sigma .* w_t
        const double cw = t == 0 ? 0.0 : 2.0 / (static_cast<double>(t) * static_cast<double>(t + 1));
        const Real cwr = static_cast<Real>(cw);
        Real v[D], s1[D], s2[D];
        Real g1[D];          // FEAT with t noise: sum of the Gaussian numerators
        // w_t = cw S except at t = 0 with a given start point (S = 0 and cw = 0 there, so the
        // origin needs no special case); one uniform branch instead of a select per asset
        const bool from_w0 = (t == 0) && P->has_w0;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            v[j] = (j < d) ? C.sz(j) * (static_cast<Real>(S[j]) * cwr) : Real(0);
            s1[j] = Real(0);
            s2[j] = Real(0);
            g1[j] = Real(0);
        }
        if (from_w0) {
#pragma unroll
            for (int j = 0; j < D; ++j) v[j] = (j < d) ? C.sz(j) * C.w0(j) : Real(0);
        }
        const bool feat_epoch = FEAT && m_in_epoch == 0;   // draws repeat within an epoch

        if constexpr (EXACT && NOISE == 0) {
            // groups of G samples hold a whole number of Philox blocks: static packing
            constexpr int G = 4 / gcd_const(D, 4);
            constexpr int NZ = G * D;
            constexpr int NB = NZ / 4;
            const uint32_t full = N / G, rem = N % G;
            PhiloxRow row{};
            if constexpr (std::is_same<Real, float>::value) row = philox_row(epoch, r, k0);
            for (uint32_t gi = 0; gi < full; ++gi) {
                Real z[NZ];
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    const Block4<Real> q = block_of_row<Real>(row, gi * NB + b, epoch, r, dom, k0, k1);
                    z[4 * b + 0] = q.z[0];
                    z[4 * b + 1] = q.z[1];
                    z[4 * b + 2] = q.z[2];
                    z[4 * b + 3] = q.z[3];
                }
#pragma unroll
                for (int s = 0; s < G; ++s) {
                    Real dot = Real(0);
#pragma unroll
                    for (int j = 0; j < D; ++j) dot = fma(z[s * D + j], v[j], dot);
#pragma unroll
                    for (int j = 0; j < D; ++j) {
                        s1[j] += z[s * D + j];
                        s2[j] = fma(z[s * D + j], dot, s2[j]);
                    }
                }
            }
            if (rem) {
                Real z[NZ];
                const uint32_t nb_needed = (rem * D + 3) / 4;
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    if (static_cast<uint32_t>(b) < nb_needed) {
                        const Block4<Real> q = block_of_row<Real>(row, full * NB + b, epoch, r, dom, k0, k1);
                        z[4 * b + 0] = q.z[0];
                        z[4 * b + 1] = q.z[1];
                        z[4 * b + 2] = q.z[2];
                        z[4 * b + 3] = q.z[3];
                    } else {
                        z[4 * b + 0] = z[4 * b + 1] = z[4 * b + 2] = z[4 * b + 3] = Real(0);
                    }
                }
#pragma unroll
                for (int s = 0; s < G; ++s) {
                    if (static_cast<uint32_t>(s) < rem) {
                        Real dot = Real(0);
#pragma unroll
                        for (int j = 0; j < D; ++j) dot = fma(z[s * D + j], v[j], dot);
#pragma unroll
                        for (int j = 0; j < D; ++j) {
                            s1[j] += z[s * D + j];
                            s2[j] = fma(z[s * D + j], dot, s2[j]);
                            }
                    }
                }
            }
        } else {
            NormalCursor<Real> cur;
            cur.seek(0u, epoch, r, dom, k0, k1);
            NormalCursor<Real> ext;
            if constexpr (NOISE == 1) ext.seek(N * static_cast<uint32_t>(d), epoch, r, dom, k0, k1);
            for (uint32_t i = 0; i < N; ++i) {
                Real z[D];
#pragma unroll
                for (int j = 0; j < D; ++j) z[j] = (j < d) ? cur.next(epoch, r, dom, k0, k1) : Real(0);
                if constexpr (FEAT && NOISE == 1) {
#pragma unroll
                    for (int j = 0; j < D; ++j) g1[j] += z[j];
                }
                if constexpr (NOISE == 1) {
                    Real ss = Real(0);
                    for (uint32_t k = 0; k < P->nu; ++k) {
                        const Real e = ext.next(epoch, r, dom, k0, k1);
                        ss = fma(e, e, ss);
                    }
                    const Real a = C.tscale() * Coef<Real>::rsqrt(ss);
#pragma unroll
                    for (int j = 0; j < D; ++j) z[j] *= a;
                }
                Real dot = Real(0);
#pragma unroll
                for (int j = 0; j < D; ++j) dot = fma(z[j], v[j], dot);
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    s1[j] += z[j];
                    s2[j] = fma(z[j], dot, s2[j]);
                }
            }
        }

        if constexpr (FEAT) {
            if (feat_epoch) {
                // the reference decision for b - sigma .* zbar (lowest index among equal minima,
                // the origin when the minimum is >= 0), weighted by the epoch's sums of (t+1)^2
                // and (t+1) over [t, min(t + M, T))
                const uint64_t t1 = (t + M < T) ? t + M : T;
                const uint64_t w2 = (M == 1) ? (t + 1) * (t + 1)
                                             : t1 * (t1 + 1) * (2 * t1 + 1) / 6 - t * (t + 1) * (2 * t + 1) / 6;
                const uint64_t w1 = (M == 1) ? t + 1 : t1 * (t1 + 1) / 2 - t * (t + 1) / 2;
                float vmin = 0.0f;
                uint32_t pick = 0;
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    if (j < d) {
                        const float u = static_cast<float>((NOISE == 1) ? g1[j] : s1[j]);
                        const float v = fmaf(-P->cv_s[j], u, P->cv_b[j]);
                        if (v < vmin) {
                            vmin = v;
                            pick = static_cast<uint32_t>(j + 1);
                        }
                    }
                }
                feat_cnt[pick * kBlock] += w2;
                fcnt1 += (pick == ftop) ? w1 : 0u;
            }
        }

        // gradient, linear subproblem over the vertices of W, Frank-Wolfe gap
        Real dot1 = Real(0);
#pragma unroll
        for (int j = 0; j < D; ++j) dot1 = fma(s1[j], v[j], dot1);
        const Real qn = dot1 * (SCHED ? inv_ns : C.inv_n());
        Real gmin = Real(0);
        int jmin = -1;
        Real gw = Real(0);
        Real gv[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            gv[j] = Real(0);
            if (j < d) {
                // c2 (s2 - s1 qn) - mu - c1 s1 with every product fused explicitly, so that each
                // kernel instantiation rounds it the same way
                const Real c1j = SCHED ? c1s[j] : C.c1(j), c2j = SCHED ? c2s[j] : C.c2(j);
                const Real g = fma(-c1j, s1[j], fma(c2j, fma(-s1[j], qn, s2[j]), -C.mu(j)));
                if (jmin < 0 || g < gmin) {
                    gmin = g;
                    jmin = j;
                }
                gv[j] = g;
                gw = fma(g, static_cast<Real>(S[j]) * cwr, gw);
            }
        }
        if (from_w0) {
            gw = Real(0);
#pragma unroll
            for (int j = 0; j < D; ++j)
                if (j < d) gw = fma(gv[j], C.w0(j), gw);
        }
        const int a = (gmin < Real(0)) ? jmin + 1 : 0;
        const Real gap = gw - (gmin < Real(0) ? gmin : Real(0));
        if (tau == kTauNone && gap <= static_cast<Real>(P->gap_eps)) tau = static_cast<uint32_t>(t);
        if (logged) B.dlog[t * P->log_count + (r - P->log_begin)] = static_cast<uint8_t>(a);

        // step 2/(t+2): the signature absorbs the update
        const WS tp1 = static_cast<WS>(t + 1);
        cnt[0] += (a == 0) ? 1u : 0u;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            const bool hit = (a == j + 1);
            S[j] += hit ? tp1 : WS(0);
            cnt[j + 1] += hit ? 1u : 0u;
        }
        if (t + 1 == next_ckpt) {
            const double c = 2.0 / (static_cast<double>(t + 1) * static_cast<double>(t + 2));
            B.fck[static_cast<uint64_t>(ck) * R + r] = objective_from_signature<D, EXACT, WS>(P, S, c);
            ++ck;
            next_ckpt = ck < n_ckpt ? P->ckpt[ck] : 0;
        }
        if (++m_in_epoch == M) {
            m_in_epoch = 0;
            ++epoch;
            if (t + 1 < T) set_epoch(epoch);
        }
    }
    res.y = objective_from_signature<D, EXACT, WS>(
        P, S, 2.0 / (static_cast<double>(T) * static_cast<double>(T + 1)));
    res.tau = tau;
    if constexpr (FEAT) {
        // x_j for vertex e_j (category j+1), x_d for the origin, x_{d+1} the (t+1)-weighted count of
        // the most probable category; the integer counts are exact in FP64 (< 2^53)
#pragma unroll
        for (int c = 0; c <= D; ++c) {
            if (c <= d) {
                const uint64_t row = (c == 0) ? static_cast<uint64_t>(d) : static_cast<uint64_t>(c - 1);
                B.feat[row * R + r] =
                    static_cast<float>((static_cast<double>(feat_cnt[c * kBlock]) - P->cv_mean[c]) * P->cv_inv[c]);
            }
        }
        B.feat[static_cast<uint64_t>(d + 1) * R + r] =
            static_cast<float>((static_cast<double>(fcnt1) - P->cv_mean1) * P->cv_inv1);
    }
}

// ---------------------------------------------------------------------------------------------
// kernel: paths + per-workgroup partials + last-workgroup finalisation
// ---------------------------------------------------------------------------------------------
template <int D, bool EXACT, typename Real, int NOISE, typename WS, bool FEAT, bool SCHED>
__global__ __launch_bounds__(kBlock) void fw_paths_kernel(const InstanceDesc *__restrict__ P,
                                                          RunBuffers B)
{
    __shared__ double sm_f[2 * (kBlock / 64)];
    __shared__ uint64_t sm_i[kBlock / 64];
    __shared__ uint32_t sm_last;
    // control-variate counts, [category][thread]: each thread owns its column
    __shared__ uint64_t sm_feat[FEAT ? (D + 1) * kBlock : 1];

    const uint64_t R = P->R;
    const uint64_t r = static_cast<uint64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const bool active = r < R;
    const int d = EXACT ? D : static_cast<int>(P->d);

    uint32_t cnt[D + 1];
    WS S[D];
    LaneResult res{0.0, kTauNone};
    if (active) {
        run_path<D, EXACT, Real, NOISE, WS, FEAT, SCHED>(P, B, static_cast<uint32_t>(r), cnt, S, res,
                                                         sm_feat + threadIdx.x);
        if ((P->flags & 8u) && !(P->flags & 1u)) B.y[r] = res.y;   // outcomes only
        if (P->flags & 1u) {
            B.y[r] = res.y;
            B.tau[r] = res.tau;
#pragma unroll
            for (int j = 0; j <= D; ++j)
                if (j <= d) B.cnt[static_cast<uint64_t>(j) * R + r] = cnt[j];
#pragma unroll
            for (int j = 0; j < D; ++j)
                if (j < d) B.wsum[static_cast<uint64_t>(j) * R + r] = static_cast<uint64_t>(S[j]);
        }
    } else {
#pragma unroll
        for (int j = 0; j <= D; ++j) cnt[j] = 0;
    }

    // per-workgroup partials: streams Y, f(w_c), RSE_c
    const uint32_t nb = B.nblocks;
    const uint32_t n_ckpt = P->n_ckpt;
    const uint32_t n_streams = 1 + 2 * n_ckpt;
    for (uint32_t s = 0; s < n_streams; ++s) {
        double x = 0.0;
        bool valid = active;
        if (active) {
            if (s == 0) {
                x = res.y;
            } else if (s <= n_ckpt) {
                x = B.fck[static_cast<uint64_t>(s - 1) * R + r];
            } else {
                const double f = B.fck[static_cast<uint64_t>(s - 1 - n_ckpt) * R + r];
                valid = (f != 0.0);
                const double e = valid ? (f - res.y) / f : 0.0;
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
        const double ymin = block_extreme<false>(active ? res.y : INFINITY, sm_f);
        const double ymax = block_extreme<true>(active ? res.y : -INFINITY, sm_f);
        if (threadIdx.x == 0) {
            double *base = B.part_f + static_cast<uint64_t>(n_streams) * kStreamFields * nb + blockIdx.x;
            store_agent(base, ymin);
            store_agent(base + nb, ymax);
        }
    }
    for (int j = 0; j <= d; ++j) {
        uint32_t cj = 0;
#pragma unroll
        for (int k = 0; k <= D; ++k)
            if (k == j) cj = cnt[k];
        const uint64_t tot = block_sum_u64(cj, sm_i);
        if (threadIdx.x == 0) store_agent(B.part_i + static_cast<uint64_t>(j) * nb + blockIdx.x, tot);
    }
    {
        const bool hit = active && res.tau != kTauNone;
        const uint64_t tc = block_sum_u64(hit ? 1u : 0u, sm_i);
        const uint64_t ts = block_sum_u64(hit ? res.tau : 0u, sm_i);
        if (threadIdx.x == 0) {
            store_agent(B.part_i + static_cast<uint64_t>(d + 1) * nb + blockIdx.x, tc);
            store_agent(B.part_i + static_cast<uint64_t>(d + 2) * nb + blockIdx.x, ts);
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
    for (int j = 0; j < d + 3; ++j) {
        uint64_t x = 0;
        for (uint32_t b = threadIdx.x; b < nb; b += kBlock) x += load_agent(B.part_i + static_cast<uint64_t>(j) * nb + b);
        x = block_sum_u64(x, sm_i);
        if (threadIdx.x == 0) B.final_i[j] = x;
    }
    if (threadIdx.x == 0) __hip_atomic_store(B.done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------------------------------------
// host dispatch over the instantiated shapes
// ---------------------------------------------------------------------------------------------
using KernelFn = void (*)(const InstanceDesc *, RunBuffers);

template <int D, bool EXACT, typename Real, int NOISE, typename WS, bool FEAT, bool SCHED = false>
constexpr KernelFn kfn()
{
    return &fw_paths_kernel<D, EXACT, Real, NOISE, WS, FEAT, SCHED>;
}

struct KernelChoice {
    KernelFn fn;
    int D;
    bool exact;
};

// Exact-width kernels pack each group of samples into whole Philox blocks at compile time; the
// generic ones read the stream through a cursor and take d <= D at run time. Runs with per-epoch
// sample sizes (SCHED) use the generic kernels, whose per-sample arithmetic and order are the
// exact-width kernels' (so a constant schedule reproduces the plain run bit for bit).
template <typename Real, typename WS, bool FEAT, bool SCHED>
static KernelChoice choose_gauss(uint32_t d)
{
    if constexpr (!SCHED) {
        switch (d) {
        case 1: return {kfn<1, true, Real, 0, WS, FEAT>(), 1, true};
        case 2: return {kfn<2, true, Real, 0, WS, FEAT>(), 2, true};
        case 3: return {kfn<3, true, Real, 0, WS, FEAT>(), 3, true};
        case 4: return {kfn<4, true, Real, 0, WS, FEAT>(), 4, true};
        case 5: return {kfn<5, true, Real, 0, WS, FEAT>(), 5, true};
        case 6: return {kfn<6, true, Real, 0, WS, FEAT>(), 6, true};
        case 8: return {kfn<8, true, Real, 0, WS, FEAT>(), 8, true};
        case 10: return {kfn<10, true, Real, 0, WS, FEAT>(), 10, true};
        case 12: return {kfn<12, true, Real, 0, WS, FEAT>(), 12, true};
        case 16: return {kfn<16, true, Real, 0, WS, FEAT>(), 16, true};
        default: break;
        }
    }
    if (d <= 16) return {kfn<16, false, Real, 0, WS, FEAT, SCHED>(), 16, false};
    if constexpr (sizeof(Real) == 4)
        if (d <= 32) return {kfn<32, false, Real, 0, WS, FEAT, SCHED>(), 32, false};
    return {nullptr, 0, false};
}

template <typename Real, typename WS, bool FEAT, bool SCHED>
static KernelChoice choose_t(uint32_t d)
{
    if (d <= 8) return {kfn<8, false, Real, 1, WS, FEAT, SCHED>(), 8, false};
    if (d <= 16) return {kfn<16, false, Real, 1, WS, FEAT, SCHED>(), 16, false};
    if constexpr (sizeof(Real) == 4)
        if (d <= 32) return {kfn<32, false, Real, 1, WS, FEAT, SCHED>(), 32, false};
    return {nullptr, 0, false};
}

template <bool SCHED>
static KernelChoice choose_plain(uint32_t d, uint32_t noise, bool fp64, bool wide)
{
    if (noise == 0) {
        if (fp64) return wide ? choose_gauss<double, uint64_t, false, SCHED>(d) : choose_gauss<double, uint32_t, false, SCHED>(d);
        return wide ? choose_gauss<float, uint64_t, false, SCHED>(d) : choose_gauss<float, uint32_t, false, SCHED>(d);
    }
    if (fp64) return wide ? choose_t<double, uint64_t, false, SCHED>(d) : choose_t<double, uint32_t, false, SCHED>(d);
    return wide ? choose_t<float, uint64_t, false, SCHED>(d) : choose_t<float, uint32_t, false, SCHED>(d);
}

// Returns 0 and launches, or a negative code: -5 unsupported shape, -3 launch failure.
// Feature-writing kernels exist for binary32 state and the 32-bit signature (T <= 92681).
int launch_fw_paths(const InstanceDesc &host_desc, const InstanceDesc *dev_desc, const RunBuffers &B,
                    bool fp64, hipStream_t stream, int *kernel_width)
{
    const bool wide = host_desc.T > kMaxNarrowT;
    const bool feat = (host_desc.flags & 4u) != 0;
    KernelChoice kc{nullptr, 0, false};
    if (feat) {
        if (fp64 || wide || B.sched_n) return -5;
        kc = host_desc.noise == 0 ? choose_gauss<float, uint32_t, true, false>(host_desc.d)
                                  : choose_t<float, uint32_t, true, false>(host_desc.d);
    } else if (B.sched_n) {
        kc = choose_plain<true>(host_desc.d, host_desc.noise, fp64, wide);
    } else {
        kc = choose_plain<false>(host_desc.d, host_desc.noise, fp64, wide);
    }
    if (!kc.fn) return -5;
    if (kernel_width) *kernel_width = kc.D;
    hipLaunchKernelGGL(kc.fn, dim3(B.nblocks), dim3(kBlock), 0, stream, dev_desc, B);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace fw
