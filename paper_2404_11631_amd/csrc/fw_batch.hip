// fw_batch.hip -- instances of uneven size and horizon, as wavefront tiles.
//
// Algorithm 1 (Section 3.1) as in fw_paths.hip, reorganised for a batch of instances with d up to
// 32 in one kernel:
//   * one wavefront per tile; every tile of the batch is in one launch, longest first, so the
//     hardware dispatcher hands the heaviest tiles out first and fills in with the lighter ones;
//   * a tile holds 64/P replications of one instance with P = Pa x Ps lanes per replication:
//     Pa lanes split the assets (a lane holds at most 8 of them: their iterate, sample sums,
//     signature and decision counts stay in registers), Ps lanes split the N samples into
//     contiguous chunks;
//   * the Pa lanes of a sample chunk draw its normals together: per round of G = 4/gcd(d,4)
//     samples (a whole number of Philox blocks) each lane draws every Pa-th block into LDS, and
//     each lane then reads its own assets' normals back; the sample's dot product with the
//     iterate is summed over the Pa lanes with an xor butterfly;
//   * after the samples the Ps partial sums are combined by an xor butterfly over the lanes that
//     hold the same assets; the gradient's dot product, the minimum of the linear subproblem
//     (lowest index among equal values), the gap and the objective at checkpoints are reduced over
//     the Pa lanes the same way. Butterflies give every lane of a replication the same bits, so all
//     of them take the same decision;
//   * each tile writes its partial sums to a slot fixed by (instance, replication block), and a
//     second kernel reduces every instance's slots in order, so the statistics do not depend on
//     the order in which tiles ran.
#include <hip/hip_runtime.h>

#include "device_reduce.hpp"
#include "device_rng.hpp"
#include "sim_types.hpp"
#include "wave_dpp.hpp"

namespace fw {

constexpr int kWave = 64;
constexpr int kBatchMaxD = 32;
constexpr int kLaneAssets = 8;                 // assets held by one lane
// LDS staging of one wavefront: a sub-group of Pa lanes draws G d <= 4 d <= 32 Pa normals per
// round, and a wavefront has 64 / Pa sub-groups. Sub-group areas are 32 Pa + 1 floats apart (131 at
// Pa = 4): with areas 32 Pa floats apart every lane of a write or read instruction would fall in
// the same few of the 64 banks (16- to 32-way conflicts); the padded stride leaves at most two
// lanes per bank for every pattern the kernel issues (checked over all d, rounds and offsets).
constexpr int kStageFloats = kBatchStageFloats;   // max over Pa of (64 / Pa) x stride
// rows of a tile's coefficient table in LDS (binary32, indexed by asset, zero past d)
constexpr int kCoefSz = 0, kCoefC1 = 1, kCoefC2 = 2, kCoefMu = 3, kCoefW0 = 4, kCoefRows = 5;
__device__ __forceinline__ uint32_t stage_stride(uint32_t Pa) { return 32u * Pa + (Pa == 4u ? 3u : 1u); }

__device__ __forceinline__ float bfly_sum(float x, uint32_t lo, uint32_t hi)
{
    for (uint32_t m = lo; m < hi; m <<= 1) x += __shfl_xor(x, m, kWave);
    return x;
}

__device__ __forceinline__ double bfly_sum(double x, uint32_t lo, uint32_t hi)
{
    for (uint32_t m = lo; m < hi; m <<= 1) x += __shfl_xor(x, m, kWave);
    return x;
}

// Sum over the Pa <= 4 lanes of a quad-aligned group by DPP quad permutes (lane xor 1, then xor 2),
// without the LDS crossbar a shuffle goes through. Addition is commutative, so every lane of the
// group ends with the same bits. Every lane of the wavefront executes it.
__device__ __forceinline__ float quad_group_sum(float x, uint32_t Pa)
{
    if (Pa >= 2) x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0xB1, 0xF, 0xF, true));
    if (Pa >= 4) x += __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x4E, 0xF, 0xF, true));
    return x;
}

// The staging area belongs to this wavefront alone (one wavefront per workgroup), and the LDS
// instructions of a wavefront complete in issue order, so draws written by some lanes are seen by
// the reads other lanes issue after them. Only the compiler must not move LDS accesses across this
// point; no workgroup barrier (and none of its waits on outstanding global loads) is needed.
__device__ __forceinline__ void wave_lds_order()
{
    asm volatile("" ::: "memory");
    __builtin_amdgcn_wave_barrier();
    asm volatile("" ::: "memory");
}

// f(w) at w = c S over this lane's assets, FP64 (Eq. (3), diagonal Sigma), summed over the Pa lanes
__device__ __forceinline__ double tile_objective(const InstanceDesc *__restrict__ P, const uint32_t (&S)[kLaneAssets],
                                                 uint32_t hibits, uint32_t a0, uint32_t acnt, uint32_t Pa, double c)
{
    double quad = 0.0, lin = 0.0;
#pragma unroll
    for (int k = 0; k < kLaneAssets; ++k) {
        if (static_cast<uint32_t>(k) < acnt) {
            const double sj = static_cast<double>(S[k]) + ((hibits >> k) & 1u ? 4294967296.0 : 0.0);
            const double w = sj * c;
            const double sw = P->sig_d[a0 + k] * w;
            quad = fma(sw, sw, quad);
            lin = fma(P->mu_d[a0 + k], w, lin);
        }
    }
    quad = bfly_sum(quad, 1u, Pa);
    lin = bfly_sum(lin, 1u, Pa);
    return fma(P->lambda, quad, -lin);
}

__device__ __forceinline__ void run_tile(const BatchBuffers &B, const Tile tile, float *stage, float (*coef)[kBatchMaxD])
{
    const InstanceDesc *P = B.inst + tile.inst;
    const uint32_t lane = threadIdx.x;
    const uint32_t Pl = tile.P, Pa = tile.Pa;
    const uint32_t g = lane / Pl;                  // replication within the tile
    const uint32_t ps = (lane % Pl) / Pa;          // sample chunk
    const uint32_t pa = lane % Pa;                 // asset slice
    const bool active = g < tile.nrep;
    const bool owner = active && ps == 0;          // writes this lane's assets of the path record
    const bool leader = owner && pa == 0;
    const uint32_t r = tile.rep0 + g;
    const uint32_t d = P->d;
    const uint32_t a0 = pa * kLaneAssets;
    const uint32_t acnt = a0 < d ? (d - a0 < kLaneAssets ? d - a0 : kLaneAssets) : 0u;
    const uint32_t N = P->N, M = P->M;
    const uint64_t T = P->T;
    const uint32_t k0 = static_cast<uint32_t>(P->seed), k1 = static_cast<uint32_t>(P->seed >> 32);
    const uint32_t dom = P->instance & 0xFFFFFFu;
    const uint32_t n_ckpt = P->n_ckpt;
    const bool tnoise = P->noise != 0;
    const uint32_t nu = P->nu;
    const bool logged = leader && (P->flags & 2u) && (static_cast<uint64_t>(r) - P->log_begin) < P->log_count;
    const uint64_t log_count = P->log_count, log_at = P->dlog_base + (static_cast<uint64_t>(r) - P->log_begin);
    const bool has_w0 = P->has_w0 != 0;
    const float inv_n = P->inv_n_f, gap_eps = static_cast<float>(P->gap_eps), tscale = P->tscale_f;

    // The instance's binary32 coefficients, copied once into this wavefront's LDS and zero past d,
    // so the iteration reads them unconditionally (a0 + k < 4 x 8 = kBatchMaxD) and its reads issue
    // together: read from the descriptor under per-asset guards, each would wait for the one before.
    if (lane < static_cast<uint32_t>(kBatchMaxD)) {
        const bool in = lane < d;
        coef[kCoefSz][lane] = in ? P->sz_f[lane] : 0.0f;
        coef[kCoefC1][lane] = in ? P->c1_f[lane] : 0.0f;
        coef[kCoefC2][lane] = in ? P->c2_f[lane] : 0.0f;
        coef[kCoefMu][lane] = in ? P->mu_f[lane] : 0.0f;
        coef[kCoefW0][lane] = (in && has_w0) ? P->w0_f[lane] : 0.0f;
    }
    wave_lds_order();

    // G = 4/gcd(d,4) samples hold a whole number of Philox blocks; lane chunks start on such a
    // group. A round is the largest multiple of G samples whose normals fit the sub-group's 32 Pa
    // floats of staging: the blocks a round does not divide evenly among the Pa lanes (drawn and
    // discarded) are then a small share of its draws.
    const uint32_t G = (d & 3u) == 0 ? 1u : ((d & 1u) == 0 ? 2u : 4u);
    const uint32_t align = tnoise ? 4u : G;
    const uint32_t Ps = Pl / Pa;
    uint32_t chunk = (N + Ps - 1) / Ps;
    chunk = (chunk + align - 1) / align * align;
    const uint32_t i0 = ps * chunk;
    const uint32_t i_end = (i0 + chunk < N) ? i0 + chunk : N;   // this lane's samples: [i0, i_end)
    uint32_t Gr = (32u * Pa) / d / G * G;
    Gr = Gr < G ? G : Gr;
    Gr = Gr > chunk ? chunk : Gr;                  // chunk is a multiple of G
    const uint32_t rounds = (chunk + Gr - 1) / Gr;
    const uint32_t nb = Gr * d / 4;                // blocks per round
    const uint32_t mb = (nb + Pa - 1) / Pa;        // blocks per lane per round (uniform)
    float *sub = stage + (lane / Pa) * stage_stride(Pa);   // this sub-group's staging area

    uint32_t S[kLaneAssets], cnt[kLaneAssets];
#pragma unroll
    for (int k = 0; k < kLaneAssets; ++k) S[k] = cnt[k] = 0u;
    uint32_t cnt0 = 0u, hibits = 0u;
    uint32_t tau = kTauNone;
    uint32_t ck = 0;
    uint64_t next_ckpt = n_ckpt ? P->ckpt[0] : 0;
    uint32_t epoch = 0, m_in_epoch = 0;

    for (uint64_t t = 0; t < T; ++t) {
        const float cw = t == 0 ? 0.0f
                                : static_cast<float>(2.0 / (static_cast<double>(t) * static_cast<double>(t + 1)));
        // past this lane's assets S = 0 and the coefficients are 0: w = v = 0 there, as required
        float w[kLaneAssets], v[kLaneAssets], s1[kLaneAssets], s2[kLaneAssets];
#pragma unroll
        for (int k = 0; k < kLaneAssets; ++k) {
            const float wk = (t == 0) ? coef[kCoefW0][a0 + k]
                                      : (static_cast<float>(S[k]) + ((hibits >> k) & 1u ? 4294967296.0f : 0.0f)) * cw;
            w[k] = wk;
            v[k] = coef[kCoefSz][a0 + k] * wk;
            s1[k] = 0.0f;
            s2[k] = 0.0f;
        }

        const PhiloxRow row = philox_row(epoch, r, k0);
        for (uint32_t rd = 0; rd < rounds; ++rd) {
            const uint32_t ib = i0 + rd * Gr;                // first sample of the round
            const uint32_t blk0 = ib * d / 4;                // its first Philox block
            // draw: blocks pa, pa + Pa, ... of the round, two at a time
            for (uint32_t m = 0; m < mb; m += 2) {
                const uint32_t b0 = pa + m * Pa, b1 = b0 + Pa;
                const Block4<float> q0 = normals_block_row(row, blk0 + b0, dom, k0, k1);
                const Block4<float> q1 = normals_block_row(row, blk0 + b1, dom, k0, k1);
                if (b0 < nb) {
                    sub[4 * b0 + 0] = q0.z[0];
                    sub[4 * b0 + 1] = q0.z[1];
                    sub[4 * b0 + 2] = q0.z[2];
                    sub[4 * b0 + 3] = q0.z[3];
                }
                if (b1 < nb) {
                    sub[4 * b1 + 0] = q1.z[0];
                    sub[4 * b1 + 1] = q1.z[1];
                    sub[4 * b1 + 2] = q1.z[2];
                    sub[4 * b1 + 3] = q1.z[3];
                }
            }
            wave_lds_order();
            for (uint32_t sidx = 0; sidx < Gr; ++sidx) {
                const uint32_t i = ib + sidx;
                const bool valid = i < i_end;
                float z[kLaneAssets];
                const float *src = sub + sidx * d + a0;
#pragma unroll
                for (int k = 0; k < kLaneAssets; ++k) z[k] = static_cast<uint32_t>(k) < acnt ? src[k] : 0.0f;
                if (tnoise) {
                    NormalCursor<float> ext;
                    ext.seek(N * d + nu * i, epoch, r, dom, k0, k1);
                    float ss = 0.0f;
#pragma unroll 1
                    for (uint32_t q = 0; q < nu; ++q) {
                        const float e = ext.next(epoch, r, dom, k0, k1);
                        ss = fmaf(e, e, ss);
                    }
                    const float a = tscale * __builtin_amdgcn_rsqf(ss);
#pragma unroll
                    for (int k = 0; k < kLaneAssets; ++k) z[k] *= a;
                }
                float dot = 0.0f;
#pragma unroll
                for (int k = 0; k < kLaneAssets; ++k) dot = fmaf(z[k], v[k], dot);
                dot = quad_group_sum(dot, Pa);
                if (valid) {
#pragma unroll
                    for (int k = 0; k < kLaneAssets; ++k) {
                        s1[k] += z[k];
                        s2[k] = fmaf(z[k], dot, s2[k]);
                    }
                }
            }
            wave_lds_order();
        }
        // combine the Ps sample chunks (lanes holding the same assets)
        for (uint32_t m = Pa; m < Pl; m <<= 1) {
#pragma unroll
            for (int k = 0; k < kLaneAssets; ++k) {
                s1[k] += __shfl_xor(s1[k], m, kWave);
                s2[k] += __shfl_xor(s2[k], m, kWave);
            }
        }

        // gradient, linear subproblem over the vertices of W, Frank-Wolfe gap
        float dot1 = 0.0f;
#pragma unroll
        for (int k = 0; k < kLaneAssets; ++k) dot1 = fmaf(s1[k], v[k], dot1);
        dot1 = bfly_sum(dot1, 1u, Pa);
        const float qn = dot1 * inv_n;
        float c1[kLaneAssets], c2[kLaneAssets], mu[kLaneAssets];
#pragma unroll
        for (int k = 0; k < kLaneAssets; ++k) {
            c1[k] = coef[kCoefC1][a0 + k];
            c2[k] = coef[kCoefC2][a0 + k];
            mu[k] = coef[kCoefMu][a0 + k];
        }
        float gmin = INFINITY, gw = 0.0f;
        uint32_t jmin = 0xFFFFFFFFu;
#pragma unroll
        for (int k = 0; k < kLaneAssets; ++k) {
            if (static_cast<uint32_t>(k) < acnt) {
                const uint32_t j = a0 + k;
                const float gj = fmaf(-c1[k], s1[k], fmaf(c2[k], fmaf(-s1[k], qn, s2[k]), -mu[k]));
                if (jmin == 0xFFFFFFFFu || gj < gmin) {
                    gmin = gj;
                    jmin = j;
                }
                gw = fmaf(gj, w[k], gw);
            }
        }
        for (uint32_t m = 1; m < Pa; m <<= 1) {
            const float og = __shfl_xor(gmin, m, kWave);
            const uint32_t oj = __shfl_xor(jmin, m, kWave);
            if (og < gmin || (og == gmin && oj < jmin)) {
                gmin = og;
                jmin = oj;
            }
        }
        gw = bfly_sum(gw, 1u, Pa);
        const uint32_t a = (gmin < 0.0f) ? jmin + 1 : 0u;
        const float gap = gw - (gmin < 0.0f ? gmin : 0.0f);
        if (tau == kTauNone && gap <= gap_eps) tau = static_cast<uint32_t>(t);
        if (logged) B.dlog[log_at + t * log_count] = static_cast<uint8_t>(a);

        // step 2/(t+2): the signature absorbs the update
        cnt0 += (a == 0u) ? 1u : 0u;
#pragma unroll
        for (int k = 0; k < kLaneAssets; ++k) {
            if (a == a0 + k + 1) {
                const uint32_t now = S[k] + static_cast<uint32_t>(t + 1);
                if (now < S[k]) hibits |= 1u << k;
                S[k] = now;
                cnt[k] += 1u;
            }
        }
        if (t + 1 == next_ckpt) {
            const double c = 2.0 / (static_cast<double>(t + 1) * static_cast<double>(t + 2));
            const double f = tile_objective(P, S, hibits, a0, acnt, Pa, c);
            if (leader) B.fck[static_cast<uint64_t>(ck) * B.total_R + P->path_base + r] = f;
            ++ck;
            next_ckpt = ck < n_ckpt ? P->ckpt[ck] : 0;
        }
        if (++m_in_epoch == M) {
            m_in_epoch = 0;
            ++epoch;
        }
    }
    const double y = tile_objective(P, S, hibits, a0, acnt, Pa, 2.0 / (static_cast<double>(T) * static_cast<double>(T + 1)));

    if (owner && B.y) {
        const uint64_t R = P->R;
        if (pa == 0) {
            B.y[P->path_base + r] = y;
            B.tau[P->path_base + r] = tau;
            B.cnt[P->cnt_base + r] = cnt0;
        }
#pragma unroll
        for (int k = 0; k < kLaneAssets; ++k) {
            if (static_cast<uint32_t>(k) < acnt) {
                const uint64_t j = a0 + k;
                B.cnt[P->cnt_base + (j + 1) * R + r] = cnt[k];
                B.wsum[P->wsum_base + j * R + r] =
                    static_cast<uint64_t>(S[k]) | (static_cast<uint64_t>((hibits >> k) & 1u) << 32);
            }
        }
    }

    // tile partials (leaders only)
    TilePartial &out = B.partials[tile.slot];
    for (uint32_t s = 0; s < kTileStreams; ++s) {
        if (s >= 1 + 2 * n_ckpt) {
            if (lane == 0)
                for (int f = 0; f < kStreamFields; ++f) out.f[s * kStreamFields + f] = 0.0;
            continue;
        }
        double x = 0.0;
        bool valid = leader;
        if (leader) {
            if (s == 0) {
                x = y;
            } else if (s <= n_ckpt) {
                x = B.fck[static_cast<uint64_t>(s - 1) * B.total_R + P->path_base + r];
            } else {
                const double f = B.fck[static_cast<uint64_t>(s - 1 - n_ckpt) * B.total_R + P->path_base + r];
                valid = (f != 0.0);
                const double e = valid ? (f - y) / f : 0.0;
                x = e * e;
            }
        }
        if (!valid) x = 0.0;
        double h = x, l = 0.0, qh = x * x, ql = fma(x, x, -(x * x)), ch = valid ? 1.0 : 0.0, cl = 0.0;
        wave_sum_dd(h, l);
        wave_sum_dd(qh, ql);
        wave_sum_dd(ch, cl);
        if (lane == 0) {
            double *o = out.f + s * kStreamFields;
            o[0] = h;
            o[1] = l;
            o[2] = qh;
            o[3] = ql;
            o[4] = ch + cl;
        }
    }
    const double mn = wave_extreme<false>(leader ? y : INFINITY);
    const double mx = wave_extreme<true>(leader ? y : -INFINITY);
    if (lane == 0) {
        out.ymin = mn;
        out.ymax = mx;
    }
    {
        const uint64_t tot = wave_sum_u64(leader ? cnt0 : 0u);
        if (lane == 0) out.dec[0] = tot;
    }
    for (uint32_t j = 0; j < static_cast<uint32_t>(kBatchMaxD); ++j) {
        uint32_t c = 0u;
#pragma unroll
        for (int k = 0; k < kLaneAssets; ++k)
            if (a0 + k == j) c = cnt[k];
        const uint64_t tot = wave_sum_u64((owner && j < d) ? c : 0u);
        if (lane == 0) out.dec[j + 1] = tot;
    }
    const bool hit = leader && tau != kTauNone;
    const uint64_t tc = wave_sum_u64(hit ? 1u : 0u);
    const uint64_t ts = wave_sum_u64(hit ? tau : 0u);
    if (lane == 0) {
        out.tau_count = tc;
        out.tau_sum = ts;
    }
}

// Sums and (value, index) minima over the 32 lanes of each half wavefront on DPP and the 16-lane row
// swap (wave_dpp.hpp); the FP64 sum keeps the shuffle butterfly (checkpoints only).
__device__ __forceinline__ float half_sum32(float x) { return dpp_sum32(x); }

__device__ __forceinline__ void half_argmin32(float &g, uint32_t &j) { dpp_argmin32(g, j); }

__device__ __forceinline__ double half_sum32(double x)
{
#pragma unroll
    for (int m = 1; m < 32; m <<= 1) x += __shfl_xor(x, m, 32);
    return x;
}

// One replication per wavefront (every tile of P = 64 lanes, Gaussian noise, N d + 3 <= the
// staging area): lane j < d holds asset j (d <= 32, so the assets sit in the first half wavefront).
// Lane i forms sample i's dot product with v = sz .* w, lane j the sums over the samples of z_ij
// and z_ij (z_i'v); the gradient, its minimum (lowest index among equal values) and g'w are reduced
// over the first half wavefront. Same formulas as the tile kernel, summed in a different order.
// A second wavefront of the workgroup draws the next epoch's N d normals (a Philox block per lane
// at a time) into the other of two LDS buffers while the first runs the iteration on the current
// one; one workgroup barrier per iteration hands the buffers over. The normals do not depend on
// the iterate, so the draw leaves the iteration's dependent chain.
__device__ __forceinline__ void run_wave(const BatchBuffers &B, const Tile tile, float *zs, float *vs, float *dots)
{
    const InstanceDesc *P = B.inst + tile.inst;
    const uint32_t lane = threadIdx.x % kWave;
    const bool drawer = threadIdx.x >= kWave;          // the second wavefront: the next epoch's normals
    const uint32_t r = tile.rep0;
    const uint32_t d = P->d, N = P->N, M = P->M, nd = N * d, nb = (nd + 3) / 4;
    const uint64_t T = P->T;
    const uint32_t k0 = static_cast<uint32_t>(P->seed), k1 = static_cast<uint32_t>(P->seed >> 32);
    const uint32_t dom = P->instance & 0xFFFFFFu;
    const uint32_t n_ckpt = P->n_ckpt;
    const bool logged = lane == 0 && (P->flags & 2u) && (static_cast<uint64_t>(r) - P->log_begin) < P->log_count;
    const uint64_t log_count = P->log_count, log_at = P->dlog_base + (static_cast<uint64_t>(r) - P->log_begin);
    const bool in = lane < d;
    const uint32_t jc = in ? lane : 0u;
    const float sz = in ? P->sz_f[jc] : 0.0f, c1 = P->c1_f[jc], c2 = P->c2_f[jc], mu = P->mu_f[jc];
    const float w0 = (in && P->has_w0) ? P->w0_f[jc] : 0.0f;
    const double sig_d = in ? P->sig_d[jc] : 0.0, mu_d = in ? P->mu_d[jc] : 0.0, lambda = P->lambda;
    const float inv_n = P->inv_n_f, gap_eps = static_cast<float>(P->gap_eps);

    uint32_t S = 0u, cnt = 0u, cnt0 = 0u, hib = 0u;
    uint32_t tau = kTauNone, ck = 0, epoch = 0, m_in_epoch = 0;
    uint64_t next_ckpt = n_ckpt ? P->ckpt[0] : 0;
    float cw = 0.0f;   // w_t = cw S for t >= 1
    // f(w) at w = c S, FP64 (Eq. (3), diagonal Sigma), summed over the assets' lanes
    auto objective = [&](double c) {
        const double w = (static_cast<double>(S) + (hib ? 4294967296.0 : 0.0)) * c;
        const double sw = sig_d * w;
        const double quad = half_sum32(in ? sw * sw : 0.0);
        const double lin = half_sum32(in ? mu_d * w : 0.0);
        return fma(lambda, quad, -lin);
    };

    // the normals of epoch e into buffer e mod 2, blocks b = first, first + stride, ...
    auto draw = [&](uint32_t e, uint32_t first, uint32_t stride) {
        const PhiloxRow row = philox_row(e, r, k0);
        float *dst = zs + (e & 1u) * kStageFloats;
        for (uint32_t b = first; b < nb; b += stride) {
            const Block4<float> q = normals_block_row(row, b, dom, k0, k1);
            dst[4 * b + 0] = q.z[0];
            dst[4 * b + 1] = q.z[1];
            dst[4 * b + 2] = q.z[2];
            dst[4 * b + 3] = q.z[3];
        }
    };
    draw(0u, threadIdx.x, 2 * kWave);
    __syncthreads();

    for (uint64_t t = 0; t < T; ++t) {
        if (drawer) {
            // epoch + 1 goes to the buffer the iteration does not read; it was last read before the
            // previous barrier
            if (m_in_epoch + 1 == M && t + 1 < T) draw(epoch + 1, lane, kWave);
        } else {
            const float *zc = zs + (epoch & 1u) * kStageFloats;
            const float w = (t == 0) ? w0 : (static_cast<float>(S) + (hib ? 4294967296.0f : 0.0f)) * cw;
            const float v = sz * w;
            if (lane < 32) vs[lane] = v;
            wave_lds_order();
            for (uint32_t i = lane; i < N; i += kWave) {
                float dot = 0.0f;
#pragma unroll 8
                for (uint32_t j = 0; j < d; ++j) dot = fmaf(zc[i * d + j], vs[j], dot);
                dots[i] = dot;
            }
            wave_lds_order();
            float s1 = 0.0f, s2 = 0.0f;
            if (in) {
#pragma unroll 8
                for (uint32_t i = 0; i < N; ++i) {
                    const float z = zc[i * d + lane];
                    s1 += z;
                    s2 = fmaf(z, dots[i], s2);
                }
            }
            wave_lds_order();                               // vs and dots are rewritten next iteration
            // the next iteration's scale 2/((t+1)(t+2)), its FP64 division beside the reductions
            // rather than at the head of the next iteration's chain
            const float cw_next =
                static_cast<float>(2.0 / (static_cast<double>(t + 1) * static_cast<double>(t + 2)));
            const float qn = half_sum32(s1 * v) * inv_n;
            float g = INFINITY;
            uint32_t jg = 0xFFFFFFFFu;
            if (in) {
                g = fmaf(-c1, s1, fmaf(c2, fmaf(-s1, qn, s2), -mu));
                jg = lane;
            }
            const float gw = half_sum32(in ? g * w : 0.0f);
            half_argmin32(g, jg);
            const uint32_t a = (g < 0.0f) ? jg + 1 : 0u;
            const float gap = gw - (g < 0.0f ? g : 0.0f);
            if (tau == kTauNone && gap <= gap_eps) tau = static_cast<uint32_t>(t);
            if (logged) B.dlog[log_at + t * log_count] = static_cast<uint8_t>(a);
            // step 2/(t+2): the signature absorbs the update
            cnt0 += (a == 0u) ? 1u : 0u;
            if (a == lane + 1) {
                const uint32_t now = S + static_cast<uint32_t>(t + 1);
                if (now < S) hib = 1u;
                S = now;
                cnt += 1u;
            }
            if (t + 1 == next_ckpt) {
                const double f = objective(2.0 / (static_cast<double>(t + 1) * static_cast<double>(t + 2)));
                if (lane == 0) B.fck[static_cast<uint64_t>(ck) * B.total_R + P->path_base + r] = f;
                ++ck;
                next_ckpt = ck < n_ckpt ? P->ckpt[ck] : 0;
            }
            cw = cw_next;
        }
        __syncthreads();   // both wavefronts: the drawn buffer is complete and the read one is free
        if (++m_in_epoch == M) {
            m_in_epoch = 0;
            ++epoch;
        }
    }
    if (drawer) return;
    const double y = objective(2.0 / (static_cast<double>(T) * static_cast<double>(T + 1)));

    if (B.y) {
        const uint64_t R = P->R;
        if (lane == 0) {
            B.y[P->path_base + r] = y;
            B.tau[P->path_base + r] = tau;
            B.cnt[P->cnt_base + r] = cnt0;
        }
        if (in) {
            B.cnt[P->cnt_base + (static_cast<uint64_t>(lane) + 1) * R + r] = cnt;
            B.wsum[P->wsum_base + static_cast<uint64_t>(lane) * R + r] =
                static_cast<uint64_t>(S) | (static_cast<uint64_t>(hib) << 32);
        }
    }

    // the tile's partial record (one replication): its streams, extremes, decision totals and tau
    TilePartial &out = B.partials[tile.slot];
    if (lane == 0) {
        for (uint32_t s = 0; s < kTileStreams; ++s) {
            double *o = out.f + s * kStreamFields;
            if (s >= 1 + 2 * n_ckpt) {
                for (int f = 0; f < kStreamFields; ++f) o[f] = 0.0;
                continue;
            }
            double x;
            bool valid = true;
            if (s == 0) {
                x = y;
            } else if (s <= n_ckpt) {
                x = B.fck[static_cast<uint64_t>(s - 1) * B.total_R + P->path_base + r];
            } else {
                const double f = B.fck[static_cast<uint64_t>(s - 1 - n_ckpt) * B.total_R + P->path_base + r];
                valid = (f != 0.0);
                const double e = valid ? (f - y) / f : 0.0;
                x = e * e;
            }
            if (!valid) x = 0.0;
            o[0] = x;
            o[1] = 0.0;
            o[2] = x * x;
            o[3] = fma(x, x, -(x * x));
            o[4] = valid ? 1.0 : 0.0;
        }
        out.ymin = y;
        out.ymax = y;
        out.dec[0] = cnt0;
        out.tau_count = tau != kTauNone ? 1u : 0u;
        out.tau_sum = tau != kTauNone ? tau : 0u;
    }
    if (lane < static_cast<uint32_t>(kBatchMaxD)) out.dec[lane + 1] = in ? cnt : 0u;
}

// One wavefront per tile, every tile of the batch, longest first.
__global__ __launch_bounds__(kWave) void fw_tile_kernel(BatchBuffers B)
{
    __shared__ float stage[kStageFloats];
    __shared__ float coef[kCoefRows][kBatchMaxD];
    const Tile tile = B.tiles[blockIdx.x];
    run_tile(B, tile, stage, coef);
}

// One replication per workgroup of two wavefronts (the iteration, the next epoch's normals), every
// tile of a batch that qualifies (BatchBuffers.wave_mode).
__global__ __launch_bounds__(2 * kWave) void fw_wave_kernel(BatchBuffers B)
{
    __shared__ float zs[2 * kStageFloats];
    __shared__ float vs[32];
    __shared__ float dots[kStageFloats];
    const Tile tile = B.tiles[blockIdx.x];
    run_wave(B, tile, zs, vs, dots);
}

// One workgroup per instance: its tile slots in order.
__global__ __launch_bounds__(kBlock) void fw_batch_reduce(BatchBuffers B)
{
    __shared__ double sm_f[2 * (kBlock / 64)];
    __shared__ uint64_t sm_i[kBlock / 64];
    const uint32_t i = blockIdx.x;
    const uint32_t b0 = B.slot_begin[i], b1 = B.slot_begin[i + 1];
    TilePartial &o = B.final_stats[i];
    for (int s = 0; s < kTileStreams; ++s) {
        double h = 0.0, l = 0.0, qh = 0.0, ql = 0.0, ch = 0.0, cl = 0.0;
        for (uint32_t b = b0 + threadIdx.x; b < b1; b += kBlock) {
            const double *f = B.partials[b].f + s * kStreamFields;
            dd_add(h, l, f[0], f[1]);
            dd_add(qh, ql, f[2], f[3]);
            dd_add(ch, cl, f[4], 0.0);
        }
        block_sum_dd(h, l, sm_f);
        block_sum_dd(qh, ql, sm_f);
        block_sum_dd(ch, cl, sm_f);
        if (threadIdx.x == 0) {
            double *f = o.f + s * kStreamFields;
            f[0] = h;
            f[1] = l;
            f[2] = qh;
            f[3] = ql;
            f[4] = ch + cl;
        }
    }
    double mn = INFINITY, mx = -INFINITY;
    for (uint32_t b = b0 + threadIdx.x; b < b1; b += kBlock) {
        mn = fmin(mn, B.partials[b].ymin);
        mx = fmax(mx, B.partials[b].ymax);
    }
    mn = block_extreme<false>(mn, sm_f);
    mx = block_extreme<true>(mx, sm_f);
    if (threadIdx.x == 0) {
        o.ymin = mn;
        o.ymax = mx;
    }
    for (int j = 0; j < 33 + 2; ++j) {
        uint64_t x = 0;
        for (uint32_t b = b0 + threadIdx.x; b < b1; b += kBlock)
            x += j < 33 ? B.partials[b].dec[j] : (j == 33 ? B.partials[b].tau_count : B.partials[b].tau_sum);
        x = block_sum_u64(x, sm_i);
        if (threadIdx.x == 0) {
            if (j < 33) o.dec[j] = x;
            else if (j == 33) o.tau_count = x;
            else o.tau_sum = x;
        }
    }
}

// the tile kernel over every tile, then the per-instance reduction, in stream order
int launch_fw_batch(const BatchBuffers &B, hipStream_t stream)
{
    if (B.n_tiles) {
        if (B.wave_mode) hipLaunchKernelGGL(fw_wave_kernel, dim3(B.n_tiles), dim3(2 * kWave), 0, stream, B);
        else hipLaunchKernelGGL(fw_tile_kernel, dim3(B.n_tiles), dim3(kWave), 0, stream, B);
    }
    hipLaunchKernelGGL(fw_batch_reduce, dim3(B.n_inst), dim3(kBlock), 0, stream, B);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace fw
