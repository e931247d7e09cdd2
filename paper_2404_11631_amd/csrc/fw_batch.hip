// fw_batch.hip -- instances of uneven size and horizon, as wavefront tiles.
//
// Algorithm 1 (Section 3.1) exactly as in fw_paths.hip, reorganised for a batch of instances:
//   * one wavefront per tile; the tiles of each (d bucket, noise) class are launched longest
//     first, so the hardware dispatcher acts as the work queue;
//   * a tile holds 64/P replications of one instance, P lanes per replication; each lane takes
//     a contiguous chunk of the N samples (chunks are multiples of 4/gcd(d,4) samples, so every
//     lane starts on a Philox block boundary and all lanes walk the stream in step), and the P
//     partial sums s1, s2 are combined with an xor butterfly, after which every lane of the group
//     holds the same bits and takes the same decision;
//   * the integer signature S_j and the decision counts live in LDS, one slot per lane
//     ([j][lane], conflict-free); the top bit of S_j (T up to 1e5 needs 33 bits) sits in a
//     per-lane bit mask;
//   * one kernel per class, specialised for d <= 4, 8, 16 and 32 (register arrays of that width);
//   * each tile writes its partial sums to a slot fixed by (instance, replication block), and a
//     second kernel reduces every instance's slots in order, so the statistics do not depend on
//     the order in which tiles ran.
#include <hip/hip_runtime.h>

#include "device_reduce.hpp"
#include "device_rng.hpp"
#include "sim_types.hpp"

namespace fw {

constexpr int kWave = 64;
constexpr int kBatchMaxD = 32;

template <int D>
struct TileLds {
    uint32_t s_lo[D][kWave];        // signature S_j mod 2^32
    uint32_t cnt[D + 1][kWave];     // decision counts, origin first
};

__device__ __forceinline__ double signature(uint32_t lo, uint32_t hibits, int j)
{
    return static_cast<double>(lo) + ((hibits >> j) & 1u ? 4294967296.0 : 0.0);
}

// f(w) at w = c S, FP64 (Eq. (3), diagonal Sigma)
template <int D>
__device__ __forceinline__ double batch_objective(const InstanceDesc *__restrict__ P, const TileLds<D> &L,
                                                  int lane, uint32_t hibits, int d, double c)
{
    double quad = 0.0, lin = 0.0;
#pragma unroll
    for (int j = 0; j < D; ++j) {
        if (j < d) {
            const double w = signature(L.s_lo[j][lane], hibits, j) * c;
            const double sw = P->sig_d[j] * w;
            quad += sw * sw;
            lin += P->mu_d[j] * w;
        }
    }
    return P->lambda * quad - lin;
}

template <int D, int NOISE>
__device__ __forceinline__ void run_tile(const BatchBuffers &B, const Tile tile, TileLds<D> &L)
{
    const InstanceDesc *P = B.inst + tile.inst;
    const int lane = threadIdx.x;
    const uint32_t Pl = tile.P;
    const uint32_t g = lane / Pl, p = lane % Pl;
    const bool active = g < tile.nrep;
    const bool leader = active && p == 0;
    const uint32_t r = tile.rep0 + g;
    const int d = static_cast<int>(P->d);
    const uint32_t N = P->N, M = P->M;
    const uint64_t T = P->T;
    const uint32_t k0 = static_cast<uint32_t>(P->seed), k1 = static_cast<uint32_t>(P->seed >> 32);
    const uint32_t dom = P->instance & 0xFFFFFFu;
    const uint32_t n_ckpt = P->n_ckpt;
    const bool logged = leader && (P->flags & 2u) && (static_cast<uint64_t>(r) - P->log_begin) < P->log_count;

    // contiguous sample chunk of this lane, aligned to whole Philox blocks
    const uint32_t align = NOISE ? 4u : ((d & 3) == 0 ? 1u : ((d & 1) == 0 ? 2u : 4u));
    uint32_t chunk = (N + Pl - 1) / Pl;
    chunk = (chunk + align - 1) / align * align;
    const uint32_t i0 = p * chunk;

#pragma unroll
    for (int j = 0; j < D; ++j) L.s_lo[j][lane] = 0u;
#pragma unroll
    for (int j = 0; j <= D; ++j) L.cnt[j][lane] = 0u;
    uint32_t hibits = 0u;
    uint32_t tau = kTauNone;
    uint32_t ck = 0;
    uint64_t next_ckpt = n_ckpt ? P->ckpt[0] : 0;
    uint32_t epoch = 0, m_in_epoch = 0;

    for (uint64_t t = 0; t < T; ++t) {
        // reload the per-instance coefficients from the scalar cache every iteration instead of
        // keeping 5 x D of them live across the sample loop
        asm volatile("" ::: "memory");
        const float cw = t == 0 ? 0.0f
                                : static_cast<float>(2.0 / (static_cast<double>(t) * static_cast<double>(t + 1)));
        float v[D], s1[D], s2[D];
#pragma unroll
        for (int j = 0; j < D; ++j) {
            float w = 0.0f;
            if (j < d) {
                w = (t == 0) ? (P->has_w0 ? P->w0_f[j] : 0.0f)
                             : (static_cast<float>(L.s_lo[j][lane]) + ((hibits >> j) & 1u ? 4294967296.0f : 0.0f)) * cw;
            }
            v[j] = (j < d) ? P->sz_f[j] * w : 0.0f;
            s1[j] = 0.0f;
            s2[j] = 0.0f;
        }

        NormalCursor<float> cur;
        cur.seek(i0 * static_cast<uint32_t>(d), epoch, r, dom, k0, k1);
        NormalCursor<float> ext;
        if constexpr (NOISE == 1) ext.seek(N * static_cast<uint32_t>(d) + P->nu * i0, epoch, r, dom, k0, k1);
#pragma unroll 1
        for (uint32_t k = 0; k < chunk; ++k) {
            const bool valid = i0 + k < N;
            float z[D];
#pragma unroll
            for (int j = 0; j < D; ++j) z[j] = (j < d) ? cur.next(epoch, r, dom, k0, k1) : 0.0f;
            if constexpr (NOISE == 1) {
                float ss = 0.0f;
#pragma unroll 1
                for (uint32_t q = 0; q < P->nu; ++q) {
                    const float e = ext.next(epoch, r, dom, k0, k1);
                    ss = fmaf(e, e, ss);
                }
                const float a = P->tscale_f * __builtin_amdgcn_rsqf(ss);
#pragma unroll
                for (int j = 0; j < D; ++j) z[j] *= a;
            }
            if (valid) {
                float dot = 0.0f;
#pragma unroll
                for (int j = 0; j < D; ++j) dot = fmaf(z[j], v[j], dot);
#pragma unroll
                for (int j = 0; j < D; ++j) {
                    s1[j] += z[j];
                    s2[j] = fmaf(z[j], dot, s2[j]);
                }
            }
        }
        // combine the P partial sums (xor butterfly: every lane of the group ends with equal bits)
        for (uint32_t m = 1; m < Pl; m <<= 1) {
#pragma unroll
            for (int j = 0; j < D; ++j) {
                if (j < d) {
                    s1[j] += __shfl_xor(s1[j], m, kWave);
                    s2[j] += __shfl_xor(s2[j], m, kWave);
                }
            }
        }

        float dot1 = 0.0f;
#pragma unroll
        for (int j = 0; j < D; ++j) dot1 = fmaf(s1[j], v[j], dot1);
        const float qn = dot1 * P->inv_n_f;
        float gmin = 0.0f, gw = 0.0f;
        int jmin = -1;
#pragma unroll
        for (int j = 0; j < D; ++j) {
            if (j < d) {
                const float gj = P->c2_f[j] * (s2[j] - s1[j] * qn) - P->mu_f[j] - P->c1_f[j] * s1[j];
                if (jmin < 0 || gj < gmin) {
                    gmin = gj;
                    jmin = j;
                }
                const float w = (t == 0) ? (P->has_w0 ? P->w0_f[j] : 0.0f)
                                         : (static_cast<float>(L.s_lo[j][lane]) + ((hibits >> j) & 1u ? 4294967296.0f : 0.0f)) * cw;
                gw = fmaf(gj, w, gw);
            }
        }
        const int a = (gmin < 0.0f) ? jmin + 1 : 0;
        const float gap = gw - (gmin < 0.0f ? gmin : 0.0f);
        if (tau == kTauNone && gap <= static_cast<float>(P->gap_eps)) tau = static_cast<uint32_t>(t);
        if (logged) B.dlog[P->dlog_base + t * P->log_count + (r - P->log_begin)] = static_cast<uint8_t>(a);

        if (active) {
            L.cnt[a][lane] += 1u;
            if (a > 0) {
                const uint32_t old = L.s_lo[a - 1][lane];
                const uint32_t now = old + static_cast<uint32_t>(t + 1);
                L.s_lo[a - 1][lane] = now;
                if (now < old) hibits |= 1u << (a - 1);
            }
        }
        if (t + 1 == next_ckpt) {
            const double c = 2.0 / (static_cast<double>(t + 1) * static_cast<double>(t + 2));
            const double f = batch_objective<D>(P, L, lane, hibits, d, c);
            if (leader) B.fck[static_cast<uint64_t>(ck) * B.total_R + P->path_base + r] = f;
            ++ck;
            next_ckpt = ck < n_ckpt ? P->ckpt[ck] : 0;
        }
        if (++m_in_epoch == M) {
            m_in_epoch = 0;
            ++epoch;
        }
    }
    const double y = batch_objective<D>(P, L, lane, hibits, d, 2.0 / (static_cast<double>(T) * static_cast<double>(T + 1)));

    if (leader && B.y) {
        const uint64_t R = P->R;
        B.y[P->path_base + r] = y;
        B.tau[P->path_base + r] = tau;
        for (int j = 0; j <= d; ++j) B.cnt[P->cnt_base + static_cast<uint64_t>(j) * R + r] = L.cnt[j][lane];
        for (int j = 0; j < d; ++j)
            B.wsum[P->wsum_base + static_cast<uint64_t>(j) * R + r] =
                static_cast<uint64_t>(L.s_lo[j][lane]) | (static_cast<uint64_t>((hibits >> j) & 1u) << 32);
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
    for (int j = 0; j <= kBatchMaxD; ++j) {
        const uint64_t tot = wave_sum_u64((leader && j <= d && j <= D) ? L.cnt[j <= D ? j : 0][lane] : 0u);
        if (lane == 0) out.dec[j] = tot;
    }
    const bool hit = leader && tau != kTauNone;
    const uint64_t tc = wave_sum_u64(hit ? 1u : 0u);
    const uint64_t ts = wave_sum_u64(hit ? tau : 0u);
    if (lane == 0) {
        out.tau_count = tc;
        out.tau_sum = ts;
    }
}

// One wavefront per tile: the tiles of one (d bucket, noise) class, longest first, so the hardware
// dispatcher hands the heaviest tiles out first and fills in with the lighter ones.
template <int D, int NOISE>
__global__ __launch_bounds__(kWave) void fw_tile_kernel(BatchBuffers B, uint32_t first_tile)
{
    __shared__ TileLds<D> L;
    const Tile tile = B.tiles[first_tile + blockIdx.x];
    run_tile<D, NOISE>(B, tile, L);
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

// tile kernels of every class present, then the per-instance reduction, in stream order;
// class_begin[c] .. class_begin[c+1] are the tiles of class c = 2 bucket + noise
int launch_fw_batch(const BatchBuffers &B, const uint32_t *class_begin, hipStream_t stream)
{
    using K = void (*)(BatchBuffers, uint32_t);
    static const K kernels[8] = {fw_tile_kernel<4, 0>, fw_tile_kernel<4, 1>, fw_tile_kernel<8, 0>,
                                 fw_tile_kernel<8, 1>, fw_tile_kernel<16, 0>, fw_tile_kernel<16, 1>,
                                 fw_tile_kernel<32, 0>, fw_tile_kernel<32, 1>};
    for (int c = 7; c >= 0; --c) {
        const uint32_t n = class_begin[c + 1] - class_begin[c];
        if (n) hipLaunchKernelGGL(kernels[c], dim3(n), dim3(kWave), 0, stream, B, class_begin[c]);
    }
    hipLaunchKernelGGL(fw_batch_reduce, dim3(B.n_inst), dim3(kBlock), 0, stream, B);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace fw
