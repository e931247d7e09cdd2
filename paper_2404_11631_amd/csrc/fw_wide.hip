// fw_wide.hip -- Algorithm 1 (Section 3.1) at the paper's experimental shape (Section 4.1): a few
// replications of an instance with many assets (d up to 1e5), Sigma = diag(sigma^2), N = 25-50
// Gaussian samples per gradient, FP32 state.
//
// Parallelism is inside a replication: a workgroup owns 128 assets (32 quads of four consecutive
// assets, one Philox block per quad and sample) and splits the N samples over 8 chunks. One
// iteration is three launches and a step:
//   sample    z_i for the workgroup's assets; z_i'v summed over the workgroup (per sample) and
//             s1 = sum_i z_i per asset; workgroup partials of s1'v,
//   dot       z_i'v and s1'v over the workgroups of the replication (fixed order),
//   gradient  z_i again (same counters), s2 = sum_i z_i (z_i'v), the gradient
//             g = c2 (s2 - s1 (s1'v)/N) - mu - c1 s1 of Eq. (4)-(5) in noise coordinates, the
//             workgroup's smallest g_j (lowest index among equal values) and its part of g'w,
//   step      the vertex over all workgroups, the Frank-Wolfe gap and tau, and the integer update
//             S_a += t + 1 of the chosen vertex (w_{t+1} = 2 S / ((t+1)(t+2)), Algorithm 1's
//             recurrence in exact arithmetic). It runs at the start of the next iteration's sample
//             launch (every workgroup reduces the same partials in the same order; the partials
//             alternate between two buffers), and in a launch of its own only before an objective
//             evaluation and after the last iteration.
// Every sum runs in a fixed order, so a run is reproducible bit for bit. The normals are those of
// the per-lane path kernels (standard normal q = i d + j of the (replication, epoch) stream),
// scaled by 1/sqrt(2 ln 2), which the host folds into sz = sqrt(2 ln 2) sigma.
#include <hip/hip_runtime.h>

#include "device_reduce.hpp"
#include "sim.h"
#include "device_rng.hpp"
#include "sim_types.hpp"
#include "wave_dpp.hpp"
#include "wide.hpp"

namespace fw {

namespace {

// Sums and (value, index) minima (lowest index among equal values) over the 32 lanes of a half
// wavefront (the lanes of one sample chunk) or over the 64 of a wavefront; every lane gets the
// result. The DPP exchanges pair lanes as the xor butterfly 1, 2, ... does, so the sums' rounding is
// that butterfly's.
__device__ __forceinline__ float half_sum(float x) { return dpp_sum32(x); }

__device__ __forceinline__ void half_argmin(float &g, uint32_t &j) { dpp_argmin32(g, j); }

__device__ __forceinline__ float wave64_sum(float x) { return dpp_sum64(x); }

__device__ __forceinline__ void wave64_argmin(float &g, uint32_t &j) { dpp_argmin64(g, j); }

// A quad's signature words, scaled sigma and start point, loaded together (d is a multiple of 4 and
// every array starts 16-byte aligned, so each is one or two 16-byte words); qc is a quad in range.
struct WideQuad {
    uint64_t S[4];
    float sz[4], w0[4];
};

__device__ __forceinline__ WideQuad wide_load_quad(const WideArgs &A, uint32_t r, uint32_t qc)
{
    WideQuad Q;
    const ulonglong2 *sp = reinterpret_cast<const ulonglong2 *>(A.S + static_cast<uint64_t>(r) * A.d + 4 * qc);
    const ulonglong2 s01 = sp[0], s23 = sp[1];
    const float4 sz = *reinterpret_cast<const float4 *>(A.sz_f + 4 * qc);
    const float4 w0 = *reinterpret_cast<const float4 *>(A.w0_f + 4 * qc);
    Q.S[0] = s01.x;
    Q.S[1] = s01.y;
    Q.S[2] = s23.x;
    Q.S[3] = s23.y;
    Q.sz[0] = sz.x;
    Q.sz[1] = sz.y;
    Q.sz[2] = sz.z;
    Q.sz[3] = sz.w;
    Q.w0[0] = w0.x;
    Q.w0[1] = w0.y;
    Q.w0[2] = w0.z;
    Q.w0[3] = w0.w;
    return Q;
}

// w_t of the quad's four assets and v = sz .* w_t (zero for a quad past the last)
__device__ __forceinline__ void wide_iterate(const WideQuad &Q, bool active, float cw, bool from_w0, float (&w)[4],
                                             float (&v)[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        w[k] = 0.0f;
        v[k] = 0.0f;
        if (active) {
            w[k] = from_w0 ? Q.w0[k] : static_cast<float>(static_cast<double>(Q.S[k])) * cw;
            v[k] = Q.sz[k] * w[k];
        }
    }
}

// The vertex over the workgroup partials of replication r (buffer par): the smallest gradient entry
// (lowest asset among equal values: the workgroups cover ascending asset ranges, so strict < over
// them in order keeps the lowest), the sum of the g'w parts, then the vertex a (0: the origin) and the
// Frank-Wolfe gap. Every thread of the kWideBlock-thread workgroup takes part and gets a; the order
// of the sums is fixed, so every workgroup that calls it gets the same bits.
__device__ __forceinline__ uint32_t wide_reduce_step(const WideArgs &A, uint32_t r, uint32_t par, float *smg, float *smw,
                                                     uint32_t *smj, float &gap)
{
    const uint32_t tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const uint64_t base = (static_cast<uint64_t>(par) * A.R + r) * A.nwg;
    float gmin = INFINITY, gw = 0.0f;
    uint32_t jmin = 0xFFFFFFFFu;
    for (uint32_t g = tid; g < A.nwg; g += kWideBlock) {
        const float x = A.wg_g[base + g];
        const uint32_t xj = A.wg_j[base + g];
        if (x < gmin || (x == gmin && xj < jmin)) {
            gmin = x;
            jmin = xj;
        }
        gw += A.wg_gw[base + g];
    }
    // within each wavefront, then over the wavefronts in order (the same in every thread)
    wave64_argmin(gmin, jmin);
    gw = wave64_sum(gw);
    if (lane == 0) {
        smg[wave] = gmin;
        smj[wave] = jmin;
        smw[wave] = gw;
    }
    __syncthreads();
    float gm = smg[0], gws = smw[0];
    uint32_t jm = smj[0];
    for (int w = 1; w < kWideBlock / 64; ++w) {
        if (smg[w] < gm || (smg[w] == gm && smj[w] < jm)) {
            gm = smg[w];
            jm = smj[w];
        }
        gws += smw[w];
    }
    const uint32_t a = (gm < 0.0f) ? jm + 1u : 0u;
    gap = gws - (gm < 0.0f ? gm : 0.0f);
    __syncthreads();                                    // smg/smj/smw may be reused after this
    return a;
}

// The records of the step of iteration t with vertex a (one thread).
// tau_now: the replication's hitting time as read before; the count is a single-writer atomic add,
// which nothing waits for.
__device__ __forceinline__ void wide_record_step(const WideArgs &A, uint32_t r, uint64_t t, uint32_t a, float gap,
                                                 uint32_t tau_now)
{
    if (tau_now == kTauNone && gap <= A.gap_eps) A.tau[r] = static_cast<uint32_t>(t);
    A.dec[static_cast<uint64_t>(r) * A.T + t] = a;
    atomicAdd(A.cnt + static_cast<uint64_t>(r) * (A.d + 1) + a, 1u);
}

}  // namespace

// With prev_t >= 0 the launch first takes the step of iteration prev_t = t - 1 from the partials the
// previous gradient launch left in buffer par ^ 1 (every workgroup computes the same vertex;
// workgroup 0 records it, and the workgroup owning that asset adds t to its signature before any
// thread reads it), which saves the separate step launch between the two iterations.
__global__ __launch_bounds__(kWideBlock) void wide_sample_kernel(WideArgs A, uint32_t epoch, uint32_t Nk, float cw,
                                                                 int from_w0, int64_t prev_t, uint32_t par)
{
    __shared__ float sm[kWideBlock * 4];
    __shared__ uint32_t st_j[kWideBlock];
    const uint32_t tid = threadIdx.x, c = tid / kWideQuads, aq = tid % kWideQuads;
    const uint32_t r = blockIdx.y, g = blockIdx.x;
    const uint32_t q = g * kWideQuads + aq;
    const bool active = q < A.nq;
    const uint32_t j0 = 4 * q;
    // the quad's signature and coefficients, loaded before the step's reduction (a thread past the
    // last quad loads the last quad and discards it)
    WideQuad Q = wide_load_quad(A, r, active ? q : A.nq - 1);
    const bool recorder = g == 0 && tid == 0 && prev_t >= 0;
    const uint32_t tau_now = recorder ? A.tau[r] : kTauNone;
    if (prev_t >= 0) {
        float gap;
        const uint32_t a = wide_reduce_step(A, r, par ^ 1u, sm, sm + kWideBlock, st_j, gap);
        if (recorder) wide_record_step(A, r, static_cast<uint64_t>(prev_t), a, gap, tau_now);
        if (a > 0 && active && a - 1 >= j0 && a - 1 < j0 + 4) {
            // every chunk's copy of the quad absorbs the step; the first chunk stores it
            const uint32_t k = a - 1 - j0;
            const uint64_t add = static_cast<uint64_t>(prev_t) + 1;
            Q.S[0] += k == 0 ? add : 0;
            Q.S[1] += k == 1 ? add : 0;
            Q.S[2] += k == 2 ? add : 0;
            Q.S[3] += k == 3 ? add : 0;
            if (c == 0)
                A.S[static_cast<uint64_t>(r) * A.d + (a - 1)] = k == 0 ? Q.S[0] : k == 1 ? Q.S[1] : k == 2 ? Q.S[2] : Q.S[3];
        }
    }
    float w[4], v[4];
    wide_iterate(Q, active, cw, from_w0 != 0, w, v);

    const PhiloxRow row = philox_row(epoch, r, A.k0);
    float s1[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (uint32_t i = c; i < Nk; i += kWideChunks) {
        const Block4<float> z = normals_block_row(row, i * A.nq + q, A.dom, A.k0, A.k1);
        float p = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            p = fmaf(z.z[k], v[k], p);
            s1[k] += z.z[k];
        }
        p = half_sum(p);
        if (aq == 0) A.part_dot[(static_cast<uint64_t>(r) * A.N + i) * A.nwg + g] = p;
    }
    // s1 over the sample chunks, in chunk order
#pragma unroll
    for (int k = 0; k < 4; ++k) sm[tid * 4 + k] = s1[k];
    __syncthreads();
    if (c == 0) {
        float tot[4], qp = 0.0f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            tot[k] = sm[aq * 4 + k];
            for (int cc = 1; cc < kWideChunks; ++cc) tot[k] += sm[(cc * kWideQuads + aq) * 4 + k];
            qp = fmaf(tot[k], v[k], qp);
        }
        if (active) {
            float4 *dst = reinterpret_cast<float4 *>(A.s1 + static_cast<uint64_t>(r) * A.d + j0);
            *dst = make_float4(tot[0], tot[1], tot[2], tot[3]);
        }
        qp = half_sum(qp);
        if (aq == 0) A.part_qn[static_cast<uint64_t>(r) * A.nwg + g] = qp;
    }
}

// block i < N_k: dot_i = sum over the workgroups of z_i'v; block N_k: s1'v. One workgroup each.
__global__ __launch_bounds__(kWideBlock) void wide_dot_kernel(WideArgs A, uint32_t Nk)
{
    __shared__ float sm[kWideBlock];
    const uint32_t i = blockIdx.x, r = blockIdx.y, tid = threadIdx.x;
    const float *src = (i < Nk) ? A.part_dot + (static_cast<uint64_t>(r) * A.N + i) * A.nwg
                                 : A.part_qn + static_cast<uint64_t>(r) * A.nwg;
    float x = 0.0f;
    for (uint32_t g = tid; g < A.nwg; g += kWideBlock) x += src[g];
    sm[tid] = x;
    __syncthreads();
    for (int h = kWideBlock / 2; h > 0; h >>= 1) {
        if (tid < static_cast<uint32_t>(h)) sm[tid] += sm[tid + h];
        __syncthreads();
    }
    if (tid == 0) {
        if (i < Nk) A.dot[static_cast<uint64_t>(r) * A.N + i] = sm[0];
        else A.qn[r] = sm[0];
    }
}

__global__ __launch_bounds__(kWideBlock) void wide_gradient_kernel(WideArgs A, uint32_t epoch, WideEpoch E, float cw,
                                                                   int from_w0)
{
    __shared__ float sm[kWideBlock * 4];
    __shared__ float s_dot[SIM_WIDE_MAX_N];
    const uint32_t tid = threadIdx.x, c = tid / kWideQuads, aq = tid % kWideQuads;
    const uint32_t r = blockIdx.y, g = blockIdx.x;
    const uint32_t q = g * kWideQuads + aq;
    const bool active = q < A.nq;
    const uint32_t j0 = 4 * q;

    // every load of the launch before the first wait: the quad's signature, coefficients and s1, the
    // replication's s1'v, and the sample dot products (into LDS)
    const uint32_t qc = active ? q : A.nq - 1;
    const WideQuad Q = wide_load_quad(A, r, qc);
    const float4 s1q = *reinterpret_cast<const float4 *>(A.s1 + static_cast<uint64_t>(r) * A.d + 4 * qc);
    const float4 c1q = *reinterpret_cast<const float4 *>(A.c1_f + 4 * qc);
    const float4 c2q = *reinterpret_cast<const float4 *>(A.c2_f + 4 * qc);
    const float4 muq = *reinterpret_cast<const float4 *>(A.mu_f + 4 * qc);
    const float qn_r = A.qn[r];
    const float *dot = A.dot + static_cast<uint64_t>(r) * A.N;
    for (uint32_t i = tid; i < E.n; i += kWideBlock) s_dot[i] = dot[i];
    __syncthreads();

    const PhiloxRow row = philox_row(epoch, r, A.k0);
    float s2[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (uint32_t i = c; i < E.n; i += kWideChunks) {
        const Block4<float> z = normals_block_row(row, i * A.nq + q, A.dom, A.k0, A.k1);
        const float di = s_dot[i];
#pragma unroll
        for (int k = 0; k < 4; ++k) s2[k] = fmaf(z.z[k], di, s2[k]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) sm[tid * 4 + k] = s2[k];
    __syncthreads();
    if (c == 0) {
        float w[4], v[4];
        wide_iterate(Q, active, cw, from_w0 != 0, w, v);
        const float qn = qn_r * E.inv_n;
        const float s1a[4] = {s1q.x, s1q.y, s1q.z, s1q.w}, c1a[4] = {c1q.x, c1q.y, c1q.z, c1q.w};
        const float c2a[4] = {c2q.x, c2q.y, c2q.z, c2q.w}, mua[4] = {muq.x, muq.y, muq.z, muq.w};
        float gmin = INFINITY, gw = 0.0f;
        uint32_t jmin = 0xFFFFFFFFu;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float s2k = sm[aq * 4 + k];
            for (int cc = 1; cc < kWideChunks; ++cc) s2k += sm[(cc * kWideQuads + aq) * 4 + k];
            if (active) {
                const uint32_t j = j0 + k;
                const float s1k = s1a[k];
                const float gj = (c2a[k] * E.sc2) * (s2k - s1k * qn) - mua[k] - (c1a[k] * E.sc1) * s1k;
                if (gj < gmin) {
                    gmin = gj;
                    jmin = j;
                }
                gw = fmaf(gj, w[k], gw);
            }
        }
        half_argmin(gmin, jmin);
        gw = half_sum(gw);
        if (aq == 0) {
            const uint64_t o = (static_cast<uint64_t>(E.par) * A.R + r) * A.nwg + g;
            A.wg_g[o] = gmin;
            A.wg_j[o] = jmin;
            A.wg_gw[o] = gw;
        }
    }
}

// The step of iteration t from buffer par on its own (before an objective evaluation and after the
// last iteration): the vertex, the gap, tau and the update.
__global__ __launch_bounds__(kWideBlock) void wide_step_kernel(WideArgs A, uint64_t t, uint32_t par)
{
    __shared__ float smg[kWideBlock], smw[kWideBlock];
    __shared__ uint32_t smj[kWideBlock];
    const uint32_t r = blockIdx.x;
    float gap;
    const uint32_t a = wide_reduce_step(A, r, par, smg, smw, smj, gap);
    if (threadIdx.x == 0) {
        wide_record_step(A, r, t, a, gap, A.tau[r]);
        if (a > 0) A.S[static_cast<uint64_t>(r) * A.d + (a - 1)] += t + 1;
    }
}

// f(w) = lambda sum_j sigma_j^2 w_j^2 - mu'w at w = c S (Eq. (3)), FP64, one workgroup per replication.
__global__ __launch_bounds__(kWideBlock) void wide_objective_kernel(WideArgs A, double c, uint32_t slot)
{
    __shared__ double sm[2 * (kWideBlock / 64)];
    const uint32_t r = blockIdx.x, tid = threadIdx.x;
    const uint64_t *S = A.S + static_cast<uint64_t>(r) * A.d;
    double quad = 0.0, lin = 0.0;
    for (uint32_t j = tid; j < A.d; j += kWideBlock) {
        const double w = static_cast<double>(S[j]) * c;
        const double sw = A.sig_d[j] * w;
        quad += sw * sw;
        lin += A.mu_d[j] * w;
    }
    double qh = quad, ql = 0.0, lh = lin, ll = 0.0;
    block_sum_dd(qh, ql, sm);
    block_sum_dd(lh, ll, sm);
    if (tid == 0) A.fval[static_cast<uint64_t>(slot) * A.R + r] = A.lambda * (qh + ql) - (lh + ll);
}

// Streams Y, f(w_c), RSE_c = ((f(w_c) - Y) / f(w_c))^2 over the replications in order, in the layout of
// the per-lane kernels (sum hi/lo, squares hi/lo, count), min and max of Y, and the origin's total.
__global__ void wide_finalize_kernel(WideArgs A, uint32_t n_ckpt)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double *Y = A.fval + static_cast<uint64_t>(n_ckpt) * A.R;
    const uint32_t n_streams = 1 + 2 * n_ckpt;
    for (uint32_t s = 0; s < n_streams; ++s) {
        double h = 0.0, l = 0.0, qh = 0.0, ql = 0.0, n = 0.0;
        for (uint32_t r = 0; r < A.R; ++r) {
            double x;
            if (s == 0) {
                x = Y[r];
            } else if (s <= n_ckpt) {
                x = A.fval[static_cast<uint64_t>(s - 1) * A.R + r];
            } else {
                const double f = A.fval[static_cast<uint64_t>(s - 1 - n_ckpt) * A.R + r];
                if (f == 0.0) continue;
                const double e = (f - Y[r]) / f;
                x = e * e;
            }
            dd_add(h, l, x, 0.0);
            dd_add(qh, ql, x * x, fma(x, x, -(x * x)));
            n += 1.0;
        }
        double *o = A.stats + s * kStreamFields;
        o[0] = h;
        o[1] = l;
        o[2] = qh;
        o[3] = ql;
        o[4] = n;
    }
    double mn = INFINITY, mx = -INFINITY;
    uint64_t origin = 0;
    for (uint32_t r = 0; r < A.R; ++r) {
        mn = fmin(mn, Y[r]);
        mx = fmax(mx, Y[r]);
        origin += A.cnt[static_cast<uint64_t>(r) * (A.d + 1)];
    }
    A.stats[n_streams * kStreamFields] = mn;
    A.stats[n_streams * kStreamFields + 1] = mx;
    *A.origin_total = origin;
}

int launch_wide_iteration(const WideArgs &A, uint64_t t, uint32_t epoch, const WideEpoch &E, float cw, bool from_w0,
                          bool fold_prev, hipStream_t s)
{
    const dim3 grid(A.nwg, A.R);
    const int64_t prev = fold_prev ? static_cast<int64_t>(t) - 1 : -1;
    hipLaunchKernelGGL(wide_sample_kernel, grid, dim3(kWideBlock), 0, s, A, epoch, E.n, cw, from_w0 ? 1 : 0, prev, E.par);
    hipLaunchKernelGGL(wide_dot_kernel, dim3(E.n + 1, A.R), dim3(kWideBlock), 0, s, A, E.n);
    hipLaunchKernelGGL(wide_gradient_kernel, grid, dim3(kWideBlock), 0, s, A, epoch, E, cw, from_w0 ? 1 : 0);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_wide_step(const WideArgs &A, uint64_t t, hipStream_t s)
{
    hipLaunchKernelGGL(wide_step_kernel, dim3(A.R), dim3(kWideBlock), 0, s, A, t, static_cast<uint32_t>(t & 1));
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_wide_objective(const WideArgs &A, double c, uint32_t slot, hipStream_t s)
{
    hipLaunchKernelGGL(wide_objective_kernel, dim3(A.R), dim3(kWideBlock), 0, s, A, c, slot);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_wide_finalize(const WideArgs &A, uint32_t n_ckpt, hipStream_t s)
{
    hipLaunchKernelGGL(wide_finalize_kernel, dim3(1), dim3(64), 0, s, A, n_ckpt);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace fw
