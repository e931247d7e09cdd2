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
#include "device_rng.hpp"
#include "sim_types.hpp"
#include "wide.hpp"

namespace fw {

namespace {

// Sum over the 32 lanes of a half wavefront (the lanes of one sample chunk); every lane gets it.
__device__ __forceinline__ float half_sum(float x)
{
#pragma unroll
    for (int m = 1; m < 32; m <<= 1) x += __shfl_xor(x, m, 32);
    return x;
}

// (value, index) minimum over the 32 lanes of a half wavefront, lowest index among equal values.
__device__ __forceinline__ void half_argmin(float &g, uint32_t &j)
{
#pragma unroll
    for (int m = 1; m < 32; m <<= 1) {
        const float og = __shfl_xor(g, m, 32);
        const uint32_t oj = __shfl_xor(j, m, 32);
        if (og < g || (og == g && oj < j)) {
            g = og;
            j = oj;
        }
    }
}

// w_t of four consecutive assets j0..j0+3 and v = sz .* w_t
__device__ __forceinline__ void wide_iterate(const WideArgs &A, uint32_t r, uint32_t j0, bool active, float cw,
                                             bool from_w0, float (&w)[4], float (&v)[4])
{
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        w[k] = 0.0f;
        v[k] = 0.0f;
        if (active) {
            w[k] = from_w0 ? A.w0_f[j0 + k]
                           : static_cast<float>(static_cast<double>(A.S[static_cast<uint64_t>(r) * A.d + j0 + k])) * cw;
            v[k] = A.sz_f[j0 + k] * w[k];
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
    const uint32_t tid = threadIdx.x;
    const uint64_t base = (static_cast<uint64_t>(par) * A.R + r) * A.nwg;
    float gmin = INFINITY, gw = 0.0f;
    uint32_t jmin = 0xFFFFFFFFu;
    for (uint32_t g = tid; g < A.nwg; g += kWideBlock) {
        const float x = A.wg_g[base + g];
        if (x < gmin) {
            gmin = x;
            jmin = A.wg_j[base + g];
        }
        gw += A.wg_gw[base + g];
    }
    smg[tid] = gmin;
    smj[tid] = jmin;
    smw[tid] = gw;
    __syncthreads();
    for (int h = kWideBlock / 2; h > 0; h >>= 1) {
        if (tid < static_cast<uint32_t>(h)) {
            const float og = smg[tid + h];
            const uint32_t oj = smj[tid + h];
            if (og < smg[tid] || (og == smg[tid] && oj < smj[tid])) {
                smg[tid] = og;
                smj[tid] = oj;
            }
            smw[tid] += smw[tid + h];
        }
        __syncthreads();
    }
    const float gm = smg[0];
    const uint32_t a = (gm < 0.0f) ? smj[0] + 1u : 0u;
    gap = smw[0] - (gm < 0.0f ? gm : 0.0f);
    __syncthreads();                                    // smg/smj/smw may be reused after this
    return a;
}

// The records of the step of iteration t with vertex a (one thread).
__device__ __forceinline__ void wide_record_step(const WideArgs &A, uint32_t r, uint64_t t, uint32_t a, float gap)
{
    if (A.tau[r] == kTauNone && gap <= A.gap_eps) A.tau[r] = static_cast<uint32_t>(t);
    A.dec[static_cast<uint64_t>(r) * A.T + t] = a;
    A.cnt[static_cast<uint64_t>(r) * (A.d + 1) + a] += 1u;
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
    if (prev_t >= 0) {
        float gap;
        const uint32_t a = wide_reduce_step(A, r, par ^ 1u, sm, sm + kWideBlock, st_j, gap);
        if (g == 0 && tid == 0) wide_record_step(A, r, static_cast<uint64_t>(prev_t), a, gap);
        if (a > 0 && c == 0 && active && a - 1 >= j0 && a - 1 < j0 + 4)
            A.S[static_cast<uint64_t>(r) * A.d + (a - 1)] += static_cast<uint64_t>(prev_t) + 1;
        __syncthreads();                                // the signature is read below by all chunks
    }
    float w[4], v[4];
    wide_iterate(A, r, j0, active, cw, from_w0 != 0, w, v);

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
    const uint32_t tid = threadIdx.x, c = tid / kWideQuads, aq = tid % kWideQuads;
    const uint32_t r = blockIdx.y, g = blockIdx.x;
    const uint32_t q = g * kWideQuads + aq;
    const bool active = q < A.nq;
    const uint32_t j0 = 4 * q;

    const PhiloxRow row = philox_row(epoch, r, A.k0);
    const float *dot = A.dot + static_cast<uint64_t>(r) * A.N;
    float s2[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    for (uint32_t i = c; i < E.n; i += kWideChunks) {
        const Block4<float> z = normals_block_row(row, i * A.nq + q, A.dom, A.k0, A.k1);
        const float di = dot[i];
#pragma unroll
        for (int k = 0; k < 4; ++k) s2[k] = fmaf(z.z[k], di, s2[k]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) sm[tid * 4 + k] = s2[k];
    __syncthreads();
    if (c == 0) {
        float w[4], v[4];
        wide_iterate(A, r, j0, active, cw, from_w0 != 0, w, v);
        const float qn = A.qn[r] * E.inv_n;
        float gmin = INFINITY, gw = 0.0f;
        uint32_t jmin = 0xFFFFFFFFu;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            float s2k = sm[aq * 4 + k];
            for (int cc = 1; cc < kWideChunks; ++cc) s2k += sm[(cc * kWideQuads + aq) * 4 + k];
            if (active) {
                const uint32_t j = j0 + k;
                const float s1k = A.s1[static_cast<uint64_t>(r) * A.d + j];
                const float gj = (A.c2_f[j] * E.sc2) * (s2k - s1k * qn) - A.mu_f[j] - (A.c1_f[j] * E.sc1) * s1k;
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
        wide_record_step(A, r, t, a, gap);
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
