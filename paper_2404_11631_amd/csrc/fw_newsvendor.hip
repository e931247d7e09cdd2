// fw_newsvendor.hip -- Algorithm 2 (Section 3.2, Task 2): the multi-product newsvendor with one
// resource row c'x <= C, by stochastic Frank-Wolfe, at the paper's shape (Section 4.1: 1e2 to 1e6
// products, S = 25-50 demand samples per product, K = 1500 iterations, one or a few replications).
//
// The gradient is separable (Eq. (8)-(9)): g_j = k_j - v_j + (h_j + v_j) #{s : d_j^(s) <= x_j} / S,
// so an iteration is a sample launch and a step:
//   sample    a thread owns four consecutive products (one Philox block per sample), draws their S
//             demand samples, counts those at or below x_j -- as standard normals against the
//             threshold (x_j - mu_j)/sigma_j, in binary32 -- forms g_j and the ratio g_j / c_j, and
//             the workgroup keeps its smallest ratio (lowest index among equal values) and its part
//             of g'x;
//   step      the vertex over all workgroups: (C/c_j) e_j for the smallest ratio when it is negative,
//             else the origin; the Frank-Wolfe gap g'x - min(0, C min_j g_j/c_j) and tau; the
//             integer update S_a += t + 1 (x_{t+1} = (C/c) .* 2 S / ((t+1)(t+2)), Algorithm 2's
//             recurrence in exact arithmetic). The step of iteration t normally runs at the start of
//             iteration t + 1's sample launch: every workgroup reduces the same partials in the same
//             order (so all get the same vertex), workgroup 0 records it and the thread owning the
//             chosen product updates its signature; a launch of its own remains only before a cost
//             evaluation and after the last iteration. The partials alternate between two buffers.
// The demand normals are standard normal s n + j of the (replication, epoch) stream in domain 4,
// scaled by 1/sqrt(2 ln 2) like every binary32 normal here; the host folds that into the threshold.
#include <hip/hip_runtime.h>

#include "device_reduce.hpp"
#include "device_rng.hpp"
#include "newsvendor.hpp"
#include "sim_types.hpp"
#include "wave_dpp.hpp"

namespace fw {

namespace {

// (value, index) minimum over a wavefront, lowest index among equal values, and a sum over it; every
// lane gets the result. The DPP exchanges pair lanes as the xor butterfly 1, 2, ..., 32 does, so
// the sums' rounding is that butterfly's.
__device__ __forceinline__ void wave_argmin(float &g, uint32_t &j) { dpp_argmin64(g, j); }

__device__ __forceinline__ float wave_sum(float x) { return dpp_sum64(x); }

// The step of iteration t over the workgroup partials of replication r (buffer par): the smallest
// ratio (lowest product among equal values; the workgroups cover ascending product ranges, so strict
// < over them in order keeps the lowest), the sum of the g'x parts, then the vertex a (0: the
// origin). Every thread of the kNvBlock-thread workgroup takes part and gets a; thread 0 also gets
// the gap. The order of the sums is fixed, so every workgroup that calls it gets the same bits.
__device__ __forceinline__ uint32_t nv_reduce_step(const NvArgs &A, uint32_t r, uint32_t par, float *smr, float *smx,
                                                   uint32_t *smj, float &gap)
{
    const uint32_t tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const uint64_t base = (static_cast<uint64_t>(par) * A.R + r) * A.nwg;
    float rm = INFINITY, gs = 0.0f;
    uint32_t jm = 0xFFFFFFFFu;
    for (uint32_t g = tid; g < A.nwg; g += kNvBlock) {
        const float x = A.wg_r[base + g];
        const uint32_t xj = A.wg_j[base + g];
        if (x < rm || (x == rm && xj < jm)) {
            rm = x;
            jm = xj;
        }
        gs += A.wg_gx[base + g];
    }
    // smallest ratio (lowest product among equal ones) and the sum: within each wavefront, then over
    // the wavefronts in order, the same in every thread
    wave_argmin(rm, jm);
    gs = wave_sum(gs);
    if (lane == 0) {
        smr[wave] = rm;
        smj[wave] = jm;
        smx[wave] = gs;
    }
    __syncthreads();
    float best = smr[0], gsum = smx[0];
    uint32_t bj = smj[0];
    for (int w = 1; w < kNvBlock / 64; ++w) {
        if (smr[w] < best || (smr[w] == best && smj[w] < bj)) {
            best = smr[w];
            bj = smj[w];
        }
        gsum += smx[w];
    }
    const uint32_t a = (best < 0.0f) ? bj + 1u : 0u;
    gap = gsum - (best < 0.0f ? A.C * best : 0.0f);
    __syncthreads();                                    // smr/smj/smx may be reused after this
    return a;
}

// f_j(x) of Eq. (6) for normal demand N(mu, sg^2), closed form: k x + h E(x - xi)^+ + v E(xi - x)^+.
__device__ __forceinline__ double nv_product_cost(double x, double mu, double sg, double k, double h, double v)
{
    double over, under;
    if (sg > 0.0) {
        const double z = (x - mu) / sg;
        const double pdf = 0.39894228040143267794 * exp(-0.5 * z * z);
        const double cdf = 0.5 * erfc(-z * 0.70710678118654752440);
        const double upper = 0.5 * erfc(z * 0.70710678118654752440);
        over = sg * (z * cdf + pdf);
        under = sg * (pdf - z * upper);
    } else {
        over = x > mu ? x - mu : 0.0;
        under = mu > x ? mu - x : 0.0;
    }
    return k * x + h * over + v * under;
}

// The records of the step of iteration t with vertex a (one thread), tau_now being the replication's
// hitting time as read before. The count is a single-writer atomic add, which nothing waits for.
__device__ __forceinline__ void nv_record_step(const NvArgs &A, uint32_t r, uint64_t t, uint32_t a, float gap,
                                               uint32_t tau_now)
{
    if (tau_now == kTauNone && gap <= A.gap_eps) A.tau[r] = static_cast<uint32_t>(t);
    A.dec[static_cast<uint64_t>(r) * A.T + t] = a;
    atomicAdd(A.cnt + static_cast<uint64_t>(r) * (A.n + 1) + a, 1u);
}

}  // namespace

// Iteration t (partials into buffer par = t & 1). With prev_t >= 0 the launch first takes the step of
// iteration prev_t = t - 1 from the other buffer (every workgroup computes the same vertex; workgroup 0
// records it, and the thread owning that product adds t to its signature before reading it), which
// saves the separate step launch between the two iterations.
__global__ __launch_bounds__(kNvBlock) void nv_sample_kernel(NvArgs A, uint32_t epoch, float cw, int from_x0,
                                                             int64_t prev_t, uint32_t par)
{
    __shared__ float sm_r[kNvBlock / 64], sm_gx[kNvBlock / 64];
    __shared__ uint32_t sm_j[kNvBlock / 64];
    __shared__ float st_r[kNvBlock], st_x[kNvBlock];
    __shared__ uint32_t st_j[kNvBlock];
    const uint32_t tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
    const uint32_t r = blockIdx.y, g = blockIdx.x;
    // P consecutive lanes per quad (aligned groups within a wavefront), quads in ascending order
    const uint32_t P = A.P, sub = tid % P;
    const uint32_t q = g * (kNvBlock / P) + tid / P;
    const bool active = q < A.nq;
    const bool lead = sub == 0;                         // the lane that carries the quad after its counts are summed
    const uint32_t j0 = 4 * q;

    // The quad's coefficients and signature words, loaded before the step's reduction and all at
    // once (n is a multiple of 4 and every array starts 16-byte aligned, so a quad is one 16-byte
    // word per coefficient). A thread past the last quad loads the last quad and discards it.
    const uint32_t jc = 4 * (active ? q : A.nq - 1);
    const float4 mu4 = *reinterpret_cast<const float4 *>(A.mu_f + jc);
    const float4 isk4 = *reinterpret_cast<const float4 *>(A.isk_f + jc);
    const float4 a4 = *reinterpret_cast<const float4 *>(A.a_f + jc);
    const float4 b4 = *reinterpret_cast<const float4 *>(A.b_f + jc);
    const float4 ic4 = *reinterpret_cast<const float4 *>(A.ic_f + jc);
    const float4 xs4 = *reinterpret_cast<const float4 *>((from_x0 ? A.x0_f : A.xs_f) + jc);
    uint64_t *sig = A.S_sig + static_cast<uint64_t>(r) * A.n + jc;
    const ulonglong2 s01 = reinterpret_cast<const ulonglong2 *>(sig)[0];
    const ulonglong2 s23 = reinterpret_cast<const ulonglong2 *>(sig)[1];
    uint64_t S4[4] = {s01.x, s01.y, s23.x, s23.y};
    const bool recorder = g == 0 && tid == 0 && prev_t >= 0;
    const uint32_t tau_now = recorder ? A.tau[r] : kTauNone;
    const float mu[4] = {mu4.x, mu4.y, mu4.z, mu4.w}, isk[4] = {isk4.x, isk4.y, isk4.z, isk4.w};
    const float ca[4] = {a4.x, a4.y, a4.z, a4.w}, cb[4] = {b4.x, b4.y, b4.z, b4.w};
    const float ic[4] = {ic4.x, ic4.y, ic4.z, ic4.w}, xs[4] = {xs4.x, xs4.y, xs4.z, xs4.w};

    if (prev_t >= 0) {
        float gap;
        const uint32_t a = nv_reduce_step(A, r, par ^ 1u, st_r, st_x, st_j, gap);
        if (recorder) nv_record_step(A, r, static_cast<uint64_t>(prev_t), a, gap, tau_now);
        if (a > 0 && active && a - 1 >= j0 && a - 1 < j0 + 4) {
            // the chosen product's signature absorbs the step (selects, not a dynamic register index)
            const uint32_t k = a - 1 - j0;
            const uint64_t add = static_cast<uint64_t>(prev_t) + 1;
            S4[0] += k == 0 ? add : 0;
            S4[1] += k == 1 ? add : 0;
            S4[2] += k == 2 ? add : 0;
            S4[3] += k == 3 ? add : 0;
            if (lead) sig[k] = k == 0 ? S4[0] : k == 1 ? S4[1] : k == 2 ? S4[2] : S4[3];
        }
    }

    float x[4], thr[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        x[k] = 0.0f;
        thr[k] = 0.0f;
        if (active) {
            x[k] = from_x0 ? xs[k] : xs[k] * (static_cast<float>(static_cast<double>(S4[k])) * cw);
            // sigma_j = 0 stores an infinite scale: the threshold is then +-infinity, and +infinity
            // (every sample counted) where x_j equals the demand exactly
            thr[k] = (x[k] - mu[k]) * isk[k];
            if (thr[k] != thr[k]) thr[k] = INFINITY;
        }
    }
    const PhiloxRow row = philox_row(epoch, r, A.k0);
    // the quad's samples s = sub, sub + P, ...; the counts are integers, so their sum over the P lanes
    // is exact whatever the split
    uint32_t count[4] = {0u, 0u, 0u, 0u};
    for (uint32_t s = sub; s < A.S; s += P) {
        const Block4<float> z = normals_block_row(row, s * A.nq + q, A.dom, A.k0, A.k1);
#pragma unroll
        for (int k = 0; k < 4; ++k) count[k] += (z.z[k] <= thr[k]) ? 1u : 0u;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) count[k] = dpp_sum_lanes(count[k], P);
    float rmin = INFINITY, gx = 0.0f;
    uint32_t jmin = 0xFFFFFFFFu;
    if (active && lead) {
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint32_t j = j0 + k;
            const float gj = ca[k] + cb[k] * static_cast<float>(count[k]);
            const float rj = gj * ic[k];
            if (rj < rmin) {
                rmin = rj;
                jmin = j;
            }
            gx = fmaf(gj, x[k], gx);
        }
    }
    wave_argmin(rmin, jmin);
    gx = wave_sum(gx);
    if (lane == 0) {
        sm_r[wave] = rmin;
        sm_j[wave] = jmin;
        sm_gx[wave] = gx;
    }
    __syncthreads();
    if (tid == 0) {   // the wavefronts cover ascending product ranges: strict < keeps the lowest index
        float rm = sm_r[0], gs = sm_gx[0];
        uint32_t jm = sm_j[0];
        for (int w = 1; w < kNvBlock / 64; ++w) {
            if (sm_r[w] < rm) {
                rm = sm_r[w];
                jm = sm_j[w];
            }
            gs += sm_gx[w];
        }
        const uint64_t o = (static_cast<uint64_t>(par) * A.R + r) * A.nwg + g;
        A.wg_r[o] = rm;
        A.wg_j[o] = jm;
        A.wg_gx[o] = gs;
    }
}

// The step of iteration t from buffer par on its own (before a cost evaluation and after the last
// iteration): the vertex, the gap, tau and the update.
__global__ __launch_bounds__(kNvBlock) void nv_step_kernel(NvArgs A, uint64_t t, uint32_t par)
{
    __shared__ float smr[kNvBlock], smx[kNvBlock];
    __shared__ uint32_t smj[kNvBlock];
    const uint32_t r = blockIdx.x;
    float gap;
    const uint32_t a = nv_reduce_step(A, r, par, smr, smx, smj, gap);
    if (threadIdx.x == 0) {
        nv_record_step(A, r, t, a, gap, A.tau[r]);
        if (a > 0) A.S_sig[static_cast<uint64_t>(r) * A.n + (a - 1)] += t + 1;
    }
}

// f(x) = sum_j k x + h E(x - xi)^+ + v E(xi - x)^+ (Eq. (6), normal demand, closed form) at
// x = (C/c) .* c S, FP64: workgroup blockIdx.x of replication blockIdx.y sums products
// [kNvCostChunk blockIdx.x, +kNvCostChunk) into a double-double partial.
__global__ __launch_bounds__(kBlock) void nv_cost_kernel(NvArgs A, double c)
{
    __shared__ double sm[2 * (kBlock / 64)];
    const uint32_t r = blockIdx.y, tid = threadIdx.x;
    const uint64_t *S = A.S_sig + static_cast<uint64_t>(r) * A.n;
    const uint32_t j1 = min(A.n, (blockIdx.x + 1) * kNvCostChunk);
    double total = 0.0;
    for (uint32_t j = blockIdx.x * kNvCostChunk + tid; j < j1; j += kBlock) {
        const double x = A.xs_d[j] * (static_cast<double>(S[j]) * c);
        total += nv_product_cost(x, A.mu_d[j], A.sig_d[j], A.k_d[j], A.h_d[j], A.v_d[j]);
    }
    double h = total, l = 0.0;
    block_sum_dd(h, l, sm);
    if (tid == 0) {
        const uint32_t nc = (A.n + kNvCostChunk - 1) / kNvCostChunk;
        double *o = A.cost_part + 2 * (static_cast<uint64_t>(r) * nc + blockIdx.x);
        o[0] = h;
        o[1] = l;
    }
}

// The partials of replication blockIdx.x in order, into fval[slot][r].
__global__ __launch_bounds__(kBlock) void nv_cost_sum_kernel(NvArgs A, uint32_t slot)
{
    __shared__ double sm[2 * (kBlock / 64)];
    const uint32_t r = blockIdx.x, tid = threadIdx.x;
    const uint32_t nc = (A.n + kNvCostChunk - 1) / kNvCostChunk;
    const double *p = A.cost_part + 2 * static_cast<uint64_t>(r) * nc;
    double h = 0.0, l = 0.0;
    for (uint32_t b = tid; b < nc; b += kBlock) dd_add(h, l, p[2 * b], p[2 * b + 1]);
    block_sum_dd(h, l, sm);
    if (tid == 0) A.fval[static_cast<uint64_t>(slot) * A.R + r] = h + l;
}

// Streams of Y, f(x_c) and RSE_c over the replications in order, in the layout of the per-lane
// kernels (sum hi/lo, squares hi/lo, count), then min and max of Y (one thread).
__device__ void nv_stream_stats(const double *fval, uint32_t R, uint32_t n_ckpt, double *stats)
{
    const double *Y = fval + static_cast<uint64_t>(n_ckpt) * R;
    const uint32_t n_streams = 1 + 2 * n_ckpt;
    for (uint32_t s = 0; s < n_streams; ++s) {
        double h = 0.0, l = 0.0, qh = 0.0, ql = 0.0, n = 0.0;
        for (uint32_t r = 0; r < R; ++r) {
            double x;
            if (s == 0) {
                x = Y[r];
            } else if (s <= n_ckpt) {
                x = fval[static_cast<uint64_t>(s - 1) * R + r];
            } else {
                const double f = fval[static_cast<uint64_t>(s - 1 - n_ckpt) * R + r];
                if (f == 0.0) continue;
                const double e = (f - Y[r]) / f;
                x = e * e;
            }
            dd_add(h, l, x, 0.0);
            dd_add(qh, ql, x * x, fma(x, x, -(x * x)));
            n += 1.0;
        }
        double *o = stats + s * kStreamFields;
        o[0] = h;
        o[1] = l;
        o[2] = qh;
        o[3] = ql;
        o[4] = n;
    }
    double mn = INFINITY, mx = -INFINITY;
    for (uint32_t r = 0; r < R; ++r) {
        mn = fmin(mn, Y[r]);
        mx = fmax(mx, Y[r]);
    }
    stats[n_streams * kStreamFields] = mn;
    stats[n_streams * kStreamFields + 1] = mx;
}

// The statistics and the origin's total.
__global__ void nv_finalize_kernel(NvArgs A, uint32_t n_ckpt)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    nv_stream_stats(A.fval, A.R, n_ckpt, A.stats);
    uint64_t origin = 0;
    for (uint32_t r = 0; r < A.R; ++r) origin += A.cnt[static_cast<uint64_t>(r) * (A.n + 1)];
    *A.origin_total = origin;
}

// ---- Algorithm 2 over X = {A x <= C, x >= 0} with M resource rows (Eq. (7)) --------------------
//
// The iterate is kept in FP64 (x + gamma (s - x), each operation rounded on its own), the gradient
// Eq. (9) in FP64 from the same demand samples as above, and the linear subproblem
// min_{s in X} s'g is a revised simplex in FP64 on [A I][s; slack] = C, one workgroup per
// replication (256 threads up to 2,048 products, 1,024 above), started from the slack basis each
// iteration; pricing is a pass over the n + M columns per pivot.

namespace {

// x + gamma (s - x) with each operation rounded on its own (contraction into a fused multiply-add is
// off here), so that any other implementation of the same formula in FP64 gets the same bits.
__device__ __forceinline__ double nv_lp_move(double x, double s, double gamma)
{
#pragma clang fp contract(off)
    const double step = gamma * (s - x);
    return x + step;
}

// Eq. (9): (k - v) + ((h + v) count) / S, each operation rounded on its own.
__device__ __forceinline__ double nv_lp_grad(double km, double hv, uint32_t count, uint32_t S)
{
#pragma clang fp contract(off)
    const double part = (hv * static_cast<double>(count)) / static_cast<double>(S);
    return km + part;
}

// s_j of the vertex recorded for iteration t of replication r: the basic value where the basis
// holds product j, else 0.
__device__ __forceinline__ double nv_lp_vertex(const NvLpArgs &A, uint32_t r, uint64_t t, uint32_t j)
{
    const uint64_t o = (static_cast<uint64_t>(r) * A.T + t) * A.M;
    double s = 0.0;
    for (uint32_t i = 0; i < A.M; ++i)
        if (A.rec_basis[o + i] == j) s = A.rec_value[o + i];
    return s;
}

}  // namespace

// Iteration t's gradient (grid: workgroups of kNvBlock threads over the product quads, P consecutive
// lanes per quad, by replication). With fold_prev each quad is first moved to x_t with the vertex of
// iteration t - 1. Every load is issued before the first wait: the previous vertex's basis and
// values, the quad's iterate and coefficients. The quad's S samples are split over its P lanes and
// the integer counts summed exactly, so the gradient does not depend on P.
__global__ __launch_bounds__(kNvBlock) void nv_lp_gradient_kernel(NvLpArgs A, uint64_t t, uint32_t epoch,
                                                                  int fold_prev)
{
    const uint32_t r = blockIdx.y, tid = threadIdx.x;
    const uint32_t P = A.P, sub = tid % P;
    const uint32_t q = blockIdx.x * (kNvBlock / P) + tid / P;
    const bool active = q < A.nq;
    const bool lead = sub == 0;                         // stores the quad's iterate and gradient
    const uint32_t j0 = 4 * (active ? q : A.nq - 1);    // past the last quad: the last, discarded
    double *x = A.x + static_cast<uint64_t>(r) * A.n;

    uint32_t vb[kNvLpMaxM];
    double vv[kNvLpMaxM];
    if (fold_prev) {
        const uint64_t o = (static_cast<uint64_t>(r) * A.T + (t - 1)) * A.M;
#pragma unroll
        for (uint32_t i = 0; i < kNvLpMaxM; ++i) {
            vb[i] = A.rec_basis[o + (i < A.M ? i : 0)];
            vv[i] = A.rec_value[o + (i < A.M ? i : 0)];
        }
    }
    double xv[4], mu[4], isk[4], km[4], hv[4];
    auto load_quad = [&](const double *p, double (&v)[4]) {
        const double2 a = reinterpret_cast<const double2 *>(p + j0)[0];
        const double2 b = reinterpret_cast<const double2 *>(p + j0)[1];
        v[0] = a.x;
        v[1] = a.y;
        v[2] = b.x;
        v[3] = b.y;
    };
    load_quad(x, xv);
    load_quad(A.mu_d, mu);
    load_quad(A.isk_d, isk);
    load_quad(A.km_d, km);
    load_quad(A.hv_d, hv);

    double thr[4];
    const double gamma = fold_prev ? 2.0 / (static_cast<double>(t - 1) + 2.0) : 0.0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (fold_prev) {
            // s_j of the previous vertex: the basic value where the basis holds product j, else 0
            double sj = 0.0;
#pragma unroll
            for (uint32_t i = 0; i < kNvLpMaxM; ++i)
                if (i < A.M && vb[i] == j0 + k) sj = vv[i];
            xv[k] = nv_lp_move(xv[k], sj, gamma);
        }
        // sigma_j = 0 has an infinite scale: the threshold is +-infinity, and +infinity (every sample
        // counted) where x_j equals the demand exactly
        thr[k] = (xv[k] - mu[k]) * isk[k];
        if (thr[k] != thr[k]) thr[k] = INFINITY;
    }
    // every thread of the workgroup has read x (its value is already used above) before the moved
    // iterate is stored: lanes of the same quad and, past the last quad, lanes reading the last one
    if (fold_prev) __syncthreads();
    if (fold_prev && active && lead) {
        reinterpret_cast<double2 *>(x + j0)[0] = make_double2(xv[0], xv[1]);
        reinterpret_cast<double2 *>(x + j0)[1] = make_double2(xv[2], xv[3]);
    }
    const PhiloxRow row = philox_row(epoch, r, A.k0);
    uint32_t count[4] = {0u, 0u, 0u, 0u};
    for (uint32_t s = sub; s < A.S; s += P) {
        const Block4<float> z = normals_block_row(row, s * A.nq + (j0 / 4), A.dom, A.k0, A.k1);
#pragma unroll
        for (int k = 0; k < 4; ++k) count[k] += (static_cast<double>(z.z[k]) <= thr[k]) ? 1u : 0u;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) count[k] = dpp_sum_lanes(count[k], P);
    if (active && lead) {
        double gq[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) gq[k] = nv_lp_grad(km[k], hv[k], count[k], A.S);   // (k - v) + ((h + v) count) / S
        double *g = A.g + static_cast<uint64_t>(r) * A.n;
        reinterpret_cast<double2 *>(g + j0)[0] = make_double2(gq[0], gq[1]);
        reinterpret_cast<double2 *>(g + j0)[1] = make_double2(gq[2], gq[3]);
    }
}

// The update of iteration t alone: x_{t+1} = x_t + gamma_t (s_t - x_t).
__global__ __launch_bounds__(kNvBlock) void nv_lp_update_kernel(NvLpArgs A, uint64_t t)
{
    const uint32_t r = blockIdx.y;
    const uint32_t j = blockIdx.x * kNvBlock + threadIdx.x;
    if (j >= A.n) return;
    double *x = A.x + static_cast<uint64_t>(r) * A.n;
    x[j] = nv_lp_move(x[j], nv_lp_vertex(A, r, t, j), 2.0 / (static_cast<double>(t) + 2.0));
}

namespace {

// (value, column) minimum with the lowest column among equal values: associative and commutative,
// so any reduction order gives the same pair.
__device__ __forceinline__ void nv_lp_better(double &v, uint32_t &j, double ov, uint32_t oj)
{
    if (ov < v || (ov == v && oj < j)) {
        v = ov;
        j = oj;
    }
}

// Column q of [A I]: A's column for a product, the unit vector for a slack.
__device__ __forceinline__ double nv_lp_col(const NvLpArgs &A, uint32_t q, uint32_t i)
{
    return q < A.n ? A.Am[static_cast<uint64_t>(i) * A.n + q] : (q - A.n == i ? 1.0 : 0.0);
}

}  // namespace

// Iteration t's linear subproblem for replication blockIdx.x (BLOCK threads).
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void nv_lp_subproblem_kernel(NvLpArgs A, uint64_t t)
{
    __shared__ double sB[kNvLpMaxM][2 * kNvLpMaxM];     // columns M..2M-1: the basis inverse
    __shared__ double sxb[kNvLpMaxM], sy[kNvLpMaxM], sd[kNvLpMaxM], sprow[kNvLpMaxM];
    __shared__ uint32_t sbasis[kNvLpMaxM];
    __shared__ double wv[BLOCK / 64];
    __shared__ uint32_t wj[BLOCK / 64];
    __shared__ double s_gx;
    __shared__ uint32_t s_q, s_leave;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    const uint32_t r = blockIdx.x, M = A.M, n = A.n;
    const double *g = A.g + static_cast<uint64_t>(r) * n;
    const double *x = A.x + static_cast<uint64_t>(r) * n;

    // g'x of the current iterate, in a fixed order (threads in order, then a tree of wavefronts)
    {
        double acc = 0.0;
        for (uint32_t j = tid; j < n; j += BLOCK) acc = __dadd_rn(acc, __dmul_rn(g[j], x[j]));
        acc = dpp_sum64(acc);   // the xor butterfly's pairing, on DPP and the lane swaps
        if (lane == 0) wv[wave] = acc;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int w = 0; w < BLOCK / 64; ++w) s = __dadd_rn(s, wv[w]);
            s_gx = s;
        }
        __syncthreads();
    }

    // the slack basis: B = I, so B^-1 = I and x_B = C (a fresh start every iteration: the resampled
    // gradient moves the optimum to other products, so the previous basis is no better a start)
    if (tid < M * M) {
        const uint32_t i = tid / M, k = tid % M;
        sB[i][M + k] = i == k ? 1.0 : 0.0;
    }
    if (tid < M) {
        sbasis[tid] = n + tid;
        sxb[tid] = A.Cv[tid];
    }
    __syncthreads();

    uint32_t pivots = 0, degenerate = 0;
    bool solved = false;
    for (;;) {
        // y' = c_B' B^-1 (c_B: the gradient of basic products, 0 for slacks)
        if (tid < M) {
            double v = 0.0;
            for (uint32_t i = 0; i < M; ++i) {
                const double cb = sbasis[i] < n ? g[sbasis[i]] : 0.0;
                v = __dadd_rn(v, __dmul_rn(cb, sB[i][M + tid]));
            }
            sy[tid] = v;
        }
        __syncthreads();
        // pricing over the n + M columns: the most negative reduced cost (Dantzig), or after 2M + 2
        // degenerate pivots in a row the lowest column with a negative one (Bland)
        const bool bland = degenerate > 2 * M + 2;
        double bv = INFINITY;
        uint32_t bj = 0xFFFFFFFFu;
        for (uint32_t j = tid; j < n + M; j += BLOCK) {
            double rc;
            if (j < n) {
                rc = g[j];
                for (uint32_t k = 0; k < M; ++k) rc = __dsub_rn(rc, __dmul_rn(sy[k], A.Am[static_cast<uint64_t>(k) * n + j]));
            } else {
                rc = -sy[j - n];
            }
            if (rc < -A.eps_r) nv_lp_better(bv, bj, bland ? 0.0 : rc, j);
        }
        dpp_argmin64(bv, bj);   // nv_lp_better's rule, the xor butterfly's pairing
        if (lane == 0) {
            wv[wave] = bv;
            wj[wave] = bj;
        }
        __syncthreads();
        if (tid == 0) {
            double v = wv[0];
            uint32_t j = wj[0];
            for (int w = 1; w < BLOCK / 64; ++w) nv_lp_better(v, j, wv[w], wj[w]);
            s_q = j;
        }
        __syncthreads();
        const uint32_t q = s_q;
        if (q == 0xFFFFFFFFu) {       // no negative reduced cost: optimal
            solved = true;
            break;
        }
        if (pivots == A.max_pivots) break;
        // d = B^-1 A_q, then the ratio test: the smallest x_B,i / d_i over d_i > eps_d (lowest i among equal ratios)
        if (tid < M) {
            double v = 0.0;
            for (uint32_t k = 0; k < M; ++k) v = __dadd_rn(v, __dmul_rn(sB[tid][M + k], nv_lp_col(A, q, k)));
            sd[tid] = v;
        }
        __syncthreads();
        if (tid == 0) {
            uint32_t leave = 0xFFFFFFFFu;
            double best = INFINITY;
            for (uint32_t i = 0; i < M; ++i)
                if (sd[i] > A.eps_d) {
                    const double ratio = __ddiv_rn(sxb[i], sd[i]);
                    if (ratio < best) {
                        best = ratio;
                        leave = i;
                    }
                }
            s_leave = leave;
        }
        __syncthreads();
        const uint32_t lv = s_leave;
        if (lv == 0xFFFFFFFFu) break;   // unbounded direction: impossible when every column has a positive entry
        const double dl = sd[lv];
        const double theta = __ddiv_rn(sxb[lv], dl);
        // the pivot: row lv divided by d_lv, the others reduced by it; x_B and the basis likewise
        if (tid < M) sprow[tid] = __ddiv_rn(sB[lv][M + tid], dl);
        __syncthreads();
        if (tid < M * M) {
            const uint32_t i = tid / M, k = tid % M;
            sB[i][M + k] = i == lv ? sprow[k] : __dsub_rn(sB[i][M + k], __dmul_rn(sd[i], sprow[k]));
        }
        if (tid < M) {
            const double v = tid == lv ? theta : __dsub_rn(sxb[tid], __dmul_rn(sd[tid], theta));
            sxb[tid] = v > 0.0 ? v : 0.0;
        }
        if (tid == 0) sbasis[lv] = q;
        degenerate = theta == 0.0 ? degenerate + 1 : 0;
        ++pivots;
        __syncthreads();
    }

    // records, the Frank-Wolfe gap g'x - g's and tau
    if (tid < M) {
        const uint64_t o = (static_cast<uint64_t>(r) * A.T + t) * M + tid;
        A.rec_basis[o] = sbasis[tid];
        A.rec_value[o] = sxb[tid];
    }
    if (tid == 0) {
        A.rec_piv[static_cast<uint64_t>(r) * A.T + t] = solved ? pivots : A.max_pivots + 1;
        double gs = 0.0;
        bool origin = true;
        for (uint32_t i = 0; i < M; ++i)
            if (sbasis[i] < n && sxb[i] > 0.0) {
                gs = __dadd_rn(gs, __dmul_rn(g[sbasis[i]], sxb[i]));
                origin = false;
            }
        if (origin) A.origin[r] += 1u;
        const double gap = __dsub_rn(s_gx, gs);
        if (A.tau[r] == kTauNone && gap <= A.gap_eps) A.tau[r] = static_cast<uint32_t>(t);
    }
}

// f(x) of Eq. (6) at the current iterate, FP64: workgroup blockIdx.x of replication blockIdx.y sums
// products [kNvCostChunk blockIdx.x, +kNvCostChunk) into a double-double partial.
__global__ __launch_bounds__(kBlock) void nv_lp_cost_kernel(NvLpArgs A)
{
    __shared__ double sm[2 * (kBlock / 64)];
    const uint32_t r = blockIdx.y, tid = threadIdx.x;
    const double *x = A.x + static_cast<uint64_t>(r) * A.n;
    const uint32_t j1 = min(A.n, (blockIdx.x + 1) * kNvCostChunk);
    double total = 0.0;
    for (uint32_t j = blockIdx.x * kNvCostChunk + tid; j < j1; j += kBlock)
        total += nv_product_cost(x[j], A.mu_d[j], A.sig_d[j], A.k_d[j], A.h_d[j], A.v_d[j]);
    double h = total, l = 0.0;
    block_sum_dd(h, l, sm);
    if (tid == 0) {
        const uint32_t nc = (A.n + kNvCostChunk - 1) / kNvCostChunk;
        double *o = A.cost_part + 2 * (static_cast<uint64_t>(r) * nc + blockIdx.x);
        o[0] = h;
        o[1] = l;
    }
}

__global__ __launch_bounds__(kBlock) void nv_lp_cost_sum_kernel(NvLpArgs A, uint32_t slot)
{
    __shared__ double sm[2 * (kBlock / 64)];
    const uint32_t r = blockIdx.x, tid = threadIdx.x;
    const uint32_t nc = (A.n + kNvCostChunk - 1) / kNvCostChunk;
    const double *p = A.cost_part + 2 * static_cast<uint64_t>(r) * nc;
    double h = 0.0, l = 0.0;
    for (uint32_t b = tid; b < nc; b += kBlock) dd_add(h, l, p[2 * b], p[2 * b + 1]);
    block_sum_dd(h, l, sm);
    if (tid == 0) A.fval[static_cast<uint64_t>(slot) * A.R + r] = h + l;
}

__global__ void nv_lp_finalize_kernel(NvLpArgs A, uint32_t n_ckpt)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    nv_stream_stats(A.fval, A.R, n_ckpt, A.stats);
    uint64_t origin = 0;
    for (uint32_t r = 0; r < A.R; ++r) origin += A.origin[r];
    *A.origin_total = origin;
}

int launch_nv_lp_gradient(const NvLpArgs &A, uint64_t t, uint32_t epoch, bool fold_prev, hipStream_t s)
{
    hipLaunchKernelGGL(nv_lp_gradient_kernel, dim3(A.nwg, A.R), dim3(kNvBlock), 0, s, A, t, epoch, fold_prev ? 1 : 0);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_nv_lp_subproblem(const NvLpArgs &A, uint64_t t, hipStream_t s)
{
    if (A.n <= kNvLpSmallN)
        hipLaunchKernelGGL(nv_lp_subproblem_kernel<kNvLpBlockSmall>, dim3(A.R), dim3(kNvLpBlockSmall), 0, s, A, t);
    else
        hipLaunchKernelGGL(nv_lp_subproblem_kernel<kNvLpBlockLarge>, dim3(A.R), dim3(kNvLpBlockLarge), 0, s, A, t);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_nv_lp_update(const NvLpArgs &A, uint64_t t, hipStream_t s)
{
    hipLaunchKernelGGL(nv_lp_update_kernel, dim3((A.n + kNvBlock - 1) / kNvBlock, A.R), dim3(kNvBlock), 0, s, A, t);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_nv_lp_cost(const NvLpArgs &A, uint32_t slot, hipStream_t s)
{
    const uint32_t nc = (A.n + kNvCostChunk - 1) / kNvCostChunk;
    hipLaunchKernelGGL(nv_lp_cost_kernel, dim3(nc, A.R), dim3(kBlock), 0, s, A);
    hipLaunchKernelGGL(nv_lp_cost_sum_kernel, dim3(A.R), dim3(kBlock), 0, s, A, slot);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_nv_lp_finalize(const NvLpArgs &A, uint32_t n_ckpt, hipStream_t s)
{
    hipLaunchKernelGGL(nv_lp_finalize_kernel, dim3(1), dim3(64), 0, s, A, n_ckpt);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_nv_sample(const NvArgs &A, uint64_t t, uint32_t epoch, float cw, bool from_x0, bool fold_prev, hipStream_t s)
{
    const int64_t prev = fold_prev ? static_cast<int64_t>(t) - 1 : -1;
    hipLaunchKernelGGL(nv_sample_kernel, dim3(A.nwg, A.R), dim3(kNvBlock), 0, s, A, epoch, cw, from_x0 ? 1 : 0, prev,
                       static_cast<uint32_t>(t & 1));
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_nv_step(const NvArgs &A, uint64_t t, hipStream_t s)
{
    hipLaunchKernelGGL(nv_step_kernel, dim3(A.R), dim3(kNvBlock), 0, s, A, t, static_cast<uint32_t>(t & 1));
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_nv_cost(const NvArgs &A, double c, uint32_t slot, hipStream_t s)
{
    const uint32_t nc = (A.n + kNvCostChunk - 1) / kNvCostChunk;
    hipLaunchKernelGGL(nv_cost_kernel, dim3(nc, A.R), dim3(kBlock), 0, s, A, c);
    hipLaunchKernelGGL(nv_cost_sum_kernel, dim3(A.R), dim3(kBlock), 0, s, A, slot);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_nv_finalize(const NvArgs &A, uint32_t n_ckpt, hipStream_t s)
{
    hipLaunchKernelGGL(nv_finalize_kernel, dim3(1), dim3(64), 0, s, A, n_ckpt);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace fw
