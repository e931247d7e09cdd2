// fw_sqn_split.hip -- Algorithms 3-4 (Section 3.3, Task 3) with each replication spread over
// one-wavefront workgroups that own 64-quad slices of the features (the launch sequence and the
// buffers are described in sqn_split.hpp). One workgroup per replication (fw_sqn.hip) streams the
// stored pairs twice per iteration through a single compute unit; here every slice streams its own
// part, and the sums over slices are taken in fixed order in the next launch.
//
// A workgroup of one wavefront has no other waves to hide a load's latency behind, so every loop
// over global memory here issues kInFlight independent loads per thread before it waits (copies
// into LDS, stored vectors in batches), and the sampled rows' bits are staged in LDS once per
// launch and read from there.
//
// Arithmetic per iteration is that of the one-workgroup kernel; only the order in which the
// dot products are summed differs (within a slice, then over slices).
#include <hip/hip_runtime.h>

#include "sqn.hpp"
#include "sqn_device.hpp"
#include "sqn_split.hpp"

namespace fw {

namespace {

constexpr uint32_t kSliceWords = 8;                      // bitmap words of a slice's 256 features
constexpr uint32_t kBitsCap = kSqnMaxB * kSliceWords;    // staged words: every row's slice
constexpr uint32_t kInFlight = 8;                        // loads issued per thread before the first wait
constexpr uint32_t kStageDoubles = 4096;                 // LDS staging of partial sums (32 KB)
constexpr uint32_t kPairBatch = 4;                       // stored pairs loaded together (two vectors each)
static_assert(kSqnMaxB >= static_cast<int>(SIM_SQN_MAX_B) && kSqnMaxM >= static_cast<int>(SIM_SQN_MAX_M) &&
                  kSqnMaxN >= SIM_SQN_MAX_N,
              "the LDS arrays hold the largest b, b_H, M and n that validation admits");
static_assert(kSplitMaxSlices * kSplitQuads * 4 >= SIM_SQN_MAX_N, "slices cover every feature");
static_assert(kStageDoubles >= kSplitMaxSlices && kStageDoubles >= 2 * kSqnMaxM * kSqnMaxM,
              "a staged block holds a row of partials and the two small matrices");

struct Slice {
    uint32_t s, rep, tid, q, qc;     // slice, replication, thread, owned quad, that quad clamped into range
    bool own;
};

__device__ __forceinline__ Slice slice_of(const SqnSplit &P)
{
    Slice c;
    c.s = blockIdx.x;
    c.rep = blockIdx.y;
    c.tid = threadIdx.x;
    c.q = c.s * kSplitQuads + c.tid;
    c.own = c.q < P.A.nq;
    c.qc = c.own ? c.q : P.A.nq - 1;
    return c;
}

// v's slice (quads owned by the workgroup, zero past n) into sv[256]
__device__ __forceinline__ void stage_slice(const Slice &c, const double (&v)[4], double *sv)
{
#pragma unroll
    for (int e = 0; e < 4; ++e) sv[4 * c.tid + e] = c.own ? v[e] : 0.0;
}

// dst[0..count) = src[0..count), global to LDS, kInFlight independent loads per thread at a time.
// count >= 1.
__device__ __forceinline__ void to_lds(const double *src, uint32_t count, double *dst)
{
    for (uint32_t base = 0; base < count; base += kInFlight * kSplitQuads) {
        double v[kInFlight];
#pragma unroll
        for (uint32_t j = 0; j < kInFlight; ++j) {
            const uint32_t u = base + j * kSplitQuads + threadIdx.x;
            v[j] = src[u < count ? u : count - 1];
        }
#pragma unroll
        for (uint32_t j = 0; j < kInFlight; ++j) {
            const uint32_t u = base + j * kSplitQuads + threadIdx.x;
            if (u < count) dst[u] = v[j];
        }
    }
}

// out[i] = sum over the W slices, in order, of part[i W + u], for i < count (count >= 1); the
// partial sums are staged through stage[kStageDoubles] a block of rows at a time. Starts and ends
// with a barrier.
__device__ __forceinline__ void reduce_slices(const double *part, uint32_t count, uint32_t W, double *stage,
                                              double *out)
{
    const uint32_t rows = kStageDoubles / W;
    for (uint32_t i0 = 0; i0 < count; i0 += rows) {
        const uint32_t cnt = min(rows, count - i0);
        __syncthreads();
        to_lds(part + static_cast<size_t>(i0) * W, cnt * W, stage);
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cnt; i += kSplitQuads) {
            double a = 0.0;
            for (uint32_t u = 0; u < W; ++u) a += stage[i * W + u];
            out[i0 + i] = a;
        }
    }
    __syncthreads();
}

// The slice's 8 bitmap words of each row idx[0..count) into bits[i * 8 + word]: two 16-byte words
// per row, kInFlight loads per thread at a time; words past the row's end are zero. The caller
// synchronises before and after.
__device__ __forceinline__ void stage_slice_bits(const SqnSplit &P, const Slice &c, const uint32_t *idx, uint32_t count,
                                                 uint32_t *bits)
{
    const SqnArgs &A = P.A;
    const uint32_t n4 = A.xw / 4, total = 2 * count;
    for (uint32_t base = 0; base < total; base += kInFlight * kSplitQuads) {
        uint4 v[kInFlight];
#pragma unroll
        for (uint32_t j = 0; j < kInFlight; ++j) {
            const uint32_t u = base + j * kSplitQuads + c.tid;
            const uint32_t uc = u < total ? u : total - 1;
            const uint32_t u4 = 2 * c.s + (uc & 1u);
            v[j] = reinterpret_cast<const uint4 *>(A.X + static_cast<size_t>(idx[uc >> 1]) * A.xw)[u4 < n4 ? u4 : n4 - 1];
        }
#pragma unroll
        for (uint32_t j = 0; j < kInFlight; ++j) {
            const uint32_t u = base + j * kSplitQuads + c.tid;
            if (u < total) {
                uint4 w = v[j];
                if (2 * c.s + (u & 1u) >= n4) w.x = w.y = w.z = w.w = 0u;
                reinterpret_cast<uint4 *>(bits)[u] = w;
            }
        }
    }
}

// Partial x_i'v over the slice for `count` staged rows, v's slice in sv: a thread per row, the
// row's eight words in order; out[i W + s].
__device__ __forceinline__ void slice_row_dots(const SqnSplit &P, const Slice &c, const uint32_t *bits, uint32_t count,
                                               const double *sv, double *out)
{
    for (uint32_t i = c.tid; i < count; i += kSplitQuads) {
        double a = 0.0;
#pragma unroll
        for (uint32_t wd = 0; wd < kSliceWords; ++wd) a += word_dot(bits[i * kSliceWords + wd], sv, 32u * wd);
        out[static_cast<size_t>(i) * P.W + c.s] = a;
    }
}

// sum over the rows of coef[i] times the owned quad's four bits (rows in order)
__device__ __forceinline__ void slice_bit_sum(const Slice &c, const uint32_t *bits, const double *coef, uint32_t count,
                                              double (&out)[4])
{
#pragma unroll
    for (int e = 0; e < 4; ++e) out[e] = 0.0;
    const uint32_t wq = c.tid >> 3, sh = 4 * (c.tid & 7);
    for (uint32_t i = 0; i < count; ++i) {
        const uint32_t x = (bits[i * kSliceWords + wq] >> sh) & 0xFu;
        const double r = coef[i];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if ((x >> e) & 1u) out[e] += r;
    }
}

// red[v][64] = vec(v)'x over the owned quad (0 for a quad past n), v < count, kInFlight vectors
// loaded at a time; vec(v) is the start of stored vector v.
template <typename PT, class VecOf>
__device__ __forceinline__ void quad_products(const Slice &c, uint32_t count, VecOf vec, const double (&x)[4], double *red)
{
    for (uint32_t v0 = 0; v0 < count; v0 += kInFlight) {
        double a[kInFlight][4];
#pragma unroll
        for (uint32_t j = 0; j < kInFlight; ++j) load4(vec(min(v0 + j, count - 1)) + 4 * c.qc, a[j]);
#pragma unroll
        for (uint32_t j = 0; j < kInFlight; ++j) {
            double p = 0.0;
#pragma unroll
            for (int e = 0; e < 4; ++e) p += a[j][e] * x[e];
            if (v0 + j < count) red[(v0 + j) * kSplitQuads + c.tid] = c.own ? p : 0.0;
        }
    }
}

// Column sums of red[v][64] for v < count (the 64 lanes' products, lanes in order) into
// out[v W + s]. Starts and ends with a barrier.
__device__ __forceinline__ void slice_column_sums(const Slice &c, double *red, uint32_t count, double *out, uint32_t W)
{
    __syncthreads();
    for (uint32_t v = c.tid; v < count; v += kSplitQuads) {
        double a = 0.0;
        for (uint32_t l = 0; l < kSplitQuads; ++l) a += red[v * kSplitQuads + l];
        out[static_cast<size_t>(v) * W + c.s] = a;
    }
    __syncthreads();
}

// w^{k+1} into the iterate and the snapshot slots, then the next iteration's partial row dot
// products (rows drawn and staged into s_idx and bits)
__device__ __forceinline__ void after_step(const SqnSplit &P, const Slice &c, const SqnSplitStep &st,
                                           const double (&w4)[4], uint32_t *s_idx, double *sv, uint32_t *bits)
{
    const SqnArgs &A = P.A;
    const size_t ld = A.ld;
    if (c.own) {
        store4(P.w + c.rep * ld + 4 * c.q, w4);
        if (st.snap >= 0) store4(A.wsnap + (static_cast<size_t>(st.snap) * A.R + c.rep) * ld + 4 * c.q, w4);
        if (st.snap_last >= 0) store4(A.wsnap + (static_cast<size_t>(st.snap_last) * A.R + c.rep) * ld + 4 * c.q, w4);
    }
    if (!st.next) return;
    __syncthreads();                                        // s_idx, sv and bits are free
    stage_slice(c, w4, sv);
    draw_rows(A, c.rep, st.k + 1, kSqnDomGrad, A.b, s_idx);
    __syncthreads();
    stage_slice_bits(P, c, s_idx, A.b, bits);
    __syncthreads();
    double *xp = P.xpart + (((st.k + 1) & 1) * A.R + c.rep) * static_cast<size_t>(A.b) * P.W;
    slice_row_dots(P, c, bits, A.b, sv, xp);
}

}  // namespace

// w^1 = 0, the window sum cleared, no pairs; the partial row dot products of iteration 1 (of w^1 = 0)
__global__ __launch_bounds__(kSplitQuads) void sqn_split_start(SqnSplit P, SqnSplitStep st)
{
    const Slice c = slice_of(P);
    const SqnArgs &A = P.A;
    const double zero[4] = {0.0, 0.0, 0.0, 0.0};
    if (c.own) {
        store4(A.acc + c.rep * static_cast<size_t>(A.ld) + 4 * c.q, zero);
        store4(P.w + c.rep * static_cast<size_t>(A.ld) + 4 * c.q, zero);
    }
    if (c.s == 0 && c.tid == 0) A.pairs[c.rep] = 0u;
    double *xp = P.xpart + ((1 & 1) * A.R + c.rep) * static_cast<size_t>(A.b) * P.W;
    for (uint32_t i = c.tid; i < A.b; i += kSplitQuads) xp[static_cast<size_t>(i) * P.W + c.s] = 0.0;
}

// Eq. (12) over the b rows of iteration k, the window sum; then the step (k <= 2L) or the partial
// S'g, Y'g (k > 2L)
template <typename PT>
__global__ __launch_bounds__(kSplitQuads) void sqn_split_grad(SqnSplit P, SqnSplitStep st)
{
    __shared__ uint32_t s_idx[kSqnMaxB];
    __shared__ double s_v[kSqnMaxB];
    __shared__ double s_coef[kSqnMaxB];
    __shared__ double sv[4 * kSplitQuads];
    __shared__ double stage[kStageDoubles];
    __shared__ union {
        uint32_t bits[kBitsCap];
        double red[2 * kSqnMaxM * kSplitQuads];
    } u;
    const Slice c = slice_of(P);
    const SqnArgs &A = P.A;
    const size_t ld = A.ld;
    const uint64_t k = st.k;

    draw_rows(A, c.rep, k, kSqnDomGrad, A.b, s_idx);
    reduce_slices(P.xpart + ((k & 1) * A.R + c.rep) * static_cast<size_t>(A.b) * P.W, A.b, P.W, stage, s_v);
    for (uint32_t i = c.tid; i < A.b; i += kSplitQuads)
        s_coef[i] = sigmoid(s_v[i]) - static_cast<double>(A.z[s_idx[i]]);
    stage_slice_bits(P, c, s_idx, A.b, u.bits);
    __syncthreads();

    double g[4], w4[4], a4[4];
    slice_bit_sum(c, u.bits, s_coef, A.b, g);
    load4(P.w + c.rep * ld + 4 * c.qc, w4);
    load4(A.acc + c.rep * ld + 4 * c.qc, a4);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        g[e] /= static_cast<double>(A.b);
        a4[e] += w4[e];
    }
    if (c.own) store4(A.acc + c.rep * ld + 4 * c.q, a4);
    const double alpha = A.beta / static_cast<double>(k);
    if (k <= 2ull * A.L) {
#pragma unroll
        for (int e = 0; e < 4; ++e) w4[e] -= alpha * g[e];
        after_step(P, c, st, w4, s_idx, sv, u.bits);
        return;
    }
    // the gradient for the direction launch, and its partial dot products with the stored pairs:
    // 2i is s_i'g, 2i + 1 is y_i'g, pair i oldest first
    if (c.own) store4(P.g + c.rep * ld + 4 * c.q, g);
    const PT *S = static_cast<const PT *>(A.S) + static_cast<size_t>(c.rep) * A.M * ld;
    const PT *Y = static_cast<const PT *>(A.Y) + static_cast<size_t>(c.rep) * A.M * ld;
    __syncthreads();                                        // the bits are read: the union turns to red
    const uint32_t head = st.head, M = A.M;
    quad_products<PT>(c, 2 * st.m, [&](uint32_t v) { return ((v & 1) ? Y : S) + ((head + (v >> 1)) % M) * ld; }, g,
                      u.red);
    slice_column_sums(c, u.red, 2 * st.m, P.dpart + static_cast<size_t>(c.rep) * 2 * A.M * P.W, P.W);
}

// S'g, Y'g over the slices; H g by the compact representation; the step
template <typename PT>
__global__ __launch_bounds__(kSplitQuads) void sqn_split_dir(SqnSplit P, SqnSplitStep st)
{
    __shared__ uint32_t s_idx[kSqnMaxB];
    __shared__ double sv[4 * kSplitQuads];
    __shared__ double stage[kStageDoubles];
    __shared__ uint32_t bits[kBitsCap];
    __shared__ double s_dots[2 * kSqnMaxM];
    __shared__ double s_cs[kSqnMaxM], s_cy[kSqnMaxM];
    const Slice c = slice_of(P);
    const SqnArgs &A = P.A;
    const size_t ld = A.ld;
    const uint32_t m = st.m;
    const double *small = P.small + static_cast<size_t>(c.rep) * kSqnSmall;

    reduce_slices(P.dpart + static_cast<size_t>(c.rep) * 2 * A.M * P.W, 2 * m, P.W, stage, s_dots);
    // R^-1 and C (their first m rows) into the staging area
    double *Ri = stage, *C = stage + kSqnMaxM * kSqnMaxM;
    to_lds(small + 2 * kSqnMaxM * kSqnMaxM, m * kSqnMaxM, Ri);
    to_lds(small + 3 * kSqnMaxM * kSqnMaxM, m * kSqnMaxM, C);
    const double gamma = small[4 * kSqnMaxM * kSqnMaxM];
    __syncthreads();
    if (c.tid < m) {
        const uint32_t i = c.tid;
        double a = 0.0, r = 0.0;
        for (uint32_t l = 0; l < m; ++l) a += C[i * kSqnMaxM + l] * s_dots[2 * l];
        for (uint32_t l = 0; l <= i; ++l) r += Ri[l * kSqnMaxM + i] * s_dots[2 * l + 1];
        s_cs[i] = a - gamma * r;
    } else if (c.tid < 2 * m) {
        const uint32_t i = c.tid - m;
        double r = 0.0;
        for (uint32_t l = i; l < m; ++l) r += Ri[i * kSqnMaxM + l] * s_dots[2 * l];
        s_cy[i] = -gamma * r;
    }
    __syncthreads();

    const PT *S = static_cast<const PT *>(A.S) + static_cast<size_t>(c.rep) * A.M * ld;
    const PT *Y = static_cast<const PT *>(A.Y) + static_cast<size_t>(c.rep) * A.M * ld;
    double g[4], w4[4], dir[4];
    load4(P.g + c.rep * ld + 4 * c.qc, g);
    load4(P.w + c.rep * ld + 4 * c.qc, w4);
#pragma unroll
    for (int e = 0; e < 4; ++e) dir[e] = gamma * g[e];
    for (uint32_t i0 = 0; i0 < m; i0 += kPairBatch) {
        double sq[kPairBatch][4], yq[kPairBatch][4];
#pragma unroll
        for (uint32_t j = 0; j < kPairBatch; ++j) {
            const size_t off = ((st.head + min(i0 + j, m - 1)) % A.M) * ld + 4 * c.qc;
            load4(S + off, sq[j]);
            load4(Y + off, yq[j]);
        }
#pragma unroll
        for (uint32_t j = 0; j < kPairBatch; ++j) {
            if (i0 + j < m) {
                const double cs = s_cs[i0 + j], cy = s_cy[i0 + j];
#pragma unroll
                for (int e = 0; e < 4; ++e) dir[e] += sq[j][e] * cs + yq[j][e] * cy;
            }
        }
    }
    const double alpha = A.beta / static_cast<double>(st.k);
#pragma unroll
    for (int e = 0; e < 4; ++e) w4[e] -= alpha * dir[e];
    after_step(P, c, st, w4, s_idx, sv, bits);
}

// The window average; s into the ring; the Hessian rows' partial dot products with wbar and s
template <typename PT>
__global__ __launch_bounds__(kSplitQuads) void sqn_split_win1(SqnSplit P, SqnSplitStep st)
{
    __shared__ uint32_t s_idx[kSqnMaxB];
    __shared__ double sv_w[4 * kSplitQuads], sv_s[4 * kSplitQuads];
    __shared__ uint32_t bits[kBitsCap];
    const Slice c = slice_of(P);
    const SqnArgs &A = P.A;
    const size_t ld = A.ld;
    double wb[4] = {0.0, 0.0, 0.0, 0.0}, sq[4] = {0.0, 0.0, 0.0, 0.0};
    PT *S = static_cast<PT *>(A.S) + static_cast<size_t>(c.rep) * A.M * ld;
    if (c.own) {
        load4(A.acc + c.rep * ld + 4 * c.q, wb);
#pragma unroll
        for (int e = 0; e < 4; ++e) wb[e] /= static_cast<double>(A.L);
        if (st.pair) {
            double pv[4];
            load4(A.wprev + c.rep * ld + 4 * c.q, pv);
#pragma unroll
            for (int e = 0; e < 4; ++e) sq[e] = wb[e] - pv[e];
            store4(S + st.slot * ld + 4 * c.q, sq);
            // s as stored (rounded to the pairs' type)
#pragma unroll
            for (int e = 0; e < 4; ++e) sq[e] = static_cast<double>(static_cast<PT>(sq[e]));
        }
        store4(A.wprev + c.rep * ld + 4 * c.q, wb);
        const double zero[4] = {0.0, 0.0, 0.0, 0.0};
        store4(A.acc + c.rep * ld + 4 * c.q, zero);
    }
    if (!st.pair) return;
    stage_slice(c, wb, sv_w);
    stage_slice(c, sq, sv_s);
    draw_rows(A, c.rep, st.k, kSqnDomHess, A.bH, s_idx);
    __syncthreads();
    stage_slice_bits(P, c, s_idx, A.bH, bits);
    __syncthreads();
    double *hp = P.hpart + static_cast<size_t>(c.rep) * 2 * A.bH * P.W;
    slice_row_dots(P, c, bits, A.bH, sv_w, hp);                                 // x_i'wbar
    slice_row_dots(P, c, bits, A.bH, sv_s, hp + static_cast<size_t>(A.bH) * P.W);   // x_i's
}

// y = Eq. (13) applied to s into the ring; the new pair's partial dot products with the stored ones
template <typename PT>
__global__ __launch_bounds__(kSplitQuads) void sqn_split_win2(SqnSplit P, SqnSplitStep st)
{
    __shared__ uint32_t s_idx[kSqnMaxB];
    __shared__ double s_v[kSqnMaxB];
    __shared__ double s_coef[kSqnMaxB];
    __shared__ double stage[kStageDoubles];
    __shared__ union {
        uint32_t bits[kBitsCap];
        double red[2 * kSqnMaxM * kSplitQuads];
    } u;
    const Slice c = slice_of(P);
    const SqnArgs &A = P.A;
    const size_t ld = A.ld;
    PT *S = static_cast<PT *>(A.S) + static_cast<size_t>(c.rep) * A.M * ld;
    PT *Y = static_cast<PT *>(A.Y) + static_cast<size_t>(c.rep) * A.M * ld;

    draw_rows(A, c.rep, st.k, kSqnDomHess, A.bH, s_idx);
    const double *hp = P.hpart + static_cast<size_t>(c.rep) * 2 * A.bH * P.W;
    reduce_slices(hp, A.bH, P.W, stage, s_v);                                    // x_i'wbar
    reduce_slices(hp + static_cast<size_t>(A.bH) * P.W, A.bH, P.W, stage, s_coef);   // x_i's
    for (uint32_t i = c.tid; i < A.bH; i += kSplitQuads) {
        const double sg = sigmoid(s_v[i]);
        s_coef[i] = sg * (1.0 - sg) * s_coef[i];
    }
    stage_slice_bits(P, c, s_idx, A.bH, u.bits);
    __syncthreads();
    double y[4], sq[4];
    slice_bit_sum(c, u.bits, s_coef, A.bH, y);
#pragma unroll
    for (int e = 0; e < 4; ++e) y[e] = c.own ? static_cast<double>(static_cast<PT>(y[e] / static_cast<double>(A.bH))) : 0.0;
    if (c.own) store4(Y + st.slot * ld + 4 * c.q, y);
    load4(S + st.slot * ld + 4 * c.qc, sq);
    __syncthreads();                                        // the bits are read: the union turns to red
    // s_i'y (v even) and y_i'y (v odd), the new pair included, oldest first. The new pair's y was
    // stored above by this thread at the quad it reads back, so the reads see it.
    const uint32_t mn = st.m_new, hn = st.head_new, M = A.M;
    quad_products<PT>(c, 2 * mn, [&](uint32_t v) { return ((v & 1) ? Y : S) + ((hn + (v >> 1)) % M) * ld; }, y,
                      u.red);
    double *yp = P.ypart + static_cast<size_t>(c.rep) * 3 * A.M * P.W;
    slice_column_sums(c, u.red, 2 * mn, yp, P.W);                 // [2i] s_i'y, [2i + 1] y_i'y
    quad_products<PT>(c, mn, [&](uint32_t v) { return Y + ((hn + v) % M) * ld; }, sq, u.red);
    slice_column_sums(c, u.red, mn, yp + static_cast<size_t>(2 * A.M) * P.W, P.W);    // s'y_i
}

// S'Y and Y'Y with the new pair, gamma, R^-1 and C = R^-T (D + gamma Y'Y) R^-1 (one workgroup
// per replication)
__global__ __launch_bounds__(kSplitQuads) void sqn_split_small(SqnSplit P, SqnSplitStep st)
{
    __shared__ double s_SY[kSqnMaxM * kSqnMaxM], s_YY[kSqnMaxM * kSqnMaxM], s_Ri[kSqnMaxM * kSqnMaxM];
    __shared__ double s_T[kSqnMaxM * kSqnMaxM];
    __shared__ double stage[kStageDoubles];
    __shared__ double s_a[2 * kSqnMaxM], s_b[kSqnMaxM];
    const uint32_t rep = blockIdx.y, tid = threadIdx.x;
    const SqnArgs &A = P.A;
    double *small = P.small + static_cast<size_t>(rep) * kSqnSmall;
    const uint32_t m_old = st.m, m = st.m_new;
    const double *yp = P.ypart + static_cast<size_t>(rep) * 3 * A.M * P.W;

    reduce_slices(yp, 2 * m, P.W, stage, s_a);                                   // s_i'y, y_i'y
    reduce_slices(yp + static_cast<size_t>(2 * A.M) * P.W, m, P.W, stage, s_b);   // s'y_i
    // the held block (oldest first), shifted by one when the oldest pair leaves
    const uint32_t sh = st.full ? 1u : 0u, keep = m_old - sh;
    if (m_old) {
        to_lds(small, 2 * kSqnMaxM * kSqnMaxM, stage);       // S'Y, then Y'Y
        __syncthreads();
        for (uint32_t v = tid; v < keep * keep; v += kSplitQuads) {
            const uint32_t i = v / keep, j = v % keep;
            s_SY[i * kSqnMaxM + j] = stage[(i + sh) * kSqnMaxM + j + sh];
            s_YY[i * kSqnMaxM + j] = stage[kSqnMaxM * kSqnMaxM + (i + sh) * kSqnMaxM + j + sh];
        }
    }
    __syncthreads();
    if (tid < m) {
        const uint32_t i = tid, n1 = m - 1;
        s_SY[n1 * kSqnMaxM + i] = s_b[i];
        s_YY[i * kSqnMaxM + n1] = s_a[2 * i + 1];
        s_YY[n1 * kSqnMaxM + i] = s_a[2 * i + 1];
    }
    __syncthreads();
    if (tid < m) s_SY[tid * kSqnMaxM + (m - 1)] = s_a[2 * tid];
    __syncthreads();
    const double gamma = s_SY[(m - 1) * kSqnMaxM + (m - 1)] / s_YY[(m - 1) * kSqnMaxM + (m - 1)];
    // R^-1 by columns: R x = e_c, back substitution
    if (tid < m) {
        const uint32_t c = tid;
        for (uint32_t i = c + 1; i < m; ++i) s_Ri[i * kSqnMaxM + c] = 0.0;
        s_Ri[c * kSqnMaxM + c] = 1.0 / s_SY[c * kSqnMaxM + c];
        for (int i = static_cast<int>(c) - 1; i >= 0; --i) {
            double acc_r = 0.0;
            for (uint32_t l = i + 1; l <= c; ++l) acc_r += s_SY[i * kSqnMaxM + l] * s_Ri[l * kSqnMaxM + c];
            s_Ri[i * kSqnMaxM + c] = -acc_r / s_SY[i * kSqnMaxM + i];
        }
    }
    __syncthreads();
    // T1 = (D + gamma Y'Y) R^-1, then C = R^-T T1
    for (uint32_t v = tid; v < m * m; v += kSplitQuads) {
        const uint32_t i = v / m, c = v % m;
        double acc_t = 0.0;
        for (uint32_t l = 0; l <= c; ++l) {
            const double dl = gamma * s_YY[i * kSqnMaxM + l] + (i == l ? s_SY[i * kSqnMaxM + i] : 0.0);
            acc_t += dl * s_Ri[l * kSqnMaxM + c];
        }
        s_T[i * kSqnMaxM + c] = acc_t;
    }
    __syncthreads();
    double *Cg = small + 3 * kSqnMaxM * kSqnMaxM;
    for (uint32_t v = tid; v < m * m; v += kSplitQuads) {
        const uint32_t i = v / m, c = v % m;
        double acc_c = 0.0;
        for (uint32_t l = 0; l <= i; ++l) acc_c += s_Ri[l * kSqnMaxM + i] * s_T[l * kSqnMaxM + c];
        Cg[i * kSqnMaxM + c] = acc_c;
    }
    for (uint32_t v = tid; v < m * m; v += kSplitQuads) {
        const uint32_t i = v / m, j = v % m;
        small[i * kSqnMaxM + j] = s_SY[i * kSqnMaxM + j];
        small[kSqnMaxM * kSqnMaxM + i * kSqnMaxM + j] = s_YY[i * kSqnMaxM + j];
        small[2 * kSqnMaxM * kSqnMaxM + i * kSqnMaxM + j] = s_Ri[i * kSqnMaxM + j];
    }
    if (tid == 0) {
        small[4 * kSqnMaxM * kSqnMaxM] = gamma;
        A.pairs[rep] = st.pairs;
    }
}

template <typename PT>
static void launch_split_kind(const SqnSplit &P, SqnSplitKernel kind, const SqnSplitStep &st, hipStream_t s)
{
    const dim3 grid(P.W, P.A.R), block(kSplitQuads);
    switch (kind) {
    case SqnSplitKernel::Start: hipLaunchKernelGGL(sqn_split_start, grid, block, 0, s, P, st); break;
    case SqnSplitKernel::Grad: hipLaunchKernelGGL(sqn_split_grad<PT>, grid, block, 0, s, P, st); break;
    case SqnSplitKernel::Dir: hipLaunchKernelGGL(sqn_split_dir<PT>, grid, block, 0, s, P, st); break;
    case SqnSplitKernel::Win1: hipLaunchKernelGGL(sqn_split_win1<PT>, grid, block, 0, s, P, st); break;
    case SqnSplitKernel::Win2: hipLaunchKernelGGL(sqn_split_win2<PT>, grid, block, 0, s, P, st); break;
    case SqnSplitKernel::Small: hipLaunchKernelGGL(sqn_split_small, dim3(1, P.A.R), block, 0, s, P, st); break;
    }
}

int launch_sqn_split(const SqnSplit &P, SqnSplitKernel kind, const SqnSplitStep &st, hipStream_t s)
{
    if (P.A.pairs_fp32) launch_split_kind<float>(P, kind, st, s);
    else launch_split_kind<double>(P, kind, st, s);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace fw
