// fw_sqn_split.hip -- Algorithms 3-4 (Section 3.3, Task 3) with each replication spread over
// workgroups that own 64-quad slices of the features (the launch sequence and the buffers are
// described in sqn_split.hpp). One workgroup per replication (fw_sqn.hip) streams the stored pairs
// twice per iteration through a single compute unit; here every slice streams its own part, and
// the sums over slices are taken in fixed order in the next launch.
//
// A launch does little work per slice, so its time is the chain of dependent global round trips.
// Each kernel therefore issues every load it will need before it waits for any: the stored vectors
// (spread over the four wavefronts by index), the slice's quads of the iterate, the sampled rows'
// bits (this iteration's and, where the launch also steps, the next iteration's, whose indices
// depend only on the counter), and the partial sums of the previous launch (a thread per sum, all
// slices' partials loaded together). Values per quad (the gradient, the direction, y) end up alike
// in every wavefront (the rows' sums are split into four contiguous quarters, one per wavefront,
// and the quarters added in order) and are stored by the first.
//
// Arithmetic per iteration is that of the one-workgroup kernel; only the order of some sums differs:
// dot products within a slice, then over slices; the direction over the pairs each wavefront holds,
// then over wavefronts; the gradient and y over quarters of the rows, then over quarters.
#include <hip/hip_runtime.h>

#include "sqn.hpp"
#include "sqn_device.hpp"
#include "sqn_split.hpp"

namespace fw {

namespace {

constexpr uint32_t kSliceWords = 8;                      // bitmap words of a slice's 256 features
constexpr uint32_t kBitsCap = kSqnMaxB * kSliceWords;    // staged words: every row's slice
constexpr uint32_t kInFlight = 8;                        // loads per thread per batch of a copy
constexpr uint32_t kVecPerWave = 2 * kSqnMaxM / kSplitWaves;   // stored vectors a thread holds (16)
constexpr uint32_t kPairPerWave = kSqnMaxM / kSplitWaves;      // stored pairs a thread holds (8)
static_assert(kSqnMaxB >= static_cast<int>(SIM_SQN_MAX_B) && kSqnMaxM >= static_cast<int>(SIM_SQN_MAX_M) &&
                  kSqnMaxN >= SIM_SQN_MAX_N,
              "the LDS arrays hold the largest b, b_H, M and n that validation admits");
static_assert(kSplitMaxSlices * kSplitQuads * 4 >= SIM_SQN_MAX_N, "slices cover every feature");
static_assert(2 * kSqnMaxM <= kSplitQuads, "a thread per stored vector in the column sums");

struct Slice {
    uint32_t s, rep, tid, ql, wv;    // slice, replication, thread, quad within the slice, wavefront
    uint32_t q, qc;                  // the quad, and the quad clamped into range (for loads)
    bool own, owner;                 // q < nq; own and in the first wavefront (stores)
};

__device__ __forceinline__ Slice slice_of(const SqnSplit &P)
{
    Slice c;
    c.s = blockIdx.x;
    c.rep = blockIdx.y;
    c.tid = threadIdx.x;
    c.ql = c.tid % kSplitQuads;
    c.wv = c.tid / kSplitQuads;
    c.q = c.s * kSplitQuads + c.ql;
    c.own = c.q < P.A.nq;
    c.owner = c.own && c.wv == 0;
    c.qc = c.own ? c.q : P.A.nq - 1;
    return c;
}

// v's slice (zero past n) into sv[256], by the first wavefront
__device__ __forceinline__ void stage_slice(const Slice &c, const double (&v)[4], double *sv)
{
    if (c.wv == 0) {
#pragma unroll
        for (int e = 0; e < 4; ++e) sv[4 * c.ql + e] = c.own ? v[e] : 0.0;
    }
}

// dst[0..count) = src[0..count), global to LDS, kInFlight loads per thread at a time. count >= 1.
__device__ __forceinline__ void to_lds(const double *src, uint32_t count, double *dst)
{
    for (uint32_t base = 0; base < count; base += kInFlight * kSplitThreads) {
        double v[kInFlight];
#pragma unroll
        for (uint32_t j = 0; j < kInFlight; ++j) {
            const uint32_t u = base + j * kSplitThreads + threadIdx.x;
            v[j] = src[u < count ? u : count - 1];
        }
#pragma unroll
        for (uint32_t j = 0; j < kInFlight; ++j) {
            const uint32_t u = base + j * kSplitThreads + threadIdx.x;
            if (u < count) dst[u] = v[j];
        }
    }
}

// The sum over the W slices, in order, of part[i W + u], all W partials loaded together.
__device__ __forceinline__ double sum_slices(const double *part, uint32_t i, uint32_t W)
{
    const double *p = part + static_cast<size_t>(i) * W;
    double v[kSplitMaxSlices];
#pragma unroll
    for (uint32_t u = 0; u < kSplitMaxSlices; ++u) v[u] = p[u < W ? u : W - 1];
    double a = 0.0;
#pragma unroll
    for (uint32_t u = 0; u < kSplitMaxSlices; ++u)
        if (u < W) a += v[u];
    return a;
}

// The slice's 8 bitmap words of each row idx[0..count) into bits[i * 8 + word]: two 16-byte words
// per row, kInFlight loads per thread at a time; words past the row's end are zero. The caller
// synchronises before and after.
__device__ __forceinline__ void stage_slice_bits(const SqnSplit &P, const Slice &c, const uint32_t *idx, uint32_t count,
                                                 uint32_t *bits)
{
    const SqnArgs &A = P.A;
    const uint32_t n4 = A.xw / 4, total = 2 * count;
    for (uint32_t base = 0; base < total; base += kInFlight * kSplitThreads) {
        uint4 v[kInFlight];
#pragma unroll
        for (uint32_t j = 0; j < kInFlight; ++j) {
            const uint32_t u = base + j * kSplitThreads + c.tid;
            const uint32_t uc = u < total ? u : total - 1;
            const uint32_t u4 = 2 * c.s + (uc & 1u);
            v[j] = reinterpret_cast<const uint4 *>(A.X + static_cast<size_t>(idx[uc >> 1]) * A.xw)[u4 < n4 ? u4 : n4 - 1];
        }
#pragma unroll
        for (uint32_t j = 0; j < kInFlight; ++j) {
            const uint32_t u = base + j * kSplitThreads + c.tid;
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
    for (uint32_t i = c.tid; i < count; i += kSplitThreads) {
        double a = 0.0;
#pragma unroll
        for (uint32_t wd = 0; wd < kSliceWords; ++wd) a += word_dot(bits[i * kSliceWords + wd], sv, 32u * wd);
        out[static_cast<size_t>(i) * P.W + c.s] = a;
    }
}

// The sum over the rows of coef[i] times the quad's four bits: each wavefront sums a contiguous
// quarter of the rows in order, then every thread adds the four quarters in order (part: LDS
// [kSplitWaves][64][4]). Every thread of the workgroup must call it; it synchronises.
__device__ __forceinline__ void slice_bit_sum(const Slice &c, const uint32_t *bits, const double *coef, uint32_t count,
                                              double (*part)[kSplitQuads][4], double (&out)[4])
{
    const uint32_t per = (count + kSplitWaves - 1) / kSplitWaves;
    const uint32_t i0 = min(count, c.wv * per), i1 = min(count, i0 + per);
    const uint32_t wq = c.ql >> 3, sh = 4 * (c.ql & 7);
    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 8
    for (uint32_t i = i0; i < i1; ++i) {
        const uint32_t x = (bits[i * kSliceWords + wq] >> sh) & 0xFu;
        const double r = coef[i];
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if ((x >> e) & 1u) a[e] += r;
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) part[c.wv][c.ql][e] = a[e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        double t = part[0][c.ql][e];
        for (uint32_t u = 1; u < kSplitWaves; ++u) t += part[u][c.ql][e];
        out[e] = t;
    }
}

__device__ __forceinline__ double dot4(const double (&a)[4], const double (&b)[4])
{
    double p = 0.0;
#pragma unroll
    for (int e = 0; e < 4; ++e) p += a[e] * b[e];
    return p;
}

// Column sums of red[v][64] for v < count (the 64 quads' products, in order) into out[v W + s].
// The caller synchronises before.
__device__ __forceinline__ void slice_column_sums(const Slice &c, const double *red, uint32_t count, double *out,
                                                  uint32_t W)
{
    for (uint32_t v = c.tid; v < count; v += kSplitThreads) {
        double a = 0.0;
#pragma unroll 16
        for (uint32_t l = 0; l < kSplitQuads; ++l) a += red[v * kSplitQuads + l];
        out[static_cast<size_t>(v) * W + c.s] = a;
    }
}

// w^{k+1} into the iterate and the snapshot slots; the next iteration's partial row dot products
// from its staged rows (bits_next). Every thread holds the same w4 for its quad.
__device__ __forceinline__ void after_step(const SqnSplit &P, const Slice &c, const SqnSplitStep &st,
                                           const double (&w4)[4], double *sv, const uint32_t *bits_next)
{
    const SqnArgs &A = P.A;
    const size_t ld = A.ld;
    if (c.owner) {
        store4(P.w + c.rep * ld + 4 * c.q, w4);
        if (st.snap >= 0) store4(A.wsnap + (static_cast<size_t>(st.snap) * A.R + c.rep) * ld + 4 * c.q, w4);
        if (st.snap_last >= 0) store4(A.wsnap + (static_cast<size_t>(st.snap_last) * A.R + c.rep) * ld + 4 * c.q, w4);
    }
    if (!st.next) return;
    stage_slice(c, w4, sv);
    __syncthreads();
    double *xp = P.xpart + (((st.k + 1) & 1) * A.R + c.rep) * static_cast<size_t>(A.b) * P.W;
    slice_row_dots(P, c, bits_next, A.b, sv, xp);
}

}  // namespace

// w^1 = 0, the window sum cleared, no pairs; the partial row dot products of iteration 1 (of w^1 = 0)
__global__ __launch_bounds__(kSplitThreads) void sqn_split_start(SqnSplit P, SqnSplitStep st)
{
    const Slice c = slice_of(P);
    const SqnArgs &A = P.A;
    const double zero[4] = {0.0, 0.0, 0.0, 0.0};
    if (c.owner) {
        store4(A.acc + c.rep * static_cast<size_t>(A.ld) + 4 * c.q, zero);
        store4(P.w + c.rep * static_cast<size_t>(A.ld) + 4 * c.q, zero);
    }
    if (c.s == 0 && c.tid == 0) A.pairs[c.rep] = 0u;
    double *xp = P.xpart + ((1 & 1) * A.R + c.rep) * static_cast<size_t>(A.b) * P.W;
    for (uint32_t i = c.tid; i < A.b; i += kSplitThreads) xp[static_cast<size_t>(i) * P.W + c.s] = 0.0;
}

// Eq. (12) over the b rows of iteration k, the window sum; then the step and the next iteration's
// partial row dot products (k <= 2L), or the gradient and the partial S'g, Y'g (k > 2L)
template <typename PT>
__global__ __launch_bounds__(kSplitThreads) void sqn_split_grad(SqnSplit P, SqnSplitStep st)
{
    __shared__ uint32_t s_idx[kSqnMaxB], s_idx_next[kSqnMaxB];
    __shared__ double s_coef[kSqnMaxB];
    __shared__ double sv[4 * kSplitQuads];
    __shared__ uint32_t bits[kBitsCap], bits_next[kBitsCap];
    __shared__ double red[2 * kSqnMaxM * kSplitQuads];
    __shared__ double s_part[kSplitWaves][kSplitQuads][4];
    const Slice c = slice_of(P);
    const SqnArgs &A = P.A;
    const size_t ld = A.ld;
    const uint64_t k = st.k;
    const bool qn = k > 2ull * A.L;                         // a quasi-Newton iteration
    const bool steps = !qn && st.next;                      // this launch also stages iteration k + 1

    draw_rows(A, c.rep, k, kSqnDomGrad, A.b, s_idx);
    if (steps) draw_rows(A, c.rep, k + 1, kSqnDomGrad, A.b, s_idx_next);
    __syncthreads();
    // every load of the launch: the stored vectors, the quad of w and of the window sum, the rows'
    // bits, the partial row dot products with the labels
    const PT *S = static_cast<const PT *>(A.S) + static_cast<size_t>(c.rep) * A.M * ld;
    const PT *Y = static_cast<const PT *>(A.Y) + static_cast<size_t>(c.rep) * A.M * ld;
    const uint32_t nv = qn ? 2 * st.m : 0u;
    double x[kVecPerWave][4];
#pragma unroll
    for (uint32_t j = 0; j < kVecPerWave; ++j) {
        const uint32_t v = c.wv + kSplitWaves * j;
        if (v < nv) load4(((v & 1) ? Y : S) + ((st.head + (v >> 1)) % A.M) * ld + 4 * c.qc, x[j]);
    }
    double w4[4], a4[4];
    load4(P.w + c.rep * ld + 4 * c.qc, w4);
    load4(A.acc + c.rep * ld + 4 * c.qc, a4);
    stage_slice_bits(P, c, s_idx, A.b, bits);
    if (steps) stage_slice_bits(P, c, s_idx_next, A.b, bits_next);
    const double *xp = P.xpart + ((k & 1) * A.R + c.rep) * static_cast<size_t>(A.b) * P.W;
    for (uint32_t i = c.tid; i < A.b; i += kSplitThreads) {
        const double zi = static_cast<double>(A.z[s_idx[i]]);
        s_coef[i] = sigmoid(sum_slices(xp, i, P.W)) - zi;
    }
    __syncthreads();

    double g[4];
    slice_bit_sum(c, bits, s_coef, A.b, s_part, g);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        g[e] /= static_cast<double>(A.b);
        a4[e] += w4[e];
    }
    if (c.owner) store4(A.acc + c.rep * ld + 4 * c.q, a4);
    if (!qn) {
        const double alpha = A.beta / static_cast<double>(k);
#pragma unroll
        for (int e = 0; e < 4; ++e) w4[e] -= alpha * g[e];
        after_step(P, c, st, w4, sv, bits_next);
        return;
    }
    // the gradient for the direction launch, and its partial dot products with the stored pairs:
    // 2i is s_i'g, 2i + 1 is y_i'g, pair i oldest first
    if (c.owner) store4(P.g + c.rep * ld + 4 * c.q, g);
#pragma unroll
    for (uint32_t j = 0; j < kVecPerWave; ++j) {
        const uint32_t v = c.wv + kSplitWaves * j;
        if (v < nv) red[v * kSplitQuads + c.ql] = c.own ? dot4(x[j], g) : 0.0;
    }
    __syncthreads();
    slice_column_sums(c, red, nv, P.dpart + static_cast<size_t>(c.rep) * 2 * A.M * P.W, P.W);
}

// S'g, Y'g over the slices; H g by the compact representation; the step; the next iteration's
// partial row dot products
template <typename PT>
__global__ __launch_bounds__(kSplitThreads) void sqn_split_dir(SqnSplit P, SqnSplitStep st)
{
    __shared__ uint32_t s_idx_next[kSqnMaxB];
    __shared__ double sv[4 * kSplitQuads];
    __shared__ uint32_t bits_next[kBitsCap];
    __shared__ double s_Ri[kSqnMaxM * kSqnMaxM], s_C[kSqnMaxM * kSqnMaxM];
    __shared__ double s_dots[2 * kSqnMaxM];
    __shared__ double s_cs[kSqnMaxM], s_cy[kSqnMaxM];
    __shared__ double s_pd[kSplitWaves][kSplitQuads][4];
    const Slice c = slice_of(P);
    const SqnArgs &A = P.A;
    const size_t ld = A.ld;
    const uint32_t m = st.m;
    const double *small = P.small + static_cast<size_t>(c.rep) * kSqnSmall;

    if (st.next) draw_rows(A, c.rep, st.k + 1, kSqnDomGrad, A.b, s_idx_next);
    __syncthreads();
    // every load of the launch: the pairs this wavefront holds (i = wv + 4 j), the quad of g and
    // of w, the next rows' bits, R^-1 and C, the partial S'g, Y'g, gamma
    const PT *S = static_cast<const PT *>(A.S) + static_cast<size_t>(c.rep) * A.M * ld;
    const PT *Y = static_cast<const PT *>(A.Y) + static_cast<size_t>(c.rep) * A.M * ld;
    double sq[kPairPerWave][4], yq[kPairPerWave][4];
#pragma unroll
    for (uint32_t j = 0; j < kPairPerWave; ++j) {
        const uint32_t i = c.wv + kSplitWaves * j;
        if (i < m) {
            const size_t off = ((st.head + i) % A.M) * ld + 4 * c.qc;
            load4(S + off, sq[j]);
            load4(Y + off, yq[j]);
        }
    }
    double g[4], w4[4];
    load4(P.g + c.rep * ld + 4 * c.qc, g);
    load4(P.w + c.rep * ld + 4 * c.qc, w4);
    if (st.next) stage_slice_bits(P, c, s_idx_next, A.b, bits_next);
    to_lds(small + 2 * kSqnMaxM * kSqnMaxM, m * kSqnMaxM, s_Ri);
    to_lds(small + 3 * kSqnMaxM * kSqnMaxM, m * kSqnMaxM, s_C);
    const double *dp = P.dpart + static_cast<size_t>(c.rep) * 2 * A.M * P.W;
    for (uint32_t v = c.tid; v < 2 * m; v += kSplitThreads) s_dots[v] = sum_slices(dp, v, P.W);
    const double gamma = small[4 * kSqnMaxM * kSqnMaxM];
    __syncthreads();
    if (c.tid < m) {
        const uint32_t i = c.tid;
        double a = 0.0, r = 0.0;
#pragma unroll 8
        for (uint32_t l = 0; l < m; ++l) a += s_C[i * kSqnMaxM + l] * s_dots[2 * l];
#pragma unroll 8
        for (uint32_t l = 0; l <= i; ++l) r += s_Ri[l * kSqnMaxM + i] * s_dots[2 * l + 1];
        s_cs[i] = a - gamma * r;
    } else if (c.tid < 2 * m) {
        const uint32_t i = c.tid - m;
        double r = 0.0;
#pragma unroll 8
        for (uint32_t l = i; l < m; ++l) r += s_Ri[i * kSqnMaxM + l] * s_dots[2 * l];
        s_cy[i] = -gamma * r;
    }
    __syncthreads();
    // this wavefront's pairs, oldest first, then the four wavefronts' sums in order
    double pd[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (uint32_t j = 0; j < kPairPerWave; ++j) {
        const uint32_t i = c.wv + kSplitWaves * j;
        if (i < m) {
            const double cs = s_cs[i], cy = s_cy[i];
#pragma unroll
            for (int e = 0; e < 4; ++e) pd[e] += sq[j][e] * cs + yq[j][e] * cy;
        }
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) s_pd[c.wv][c.ql][e] = pd[e];
    __syncthreads();
    const double alpha = A.beta / static_cast<double>(st.k);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
        double dir = gamma * g[e];
        for (uint32_t u = 0; u < kSplitWaves; ++u) dir += s_pd[u][c.ql][e];
        w4[e] -= alpha * dir;
    }
    after_step(P, c, st, w4, sv, bits_next);
}

// The window average; s into the ring; the Hessian rows' partial dot products with wbar and s
template <typename PT>
__global__ __launch_bounds__(kSplitThreads) void sqn_split_win1(SqnSplit P, SqnSplitStep st)
{
    __shared__ uint32_t s_idx[kSqnMaxB];
    __shared__ double sv_w[4 * kSplitQuads], sv_s[4 * kSplitQuads];
    __shared__ uint32_t bits[kBitsCap];
    const Slice c = slice_of(P);
    const SqnArgs &A = P.A;
    const size_t ld = A.ld;
    PT *S = static_cast<PT *>(A.S) + static_cast<size_t>(c.rep) * A.M * ld;
    if (st.pair) {
        draw_rows(A, c.rep, st.k, kSqnDomHess, A.bH, s_idx);
        __syncthreads();
    }
    double wb[4], pv[4], sq[4] = {0.0, 0.0, 0.0, 0.0};
    load4(A.acc + c.rep * ld + 4 * c.qc, wb);
    load4(A.wprev + c.rep * ld + 4 * c.qc, pv);
    if (st.pair) stage_slice_bits(P, c, s_idx, A.bH, bits);
#pragma unroll
    for (int e = 0; e < 4; ++e) wb[e] /= static_cast<double>(A.L);
    if (st.pair) {
#pragma unroll
        for (int e = 0; e < 4; ++e) sq[e] = wb[e] - pv[e];
        if (c.owner) store4(S + st.slot * ld + 4 * c.q, sq);
        // s as stored (rounded to the pairs' type)
#pragma unroll
        for (int e = 0; e < 4; ++e) sq[e] = static_cast<double>(static_cast<PT>(sq[e]));
    }
    if (c.owner) {
        store4(A.wprev + c.rep * ld + 4 * c.q, wb);
        const double zero[4] = {0.0, 0.0, 0.0, 0.0};
        store4(A.acc + c.rep * ld + 4 * c.q, zero);
    }
    if (!st.pair) return;
    stage_slice(c, wb, sv_w);
    stage_slice(c, sq, sv_s);
    __syncthreads();
    double *hp = P.hpart + static_cast<size_t>(c.rep) * 2 * A.bH * P.W;
    slice_row_dots(P, c, bits, A.bH, sv_w, hp);                                     // x_i'wbar
    slice_row_dots(P, c, bits, A.bH, sv_s, hp + static_cast<size_t>(A.bH) * P.W);   // x_i's
}

// y = Eq. (13) applied to s into the ring; the new pair's partial dot products with the stored ones
template <typename PT>
__global__ __launch_bounds__(kSplitThreads) void sqn_split_win2(SqnSplit P, SqnSplitStep st)
{
    __shared__ uint32_t s_idx[kSqnMaxB];
    __shared__ double s_coef[kSqnMaxB];
    __shared__ uint32_t bits[kBitsCap];
    __shared__ double red[2 * kSqnMaxM * kSplitQuads], red_s[kSqnMaxM * kSplitQuads];
    __shared__ double s_part[kSplitWaves][kSplitQuads][4];
    const Slice c = slice_of(P);
    const SqnArgs &A = P.A;
    const size_t ld = A.ld;
    PT *S = static_cast<PT *>(A.S) + static_cast<size_t>(c.rep) * A.M * ld;
    PT *Y = static_cast<PT *>(A.Y) + static_cast<size_t>(c.rep) * A.M * ld;
    const uint32_t mn = st.m_new, hn = st.head_new;

    draw_rows(A, c.rep, st.k, kSqnDomHess, A.bH, s_idx);
    __syncthreads();
    // every load of the launch: the pairs this wavefront holds after the insertion (the new pair's
    // y is formed below and taken from registers), s, the rows' bits, the partial row dot products
    double sp[kPairPerWave][4], yp[kPairPerWave][4], sq[4];
#pragma unroll
    for (uint32_t j = 0; j < kPairPerWave; ++j) {
        const uint32_t i = c.wv + kSplitWaves * j;
        if (i < mn) {
            const size_t off = ((hn + i) % A.M) * ld + 4 * c.qc;
            load4(S + off, sp[j]);
            load4(Y + off, yp[j]);
        }
    }
    load4(S + st.slot * ld + 4 * c.qc, sq);
    stage_slice_bits(P, c, s_idx, A.bH, bits);
    const double *hp = P.hpart + static_cast<size_t>(c.rep) * 2 * A.bH * P.W;
    for (uint32_t i = c.tid; i < A.bH; i += kSplitThreads) {
        const double sg = sigmoid(sum_slices(hp, i, P.W));
        s_coef[i] = sg * (1.0 - sg) * sum_slices(hp + static_cast<size_t>(A.bH) * P.W, i, P.W);
    }
    __syncthreads();
    double y[4];
    slice_bit_sum(c, bits, s_coef, A.bH, s_part, y);
#pragma unroll
    for (int e = 0; e < 4; ++e) y[e] = static_cast<double>(static_cast<PT>(y[e] / static_cast<double>(A.bH)));
    if (c.owner) store4(Y + st.slot * ld + 4 * c.q, y);
    // [2i] s_i'y, [2i + 1] y_i'y into red; s'y_i into red_s
#pragma unroll
    for (uint32_t j = 0; j < kPairPerWave; ++j) {
        const uint32_t i = c.wv + kSplitWaves * j;
        if (i < mn) {
            const bool fresh = (hn + i) % A.M == st.slot;
            double yi[4];
#pragma unroll
            for (int e = 0; e < 4; ++e) yi[e] = fresh ? y[e] : yp[j][e];
            red[(2 * i) * kSplitQuads + c.ql] = c.own ? dot4(sp[j], y) : 0.0;
            red[(2 * i + 1) * kSplitQuads + c.ql] = c.own ? dot4(yi, y) : 0.0;
            red_s[i * kSplitQuads + c.ql] = c.own ? dot4(yi, sq) : 0.0;
        }
    }
    __syncthreads();
    double *ypt = P.ypart + static_cast<size_t>(c.rep) * 3 * A.M * P.W;
    slice_column_sums(c, red, 2 * mn, ypt, P.W);
    slice_column_sums(c, red_s, mn, ypt + static_cast<size_t>(2 * A.M) * P.W, P.W);
}

// S'Y and Y'Y with the new pair, gamma, R^-1 and C = R^-T (D + gamma Y'Y) R^-1 (one workgroup
// per replication)
__global__ __launch_bounds__(kSplitThreads) void sqn_split_small(SqnSplit P, SqnSplitStep st)
{
    __shared__ double s_SY[kSqnMaxM * kSqnMaxM], s_YY[kSqnMaxM * kSqnMaxM], s_Ri[kSqnMaxM * kSqnMaxM];
    __shared__ double s_T[kSqnMaxM * kSqnMaxM];
    __shared__ double stage[2 * kSqnMaxM * kSqnMaxM];
    __shared__ double s_a[2 * kSqnMaxM], s_b[kSqnMaxM];
    const uint32_t rep = blockIdx.y, tid = threadIdx.x;
    const SqnArgs &A = P.A;
    double *small = P.small + static_cast<size_t>(rep) * kSqnSmall;
    const uint32_t m_old = st.m, m = st.m_new;
    const double *ypt = P.ypart + static_cast<size_t>(rep) * 3 * A.M * P.W;

    if (m_old) to_lds(small, 2 * kSqnMaxM * kSqnMaxM, stage);      // S'Y, then Y'Y
    for (uint32_t v = tid; v < 2 * m; v += kSplitThreads) s_a[v] = sum_slices(ypt, v, P.W);            // s_i'y, y_i'y
    for (uint32_t v = tid; v < m; v += kSplitThreads) s_b[v] = sum_slices(ypt + 2 * A.M * P.W, v, P.W);   // s'y_i
    __syncthreads();
    // the held block (oldest first), shifted by one when the oldest pair leaves
    const uint32_t sh = st.full ? 1u : 0u, keep = m_old - sh;
    for (uint32_t v = tid; v < keep * keep; v += kSplitThreads) {
        const uint32_t i = v / keep, j = v % keep;
        s_SY[i * kSqnMaxM + j] = stage[(i + sh) * kSqnMaxM + j + sh];
        s_YY[i * kSqnMaxM + j] = stage[kSqnMaxM * kSqnMaxM + (i + sh) * kSqnMaxM + j + sh];
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
#pragma unroll 8
            for (uint32_t l = i + 1; l <= c; ++l) acc_r += s_SY[i * kSqnMaxM + l] * s_Ri[l * kSqnMaxM + c];
            s_Ri[i * kSqnMaxM + c] = -acc_r / s_SY[i * kSqnMaxM + i];
        }
    }
    __syncthreads();
    // T1 = (D + gamma Y'Y) R^-1, then C = R^-T T1
    for (uint32_t v = tid; v < m * m; v += kSplitThreads) {
        const uint32_t i = v / m, c = v % m;
        double acc_t = 0.0;
#pragma unroll 8
        for (uint32_t l = 0; l <= c; ++l) {
            const double dl = gamma * s_YY[i * kSqnMaxM + l] + (i == l ? s_SY[i * kSqnMaxM + i] : 0.0);
            acc_t += dl * s_Ri[l * kSqnMaxM + c];
        }
        s_T[i * kSqnMaxM + c] = acc_t;
    }
    __syncthreads();
    double *Cg = small + 3 * kSqnMaxM * kSqnMaxM;
    for (uint32_t v = tid; v < m * m; v += kSplitThreads) {
        const uint32_t i = v / m, c = v % m;
        double acc_c = 0.0;
#pragma unroll 8
        for (uint32_t l = 0; l <= i; ++l) acc_c += s_Ri[l * kSqnMaxM + i] * s_T[l * kSqnMaxM + c];
        Cg[i * kSqnMaxM + c] = acc_c;
    }
    for (uint32_t v = tid; v < m * m; v += kSplitThreads) {
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
    const dim3 grid(P.W, P.A.R), block(kSplitThreads);
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
