// mlp.hip -- the control-variate surrogate h: F -> 64 -> 64 -> 1 with exact GELU (x Phi(x)),
// trained and evaluated on the matrix cores (v_mfma_f32_32x32x16_bf16: bfloat16 operands, FP32
// accumulation), plus the draws from the exact law of the path features and the FP64 moment
// reductions of the control-variate estimator.
//
// Wavefront layout: a wavefront holds 32 rows (samples), lane l = (j, h) with j = l mod 32 the row
// and h = l / 32 the half. A layer with input width K is (64 x K) x (K x 32) on the matrix cores:
// the weights are the A operand, the activations the B operand. Lane (j, h) holds, for K-step kk,
// the eight inputs u(kk, h, e) = 16 kk + 8 (e div 4) + 4 h + (e mod 4) of its row; the product
// leaves output unit U(mt, r, h) = 32 mt + 8 (r div 4) + 4 h + (r mod 4) in register r of tile mt,
// which is exactly input u(kk, h, e) of the next layer for kk = 2 mt + r div 8, e = r mod 8, so
// activations pass from layer to layer without any data movement. The A operands are bfloat16
// copies of W1, W2 and W2' laid out in that lane order (written by the parameter update), one
// 16-byte load per lane per K-step.
//
// Weight gradients contract over rows: each wavefront stores its bfloat16 gradients and
// activations transposed ([unit][row]) in LDS, and the products read eight consecutive rows per
// lane. Bias and w3 gradients, the loss, and the cross-workgroup sums stay in FP32 (fixed order),
// the FP32 master weights take an Adam step.
#include <hip/hip_runtime.h>

#include "device_reduce.hpp"
#include "device_rng.hpp"
#include "mlp.hpp"
#include "wave_dpp.hpp"

namespace fw {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef uint16_t u16x8 __attribute__((ext_vector_type(8)));

constexpr int kRowPitch = 136;   // LDS pitch (bf16 elements) of [unit][row] tiles: 272 B rows

// bfloat16 bits of x, rounded to nearest even (inputs are finite)
__device__ __forceinline__ uint16_t bf16_bits(float x)
{
    uint32_t u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return static_cast<uint16_t>(u >> 16);
}

__device__ __forceinline__ int in_unit(int kk, int h, int e) { return 16 * kk + 8 * (e >> 2) + 4 * h + (e & 3); }
__device__ __forceinline__ int out_unit(int i, int h) { return 32 * (i >> 4) + 8 * ((i & 15) >> 2) + 4 * h + (i & 3); }

__device__ __forceinline__ float gelu(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad(float a)
{
    return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) + a * 0.39894228040143268f * __expf(-0.5f * a * a);
}

__device__ __forceinline__ bf16x8 load_operand(const uint16_t *p)
{
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(p));
}

// 64 x K product of one layer for the 32 rows of this wavefront: out[16 mt + r] = unit U(mt, r, h)
template <int KS>
__device__ __forceinline__ void layer(const uint16_t *A, const bf16x8 (&b)[KS], float (&out)[32], int lane)
{
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
        f32x16 acc = {0.0f};
#pragma unroll
        for (int kk = 0; kk < KS; ++kk)
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(load_operand(A + ((mt * KS + kk) * 64 + lane) * 8), b[kk],
                                                          acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 16; ++r) out[16 * mt + r] = acc[r];
    }
}

// 32 activations of D layout -> the four K-steps of the next layer's B operand
__device__ __forceinline__ void to_operand(const float (&v)[32], bf16x8 (&b)[4])
{
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
        u16x8 u;
#pragma unroll
        for (int e = 0; e < 8; ++e) u[e] = bf16_bits(v[8 * kk + e]);
        b[kk] = __builtin_bit_cast(bf16x8, u);
    }
}

// Forward pass of the 32 rows of this wavefront. x: feature-major [F][ldx]; row index src (or
// invalid). Returns the network output (both halves), keeps pre-activations and the inputs.
template <int KS1>
__device__ __forceinline__ float forward_rows(const MlpDev &m, const float *x, uint64_t ldx, uint64_t src, bool valid,
                                             int lane, bf16x8 (&xb)[KS1], float (&a1)[32], float (&a2)[32])
{
    const int h = lane >> 5;
#pragma unroll
    for (int kk = 0; kk < KS1; ++kk) {
        u16x8 u;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int f = in_unit(kk, h, e);
            const float v = (valid && f < m.F) ? x[static_cast<uint64_t>(f) * ldx + src] : 0.0f;
            u[e] = bf16_bits(v);
        }
        xb[kk] = __builtin_bit_cast(bf16x8, u);
    }
    const float *b1 = m.theta + m.off_b1, *b2 = m.theta + m.off_b2, *w3 = m.theta + m.off_w3;
    layer<KS1>(m.w1a, xb, a1, lane);
    float h1[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        a1[i] += b1[out_unit(i, h)];
        h1[i] = gelu(a1[i]);
    }
    bf16x8 hb[4];
    to_operand(h1, hb);
    layer<4>(m.w2a, hb, a2, lane);
    float part = 0.0f;
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        a2[i] += b2[out_unit(i, h)];
        part = fmaf(w3[out_unit(i, h)], gelu(a2[i]), part);
    }
    // the two halves' partial sums over the hidden units: lane ^ 32 by the 32-lane swap
    const auto hp = __builtin_amdgcn_permlane32_swap(__float_as_uint(part), __float_as_uint(part), false, false);
    return (__uint_as_float(hp[0]) + __uint_as_float(hp[1])) + m.theta[m.off_b3];
}

template <int KS1>
__global__ __launch_bounds__(256) void mlp_forward_kernel(MlpDev m, const float *x, uint64_t ldx, uint64_t n,
                                                          float shift, float scale, float *out)
{
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint64_t row = static_cast<uint64_t>(blockIdx.x) * 128 + wave * 32 + (lane & 31);
    const bool valid = row < n;
    bf16x8 xb[KS1];
    float a1[32], a2[32];
    const float o = forward_rows<KS1>(m, x, ldx, row, valid, lane, xb, a1, a2);
    if (valid && lane < 32) out[row] = shift + scale * o;
}

// Sum over the 32 rows of one half-wavefront; every lane of the half gets the total (DPP and the
// 16-lane row swap; the pairing is the xor butterfly's, so is the rounding).
__device__ __forceinline__ float half_sum(float v) { return dpp_sum32(v); }

// Loss and gradient partials of one workgroup (128 rows): part[blockIdx][P + 1], loss at P.
// Rows: q = q0 + 128 blockIdx + 32 wave + j, data row (a q + c) mod n_data, valid while q < q_end.
template <int KS1>
__global__ __launch_bounds__(256) void mlp_grad_kernel(MlpDev m, const float *x, uint64_t ldx, const float *y,
                                                       uint64_t q0, uint64_t q_end, uint64_t a, uint64_t c,
                                                       uint64_t n_data, float inv_batch, float *part)
{
    constexpr int NF = (16 * KS1 + 31) / 32;   // 32-wide feature tiles of dW1
    // 16-byte aligned: the products read eight consecutive bfloat16 values per lane
    __shared__ __attribute__((aligned(16))) uint16_t sT2[64 * kRowPitch];   // dA2, [unit][row]
    __shared__ __attribute__((aligned(16))) uint16_t sH1[64 * kRowPitch];   // h1
    __shared__ __attribute__((aligned(16))) uint16_t sT1[64 * kRowPitch];   // dA1
    __shared__ __attribute__((aligned(16))) uint16_t sX[32 * NF * kRowPitch];
    __shared__ float sRed[4][3][64];           // per-wave sums of dA2, dA1, dout h2
    __shared__ float sRow[4][2];               // per-wave sums of dout and squared error

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int h = lane >> 5, j = lane & 31;
    const int rb = wave * 32 + j;              // row within the workgroup
    const uint64_t q = q0 + static_cast<uint64_t>(blockIdx.x) * 128 + rb;
    const bool valid = q < q_end;
    const uint64_t src = valid ? (a * q + c) % n_data : 0;
    const float *w3 = m.theta + m.off_w3;

    bf16x8 xb[KS1];
    float a1[32], a2[32];
    const float out = forward_rows<KS1>(m, x, ldx, src, valid, lane, xb, a1, a2);
    const float err = valid ? out - y[src] : 0.0f;
    const float dout = 2.0f * err * inv_batch;

    // backward through layer 3 and the second GELU; keep h2 for the w3 gradient
    float g2[32], hw3[32];
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const int u = out_unit(i, h);
        hw3[i] = dout * gelu(a2[i]);
        g2[i] = dout * w3[u] * gelu_grad(a2[i]);
    }
    // dH1 = W2' dA2, then the first GELU
    bf16x8 gb[4];
    to_operand(g2, gb);
    float g1[32];
    layer<4>(m.w2t, gb, g1, lane);
#pragma unroll
    for (int i = 0; i < 32; ++i) g1[i] *= gelu_grad(a1[i]);

    // transposed bfloat16 tiles for the weight gradients
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const int u = out_unit(i, h);
        sT2[u * kRowPitch + rb] = bf16_bits(g2[i]);
        sH1[u * kRowPitch + rb] = bf16_bits(gelu(a1[i]));
        sT1[u * kRowPitch + rb] = bf16_bits(g1[i]);
    }
#pragma unroll
    for (int kk = 0; kk < KS1; ++kk) {
        const u16x8 u = __builtin_bit_cast(u16x8, xb[kk]);
#pragma unroll
        for (int e = 0; e < 8; ++e) sX[in_unit(kk, h, e) * kRowPitch + rb] = u[e];
    }
    if constexpr (32 * NF > 16 * KS1) {
        for (int f = 16 * KS1; f < 32 * NF; ++f)
            if (h == 0) sX[f * kRowPitch + rb] = 0;
    }

    // bias, w3, loss: FP32 sums over rows in a fixed tree
#pragma unroll
    for (int i = 0; i < 32; ++i) {
        const float s2 = half_sum(g2[i]);
        const float s1 = half_sum(g1[i]);
        const float s3 = half_sum(hw3[i]);
        if (j == 0) {
            const int u = out_unit(i, h);
            sRed[wave][0][u] = s2;
            sRed[wave][1][u] = s1;
            sRed[wave][2][u] = s3;
        }
    }
    {
        const float sd = half_sum(dout);
        const float se = half_sum(err * err);
        if (lane == 0) {
            sRow[wave][0] = sd;
            sRow[wave][1] = se;
        }
    }
    __syncthreads();

    const int F = m.F;
    const int P = m.P;
    float *out_p = part + static_cast<uint64_t>(blockIdx.x) * (P + 1);
    // dW2: one 32 x 32 tile per wavefront, K = the 128 rows of the workgroup
    {
        const int mo = wave >> 1, mi = wave & 1;
        f32x16 acc = {0.0f};
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            const bf16x8 A = load_operand(sT2 + (32 * mo + j) * kRowPitch + 16 * kk + 8 * h);
            const bf16x8 Bv = load_operand(sH1 + (32 * mi + j) * kRowPitch + 16 * kk + 8 * h);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, Bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int o = 32 * mo + 8 * (r >> 2) + 4 * h + (r & 3);
            out_p[m.off_w2 + o * 64 + 32 * mi + j] = acc[r];
        }
    }
    // dW1: 2 x NF tiles over the wavefronts
    for (int t = wave; t < 2 * NF; t += 4) {
        const int mo = t & 1, mf = t >> 1;
        f32x16 acc = {0.0f};
#pragma unroll
        for (int kk = 0; kk < 8; ++kk) {
            const bf16x8 A = load_operand(sT1 + (32 * mo + j) * kRowPitch + 16 * kk + 8 * h);
            const bf16x8 Bv = load_operand(sX + (32 * mf + j) * kRowPitch + 16 * kk + 8 * h);
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, Bv, acc, 0, 0, 0);
        }
        const int f = 32 * mf + j;
        if (f < F) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int o = 32 * mo + 8 * (r >> 2) + 4 * h + (r & 3);
                out_p[o * F + f] = acc[r];
            }
        }
    }
    if (threadIdx.x < 64) {
        const int u = threadIdx.x;
        float s2 = 0.0f, s1 = 0.0f, s3 = 0.0f;
        for (int w = 0; w < 4; ++w) {
            s2 += sRed[w][0][u];
            s1 += sRed[w][1][u];
            s3 += sRed[w][2][u];
        }
        out_p[m.off_b2 + u] = s2;
        out_p[m.off_b1 + u] = s1;
        out_p[m.off_w3 + u] = s3;
        if (u == 0) {
            float sd = 0.0f, se = 0.0f;
            for (int w = 0; w < 4; ++w) {
                sd += sRow[w][0];
                se += sRow[w][1];
            }
            out_p[m.off_b3] = sd;
            out_p[P] = se;
        }
    }
}

// Position of parameter W[o][in] (K inputs, KS = K/16 steps) in the A-operand copy.
__device__ __forceinline__ int a_pos(int o, int in, int KS)
{
    const int mt = o >> 5, il = o & 31;
    const int kk = in >> 4, rem = in & 15;
    const int hh = (rem >> 2) & 1, e = 4 * (rem >> 3) + (rem & 3);
    return ((mt * KS + kk) * 64 + il + 32 * hh) * 8 + e;
}

__device__ __forceinline__ void write_copies(const MlpDev &m, int i, float w)
{
    const uint16_t b = bf16_bits(w);
    if (i < m.off_b1) {
        const int o = i / m.F, f = i - o * m.F;
        m.w1a[a_pos(o, f, m.KS1)] = b;
    } else if (i >= m.off_w2 && i < m.off_b2) {
        const int k = i - m.off_w2;
        const int o = k >> 6, in = k & 63;
        m.w2a[a_pos(o, in, 4)] = b;
        m.w2t[a_pos(in, o, 4)] = b;
    }
}

// Sum of the workgroup partials in workgroup order, then (mode 1) one Adam step on the FP32
// master weights and their bfloat16 operand copies. grad_out (optional) receives the summed
// gradient and, at P, the summed squared error; loss_out (optional) the squared error too.
__global__ __launch_bounds__(256) void mlp_reduce_kernel(MlpDev m, const float *part, uint32_t n_parts, int mode,
                                                         AdamStep s, float *mom1, float *mom2, float *grad_out,
                                                         float *loss_out)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    const int P = m.P;
    if (i > P) return;
    float g = 0.0f;
    for (uint32_t w = 0; w < n_parts; ++w) g += part[static_cast<uint64_t>(w) * (P + 1) + i];
    if (grad_out) grad_out[i] = g;
    if (i == P) {
        if (loss_out) *loss_out = g;
        return;
    }
    if (mode != 1) return;
    const float m1 = s.beta1 * mom1[i] + (1.0f - s.beta1) * g;
    const float m2 = s.beta2 * mom2[i] + (1.0f - s.beta2) * g * g;
    mom1[i] = m1;
    mom2[i] = m2;
    const float w = m.theta[i] - s.lr * (m1 * s.bc1) / (__builtin_sqrtf(m2 * s.bc2) + s.eps);
    m.theta[i] = w;
    write_copies(m, i, w);
}

// bfloat16 operand copies of the current master weights (after initialisation or an upload).
__global__ __launch_bounds__(256) void mlp_copies_kernel(MlpDev m)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < m.P) write_copies(m, i, m.theta[i]);
}

// Initial weights: W ~ N(0, 1/fan_in) from Philox stream domain 3, biases 0.
__global__ __launch_bounds__(256) void mlp_init_kernel(MlpDev m, uint64_t seed, uint32_t instance)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= m.P) return;
    const uint32_t dom = (3u << 24) | (instance & 0xFFFFFFu);
    const Block4<double> q = normals_block<double>(static_cast<uint32_t>(i) >> 2, 0u, 0u, dom,
                                                   static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
    const double z = q.z[i & 3];
    double w = 0.0;
    if (i < m.off_b1) w = z / sqrt(static_cast<double>(m.F));
    else if (i >= m.off_w2 && i < m.off_b2) w = z / 8.0;
    else if (i >= m.off_w3 && i < m.off_b3) w = z / 8.0;
    m.theta[i] = static_cast<float>(w);
}

// Draws k0 .. k0+n-1 from the exact joint law of the path features (stream domain 2 of the seed):
// per epoch e a category from the 53-bit uniform ((a >> 5) 2^26 + (b >> 6) + 1/2) 2^-53 of words
// (a, b) = (x0, x1) for even e, (x2, x3) for odd e of Philox block (e/2, 1, k, ...), weighted by the
// epoch's sums of (t+1)^2 (every category) and (t+1) (category `top`). D bounds d; BS threads per
// workgroup; CT the per-category counter (32 bits only where T(T+1)(2T+1)/6 < 2^32: d = 64 arises
// only with a dense factor, whose features need T <= 2343).
template <int D, int BS, typename CT>
__global__ __launch_bounds__(BS) void cv_aux_kernel(AuxLaw law, uint64_t k0, uint64_t n, float *x, uint64_t ldx)
{
    constexpr int LEN = D + 1;                 // categories 0..D; entries beyond d hold 2 (never <= u)
    constexpr int TOP = (LEN > 64) ? 128 : (LEN > 32) ? 64 : (LEN > 16) ? 32 : (LEN > 8) ? 16 : (LEN > 4) ? 8 : 4;
    __shared__ double s_cum[LEN];
    __shared__ CT s_cnt[LEN * BS];             // [category][thread]: integer sums of (t+1)^2
    const int tid = threadIdx.x;
    const int d = law.d;
    for (int c = tid; c < LEN; c += BS) s_cum[c] = (c <= d) ? law.cum[c] : 2.0;
#pragma unroll
    for (int c = 0; c < LEN; ++c) s_cnt[c * BS + tid] = 0;
    __syncthreads();
    const uint64_t idx = static_cast<uint64_t>(blockIdx.x) * BS + tid;
    if (idx >= n) return;
    const uint32_t k = static_cast<uint32_t>(k0 + idx);
    const uint32_t dom = (2u << 24) | (law.instance & 0xFFFFFFu);
    const uint32_t s0 = static_cast<uint32_t>(law.seed), s1 = static_cast<uint32_t>(law.seed >> 32);
    const uint64_t T = law.T, M = law.M;
    const int top = static_cast<int>(law.top);

    uint64_t cnt1 = 0;
    Words4 w{0u, 0u, 0u, 0u};
    uint32_t e = 0;
    for (uint64_t t0 = 0; t0 < T; t0 += M, ++e) {
        if ((e & 1u) == 0) w = philox4x32_10(e >> 1, 1u, k, dom, s0, s1);
        const uint32_t a = (e & 1u) ? w.x2 : w.x0, b = (e & 1u) ? w.x3 : w.x1;
        const double u = (static_cast<double>(a >> 5) * 67108864.0 + static_cast<double>(b >> 6) + 0.5) *
                         (1.0 / 9007199254740992.0);
        // category = the number of cumulative bounds <= u (the smallest c with u < cum[c])
        int c = 0;
#pragma unroll
        for (int step = TOP; step >= 1; step >>= 1)
            if (c + step <= LEN && s_cum[c + step - 1] <= u) c += step;
        const uint64_t t1 = (t0 + M < T) ? t0 + M : T;
        const uint64_t w2 = (M == 1) ? (t0 + 1) * (t0 + 1)
                                     : t1 * (t1 + 1) * (2 * t1 + 1) / 6 - t0 * (t0 + 1) * (2 * t0 + 1) / 6;
        const uint64_t w1 = (M == 1) ? t0 + 1 : t1 * (t1 + 1) / 2 - t0 * (t0 + 1) / 2;
        s_cnt[c * BS + tid] += static_cast<CT>(w2);
        cnt1 += (c == top) ? w1 : 0u;
    }
    for (int c = 0; c <= d; ++c) {
        const uint64_t row = (c == 0) ? static_cast<uint64_t>(d) : static_cast<uint64_t>(c - 1);
        x[row * ldx + idx] = static_cast<float>((static_cast<double>(s_cnt[c * BS + tid]) - law.mean[c]) * law.inv[c]);
    }
    x[static_cast<uint64_t>(d + 1) * ldx + idx] = static_cast<float>((static_cast<double>(cnt1) - law.mean1) * law.inv1);
}

// Double-double sums of a = A - sa, b = B - sb, a^2, b^2, a b over n pairs (A FP64 or absent,
// B FP32): per-workgroup partials, the last workgroup reduces them in order into out[10]
// (hi, lo per moment).
__global__ __launch_bounds__(256) void cv_moments_kernel(const double *A, const float *Bv, uint64_t n, double sa,
                                                         double sb, double *part, uint32_t nb, double *out,
                                                         uint32_t *done)
{
    __shared__ double sm[2 * 4];
    __shared__ uint32_t last;
    double hs[5] = {0, 0, 0, 0, 0}, ls[5] = {0, 0, 0, 0, 0};
    for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * 256) {
        const double a = A ? A[i] - sa : 0.0;
        const double b = Bv ? static_cast<double>(Bv[i]) - sb : 0.0;
        const double v[5] = {a, b, a * a, b * b, a * b};
#pragma unroll
        for (int s = 0; s < 5; ++s) dd_add(hs[s], ls[s], v[s], 0.0);
    }
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        block_sum_dd(hs[s], ls[s], sm);
        if (threadIdx.x == 0) {
            store_agent(part + (2 * s) * nb + blockIdx.x, hs[s]);
            store_agent(part + (2 * s + 1) * nb + blockIdx.x, ls[s]);
        }
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t prev = __hip_atomic_fetch_add(done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        last = (prev == nb - 1) ? 1u : 0u;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
#pragma unroll
    for (int s = 0; s < 5; ++s) {
        double h = 0.0, l = 0.0;
        for (uint32_t b = threadIdx.x; b < nb; b += 256)
            dd_add(h, l, load_agent(part + (2 * s) * nb + b), load_agent(part + (2 * s + 1) * nb + b));
        block_sum_dd(h, l, sm);
        if (threadIdx.x == 0) {
            out[2 * s] = h;
            out[2 * s + 1] = l;
        }
    }
    if (threadIdx.x == 0) __hip_atomic_store(done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// (Y - mean) / sd as the FP32 training target
__global__ __launch_bounds__(256) void cv_target_kernel(const double *Y, uint64_t n, double mean, double inv_sd,
                                                        float *t)
{
    const uint64_t i = static_cast<uint64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (i < n) t[i] = static_cast<float>((Y[i] - mean) * inv_sd);
}

// ---- launchers -------------------------------------------------------------------------------

int launch_mlp_forward(const MlpDev &m, const float *x, uint64_t ldx, uint64_t n, float shift, float scale,
                       float *out, hipStream_t st)
{
    if (n == 0) return 0;
    const dim3 g(static_cast<uint32_t>((n + 127) / 128)), b(256);
    switch (m.KS1) {
    case 1: hipLaunchKernelGGL(mlp_forward_kernel<1>, g, b, 0, st, m, x, ldx, n, shift, scale, out); break;
    case 2: hipLaunchKernelGGL(mlp_forward_kernel<2>, g, b, 0, st, m, x, ldx, n, shift, scale, out); break;
    case 3: hipLaunchKernelGGL(mlp_forward_kernel<3>, g, b, 0, st, m, x, ldx, n, shift, scale, out); break;
    case 4: hipLaunchKernelGGL(mlp_forward_kernel<4>, g, b, 0, st, m, x, ldx, n, shift, scale, out); break;
    case 5: hipLaunchKernelGGL(mlp_forward_kernel<5>, g, b, 0, st, m, x, ldx, n, shift, scale, out); break;
    default: return -5;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_mlp_grad(const MlpDev &m, const float *x, uint64_t ldx, const float *y, uint64_t q0, uint64_t rows,
                    uint64_t a, uint64_t c, uint64_t n_data, float inv_batch, float *part, hipStream_t st)
{
    const dim3 g(static_cast<uint32_t>((rows + 127) / 128)), b(256);
    const uint64_t q_end = q0 + rows;
    switch (m.KS1) {
    case 1: hipLaunchKernelGGL(mlp_grad_kernel<1>, g, b, 0, st, m, x, ldx, y, q0, q_end, a, c, n_data, inv_batch, part); break;
    case 2: hipLaunchKernelGGL(mlp_grad_kernel<2>, g, b, 0, st, m, x, ldx, y, q0, q_end, a, c, n_data, inv_batch, part); break;
    case 3: hipLaunchKernelGGL(mlp_grad_kernel<3>, g, b, 0, st, m, x, ldx, y, q0, q_end, a, c, n_data, inv_batch, part); break;
    case 4: hipLaunchKernelGGL(mlp_grad_kernel<4>, g, b, 0, st, m, x, ldx, y, q0, q_end, a, c, n_data, inv_batch, part); break;
    case 5: hipLaunchKernelGGL(mlp_grad_kernel<5>, g, b, 0, st, m, x, ldx, y, q0, q_end, a, c, n_data, inv_batch, part); break;
    default: return -5;
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_mlp_reduce(const MlpDev &m, const float *part, uint32_t n_parts, int mode, const AdamStep &s, float *mom1,
                      float *mom2, float *grad_out, float *loss_out, hipStream_t st)
{
    hipLaunchKernelGGL(mlp_reduce_kernel, dim3((m.P + 1 + 255) / 256), dim3(256), 0, st, m, part, n_parts, mode, s,
                       mom1, mom2, grad_out, loss_out);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_mlp_copies(const MlpDev &m, hipStream_t st)
{
    hipLaunchKernelGGL(mlp_copies_kernel, dim3((m.P + 255) / 256), dim3(256), 0, st, m);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_mlp_init(const MlpDev &m, uint64_t seed, uint32_t instance, hipStream_t st)
{
    hipLaunchKernelGGL(mlp_init_kernel, dim3((m.P + 255) / 256), dim3(256), 0, st, m, seed, instance);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_cv_aux(const AuxLaw &law, uint64_t k0, uint64_t n, float *x, uint64_t ldx, hipStream_t st)
{
    if (n == 0) return 0;
    const dim3 g(static_cast<uint32_t>((n + 255) / 256)), b(256);
    if (law.d <= 4) hipLaunchKernelGGL((cv_aux_kernel<4, 256, uint64_t>), g, b, 0, st, law, k0, n, x, ldx);
    else if (law.d <= 8) hipLaunchKernelGGL((cv_aux_kernel<8, 256, uint64_t>), g, b, 0, st, law, k0, n, x, ldx);
    else if (law.d <= 16) hipLaunchKernelGGL((cv_aux_kernel<16, 256, uint64_t>), g, b, 0, st, law, k0, n, x, ldx);
    else if (law.d <= 32) hipLaunchKernelGGL((cv_aux_kernel<32, 256, uint64_t>), g, b, 0, st, law, k0, n, x, ldx);
    else if (law.d <= 64 && law.T <= 2343)
        hipLaunchKernelGGL((cv_aux_kernel<64, 128, uint32_t>), dim3(static_cast<uint32_t>((n + 127) / 128)), dim3(128), 0,
                           st, law, k0, n, x, ldx);
    else return -5;
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_cv_moments(const double *A, const float *B, uint64_t n, double sa, double sb, double *part, uint32_t nb,
                      double *out, uint32_t *done, hipStream_t st)
{
    hipLaunchKernelGGL(cv_moments_kernel, dim3(nb), dim3(256), 0, st, A, B, n, sa, sb, part, nb, out, done);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

int launch_cv_target(const double *Y, uint64_t n, double mean, double inv_sd, float *t, hipStream_t st)
{
    if (n == 0) return 0;
    hipLaunchKernelGGL(cv_target_kernel, dim3(static_cast<uint32_t>((n + 255) / 256)), dim3(256), 0, st, Y, n, mean,
                       inv_sd, t);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}  // namespace fw
