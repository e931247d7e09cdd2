// fw_sqn.hip -- Algorithms 3-4 (Section 3.3, Task 3): stochastic quasi-Newton (SQN) for the
// logistic loss Eq. (10)-(11) over N rows of n binary features, many independent replications.
//
// One workgroup of 1024 threads runs one replication through all K iterations (no grid-wide
// synchronisation). Two mappings share the work:
//   element owner   thread t owns the feature quads t (and t + 1024 when n > 4096): w in registers,
//                   the gradient Eq. (12) and y = Eq. (13) s summed over the sampled rows in order,
//                   the direction and the step, the window sum (in HBM, own features only);
//   groups          G lanes (a power of two) take one row or one stored vector at a time for the dot
//                   products x_i'v and s_i'v / y_i'v, against a copy of v staged in LDS; a butterfly
//                   over the G lanes, no workgroup reduction; only the set bits of a row touch LDS.
// The features are a bitmap in HBM (bit j of row i = x_ij, rows padded to 16 bytes), an eighth of
// the bytes and a single 16-byte load per 128 features.
// An iteration:
//   rows       b rows drawn uniformly with replacement (Philox domain 5, counter (q/4, k, rep));
//   gradient   x_i'w, c(x_i'w) - z_i, then Eq. (12) divided by b;
//   direction  for k <= 2L the gradient; after that H_t g by the compact representation of the
//              BFGS matrix (Byrd, Nocedal and Schnabel): with S, Y the stored pairs (oldest first),
//              R the upper triangle of S'Y, D its diagonal and gamma = s_t'y_t / y_t'y_t,
//                H g = gamma g + S (C S'g - gamma R^-T Y'g) - gamma Y R^-1 S'g,
//                C = R^-T (D + gamma Y'Y) R^-1,
//              which equals Algorithm 4's chain of rank-two updates from gamma I applied to g, in
//              O(M n) per iteration instead of forming the n x n matrix;
//   step       w -= (beta / k) direction;
//   window     every L iterations the average of the window's iterates; from the second window on
//              the pair s = wbar_t - wbar_{t-1}, y = Eq. (13) at wbar_t applied to s over b_H rows
//              (Philox domain 6, counter (q/4, k, rep)), stored in the replication's ring of M
//              slots; the new row and column of S'Y and Y'Y, then R^-1 and C, rebuilt in LDS.
// Everything is FP64; the stored pairs live in HBM ([R][M][ld] per array), in binary64 or, on
// request, binary32 (s rounded before y is formed from it, y rounded when stored: half the bytes of
// the two passes over them). The loss Eq. (10) at the checkpoints and at w^{K+1} is a separate
// launch over the whole data set.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device_reduce.hpp"
#include "device_rng.hpp"
#include "sim_types.hpp"
#include "sqn.hpp"
#include "sqn_device.hpp"

namespace fw {

namespace {

constexpr int kRunBlock = 1024;

// Rows idx[i0 .. i0 + cnt) of the bitmap into rows[r][xw] of LDS (cnt xw <= kStageWords), 16-byte
// loads spread over the workgroup. The caller synchronises before and after.
constexpr uint32_t kStageWords = 32 * (kSqnMaxN / 32);      // 32 KB: 32 rows at the largest n

__device__ __forceinline__ void stage_rows(const SqnArgs &A, const uint32_t *idx, uint32_t i0, uint32_t cnt,
                                           uint32_t *rows)
{
    const uint32_t q4 = A.xw / 4, total = cnt * q4;
    for (uint32_t u = threadIdx.x; u < total; u += blockDim.x) {
        const uint32_t r = u / q4, wq = u % q4;
        reinterpret_cast<uint4 *>(rows + r * A.xw)[wq] =
            reinterpret_cast<const uint4 *>(A.X + static_cast<size_t>(idx[i0 + r]) * A.xw)[wq];
    }
}

// Sum over the G lanes of a group (G a power of two <= 64, groups aligned in the wavefront); every
// lane of the wavefront must take part.
__device__ __forceinline__ double group_sum(double a, uint32_t G)
{
    for (uint32_t off = G >> 1; off >= 1; off >>= 1) a += __shfl_xor(a, static_cast<int>(off), 64);
    return a;
}

// out[i] = x_{idx[i]}'v for i < count, v staged in LDS, G lanes per row, each lane four words (128
// features) per load. Ends with a barrier.
__device__ __forceinline__ void row_dots(const SqnArgs &A, const uint32_t *idx, uint32_t count, const double *v,
                                         double *out, uint32_t G)
{
    const uint32_t sub = threadIdx.x & (G - 1), group = threadIdx.x / G, ngroups = blockDim.x / G;
    const uint32_t n4 = A.xw / 4;
    for (uint32_t i0 = 0; i0 < count; i0 += ngroups) {
        const uint32_t i = i0 + group;
        double a = 0.0;
        if (i < count) {
            const uint4 *row = reinterpret_cast<const uint4 *>(A.X + static_cast<size_t>(idx[i]) * A.xw);
#pragma unroll 4
            for (uint32_t k4 = sub; k4 < n4; k4 += G) {
                const uint4 x = row[k4];
                const uint32_t j0 = 128u * k4;
                a += word_dot(x.x, v, j0);
                a += word_dot(x.y, v, j0 + 32);
                a += word_dot(x.z, v, j0 + 64);
                a += word_dot(x.w, v, j0 + 96);
            }
        }
        a = group_sum(a, G);
        if (sub == 0 && i < count) out[i] = a;
    }
    __syncthreads();
}

// *out(u) = vec(u)'v for u < count, vec(u) a stored vector in HBM, v staged in LDS, G lanes per
// vector. Ends with a barrier.
template <class VecOf, class OutOf>
__device__ __forceinline__ void vec_dots(const SqnArgs &A, uint32_t count, VecOf vec, const double *v, OutOf out,
                                         uint32_t G)
{
    const uint32_t sub = threadIdx.x & (G - 1), group = threadIdx.x / G, ngroups = blockDim.x / G;
    for (uint32_t u0 = 0; u0 < count; u0 += ngroups) {
        const uint32_t u = u0 + group;
        double a = 0.0;
        if (u < count) {
            const auto *p = vec(u);
#pragma unroll 4
            for (uint32_t qq = sub; qq < A.nq; qq += G) {
                double x[4];
                load4(p + 4 * qq, x);
#pragma unroll
                for (int c = 0; c < 4; ++c) a += x[c] * v[4 * qq + c];
            }
        }
        a = group_sum(a, G);
        if (sub == 0 && u < count) *out(u) = a;
    }
    __syncthreads();
}

}  // namespace

// PT: the storage type of the pairs (double, or float when they are kept in binary32)
template <int EQ, typename PT>
__global__ __launch_bounds__(kRunBlock) void sqn_run_kernel(SqnArgs A)
{
    __shared__ double s_stage[kSqnMaxN];                 // the vector the group dot products read
    __shared__ uint32_t s_idx[kSqnMaxB];
    __shared__ double s_v[kSqnMaxB];                     // row dots x_i'w, x_i'wbar
    __shared__ double s_coef[kSqnMaxB];                  // residuals / curvature weights; matrix scratch
    __shared__ double s_dots[3 * kSqnMaxM];
    __shared__ double s_SY[kSqnMaxM * kSqnMaxM];         // s_i'y_j, chronological
    __shared__ double s_YY[kSqnMaxM * kSqnMaxM];         // y_i'y_j
    __shared__ double s_Ri[kSqnMaxM * kSqnMaxM];         // R^-1 (upper triangular)
    __shared__ double s_C[kSqnMaxM * kSqnMaxM];          // R^-T (D + gamma Y'Y) R^-1
    __shared__ double s_cs[kSqnMaxM], s_cy[kSqnMaxM];    // coefficients of S and Y in H g
    __shared__ uint32_t s_rows[kStageWords];             // a chunk of sampled rows' bits
    const uint32_t chunk = kStageWords / A.xw;           // rows per chunk: 32 at n = 8192, 2048 at n = 50

    const uint32_t rep = blockIdx.x;
    const uint32_t tid = threadIdx.x, T = blockDim.x;
    const uint32_t ld = A.ld, M = A.M, G = A.G, xw = A.xw;
    const size_t vs = static_cast<size_t>(ld);
    PT *Srep = static_cast<PT *>(A.S) + static_cast<size_t>(rep) * M * ld;
    PT *Yrep = static_cast<PT *>(A.Y) + static_cast<size_t>(rep) * M * ld;
    double *wprev = A.wprev + static_cast<size_t>(rep) * ld;
    double *acc = A.acc + static_cast<size_t>(rep) * ld;

    uint32_t q[EQ];
    bool own[EQ];
    double w[EQ][4];
#pragma unroll
    for (int e = 0; e < EQ; ++e) {
        q[e] = tid + e * T;
        own[e] = q[e] < A.nq;
#pragma unroll
        for (int c = 0; c < 4; ++c) w[e][c] = 0.0;
        if (own[e]) store4(acc + 4 * q[e], w[e]);
    }

    uint32_t m = 0, head = 0, pairs = 0, ck = 0;
    int64_t t = -1;
    double gamma = 0.0;

    for (uint64_t k = 1; k <= A.K; ++k) {
        __syncthreads();                                   // the previous rows and coefficients are read
        // rows and x_i'w (w staged)
#pragma unroll
        for (int e = 0; e < EQ; ++e)
            if (own[e]) store4(s_stage + 4 * q[e], w[e]);
        draw_rows(A, rep, k, kSqnDomGrad, A.b, s_idx);
        __syncthreads();
        row_dots(A, s_idx, A.b, s_stage, s_v, G);
        for (uint32_t i = tid; i < A.b; i += T) s_coef[i] = sigmoid(s_v[i]) - static_cast<double>(A.z[s_idx[i]]);
        __syncthreads();

        // Eq. (12), and the window sum
        double g[EQ][4];
#pragma unroll
        for (int e = 0; e < EQ; ++e) {
#pragma unroll
            for (int c = 0; c < 4; ++c) g[e][c] = 0.0;
        }
        // Eq. (12): the rows in order, staged through LDS a chunk at a time
        for (uint32_t i0 = 0; i0 < A.b; i0 += chunk) {
            const uint32_t cnt = min(chunk, A.b - i0);
            __syncthreads();
            stage_rows(A, s_idx, i0, cnt, s_rows);
            __syncthreads();
#pragma unroll
            for (int e = 0; e < EQ; ++e) {
                if (!own[e]) continue;
                const uint32_t wq = q[e] >> 3, sh = 4 * (q[e] & 7);
                for (uint32_t i = 0; i < cnt; ++i) {
                    const uint32_t x = (s_rows[i * xw + wq] >> sh) & 0xFu;
                    const double r = s_coef[i0 + i];
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        if ((x >> c) & 1u) g[e][c] += r;
                }
            }
        }
#pragma unroll
        for (int e = 0; e < EQ; ++e) {
            if (!own[e]) continue;
            double a4[4];
            load4(acc + 4 * q[e], a4);
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                g[e][c] /= static_cast<double>(A.b);
                a4[c] += w[e][c];
            }
            store4(acc + 4 * q[e], a4);
        }
        const double alpha = A.beta / static_cast<double>(k);

        if (k <= 2ull * A.L) {
#pragma unroll
            for (int e = 0; e < EQ; ++e)
#pragma unroll
                for (int c = 0; c < 4; ++c) w[e][c] -= alpha * g[e][c];
        } else {
            // S'g and Y'g (g staged), interleaved: 2i is s_i'g, 2i + 1 is y_i'g, pair i oldest first
#pragma unroll
            for (int e = 0; e < EQ; ++e)
                if (own[e]) store4(s_stage + 4 * q[e], g[e]);
            __syncthreads();
            const uint32_t hd = head, mm = m;
            vec_dots(A, 2 * m, [&](uint32_t u) { return ((u & 1) ? Yrep : Srep) + ((hd + (u >> 1)) % M) * vs; },
                     s_stage, [&](uint32_t u) { return s_dots + u; }, A.GV);
            if (tid < mm) {
                const uint32_t i = tid;
                double a = 0.0, r = 0.0;
                for (uint32_t l = 0; l < mm; ++l) a += s_C[i * kSqnMaxM + l] * s_dots[2 * l];
                for (uint32_t l = 0; l <= i; ++l) r += s_Ri[l * kSqnMaxM + i] * s_dots[2 * l + 1];
                s_cs[i] = a - gamma * r;
            } else if (tid < 2 * mm) {
                const uint32_t i = tid - mm;
                double r = 0.0;
                for (uint32_t l = i; l < mm; ++l) r += s_Ri[i * kSqnMaxM + l] * s_dots[2 * l];
                s_cy[i] = -gamma * r;
            }
            __syncthreads();
#pragma unroll
            for (int e = 0; e < EQ; ++e) {
                if (!own[e]) continue;
                double dir[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) dir[c] = gamma * g[e][c];
#pragma unroll 4
                for (uint32_t i = 0; i < mm; ++i) {
                    const size_t off = ((hd + i) % M) * vs + 4 * q[e];
                    double sv[4], yv[4];
                    load4(Srep + off, sv);
                    load4(Yrep + off, yv);
                    const double cs = s_cs[i], cy = s_cy[i];
#pragma unroll
                    for (int c = 0; c < 4; ++c) dir[c] += sv[c] * cs + yv[c] * cy;
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) w[e][c] -= alpha * dir[c];
            }
        }

        if (k % A.L == 0) {
            ++t;
            const bool pair = t > 0;
            const bool full = m == M;
            const uint32_t slot = full ? head : (head + m) % M;
            // wbar (staged), s = wbar - wbar_prev into the ring, wbar_prev = wbar, the window sum cleared
#pragma unroll
            for (int e = 0; e < EQ; ++e)
                if (own[e]) {
                    double wb[4], pv[4], sv[4];
                    load4(acc + 4 * q[e], wb);
#pragma unroll
                    for (int c = 0; c < 4; ++c) wb[c] /= static_cast<double>(A.L);
                    if (pair) {
                        load4(wprev + 4 * q[e], pv);
#pragma unroll
                        for (int c = 0; c < 4; ++c) sv[c] = wb[c] - pv[c];
                        store4(Srep + slot * vs + 4 * q[e], sv);
                    }
                    store4(wprev + 4 * q[e], wb);
                    store4(s_stage + 4 * q[e], wb);
                    double zero[4] = {0.0, 0.0, 0.0, 0.0};
                    store4(acc + 4 * q[e], zero);
                }
            if (pair) {
                __syncthreads();                               // the gradient rows are read
                draw_rows(A, rep, k, kSqnDomHess, A.bH, s_idx);
                __syncthreads();
                row_dots(A, s_idx, A.bH, s_stage, s_v, G);                 // x_i'wbar
#pragma unroll
                for (int e = 0; e < EQ; ++e)
                    if (own[e]) {
                        double sv[4];
                        load4(Srep + slot * vs + 4 * q[e], sv);
                        store4(s_stage + 4 * q[e], sv);
                    }
                __syncthreads();
                row_dots(A, s_idx, A.bH, s_stage, s_coef, G);              // x_i's
                for (uint32_t i = tid; i < A.bH; i += T) {
                    const double c = sigmoid(s_v[i]);
                    s_coef[i] = c * (1.0 - c) * s_coef[i];
                }
                __syncthreads();
                // Eq. (13) applied to s (the rows in order, staged through LDS a chunk at a time),
                // into the ring and staged
                double y[EQ][4];
#pragma unroll
                for (int e = 0; e < EQ; ++e)
#pragma unroll
                    for (int c = 0; c < 4; ++c) y[e][c] = 0.0;
                for (uint32_t i0 = 0; i0 < A.bH; i0 += chunk) {
                    const uint32_t cnt = min(chunk, A.bH - i0);
                    __syncthreads();
                    stage_rows(A, s_idx, i0, cnt, s_rows);
                    __syncthreads();
#pragma unroll
                    for (int e = 0; e < EQ; ++e) {
                        if (!own[e]) continue;
                        const uint32_t wq = q[e] >> 3, sh = 4 * (q[e] & 7);
                        for (uint32_t i = 0; i < cnt; ++i) {
                            const uint32_t x = (s_rows[i * xw + wq] >> sh) & 0xFu;
                            const double cf = s_coef[i0 + i];
#pragma unroll
                            for (int c = 0; c < 4; ++c)
                                if ((x >> c) & 1u) y[e][c] += cf;
                        }
                    }
                }
#pragma unroll
                for (int e = 0; e < EQ; ++e) {
                    if (!own[e]) continue;
#pragma unroll
                    for (int c = 0; c < 4; ++c)
                        y[e][c] = static_cast<double>(static_cast<PT>(y[e][c] / static_cast<double>(A.bH)));
                    store4(Yrep + slot * vs + 4 * q[e], y[e]);
                    store4(s_stage + 4 * q[e], y[e]);
                }
                if (full) head = (head + 1) % M;
                else ++m;
                __syncthreads();
                // the new row and column of S'Y and Y'Y: 3i = s_i'y, 3i + 1 = s'y_i, 3i + 2 = y_i'y
                const uint32_t hd = head;
                vec_dots(A, 2 * m, [&](uint32_t u) { return ((u & 1) ? Yrep : Srep) + ((hd + (u >> 1)) % M) * vs; },
                         s_stage, [&](uint32_t u) { return s_dots + 3 * (u >> 1) + ((u & 1) ? 2 : 0); }, A.GV);
#pragma unroll
                for (int e = 0; e < EQ; ++e)
                    if (own[e]) {
                        double sv[4];
                        load4(Srep + slot * vs + 4 * q[e], sv);
                        store4(s_stage + 4 * q[e], sv);
                    }
                __syncthreads();
                vec_dots(A, m, [&](uint32_t u) { return Yrep + ((hd + u) % M) * vs; }, s_stage,
                         [&](uint32_t u) { return s_dots + 3 * u + 1; }, A.GV);
                // drop the oldest pair's row and column when the ring was full (through s_v, free here)
                if (full) {
                    const uint32_t mm = m - 1;
                    for (uint32_t u = tid; u < mm * mm; u += T) {
                        const uint32_t i = u / mm, j = u % mm;
                        s_v[u] = s_SY[(i + 1) * kSqnMaxM + j + 1];
                    }
                    for (uint32_t u = tid; u < mm * mm; u += T) {
                        const uint32_t i = u / mm, j = u % mm;
                        s_coef[u] = s_YY[(i + 1) * kSqnMaxM + j + 1];
                    }
                    __syncthreads();
                    for (uint32_t u = tid; u < mm * mm; u += T) {
                        const uint32_t i = u / mm, j = u % mm;
                        s_SY[i * kSqnMaxM + j] = s_v[u];
                        s_YY[i * kSqnMaxM + j] = s_coef[u];
                    }
                    __syncthreads();
                }
                if (tid < m) {
                    const uint32_t i = tid, n1 = m - 1;
                    s_SY[n1 * kSqnMaxM + i] = s_dots[3 * i + 1];
                    s_YY[i * kSqnMaxM + n1] = s_dots[3 * i + 2];
                    s_YY[n1 * kSqnMaxM + i] = s_dots[3 * i + 2];
                }
                __syncthreads();
                if (tid < m) s_SY[tid * kSqnMaxM + (m - 1)] = s_dots[3 * tid];
                __syncthreads();
                gamma = s_SY[(m - 1) * kSqnMaxM + (m - 1)] / s_YY[(m - 1) * kSqnMaxM + (m - 1)];
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
                // T1 = (D + gamma Y'Y) R^-1 into s_coef, then C = R^-T T1
                for (uint32_t u = tid; u < m * m; u += T) {
                    const uint32_t i = u / m, c = u % m;
                    double acc_t = 0.0;
                    for (uint32_t l = 0; l <= c; ++l) {
                        const double dl = gamma * s_YY[i * kSqnMaxM + l] + (i == l ? s_SY[i * kSqnMaxM + i] : 0.0);
                        acc_t += dl * s_Ri[l * kSqnMaxM + c];
                    }
                    s_coef[i * kSqnMaxM + c] = acc_t;
                }
                __syncthreads();
                for (uint32_t u = tid; u < m * m; u += T) {
                    const uint32_t i = u / m, c = u % m;
                    double acc_c = 0.0;
                    for (uint32_t l = 0; l <= i; ++l) acc_c += s_Ri[l * kSqnMaxM + i] * s_coef[l * kSqnMaxM + c];
                    s_C[i * kSqnMaxM + c] = acc_c;
                }
                ++pairs;
            }
            __syncthreads();
        }

        while (ck < A.n_ckpt && A.ckpt[ck] == k) {
            double *dst = A.wsnap + (static_cast<size_t>(ck) * A.R + rep) * ld;
#pragma unroll
            for (int e = 0; e < EQ; ++e)
                if (own[e]) store4(dst + 4 * q[e], w[e]);
            ++ck;
        }
    }
    double *dst = A.wsnap + (static_cast<size_t>(A.n_ckpt) * A.R + rep) * ld;
#pragma unroll
    for (int e = 0; e < EQ; ++e)
        if (own[e]) store4(dst + 4 * q[e], w[e]);
    if (tid == 0) A.pairs[rep] = pairs;
}

// Eq. (10) at one stored iterate (blockIdx.y = checkpoint * R + replication) over kSqnLossRows rows:
// a wavefront per row, lanes over 128-feature blocks of the row's bits, the terms log(1 + e^{-a}) + (1 - z) a summed in
// double-double, wavefront partials in order.
__global__ __launch_bounds__(kSqnLossBlock) void sqn_loss_kernel(SqnArgs A)
{
    __shared__ double s_w[kSqnMaxN];
    __shared__ double s_part[2 * kSqnLossBlock / 64];
    const uint32_t snap = blockIdx.y;
    const double *wv = A.wsnap + static_cast<size_t>(snap) * A.ld;
    for (uint32_t j = threadIdx.x; j < A.ld; j += blockDim.x) s_w[j] = wv[j];
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t r0 = blockIdx.x * kSqnLossRows;
    const uint32_t r1 = min(A.N, r0 + kSqnLossRows);
    double h = 0.0, l = 0.0;
    for (uint32_t row = r0 + wave; row < r1; row += nw) {
        double a = 0.0;
        const uint4 *xr = reinterpret_cast<const uint4 *>(A.X + static_cast<size_t>(row) * A.xw);
#pragma unroll 2
        for (uint32_t k4 = lane; k4 < A.xw / 4; k4 += 64) {
            const uint4 x = xr[k4];
            const uint32_t j0 = 128u * k4;
            a += word_dot(x.x, s_w, j0);
            a += word_dot(x.y, s_w, j0 + 32);
            a += word_dot(x.z, s_w, j0 + 64);
            a += word_dot(x.w, s_w, j0 + 96);
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off, 64);
        if (lane == 0) {
            const double sp = a > 0.0 ? log1p(exp(-a)) : log1p(exp(a)) - a;
            dd_add(h, l, sp + (A.z[row] ? 0.0 : a), 0.0);
        }
    }
    if (lane == 0) {
        s_part[2 * wave] = h;
        s_part[2 * wave + 1] = l;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        h = s_part[0];
        l = s_part[1];
        for (uint32_t k = 1; k < nw; ++k) dd_add(h, l, s_part[2 * k], s_part[2 * k + 1]);
        double *o = A.loss_part + (static_cast<size_t>(snap) * A.nblk + blockIdx.x) * 2;
        o[0] = h;
        o[1] = l;
    }
}

// wt[j][s] = wsnap[s][j]: the stored iterates feature-major, for sqn_loss_many_kernel. 32 x 32 tiles.
__global__ __launch_bounds__(256) void sqn_transpose_kernel(SqnArgs A, uint32_t n_snap)
{
    __shared__ double tile[32][33];
    const uint32_t j0 = blockIdx.x * 32, s0 = blockIdx.y * 32;
    const uint32_t tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (uint32_t r = ty; r < 32; r += 8) {
        const uint32_t sn = s0 + r, j = j0 + tx;
        tile[r][tx] = (sn < n_snap && j < A.ld) ? A.wsnap[static_cast<size_t>(sn) * A.ld + j] : 0.0;
    }
    __syncthreads();
    for (uint32_t r = ty; r < 32; r += 8) {
        const uint32_t j = j0 + r, sn = s0 + tx;
        if (j < A.ld && sn < n_snap) A.wt[static_cast<size_t>(j) * n_snap + sn] = tile[tx][r];
    }
}

// Eq. (10) at many stored iterates at once: a lane per iterate (64 per workgroup, blockIdx.y picks
// them), the four wavefronts over the rows of the block (row r0 + wave, + 4, ...). Each row's set
// bits are walked once per wavefront from scalar registers and every lane adds its iterate's w_j,
// lowest j first; the terms in double-double, the wavefronts' partials in order.
__global__ __launch_bounds__(kSqnLossBlock) void sqn_loss_many_kernel(SqnArgs A, uint32_t n_snap)
{
    __shared__ double s_part[2 * kSqnLossBlock];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
    const uint32_t snap = blockIdx.y * 64 + lane;
    const bool act = snap < n_snap;
    const double *wt = A.wt + (act ? snap : 0);
    const uint32_t r0 = blockIdx.x * kSqnLossRows;
    const uint32_t r1 = min(A.N, r0 + kSqnLossRows);
    double h = 0.0, l = 0.0;
    for (uint32_t row = r0 + wave; row < r1; row += nw) {
        const uint32_t rr = __builtin_amdgcn_readfirstlane(row);
        const uint32_t *xr = A.X + static_cast<size_t>(rr) * A.xw;
        double a = 0.0;
        for (uint32_t wi = 0; wi < A.xw; ++wi) {
            uint32_t bits = __builtin_amdgcn_readfirstlane(xr[wi]);
            while (bits) {
                const uint32_t j = 32u * wi + static_cast<uint32_t>(__builtin_ctz(bits));
                a += wt[static_cast<size_t>(j) * n_snap];
                bits &= bits - 1;
            }
        }
        const double sp = a > 0.0 ? log1p(exp(-a)) : log1p(exp(a)) - a;
        dd_add(h, l, sp + (A.z[rr] ? 0.0 : a), 0.0);
    }
    s_part[2 * threadIdx.x] = h;
    s_part[2 * threadIdx.x + 1] = l;
    __syncthreads();
    if (wave == 0 && act) {
        for (uint32_t k = 1; k < nw; ++k) dd_add(h, l, s_part[2 * (k * 64 + lane)], s_part[2 * (k * 64 + lane) + 1]);
        double *o = A.loss_part + (static_cast<size_t>(snap) * A.nblk + blockIdx.x) * 2;
        o[0] = h;
        o[1] = l;
    }
}

// ---- Algorithm 4's matrix, formed (sim_sqn_hessian) ---------------------------------------------
// H_t = gamma I + U W U' with U = [S, gamma Y] (n x 2m, pairs oldest first) and
// W = [[C, -R^-T], [-R^-1, 0]] from the compact representation; four launches: the Gram entries
// s_i'y_j and y_i'y_j, the 2m x 2m middle matrix, V = U W and U' feature-major, and the n x n
// product V U' on the FP64 matrix cores.

typedef double f64x4 __attribute__((ext_vector_type(4)));

// SY[i][j] = s_i'y_j, YY[i][j] = y_i'y_j (chronological i, j < m) of replication rep: a workgroup
// per (i, j), a fixed-order tree over the features.
template <typename PT>
__global__ __launch_bounds__(256) void sqn_gram_kernel(SqnArgs A, uint32_t rep, uint32_t head, uint32_t m, double *SY,
                                                       double *YY)
{
    __shared__ double s_a[256], s_b[256];
    const uint32_t i = blockIdx.x, j = blockIdx.y, M = A.M;
    const size_t base = static_cast<size_t>(rep) * M * A.ld;
    const PT *si = static_cast<const PT *>(A.S) + base + static_cast<size_t>((head + i) % M) * A.ld;
    const PT *yi = static_cast<const PT *>(A.Y) + base + static_cast<size_t>((head + i) % M) * A.ld;
    const PT *yj = static_cast<const PT *>(A.Y) + base + static_cast<size_t>((head + j) % M) * A.ld;
    double a = 0.0, b = 0.0;
    for (uint32_t k = threadIdx.x; k < A.ld; k += blockDim.x) {
        a += static_cast<double>(si[k]) * static_cast<double>(yj[k]);
        b += static_cast<double>(yi[k]) * static_cast<double>(yj[k]);
    }
    s_a[threadIdx.x] = a;
    s_b[threadIdx.x] = b;
    __syncthreads();
    for (uint32_t h = blockDim.x / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) {
            s_a[threadIdx.x] += s_a[threadIdx.x + h];
            s_b[threadIdx.x] += s_b[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        SY[i * m + j] = s_a[0];
        YY[i * m + j] = s_b[0];
    }
}

// W (Kp x Kp, zero beyond 2m) and gamma from SY, YY: R^-1 by column back substitution, then
// C = R^-T (D + gamma Y'Y) R^-1. One workgroup.
__global__ __launch_bounds__(256) void sqn_middle_kernel(uint32_t m, uint32_t Kp, const double *SYg, const double *YYg,
                                                         double *W, double *gamma_out)
{
    __shared__ double SY[kSqnMaxM * kSqnMaxM], YY[kSqnMaxM * kSqnMaxM];
    __shared__ double s_Ri[kSqnMaxM * kSqnMaxM], s_T[kSqnMaxM * kSqnMaxM];
    const uint32_t tid = threadIdx.x, T = blockDim.x;
    for (uint32_t u = tid; u < m * m; u += T) {
        SY[u] = SYg[u];
        YY[u] = YYg[u];
    }
    __syncthreads();
    const double gamma = SY[(m - 1) * m + (m - 1)] / YY[(m - 1) * m + (m - 1)];
    if (tid < m) {
        const uint32_t c = tid;
        for (uint32_t i = c + 1; i < m; ++i) s_Ri[i * kSqnMaxM + c] = 0.0;
        s_Ri[c * kSqnMaxM + c] = 1.0 / SY[c * m + c];
        for (int i = static_cast<int>(c) - 1; i >= 0; --i) {
            double acc = 0.0;
            for (uint32_t l = i + 1; l <= c; ++l) acc += SY[i * m + l] * s_Ri[l * kSqnMaxM + c];
            s_Ri[i * kSqnMaxM + c] = -acc / SY[i * m + i];
        }
    }
    __syncthreads();
    for (uint32_t u = tid; u < m * m; u += T) {
        const uint32_t i = u / m, c = u % m;
        double acc = 0.0;
        for (uint32_t l = 0; l <= c; ++l) acc += (gamma * YY[i * m + l] + (i == l ? SY[i * m + i] : 0.0)) * s_Ri[l * kSqnMaxM + c];
        s_T[i * kSqnMaxM + c] = acc;
    }
    __syncthreads();
    for (uint32_t u = tid; u < Kp * Kp; u += T) {
        const uint32_t r = u / Kp, c = u % Kp;
        double v = 0.0;
        if (r < m && c < m) {
            for (uint32_t l = 0; l <= r; ++l) v += s_Ri[l * kSqnMaxM + r] * s_T[l * kSqnMaxM + c];
        } else if (r < m && c < 2 * m) {
            v = -s_Ri[(c - m) * kSqnMaxM + r];            // -R^-T
        } else if (r < 2 * m && c < m) {
            v = -s_Ri[(r - m) * kSqnMaxM + c];            // -R^-1
        }
        W[u] = v;
    }
    if (tid == 0) *gamma_out = gamma;
}

// Ut[a][k] = U[a][k] and V[a][c] = sum_k U[a][k] W[k][c], feature-major (Kp per feature, zero
// padded): a wavefront per feature a, a lane per column c.
template <typename PT>
__global__ __launch_bounds__(256) void sqn_uv_kernel(SqnArgs A, uint32_t rep, uint32_t head, uint32_t m, uint32_t Kp,
                                                     const double *W, const double *gamma_p, double *V, double *Ut)
{
    __shared__ double s_W[2 * kSqnMaxM * 2 * kSqnMaxM];
    __shared__ double s_u[4][2 * kSqnMaxM];
    for (uint32_t u = threadIdx.x; u < Kp * Kp; u += blockDim.x) s_W[u] = W[u];
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t a = blockIdx.x * 4 + wave;
    const double gamma = *gamma_p;
    const uint32_t M = A.M;
    const size_t base = static_cast<size_t>(rep) * M * A.ld;
    double x = 0.0;
    if (a < A.n) {
        const PT *S = static_cast<const PT *>(A.S), *Y = static_cast<const PT *>(A.Y);
        if (lane < m) x = S[base + static_cast<size_t>((head + lane) % M) * A.ld + a];
        else if (lane < 2 * m) x = gamma * static_cast<double>(Y[base + static_cast<size_t>((head + lane - m) % M) * A.ld + a]);
    }
    s_u[wave][lane] = x;
    __syncthreads();
    if (a >= A.n || lane >= Kp) return;
    Ut[static_cast<size_t>(a) * Kp + lane] = x;
    double v = 0.0;
    for (uint32_t k = 0; k < 2 * m; ++k) v += s_u[wave][k] * s_W[k * Kp + lane];
    V[static_cast<size_t>(a) * Kp + lane] = v;
}

// H[a][b] = gamma [a == b] + sum_k V[a][k] Ut[b][k] in 64 x 64 tiles. Workgroup (g, y) owns the 64
// rows of row block y and the column tiles g, g + G, ... (G groups chosen so that the whole grid is
// resident at once): V's block is staged in LDS once; each wavefront then walks the tiles on its own,
// with no barrier: it loads its B operands from Ut (L2-resident) into registers, half of k at a
// time (so that five workgroups fit a compute unit), runs the products with A read from LDS, and
// stores its results from the accumulators, 16 consecutive columns per row. Each wavefront computes a 32 x 32 quarter as
// 2 x 2 tiles of v_mfma_f64_16x16x4f64 (A operand: row lane % 16, k lane / 16; B operand: k lane / 16,
// column lane % 16; result register i: row lane / 16 + 4 i, column lane % 16, as measured on gfx950 --
// unlike the 4 (lane / 16) + i rows of the binary32 16x16x4 form).
__global__ __launch_bounds__(256, 5) void sqn_hessian_mfma_kernel(uint32_t n, uint32_t ldh, uint32_t Kp,
                                                                  const double *V, const double *Ut,
                                                                  const double *gamma_p, double *H)
{
    // 64 rows of V are contiguous (64 Kp doubles): 16-byte loads, stored k-major in LDS with a pitch of
    // 65 doubles, so the 16 rows an operand read spans fall in consecutive banks (Kp 65 doubles of
    // dynamic LDS: 27 KB at Kp = 52).
    constexpr uint32_t P = kSqnHessianPitch;
    constexpr uint32_t kPass = 32 * 2 * kSqnMaxM / 256;              // 16-byte pairs per thread at Kp = 64
    constexpr uint32_t kHalf = 2 * kSqnMaxM / 8;                     // half the k steps of 4 at Kp = 64
    extern __shared__ double s_A[];
    const uint32_t nt = (n + 63) / 64, G = gridDim.x;
    const uint32_t ra = blockIdx.y * 64, tid = threadIdx.x;
    {
        // all loads of the block are issued before the first wait
        const uint32_t nv = min(64u, n - ra) * Kp;
        const double2 *g = reinterpret_cast<const double2 *>(V + static_cast<size_t>(ra) * Kp);
        double2 xa[kPass];
#pragma unroll
        for (uint32_t p = 0; p < kPass; ++p) {
            const uint32_t u = tid + 256 * p;
            xa[p] = 2 * u < nv ? g[u] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (uint32_t p = 0; p < kPass; ++p) {
            const uint32_t u = tid + 256 * p;
            if (u < 32 * Kp) {
                const uint32_t row = (2 * u) / Kp, k = (2 * u) % Kp; // Kp is a multiple of 4: k, k + 1 share the row
                s_A[k * P + row] = xa[p].x;
                s_A[(k + 1) * P + row] = xa[p].y;
            }
        }
    }
    __syncthreads();                                                 // s_A is only read from here on
    const double gamma = *gamma_p;
    const uint32_t lane = tid & 63, wave = tid >> 6;
    const uint32_t ta = (wave >> 1) * 32, tb = (wave & 1) * 32;      // the wavefront's quarter of a tile
    const uint32_t lr = lane & 15, lk = lane >> 4;
    const uint32_t steps = Kp / 4;
    for (uint32_t cb = blockIdx.x; cb < nt; cb += G) {
        const uint32_t rb = cb * 64;
        f64x4 acc[2][2];
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y) acc[x][y] = f64x4{0.0, 0.0, 0.0, 0.0};
        // the k range in two halves of at most kHalf steps: the B operands of a half in registers
        for (uint32_t h0 = 0; h0 < steps; h0 += kHalf) {
            double bv[kHalf][2];
#pragma unroll
            for (uint32_t s2 = 0; s2 < kHalf; ++s2)
#pragma unroll
                for (int y = 0; y < 2; ++y) {
                    const uint32_t st = h0 + s2, col = rb + tb + 16 * y + lr;
                    bv[s2][y] = (st < steps && col < n) ? Ut[static_cast<size_t>(col) * Kp + 4 * st + lk] : 0.0;
                }
#pragma unroll
            for (uint32_t s2 = 0; s2 < kHalf; ++s2) {
                const uint32_t st = h0 + s2;
                if (st < steps) {
                    double av[2];
#pragma unroll
                    for (int x = 0; x < 2; ++x) av[x] = s_A[(4 * st + lk) * P + ta + 16 * x + lr];
#pragma unroll
                    for (int x = 0; x < 2; ++x)
#pragma unroll
                        for (int y = 0; y < 2; ++y)
                            acc[x][y] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[x], bv[s2][y], acc[x][y], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int x = 0; x < 2; ++x)
#pragma unroll
            for (int y = 0; y < 2; ++y)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const uint32_t row = ra + ta + 16 * x + lk + 4 * i, col = rb + tb + 16 * y + lr;
                    double h = acc[x][y][i];
                    if (row == col) h += gamma;
                    if (row < n && col < n) H[static_cast<size_t>(row) * ldh + col] = h;
                }
    }
}

int launch_sqn_hessian(const SqnArgs &A, uint32_t rep, uint32_t head, uint32_t m, double *scratch, double *H,
                       uint32_t ldh, hipStream_t s)
{
    const uint32_t Kp = (2 * m + 3) / 4 * 4;
    double *SY = scratch, *YY = SY + kSqnMaxM * kSqnMaxM, *W = YY + kSqnMaxM * kSqnMaxM;
    double *gamma = W + 4 * kSqnMaxM * kSqnMaxM;
    double *V = gamma + 4, *Ut = V + static_cast<size_t>(A.n) * Kp;
    if (A.pairs_fp32)
        hipLaunchKernelGGL(sqn_gram_kernel<float>, dim3(m, m), dim3(256), 0, s, A, rep, head, m, SY, YY);
    else
        hipLaunchKernelGGL(sqn_gram_kernel<double>, dim3(m, m), dim3(256), 0, s, A, rep, head, m, SY, YY);
    hipLaunchKernelGGL(sqn_middle_kernel, dim3(1), dim3(256), 0, s, m, Kp, SY, YY, W, gamma);
    if (A.pairs_fp32)
        hipLaunchKernelGGL(sqn_uv_kernel<float>, dim3((A.n + 3) / 4), dim3(256), 0, s, A, rep, head, m, Kp, W, gamma, V, Ut);
    else
        hipLaunchKernelGGL(sqn_uv_kernel<double>, dim3((A.n + 3) / 4), dim3(256), 0, s, A, rep, head, m, Kp, W, gamma, V, Ut);
    // column groups: one tile per workgroup while nt^2 workgroups fit at once, fewer groups beyond
    // that (resident workgroups: as many as the LDS of a compute unit holds, at most five)
    const uint32_t nt = (A.n + 63) / 64;
    const uint32_t lds = Kp * kSqnHessianPitch * sizeof(double);
    const uint32_t slots = kSqnComputeUnits * std::min(5u, kSqnLdsPerCu / lds);
    const uint32_t groups = std::min(nt, std::max(1u, slots / nt));
    hipLaunchKernelGGL(sqn_hessian_mfma_kernel, dim3(groups, nt), dim3(256), lds, s, A.n, ldh, Kp, V, Ut, gamma, H);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// F per stored iterate: the workgroups' partials in order, divided by N.
__global__ void sqn_loss_final_kernel(SqnArgs A, uint32_t n_snap)
{
    const uint32_t snap = blockIdx.x * blockDim.x + threadIdx.x;
    if (snap >= n_snap) return;
    const double *p = A.loss_part + static_cast<size_t>(snap) * A.nblk * 2;
    double h = 0.0, l = 0.0;
    for (uint32_t b = 0; b < A.nblk; ++b) dd_add(h, l, p[2 * b], p[2 * b + 1]);
    A.fval[snap] = (h + l) / static_cast<double>(A.N);
}

// Statistics across replications: streams F(w^{K+1}), F at each checkpoint, and the relative
// squared error ((F_c - F_K) / F_c)^2 of Table 2, each as double-double sums of values and squares.
__global__ void sqn_stats_kernel(SqnArgs A)
{
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint32_t nc = A.n_ckpt;
    const double *Yv = A.fval + static_cast<size_t>(nc) * A.R;
    const uint32_t n_streams = 1 + 2 * nc;
    for (uint32_t s = 0; s < n_streams; ++s) {
        double h = 0.0, l = 0.0, qh = 0.0, ql = 0.0, cnt = 0.0;
        for (uint32_t r = 0; r < A.R; ++r) {
            double x;
            if (s == 0) {
                x = Yv[r];
            } else if (s <= nc) {
                x = A.fval[static_cast<size_t>(s - 1) * A.R + r];
            } else {
                const double f = A.fval[static_cast<size_t>(s - 1 - nc) * A.R + r];
                if (f == 0.0) continue;
                const double e = (f - Yv[r]) / f;
                x = e * e;
            }
            dd_add(h, l, x, 0.0);
            dd_add(qh, ql, x * x, fma(x, x, -(x * x)));
            cnt += 1.0;
        }
        double *o = A.stats + s * kStreamFields;
        o[0] = h;
        o[1] = l;
        o[2] = qh;
        o[3] = ql;
        o[4] = cnt;
    }
    double mn = INFINITY, mx = -INFINITY;
    for (uint32_t r = 0; r < A.R; ++r) {
        mn = fmin(mn, Yv[r]);
        mx = fmax(mx, Yv[r]);
    }
    A.stats[n_streams * kStreamFields] = mn;
    A.stats[n_streams * kStreamFields + 1] = mx;
}

int launch_sqn_run(const SqnArgs &A, hipStream_t s)
{
    const bool one = A.nq <= static_cast<uint32_t>(kRunBlock);
    if (A.pairs_fp32) {
        if (one) hipLaunchKernelGGL((sqn_run_kernel<1, float>), dim3(A.R), dim3(kRunBlock), 0, s, A);
        else hipLaunchKernelGGL((sqn_run_kernel<2, float>), dim3(A.R), dim3(kRunBlock), 0, s, A);
    } else {
        if (one) hipLaunchKernelGGL((sqn_run_kernel<1, double>), dim3(A.R), dim3(kRunBlock), 0, s, A);
        else hipLaunchKernelGGL((sqn_run_kernel<2, double>), dim3(A.R), dim3(kRunBlock), 0, s, A);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_sqn_loss(const SqnArgs &A, hipStream_t s)
{
    const uint32_t n_snap = (A.n_ckpt + 1) * A.R;
    if (n_snap >= kSqnManySnap) {
        hipLaunchKernelGGL(sqn_transpose_kernel, dim3((A.ld + 31) / 32, (n_snap + 31) / 32), dim3(256), 0, s, A, n_snap);
        hipLaunchKernelGGL(sqn_loss_many_kernel, dim3(A.nblk, (n_snap + 63) / 64), dim3(kSqnLossBlock), 0, s, A, n_snap);
    } else {
        hipLaunchKernelGGL(sqn_loss_kernel, dim3(A.nblk, n_snap), dim3(kSqnLossBlock), 0, s, A);
    }
    hipLaunchKernelGGL(sqn_loss_final_kernel, dim3((n_snap + 63) / 64), dim3(64), 0, s, A, n_snap);
    hipLaunchKernelGGL(sqn_stats_kernel, dim3(1), dim3(64), 0, s, A);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace fw
