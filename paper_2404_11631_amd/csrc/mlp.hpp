// mlp.hpp -- device-side description of the control-variate surrogate and its launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fw {

// The surrogate F -> 64 -> 64 -> 1: FP32 master parameters in the flat order
// W1 [64][F], b1 [64], W2 [64][64], b2 [64], w3 [64], b3, and the bfloat16 A-operand copies of W1
// ([2][KS1][64][8]), W2 and W2' ([2][4][64][8]), KS1 = ceil(F / 16).
struct MlpDev {
    float *theta;
    uint16_t *w1a, *w2a, *w2t;
    int F, KS1, P;
    int off_b1, off_w2, off_b2, off_w3, off_b3;
};

inline MlpDev mlp_layout(int F)
{
    MlpDev m{};
    m.F = F;
    m.KS1 = (F + 15) / 16;
    m.off_b1 = 64 * F;
    m.off_w2 = m.off_b1 + 64;
    m.off_b2 = m.off_w2 + 64 * 64;
    m.off_w3 = m.off_b2 + 64;
    m.off_b3 = m.off_w3 + 64;
    m.P = m.off_b3 + 1;
    return m;
}

// One Adam step: w -= lr (m1 bc1) / (sqrt(m2 bc2) + eps), bc = 1 / (1 - beta^t).
struct AdamStep {
    float lr, beta1, beta2, eps, bc1, bc2;
};

// Law of the path features for the aux draws (stream domain 2 of `seed`, `instance`): reference
// decisions i.i.d. over epochs with cumulative probabilities cum (origin first, last entry 2), the
// counts standardized by mean and inv, and the (t+1)-weighted count of category `top` by mean1, inv1.
struct AuxLaw {
    uint64_t seed;
    uint32_t instance;
    int d;
    uint64_t T;
    uint32_t M, top;
    double mean1, inv1;
    double cum[65], mean[65], inv[65];
};

int launch_mlp_forward(const MlpDev &m, const float *x, uint64_t ldx, uint64_t n, float shift, float scale,
                       float *out, hipStream_t st);
int launch_mlp_grad(const MlpDev &m, const float *x, uint64_t ldx, const float *y, uint64_t q0, uint64_t rows,
                    uint64_t a, uint64_t c, uint64_t n_data, float inv_batch, float *part, hipStream_t st);
int launch_mlp_reduce(const MlpDev &m, const float *part, uint32_t n_parts, int mode, const AdamStep &s, float *mom1,
                      float *mom2, float *grad_out, float *loss_out, hipStream_t st);
int launch_mlp_copies(const MlpDev &m, hipStream_t st);
int launch_mlp_init(const MlpDev &m, uint64_t seed, uint32_t instance, hipStream_t st);
int launch_cv_aux(const AuxLaw &law, uint64_t k0, uint64_t n, float *x, uint64_t ldx, hipStream_t st);
int launch_cv_moments(const double *A, const float *B, uint64_t n, double sa, double sb, double *part, uint32_t nb,
                      double *out, uint32_t *done, hipStream_t st);
int launch_cv_target(const double *Y, uint64_t n, double mean, double inv_sd, float *t, hipStream_t st);

}  // namespace fw
