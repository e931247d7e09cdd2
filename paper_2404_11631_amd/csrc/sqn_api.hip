// sqn_api.hip -- host side of Algorithms 3-4 (sim_sqn_load, sim_run_sqn): the data set upload,
// validation, device buffers, the launches, and the statistics and records of the last run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "engine.hpp"
#include "sqn.hpp"
#include "sqn_split.hpp"

using namespace fw::host;

extern "C" {

int sim_sqn_load(sim_ctx *ctx, const uint8_t *X, const uint8_t *z, uint64_t N, uint32_t n)
{
    if (!ctx) return SIM_EINVAL;
    if (!X || !z) return set_err(ctx, SIM_EINVAL, "X and z are required");
    if (n < 1 || n > SIM_SQN_MAX_N) return set_err(ctx, SIM_EINVAL, "n=%u outside [1, %u]", n, SIM_SQN_MAX_N);
    if (N < 1 || N >= (1ull << 31)) return set_err(ctx, SIM_EINVAL, "N=%llu outside [1, 2^31)", (unsigned long long)N);
    if (N * n >= (1ull << 40)) return set_err(ctx, SIM_EINVAL, "N n above 2^40");
    for (uint64_t i = 0; i < N; ++i) {
        if (z[i] > 1) return set_err(ctx, SIM_EINVAL, "label z[%llu] = %u is not 0 or 1", (unsigned long long)i, z[i]);
        const uint8_t *row = X + i * n;
        uint8_t any = 0;
        for (uint32_t j = 0; j < n; ++j) any |= row[j];
        if (any > 1)
            for (uint32_t j = 0; j < n; ++j)
                if (row[j] > 1)
                    return set_err(ctx, SIM_EINVAL, "X[%llu][%u] = %u is not 0 or 1", (unsigned long long)i, j, row[j]);
    }
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    SqnState &q = ctx->sqn;
    q.have_data = q.have = false;
    // bitmap rows: bit j % 32 of word j / 32, rows padded to a multiple of four words (16 bytes);
    // packed on the host a block of rows at a time (at most 64 MB of staging) and copied up
    const uint32_t xw = ((n + 31) / 32 + 3) / 4 * 4;
    const uint64_t block = 65536;
    std::vector<uint32_t> bits;
    try {
        bits.resize(static_cast<size_t>(std::min<uint64_t>(N, block)) * xw);
    } catch (const std::bad_alloc &) {
        return set_err(ctx, SIM_ENOMEM, "host staging for the feature bitmap");
    }
    int rc;
    if ((rc = ensure(ctx, q.X, sizeof(uint32_t) * static_cast<size_t>(N) * xw)) || (rc = ensure(ctx, q.z, N))) return rc;
    hipStream_t st = ctx->stream;
    for (uint64_t i0 = 0; i0 < N; i0 += block) {
        const uint64_t rows = std::min<uint64_t>(block, N - i0);
        std::fill(bits.begin(), bits.end(), 0u);
        for (uint64_t i = 0; i < rows; ++i) {
            const uint8_t *row = X + (i0 + i) * n;
            uint32_t *dst = bits.data() + i * xw;
            for (uint32_t j = 0; j < n; ++j) dst[j >> 5] |= static_cast<uint32_t>(row[j]) << (j & 31);
        }
        HIP_TRY(ctx, hipStreamSynchronize(st));     // the previous block's copy has read the staging
        HIP_TRY(ctx, hipMemcpyAsync(static_cast<uint32_t *>(q.X.ptr) + i0 * xw, bits.data(),
                                    sizeof(uint32_t) * rows * xw, hipMemcpyHostToDevice, st));
    }
    HIP_TRY(ctx, hipMemcpyAsync(q.z.ptr, z, N, hipMemcpyHostToDevice, st));
    HIP_TRY(ctx, hipStreamSynchronize(st));
    q.xw = xw;
    const uint32_t ld = (n + 3) / 4 * 4;
    q.N = N;
    q.n = n;
    q.ld = ld;
    q.have_data = true;
    return SIM_OK;
}

int sim_validate_sqn(const sim_sqn_params *p, uint64_t N, uint32_t n, uint64_t R, uint64_t K, char *msg, size_t len)
{
    char err[kErrLen] = {0};
    const int rc = validate_sqn(err, p, N, n, R, K);
    if (msg && len) std::snprintf(msg, len, "%s", rc ? err : "");
    return rc;
}

// Validation, the run's buffers and the kernels' arguments, shared by both run entry points.
static int sqn_prepare(sim_ctx *ctx, const sim_sqn_params *p, uint64_t R, uint64_t K, uint64_t seed,
                       fw::SqnArgs &A)
{
    if (!ctx) return SIM_EINVAL;
    SqnState &q = ctx->sqn;
    if (!q.have_data) return set_err(ctx, SIM_ESTATE, "no data set loaded (sim_sqn_load)");
    if (int rc = validate_sqn(ctx->err, p, q.N, q.n, R, K)) return rc;
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    q.have = false;
    for (hipEvent_t *e : {&q.ev0, &q.ev1, &q.ev2})
        if (!*e) HIP_TRY(ctx, hipEventCreate(e));
    const uint32_t nc = p->n_checkpoints;
    const size_t ld = q.ld;
    const uint32_t nblk = static_cast<uint32_t>((q.N + fw::kSqnLossRows - 1) / fw::kSqnLossRows);
    const size_t n_snap = static_cast<size_t>(nc + 1) * R;
    int rc;
    const size_t pb = p->pairs_fp32 ? sizeof(float) : sizeof(double);
    if ((rc = ensure(ctx, q.S, pb * R * p->M * ld)) || (rc = ensure(ctx, q.Y, pb * R * p->M * ld)) ||
        (rc = ensure(ctx, q.wprev, sizeof(double) * R * ld)) || (rc = ensure(ctx, q.acc, sizeof(double) * R * ld)) || (rc = ensure(ctx, q.wsnap, sizeof(double) * n_snap * ld)) ||
        (rc = ensure(ctx, q.pairs, sizeof(uint32_t) * R)) ||
        (n_snap >= fw::kSqnManySnap && (rc = ensure(ctx, q.wt, sizeof(double) * n_snap * ld))) ||
        (rc = ensure(ctx, q.loss_part, sizeof(double) * 2 * n_snap * nblk)) ||
        (rc = ensure(ctx, q.fval, sizeof(double) * n_snap)) ||
        (rc = ensure(ctx, q.stats, sizeof(double) * (fw::kMaxStreams * fw::kStreamFields + 2))))
        return rc;

    A = fw::SqnArgs{};
    A.n = q.n;
    A.ld = q.ld;
    A.nq = q.ld / 4;
    A.N = static_cast<uint32_t>(q.N);
    A.L = p->L;
    A.M = p->M;
    A.b = p->b;
    A.bH = p->b_H;
    A.k0 = static_cast<uint32_t>(seed);
    A.k1 = static_cast<uint32_t>(seed >> 32);
    A.inst = p->instance_id & 0xFFFFFFu;
    A.R = static_cast<uint32_t>(R);
    A.n_ckpt = nc;
    A.xw = q.xw;
    uint32_t G = 1;                                     // at most four 16-byte loads per lane and row
    while (G < 64 && G * 4 < A.xw / 4) G *= 2;
    A.G = G;
    uint32_t GV = 1;                                    // at most 32 quads per lane and stored vector
    while (GV < 64 && GV * 32 < A.nq) GV *= 2;
    A.GV = GV;
    A.K = K;
    A.beta = p->beta;
    for (uint32_t c = 0; c < nc; ++c) A.ckpt[c] = p->checkpoints[c];
    A.X = static_cast<const uint32_t *>(q.X.ptr);
    A.z = static_cast<const uint8_t *>(q.z.ptr);
    A.S = q.S.ptr;
    A.Y = q.Y.ptr;
    A.pairs_fp32 = p->pairs_fp32 ? 1u : 0u;
    A.wprev = static_cast<double *>(q.wprev.ptr);
    A.acc = static_cast<double *>(q.acc.ptr);
    A.wsnap = static_cast<double *>(q.wsnap.ptr);
    A.wt = static_cast<double *>(q.wt.ptr);
    A.pairs = static_cast<uint32_t *>(q.pairs.ptr);
    A.loss_part = static_cast<double *>(q.loss_part.ptr);
    A.nblk = nblk;
    A.fval = static_cast<double *>(q.fval.ptr);
    A.stats = static_cast<double *>(q.stats.ptr);

    return SIM_OK;
}

// The loss launches after the iterations, and the record of the run.
static int sqn_finish(sim_ctx *ctx, const sim_sqn_params *p, const fw::SqnArgs &A, uint64_t R, uint64_t K)
{
    SqnState &q = ctx->sqn;
    hipStream_t st = ctx->stream;
    HIP_TRY(ctx, hipEventRecord(q.ev1, st));
    if (fw::launch_sqn_loss(A, st)) return set_err(ctx, SIM_EDEVICE, "SQN loss launch failed");
    HIP_TRY(ctx, hipEventRecord(q.ev2, st));
    q.params = *p;
    q.R = R;
    q.K = K;
    q.nblk = A.nblk;
    q.have = true;
    return SIM_OK;
}

int sim_run_sqn(sim_ctx *ctx, const sim_sqn_params *p, uint64_t R, uint64_t K, uint64_t seed)
{
    if (!ctx) return SIM_EINVAL;
    fw::SqnArgs A;
    if (int rc = sqn_prepare(ctx, p, R, K, seed, A)) return rc;
    SqnState &q = ctx->sqn;
    hipStream_t st = ctx->stream;
    HIP_TRY(ctx, hipEventRecord(q.ev0, st));
    if (fw::launch_sqn_run(A, st)) return set_err(ctx, SIM_EDEVICE, "SQN launch failed");
    return sqn_finish(ctx, p, A, R, K);
}

int sim_run_sqn_split(sim_ctx *ctx, const sim_sqn_params *p, uint64_t R, uint64_t K, uint64_t seed)
{
    if (!ctx) return SIM_EINVAL;
    if (R > fw::kSplitMaxR)
        return set_err(ctx, SIM_EINVAL, "R=%llu above %u, the replications of a split run", (unsigned long long)R,
                       fw::kSplitMaxR);
    fw::SqnArgs A;
    if (int rc = sqn_prepare(ctx, p, R, K, seed, A)) return rc;
    SqnState &q = ctx->sqn;
    fw::SqnSplit P{};
    P.A = A;
    P.W = fw::sqn_split_slices(A.nq);
    const size_t ld = A.ld, W = P.W;
    int rc;
    if ((rc = ensure(ctx, q.sw, sizeof(double) * R * ld)) || (rc = ensure(ctx, q.sg, sizeof(double) * R * ld)) ||
        (rc = ensure(ctx, q.sxpart, sizeof(double) * 2 * R * A.b * W)) ||
        (rc = ensure(ctx, q.sdpart, sizeof(double) * R * 2 * A.M * W)) ||
        (rc = ensure(ctx, q.shpart, sizeof(double) * R * 2 * A.bH * W)) ||
        (rc = ensure(ctx, q.sypart, sizeof(double) * R * 3 * A.M * W)) ||
        (rc = ensure(ctx, q.ssmall, sizeof(double) * R * fw::kSqnSmall)))
        return rc;
    P.w = static_cast<double *>(q.sw.ptr);
    P.g = static_cast<double *>(q.sg.ptr);
    P.xpart = static_cast<double *>(q.sxpart.ptr);
    P.dpart = static_cast<double *>(q.sdpart.ptr);
    P.hpart = static_cast<double *>(q.shpart.ptr);
    P.ypart = static_cast<double *>(q.sypart.ptr);
    P.small = static_cast<double *>(q.ssmall.ptr);
    hipStream_t st = ctx->stream;
    HIP_TRY(ctx, hipEventRecord(q.ev0, st));
    const int lrc = fw::sqn_split_sequence(K, A.L, A.M, A.n_ckpt, A.ckpt,
                                           [&](fw::SqnSplitKernel kind, const fw::SqnSplitStep &step) {
                                               return fw::launch_sqn_split(P, kind, step, st);
                                           });
    if (lrc) return set_err(ctx, SIM_EDEVICE, "SQN split launch failed: %s", hipGetErrorString(hipGetLastError()));
    return sqn_finish(ctx, p, A, R, K);
}

int sim_sqn_stats(sim_ctx *ctx, sim_stats_out *out)
{
    if (!ctx || !out) return SIM_EINVAL;
    SqnState &q = ctx->sqn;
    if (!q.have) return set_err(ctx, SIM_ESTATE, "no SQN run yet");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipEventSynchronize(q.ev2));
    const uint32_t nc = q.params.n_checkpoints, n_streams = 1 + 2 * nc;
    double F[fw::kMaxStreams * fw::kStreamFields + 2];
    HIP_TRY(ctx, hipMemcpy(F, q.stats.ptr, sizeof(double) * (n_streams * fw::kStreamFields + 2), hipMemcpyDeviceToHost));
    float ms = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, q.ev0, q.ev1));
    const uint64_t none = 0;
    fill_stats(out, F, nc, q.params.checkpoints, F[n_streams * fw::kStreamFields], F[n_streams * fw::kStreamFields + 1],
               &none, 0, 0, 0, q.R, q.K, NAN, ms, static_cast<double>(q.R) * static_cast<double>(q.K));
    return SIM_OK;
}

int sim_sqn_paths(sim_ctx *ctx, sim_sqn_view *out)
{
    if (!ctx || !out) return SIM_EINVAL;
    SqnState &q = ctx->sqn;
    if (!q.have) return set_err(ctx, SIM_ESTATE, "no SQN run yet");
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipEventSynchronize(q.ev2));
    std::memset(out, 0, sizeof(*out));
    const uint32_t nc = q.params.n_checkpoints;
    out->R = q.R;
    out->K = q.K;
    out->n = q.n;
    out->ld = q.ld;
    out->n_checkpoints = nc;
    const double *fv = static_cast<const double *>(q.fval.ptr);
    const double *ws = static_cast<const double *>(q.wsnap.ptr);
    out->F = fv + static_cast<size_t>(nc) * q.R;
    out->F_ckpt = nc ? fv : nullptr;
    out->w = ws + static_cast<size_t>(nc) * q.R * q.ld;
    out->w_ckpt = nc ? ws : nullptr;
    out->pairs = static_cast<const uint32_t *>(q.pairs.ptr);
    out->M = q.params.M;
    out->pairs_fp32 = q.params.pairs_fp32 ? 1u : 0u;
    out->S = q.S.ptr;
    out->Y = q.Y.ptr;
    return SIM_OK;
}

int sim_sqn_hessian(sim_ctx *ctx, uint64_t rep, sim_sqn_hessian_view *out)
{
    if (!ctx || !out) return SIM_EINVAL;
    SqnState &q = ctx->sqn;
    if (!q.have) return set_err(ctx, SIM_ESTATE, "no SQN run yet");
    if (rep >= q.R) return set_err(ctx, SIM_EINVAL, "rep=%llu outside [0, %llu)", (unsigned long long)rep, (unsigned long long)q.R);
    HIP_TRY(ctx, hipSetDevice(ctx->device));
    HIP_TRY(ctx, hipEventSynchronize(q.ev2));
    uint32_t P = 0;
    HIP_TRY(ctx, hipMemcpy(&P, static_cast<const uint32_t *>(q.pairs.ptr) + rep, sizeof(uint32_t), hipMemcpyDeviceToHost));
    const uint32_t M = q.params.M;
    const uint32_t m = P < M ? P : M, head = P >= M ? P % M : 0;
    if (m == 0) return set_err(ctx, SIM_ESTATE, "replication %llu has no correction pair yet", (unsigned long long)rep);
    for (hipEvent_t *e : {&q.ev3, &q.ev4})
        if (!*e) HIP_TRY(ctx, hipEventCreate(e));
    int rc;
    const uint32_t ldh = fw::sqn_hessian_ld(q.n);
    if ((rc = ensure(ctx, q.H, sizeof(double) * q.n * ldh)) ||
        (rc = ensure(ctx, q.hscratch, sizeof(double) * fw::sqn_hessian_scratch(q.n))))
        return rc;
    fw::SqnArgs A{};
    A.n = q.n;
    A.ld = q.ld;
    A.M = M;
    A.S = q.S.ptr;
    A.Y = q.Y.ptr;
    A.pairs_fp32 = q.params.pairs_fp32 ? 1u : 0u;
    hipStream_t st = ctx->stream;
    HIP_TRY(ctx, hipEventRecord(q.ev3, st));
    if (fw::launch_sqn_hessian(A, static_cast<uint32_t>(rep), head, m, static_cast<double *>(q.hscratch.ptr),
                               static_cast<double *>(q.H.ptr), ldh, st))
        return set_err(ctx, SIM_EDEVICE, "Hessian launch failed");
    HIP_TRY(ctx, hipEventRecord(q.ev4, st));
    HIP_TRY(ctx, hipEventSynchronize(q.ev4));
    double gamma = 0.0;
    const double *gp = static_cast<const double *>(q.hscratch.ptr) + 6 * fw::kSqnMaxM * fw::kSqnMaxM;
    HIP_TRY(ctx, hipMemcpy(&gamma, gp, sizeof(double), hipMemcpyDeviceToHost));
    float ms = 0.0f;
    HIP_TRY(ctx, hipEventElapsedTime(&ms, q.ev3, q.ev4));
    out->n = q.n;
    out->ld = ldh;
    out->m = m;
    out->gamma = gamma;
    out->H = static_cast<const double *>(q.H.ptr);
    out->device_ms = ms;
    return SIM_OK;
}

}  // extern "C"
