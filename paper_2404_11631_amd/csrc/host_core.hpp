// host_core.hpp -- device-free host logic shared by the C-ABI translation units.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/sim.h"
#include "sim_types.hpp"

namespace fw {
namespace host {

constexpr size_t kErrLen = 512;
// dense-L runs keep per-path decision counts in 16 bits
constexpr uint64_t kMaxDenseT = 65535;

int fail(char *err, int code, const char *fmt, ...);
int validate(char *err, const sim_params *p, uint64_t R, uint64_t T);
// the wide path (sim_run_wide): many assets, diagonal Sigma, Gaussian noise, FP32, few replications
int validate_wide(char *err, const sim_params *p, uint64_t R, uint64_t T);
// Algorithm 2, the newsvendor (sim_run_newsvendor)
int validate_newsvendor(char *err, const sim_nv_params *p, uint64_t R, uint64_t T);
int validate_newsvendor_lp(char *err, const sim_nv_params *p, const sim_nv_constraints *con, uint64_t R, uint64_t T);
int validate_sqn(char *err, const sim_sqn_params *p, uint64_t N, uint32_t n, uint64_t R, uint64_t K);
void fill_desc(InstanceDesc &D, const sim_params *p, uint64_t R, uint64_t T, uint64_t seed);
// Per-epoch table of a sample-size schedule (sim_params.n_schedule): N_k, 1/N_k and the
// coefficients c1 = sigma/N_k, c2 = 2 lambda sigma/(N_k - 1) of every epoch k, in both
// precisions, rounded exactly as fill_desc rounds the plain run's (so a constant schedule
// reproduces it bit for bit). Byte offsets of each array in one buffer.
struct SchedLayout {
    uint64_t epochs = 0, bytes = 0;
    uint64_t off_n = 0, off_inv_f = 0, off_inv_d = 0, off_c_f = 0, off_c_d = 0;   // c: [E][2 d] (c1 | c2)
};
void fill_schedule(const sim_params *p, uint64_t T, std::vector<unsigned char> &buf, SchedLayout &L);
// Law of the control-variate features of a run (diagonal Sigma, reference gradient p->cv_ref):
// reference-decision probabilities p (0 origin, j+1 vertex e_j) and their running sums, the
// weights S2 = sum_e W2_e, S4 = sum_e W2_e^2, S1 = sum_e W1_e, S11 = sum_e W1_e^2 (W2_e, W1_e the
// epoch sums of (t+1)^2 and (t+1)), the standardization of the counts, the most probable category.
struct CvLaw {
    double p[kMaxD + 1], cum[kMaxD + 1], mean[kMaxD + 1], inv[kMaxD + 1];
    double S2, S4, S1, S11, mean1, inv1;
    uint32_t top;
    uint64_t epochs;
};
// The per-asset scale of the features' reference decision: sigma_j, or L_jj for a dense factor
// (the decision then reads each noise coordinate against its own diagonal entry, which keeps the
// product form of the law).
double cv_scale(const sim_params *p, uint32_t j);
// dense features keep their per-category sums of (t+1)^2 in 32 bits: T(T+1)(2T+1)/6 < 2^32
constexpr uint64_t kMaxDenseFeatT = 2343;
void cv_pick_probs(uint32_t d, const double *b, const double *s, double *p);
CvLaw cv_law(const sim_params *p, uint64_t T);

// The two FP32 operands of the dense-L kernels, sqrt(2 ln 2) L (for g = L h) and its transpose
// (for v = L'w), each [d/16][d/4][64] in the lane order of v_mfma_f32_16x16x4f32 (row 16 mt +
// lane mod 16, column the asset that lane lane/16 holds in register kk), and L copied in FP64.
void dense_operands(const double *L, uint32_t d, float *Ag, float *Av, double *L64);
double kkt_fstar(const double *mu, const double *sigma, uint32_t d, double lambda);
// statistics from the reduced stream layout (per stream: sum hi/lo, squares hi/lo, count)
void fill_stats(sim_stats_out *out, const double *F, uint32_t n_ckpt, const uint64_t *ckpts, double ymin,
                double ymax, const uint64_t *dec, uint32_t d, uint64_t tau_count, uint64_t tau_sum, uint64_t R,
                uint64_t T, double fstar, double ms, double path_steps);

// lanes splitting the assets of one replication in a batched tile: 8 assets per lane at most
uint32_t asset_lanes(uint32_t d);
// samples per lane: ceil(N / Ps) rounded up to whole Philox-block rounds
uint32_t chunk_of(uint32_t N, uint32_t d, uint32_t Ps, bool t_noise);
// modelled VALU work of one lane of a batched tile with P lanes per replication
double lane_cost(const sim_params &p, uint64_t T, uint32_t P);

// The work plan of a batched run.
struct BatchPlan {
    std::vector<uint32_t> P, tiles_of, slot_begin;
    std::vector<uint64_t> path_base, cnt_base, wsum_base, dlog_base;
    std::vector<InstanceDesc> desc;
    std::vector<double> fstar;
    std::vector<Tile> tiles;             // longest first
    uint32_t n_tiles = 0, max_ckpt = 1;
    bool wave_mode = false;              // every instance at 64 lanes per replication, Gaussian, N d small
    uint64_t total_R = 0, total_steps = 0, cnt_total = 0, wsum_total = 0, dlog_total = 0;
};

int plan_batch(char *err, uint32_t n_inst, const sim_params *p, const uint64_t *R, const uint64_t *T,
               uint64_t seed, const sim_batch_config *cfg, uint32_t n_cu, BatchPlan &out);

}  // namespace host
}  // namespace fw
