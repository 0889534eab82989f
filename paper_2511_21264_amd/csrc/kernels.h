// Kernel declarations and the launch-argument records shared by the kernel
// and host translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "devmodel.h"

namespace mppi {

struct RolloutArgs {
    const DevModel *md;
    const float *x0;      // [K][NX] or one shared state
    int x0_shared;
    const float *nu;      // [H][14] mean (sampling mode)
    const float *sigma;   // [14] or [H][14]
    int sigma_per_step;
    const float *U;       // [K][H][14] explicit controls (simulation mode) or null
    uint32_t key0, key1;
    int m, K, H, n_sub;
    float *costs;         // [K]
    float *terms;         // [K][7] or null
    float *xout;          // [K][NX] or [K][H][NX] (traj) or null
    int traj;
    int *counters;        // [K][4] or null: contacts, np tests, box tests, overflow
    const int *diverged;  // sticky flag of the plan (skip work when set) or null
    float *dist;          // [n_cost][K] collision-distance history (scratch of the launch)
};

// Per-plan device-side statistics (one record per plan in flight).
struct PlanStats {
    double cmin;
    double wsum;
    double ess;
    int best;
    int n_finite;
    int diverged;
    int pad;
    double cmin_iter[64];
    unsigned long long counters[4];
};

struct StatsArgs {
    const float *costs;
    int K;
    double inv_lambda;
    int n_elite;
    double *weights;        // [K] normalized weights
    PlanStats *st;
    int iter;
    const int *counters;    // [K][4] or null
    int fp32;               // weights and their sums in FP32 (precision study) instead of FP64
};

struct UpdateArgs {
    const double *weights;
    int K, H;
    const float *nu_in;
    const float *sigma;
    int sigma_per_step;
    float u_max;
    uint32_t key0, key1;
    int m;
    double eta;
    const PlanStats *st;
    float *nu_out;
    double *nu_out64;
    int fp32;               // weighted mean accumulated in FP32 instead of FP64
    const float *U;         // [K][H][14] the samples as given (QP-smoothed plans), or null: regenerated
};

// End of a served request: nu := nominal when the plan diverged, copied to
// the caller's device output and, shifted by `shift` control steps (the tail
// repeats the last row), to the cell's resident nominal.
struct FinishArgs {
    const PlanStats *st;
    const float *nom;
    float *nu;
    float *out;
    float *cell_nu;
    int H, shift;
};

// sample-to-lane mapping of the rollout
constexpr int MAP_AUTO = 0, MAP_LANE = 1, MAP_TEAM = 2, MAP_WAVE = 3, MAP_SPLIT = 4;
// the forms that carry the box-shaped object and the further task terms
// (scenes with obj_box or ext run only in these): one lane per sample, and
// one or two waves per sample (bit-identical to each other)
constexpr int MAP_TASK = 5, MAP_TASK_WAVE = 6, MAP_TASK_SPLIT = 7;
int pick_mapping(int K, int requested);
void launch_rollout(const RolloutArgs &a, int ncmax, hipStream_t s, int mapping = MAP_AUTO);
// the plain form: control step k of every sample (one sample per lane), the
// per-sample carry in ps ([PLAIN_FIELDS][K] words) between the launches
constexpr int PLAIN_FIELDS = NX + NU + NTERMS + 16 + 4;
void launch_rollout_step(const RolloutArgs &a, int ncmax, float *ps, int k, bool task, hipStream_t s);
int samples_per_block(int mapping);
// packed launches: tables live in device memory; block b of a rollout launch
// covers block blk[2b+1] of scene blk[2b]; update blocks are (scene, step)
// pairs; m >= 0 is the iteration of every entry, m < 0 keeps each entry's own
void launch_rollout_batch(const RolloutArgs *d_tab, const int *d_blk, int nblk, int ncmax, int m, int mapping,
                          hipStream_t s);
void launch_stats_batch(const StatsArgs *d_tab, int n, int m, hipStream_t s);
void launch_update_batch(const UpdateArgs *d_tab, const int *d_blk, int nblk, int m, hipStream_t s);
void launch_stats(const StatsArgs &a, hipStream_t s);
// QP smoothing of sampled sequences (one workgroup per sample, one wave per
// joint, one horizon step per lane; H <= 64)
struct ProjectArgs {
    const float *P;         // [H][S] (I + rho A^T A)^-1, rows padded with zeros to S floats
    int S;                  // row stride of P: a multiple of 4, >= H rounded up to 4
    const float *U_in;      // [K][H][14] samples, or null: nu + sigma * z from the Philox counters
    float *U_out;           // [K][H][14] projected samples
    const float *x0;        // [K][NX] start states (commanded positions), or one shared
    int x0_shared;
    const float *nu, *sigma;
    int sigma_per_step;
    uint32_t key0, key1;
    int m;
    int K, H;
    float dt, u_max, dacc, djerk;  // control step, velocity box, acc_max dt, jerk_max dt^2
    float pos_lo[NU], pos_hi[NU];
    float rho, alpha;
    int iters;
};
void launch_project(const ProjectArgs &a, hipStream_t s);

// Covariance adaptation and full-covariance sampling over the n = 14 H
// vector of a sequence (step-major: index 14 k + d)
struct CovArgs {
    const float *U;         // [K][n] the samples as rolled out
    const double *w;        // [K] weights (any positive scale; normalised by their sum)
    const double *nu;       // [n] the updated mean nu_{m+1}
    const double *S_in;     // [n][n] Sigma_m (lower triangle read)
    double *S_out;          // [n][n] Sigma_{m+1}, full symmetric (may be S_in)
    int K, n;
    double eta, eps;
};
void launch_cov_update(const CovArgs &a, hipStream_t s);

struct CholArgs {
    const double *S;  // [n][n] (lower triangle read)
    double *A;        // [n][n] work copy (lower), updated in place
    double *L;        // [n][n] factor (upper triangle zeroed); may be S
    float *L32;       // [n][n] the factor in single precision (nullable)
    double *Linv;     // [2][32][32] inverses of the diagonal blocks (block b in half b & 1)
    int *flag;        // first column with a non-positive pivot, n if none
    int n;
    int reset_flag;   // set *flag = n first (else failures of earlier calls stay recorded)
};
void launch_cholesky(const CholArgs &a, hipStream_t s);

struct SampleFullArgs {
    float *Z;           // [K][n] scratch: the Philox normals of iteration m
    const float *L32;   // [n][n] lower factor, upper triangle zero
    const float *nu;    // [n] mean
    float *U;           // [K][n] clip(nu + L z_j)
    int K, n;
    uint32_t key0, key1;
    int m;
    float u_max;
};
void launch_sample_full(const SampleFullArgs &a, hipStream_t s);
// Sigma = diag(sigma^2) over n = 14 H (sigma[14] or [H][14])
void launch_diag_sigma(const float *sigma, int sps, int n, double *S, hipStream_t s);
void launch_to_f32(const double *src, float *dst, long n, hipStream_t s);
void launch_lower_f32(float *L, int n, hipStream_t s);  // zero the upper triangle

// The best sample's sequence of an iteration (Alg. 1 returns the lowest-cost
// sequence of the final iteration): row st->best of the stored samples, or
// regenerated from (nu, sigma, the Philox counters); the mean when no sample
// had a finite cost
struct BestArgs {
    const PlanStats *st;
    const float *U;      // [K][H][14] stored samples, or null
    const float *nu;     // [H][14] the mean the samples were drawn around
    const float *sigma;
    int sigma_per_step;
    float u_max;
    uint32_t key0, key1;
    int m, H;
    float *out;          // [H][14]
};
void launch_best(const BestArgs &a, hipStream_t s);

void launch_update(const UpdateArgs &a, hipStream_t s);
void launch_sample(const DevModel *md, const float *nu, const float *sigma, int sps, uint32_t k0, uint32_t k1,
                   int m, int K, int H, float *U, float *z, uint32_t *words, hipStream_t s);
void launch_broadphase(const DevModel *md, const float *lo, const float *hi, int n, int ngeom, float margin,
                       int *flags, hipStream_t s);
void launch_narrowphase(const DevModel *md, const float *X, int n, float *phi, float *nrm, float *pt, float *lo,
                        float *hi, hipStream_t s);
void launch_reset_stats(PlanStats *st, hipStream_t s, int n = 1);
void launch_finish_batch(const FinishArgs *d_tab, int n, hipStream_t s);

}  // namespace mppi
