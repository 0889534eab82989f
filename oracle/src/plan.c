/*
 * Oracle MPPI planner (Alg. 1), FP64.
 *
 * For m = 1..M: draw n sequences from N(nu_m, Sigma_m) with diagonal
 * Sigma (per-joint sigma, optionally per step); project each onto the
 * velocity box (the QP of Eqs. proj_cost/proj_bounds with only
 * |u| <= u_max reduces to an elementwise clamp, the Euclidean projection
 * onto a box); roll every sequence out from the same x0; sum its cost;
 * keep the n_e lowest costs (ties by index); update
 *   nu_{m+1} = (1 - eta) nu_m + eta sum_j s_j u_j / sum_j s_j,
 *   s_j = exp(-(c_j - c_min) / lambda)                (Eqs. mean_update,
 * s_formula; the common factor exp(c_min / lambda) cancels), with the
 * projected u_j.  Non-finite costs get weight 0.  Returns nu_M, the last
 * iteration's costs and the index of its lowest cost.
 * TEST INFRASTRUCTURE ONLY.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "oracle.h"

typedef struct { double c; int j; } CostIdx;

static int cmp_cost(const void *a, const void *b)
{
    const CostIdx *x = (const CostIdx *)a, *y = (const CostIdx *)b;
    if (x->c < y->c) return -1;
    if (x->c > y->c) return 1;
    return x->j - y->j;
}

/* clamped sample u_j (H x 14) of iteration m */
static void sample_u(const OScene *s, const double *nu, const double *sigma, int sigma_per_step, uint64_t seed,
                     int j, int m, int H, double *u)
{
    for (int k = 0; k < H; ++k) {
        double z[14];
        or_normals14(seed, (uint32_t)j, (uint32_t)k, (uint32_t)m, z);
        for (int d = 0; d < 14; ++d) {
            double sg = sigma_per_step ? sigma[14 * k + d] : sigma[d];
            double v = nu[14 * k + d] + sg * z[d];
            if (v > s->u_max) v = s->u_max;
            if (v < -s->u_max) v = -s->u_max;
            u[14 * k + d] = v;
        }
    }
}

void oracle_sample(const OScene *s, const double *nu, const double *sigma, int sigma_per_step, uint64_t seed, int K,
                   int H, int m, double *U)
{
    for (int j = 0; j < K; ++j) sample_u(s, nu, sigma, sigma_per_step, seed, j, m, H, U + (long)j * H * 14);
}

/* MPPI update from given samples and costs; returns number of finite costs */
int oracle_update(const double *U, const double *costs, int K, int H, double lambda, double eta, int n_elite,
                  const double *nu_in, double *nu_out, double *wsum_out, double *ess_out)
{
    CostIdx *ci = (CostIdx *)malloc(sizeof(CostIdx) * K);
    int nf = 0;
    for (int j = 0; j < K; ++j)
        if (isfinite(costs[j])) { ci[nf].c = costs[j]; ci[nf].j = j; ++nf; }
    if (nf == 0) {
        memcpy(nu_out, nu_in, sizeof(double) * H * 14);
        free(ci);
        return 0;
    }
    qsort(ci, nf, sizeof(CostIdx), cmp_cost);
    int ne = n_elite < nf ? n_elite : nf;
    double cmin = ci[0].c;
    double *acc = (double *)calloc((size_t)H * 14, sizeof(double));
    double ws = 0.0, ws2 = 0.0;
    for (int e = 0; e < ne; ++e) {
        double w = exp(-(ci[e].c - cmin) / lambda);
        const double *u = U + (long)ci[e].j * H * 14;
        for (int i = 0; i < H * 14; ++i) acc[i] += w * u[i];
        ws += w;
        ws2 += w * w;
    }
    for (int i = 0; i < H * 14; ++i) nu_out[i] = (1.0 - eta) * nu_in[i] + eta * acc[i] / ws;
    if (wsum_out) *wsum_out = ws;
    if (ess_out) *ess_out = ws * ws / ws2;
    free(acc);
    free(ci);
    return nf;
}

/* full plan; returns 0 ok, -4 when every sample diverged (nu_out = nominal) */
int oracle_plan(const OScene *s, const double *x0, const double *nominal, int K, int H, double lambda,
                const double *sigma, int sigma_per_step, int M, uint64_t seed, double eta, int n_elite,
                double *nu_out, double *costs_out, int *best_out, double *cmin_iter, int nthreads)
{
    OModel md;
    or_model(s, &md);
    double *nu = (double *)malloc(sizeof(double) * H * 14);
    double *nu2 = (double *)malloc(sizeof(double) * H * 14);
    double *U = (double *)malloc(sizeof(double) * (size_t)K * H * 14);
    memcpy(nu, nominal, sizeof(double) * H * 14);
    int rc = 0;
    for (int m = 0; m < M; ++m) {
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads)
        for (int j = 0; j < K; ++j) {
            double *u = U + (long)j * H * 14;
            sample_u(s, nu, sigma, sigma_per_step, seed, j, m, H, u);
            costs_out[j] = or_rollout(s, &md, x0, u, H, NULL, NULL);
        }
        int nf = oracle_update(U, costs_out, K, H, lambda, eta, n_elite, nu, nu2, NULL, NULL);
        double cmin = INFINITY;
        int best = -1;
        for (int j = 0; j < K; ++j)
            if (costs_out[j] < cmin) { cmin = costs_out[j]; best = j; }
        if (cmin_iter) cmin_iter[m] = cmin;
        if (best_out) *best_out = best;
        if (nf == 0) {
            memcpy(nu_out, nominal, sizeof(double) * H * 14);
            rc = -4;
            goto done;
        }
        memcpy(nu, nu2, sizeof(double) * H * 14);
    }
    memcpy(nu_out, nu, sizeof(double) * H * 14);
done:
    free(nu);
    free(nu2);
    free(U);
    return rc;
}
