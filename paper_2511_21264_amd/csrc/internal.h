// Host-side definitions shared by the translation units of the C ABI
// (api.hip: contexts, scenes, plans; serve.hip: the serving loop).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/mppi.h"
#include "kernels.h"

namespace mppi_host {

// records the message of the last failure of the calling thread; returns code
int fail(int code, const char *fmt, ...);

#define HIPCHK(expr)                                                                                     \
    do {                                                                                                 \
        hipError_t e_ = (expr);                                                                          \
        if (e_ != hipSuccess) return fail(MPPI_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct Buf {
    void *p = nullptr;
    size_t cap = 0;
};

enum Slot {
    S_X0, S_SIGMA, S_NU, S_NOM, S_COSTS, S_W, S_CNT, S_DIST, S_IN0, S_IN1, S_OUT0, S_OUT1, S_OUT2, S_OUT3,
    S_BTAB, S_BST, S_BIN, S_BNU, S_BCOST, S_BW, S_BCNT, S_BDIST, S_QPP, S_QPU,
    S_COVS, S_COVA, S_COVL, S_COVL32, S_COVLI, S_COVZ, S_COVU, S_NU64, S_N
};

int mapping_of(unsigned flags);
// the mapping of a launch over K samples: pinned by the flags, else the
// context's measured choice for K's class, else the built-in rule
int resolve_mapping(const mppi_ctx *c, long K, unsigned flags);
int k_class(long K);
bool all_finite(const float *p, size_t n);

}  // namespace mppi_host

// an instantiated HIP graph of one plan's launch sequence and what it baked in
struct PlanGraph {
    std::vector<uintptr_t> key;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned long long last_use = 0;
};

struct mppi_ctx {
    int device = 0;
    // measured rollout mapping per sample-count class (MPPI_MAP_* of the
    // fastest launch); index: ceil(log2 K)), 0 = not tuned
    int tuned_map[21] = {0};
    std::vector<PlanGraph> graphs;  // small LRU cache (MPPI_GRAPH)
    hipStream_t capture = nullptr;  // private stream the plan graphs are captured on
    unsigned long long graph_clock = 0;
    mppi_host::Buf buf[mppi_host::S_N];
    mppi::PlanStats *st = nullptr;
    std::vector<hipEvent_t> ev;
    // pinned host staging of packed-batch tables
    void *host_tab = nullptr;
    size_t host_tab_cap = 0;
    // the QP smoothing's (I + rho A^T A)^-1 in buf[S_QPP], for this horizon and penalty
    int qp_H = 0;
    double qp_rho = 0.0;
    int qp_S = 0;
};

struct mppi_scene {
    mppi_ctx *ctx = nullptr;
    mppi_scene_desc desc;
    mppi::DevModel host;
    mppi::DevModel *dev = nullptr;
};

namespace mppi_host {
int set_device(mppi_ctx *c);
// a plan with any of the options (qp, cov nullable) and the best sequence of
// the final iteration in U_best (nullable), as the public entry points run it
int plan_with(mppi_ctx *ctx, const mppi_scene *scene, const float *x0, const float *nominal_U, int K, int H,
              double lambda, const float *sigma, const mppi_opts *opts, const mppi_qp *qp, const mppi_cov *cov,
              float *U_new, float *U_best, float *costs, mppi_stats *stats, void *stream);
}
