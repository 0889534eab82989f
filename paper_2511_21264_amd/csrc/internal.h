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
    S_COVS, S_COVA, S_COVL, S_COVL32, S_COVLI, S_COVZ, S_COVU, S_NU64, S_PLAIN, S_N
};

int mapping_of(unsigned flags);
// the mapping of a launch over K samples: pinned by the flags, else the
// context's measured choice for K's class, else the built-in rule
int resolve_mapping(const mppi_ctx *c, long K, unsigned flags);
// Mappings whose rollouts agree bit for bit form one family: the 16-lane
// team, the one-wave and the two-wave forms evaluate every value by the
// same operations; the one-lane form rounds differently.  A request's
// results are those of its own mapping's family, whatever it is batched with.
inline int map_family(int map) { return map == mppi::MAP_LANE ? mppi::MAP_LANE : mppi::MAP_TEAM; }
// launch groups of packed batches and of the server's iterations: mapping
// family (one lane; the team family; the task forms' one lane; the task
// forms' one or two waves) x contact-list instantiation (up to 4, up to 8)
constexpr int NGROUP = 8;
inline int group_index(int family, int n_cmax)
{
    const int f = family == mppi::MAP_LANE ? 0 : family == mppi::MAP_TASK ? 2 : family == mppi::MAP_TASK_WAVE ? 3 : 1;
    return 2 * f + (n_cmax > 4 ? 1 : 0);
}
inline int group_family(int g)
{
    const int f = g >> 1;
    return f == 0 ? mppi::MAP_LANE : f == 1 ? mppi::MAP_TEAM : f == 2 ? mppi::MAP_TASK : mppi::MAP_TASK_WAVE;
}
// the family of a request of K samples planned alone with these flags
// (scenes with a box object or the further task-cost terms run one sample
// per lane)
inline int request_family(const mppi_ctx *c, const mppi_scene *s, long K, unsigned flags);
// the mapping of a packed launch of total_k samples whose requests all belong
// to `family` (a pinned mapping wins; else the measured or built-in choice
// for total_k, kept inside the family)
int family_launch_mapping(const mppi_ctx *c, int family, long total_k, unsigned flags);
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
    // Calls on one context share its scratch buffers.  Each call records
    // order_ev on its stream when it has enqueued its work; a call on another
    // stream than the previous one first waits for that event, so calls on one
    // context run in call order whatever streams they name.
    hipEvent_t order_ev = nullptr;
    hipStream_t last_stream = nullptr;
    bool has_last = false;
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
    uint64_t gen = 0;  // unique per scene created in this process (keys of cached graphs)
    mppi_scene_desc desc;
    mppi::DevModel host;
    mppi::DevModel *dev = nullptr;
};

namespace mppi_host {
int set_device(mppi_ctx *c);

// the mapping of a launch over K samples of scene s (see resolve_mapping);
// MPPI_E_INVAL when the flags pin a mapping the scene cannot run in
int scene_mapping(const mppi_ctx *c, const mppi_scene *s, long K, unsigned flags, int *map);

inline int request_family(const mppi_ctx *c, const mppi_scene *s, long K, unsigned flags)
{
    if (s->host.task_form) {
        int map = mppi::MAP_TASK;
        scene_mapping(c, s, K, flags, &map);  // the callers have validated the flags
        return map == mppi::MAP_TASK ? mppi::MAP_TASK : mppi::MAP_TASK_WAVE;
    }
    return map_family(resolve_mapping(c, K, flags));
}


// Orders a call on stream s after the context's previous call (see
// mppi_ctx::order_ev): begin() before the first enqueue; the destructor
// records the call's end on s.
class CtxStream {
public:
    CtxStream(mppi_ctx *c, hipStream_t s) : c_(c), s_(s) {}
    int begin()
    {
        if (c_->has_last && c_->last_stream != s_) HIPCHK(hipStreamWaitEvent(s_, c_->order_ev, 0));
        began_ = true;
        return MPPI_OK;
    }
    ~CtxStream()
    {
        if (!began_) return;
        if (hipEventRecord(c_->order_ev, s_) == hipSuccess) {
            c_->last_stream = s_;
            c_->has_last = true;
        }
    }
    CtxStream(const CtxStream &) = delete;
    CtxStream &operator=(const CtxStream &) = delete;

private:
    mppi_ctx *c_;
    hipStream_t s_;
    bool began_ = false;
};
// drops every cached graph of the context (their nodes bake in buffer addresses)
void drop_graphs(mppi_ctx *c);
// a plan with any of the options (qp, cov nullable) and the best sequence of
// the final iteration in U_best (nullable), as the public entry points run it
int plan_with(mppi_ctx *ctx, const mppi_scene *scene, const float *x0, const float *nominal_U, int K, int H,
              double lambda, const float *sigma, const mppi_opts *opts, const mppi_qp *qp, const mppi_cov *cov,
              float *U_new, float *U_best, float *costs, mppi_stats *stats, void *stream);
}
