// Serving loop of the C ABI: continuous batching of MPPI iterations over
// replanning requests from many cells (mppi_server_*, mppi_cell_*,
// mppi_submit, mppi_poll, mppi_cancel).
//
// One worker thread per server owns a non-blocking stream.  Each pass of
// its loop: admit queued requests (scheduler in sched.h: FIFO, per-cell
// order, device-memory admission against a fixed arena), stage their
// inputs, launch ONE packed MPPI iteration over every active request (each
// at its own iteration index: rollout, statistics and update launches
// driven by per-request argument tables), then, for requests that just ran
// their last iteration, launch the finishing work (divergence fallback,
// output copies, warm-start shift of the cell's nominal and the plant
// advance of the cell's state).  Argument tables are double-buffered, so
// the worker builds iteration i+1 while iteration i runs and retires the
// requests of iteration i-1 as soon as it completes.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"
#include "sched.h"

using namespace mppi;
using namespace mppi_host;

namespace {

struct Cell {
    const mppi_scene *scene = nullptr;
    int H = 0;
    float *x = nullptr;   // device [NX]
    float *nu = nullptr;  // device [H][14]
};

size_t al(size_t b) { return (b + 255) / 256 * 256; }

// byte offsets of a request's slices in the device and pinned arenas
struct Layout {
    size_t x0, sig, nom, nu, cost, w, cnt, dist, st, adv_cost, adv_dist, dev_total;
    size_t h_x0, h_sig, h_nom, h_st, h_U, h_cost, host_total;
};

Layout make_layout(int K, int H, size_t nsig)
{
    Layout L;
    size_t o = 0;
    auto take = [&](size_t b) {
        const size_t r = o;
        o += al(b);
        return r;
    };
    L.x0 = take(NX * sizeof(float));
    L.sig = take(nsig * sizeof(float));
    L.nom = take((size_t)H * NU * sizeof(float));
    L.nu = take((size_t)H * NU * sizeof(float));
    L.cost = take((size_t)K * sizeof(float));
    L.w = take((size_t)K * sizeof(double));
    L.cnt = take((size_t)K * 4 * sizeof(int));
    L.dist = take((size_t)K * MAXCOST * sizeof(float));
    L.st = take(sizeof(PlanStats));
    L.adv_cost = take(sizeof(float));
    L.adv_dist = take(MAXCOST * sizeof(float));
    L.dev_total = o;
    o = 0;
    L.h_x0 = take(NX * sizeof(float));
    L.h_sig = take(nsig * sizeof(float));
    L.h_nom = take((size_t)H * NU * sizeof(float));
    L.h_st = take(sizeof(PlanStats));
    L.h_U = take((size_t)H * NU * sizeof(float));
    L.h_cost = take((size_t)K * sizeof(float));
    L.host_total = o;
    return L;
}

struct Req {
    uint64_t id = 0;
    mppi_request r{};  // the caller's request (output pointers are written at completion)
    const mppi_scene *scene = nullptr;
    Cell *cp = nullptr;  // the cell (stable address) or null
    int cell = -1, advance = 0, K = 0, H = 0, M = 0;
    bool dev_io = false, sps = false, x0_from_cell = false, nom_from_cell = false;
    size_t nsig = 0;
    std::vector<float> x0, nom, sig;  // host copies of host inputs
    Layout L{};
    char *d = nullptr, *h = nullptr;  // arena slices (while admitted)
    int status = MPPI_OK, iters = 0;
    bool done = false, cancelled = false;
    double t_submit = 0, t_admit = -1, t_done = -1, t_deadline = INFINITY;

    template <class T> T *dp(size_t off) const { return (T *)(d + off); }
    template <class T> T *hp(size_t off) const { return (T *)(h + off); }
};

}  // namespace

struct mppi_server {
    mppi_ctx *ctx = nullptr;
    mppi_server_opts o{};
    hipStream_t s = nullptr;
    char *dbase = nullptr, *hbase = nullptr;
    Scheduler sched;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    std::unordered_map<uint64_t, Req> reqs;
    std::vector<std::unique_ptr<Cell>> cells;  // accessed under mu; Cell addresses are stable
    uint64_t next_id = 1;
    mppi_server_info info{};
    std::chrono::steady_clock::time_point t0;
    // double-buffered argument tables and the requests each buffer retires
    void *dtab[2] = {nullptr, nullptr}, *htab[2] = {nullptr, nullptr};
    size_t tcap[2] = {0, 0};
    hipEvent_t ev[2] = {nullptr, nullptr};
    // timing of each buffer's packed iteration, its load (sum of K * H), and
    // the recent (load, ms) pairs the iteration model is fitted to
    hipEvent_t tev0[2] = {nullptr, nullptr}, tev1[2] = {nullptr, nullptr};
    double load_at[2] = {0.0, 0.0};
    std::vector<std::pair<double, double>> meas;
    size_t meas_next = 0;
    // completion minus predicted end of recent requests (the model's margin)
    std::vector<double> lateness;
    size_t late_next = 0;
    IterModel model;
    bool inflight[2] = {false, false};
    std::vector<uint64_t> fin_at[2], drop_at[2];
    int worker_rc = MPPI_OK;
    std::string worker_err;

    double now_ms() const
    {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace {

void fill_stats(const Req &R, const PlanStats &p, mppi_stats *st)
{
    std::memset(st, 0, sizeof *st);
    st->ess = p.ess;
    st->c_min = p.cmin;
    st->best = p.best;
    st->n_nonfinite = R.K - p.n_finite;
    st->diverged = p.diverged;
    st->iterations = R.M;
    for (int q = 0; q < 64 && q < R.M; ++q) st->cmin_iter[q] = p.cmin_iter[q];
    st->contacts = (double)p.counters[0];
    st->np_tests = (double)p.counters[1];
    st->box_tests = (double)p.counters[2];
    st->overflow = (double)p.counters[3];
    st->rollout_launches = R.M;
}

// Wait for the work of buffer `b` and retire its requests.
// The iteration model from the recent measured packed iterations: floor =
// the fastest of them; base + slope * W by least squares (slope 0 and base
// their mean when the loads do not vary; both kept >= 0).  Until 8 are
// measured the model given at creation stands.
void fit_model(mppi_server *S)
{
    const size_t n = S->meas.size();
    if (n < 8) return;
    double fl = S->meas[0].second;
    for (auto &m : S->meas) fl = std::min(fl, m.second);
    S->model.floor_ms = fl;
    double sw = 0, st = 0, sww = 0, swt = 0;
    for (auto &m : S->meas) {
        sw += m.first;
        st += m.second;
        sww += m.first * m.first;
        swt += m.first * m.second;
    }
    const double mw = sw / n, mt = st / n, vw = sww / n - mw * mw, cwt = swt / n - mw * mt;
    double slope = vw > 1e-9 * (mw * mw + 1.0) ? cwt / vw : 0.0;
    slope = std::max(slope, 0.0);
    S->model.ms_per_work = slope;
    S->model.base_ms = std::max(mt - slope * mw, 0.0);
}

int retire(mppi_server *S, int b)
{
    if (!S->inflight[b]) return MPPI_OK;
    HIPCHK(hipEventSynchronize(S->ev[b]));
    float it_ms = -1.f;
    if (S->load_at[b] > 0 && hipEventElapsedTime(&it_ms, S->tev0[b], S->tev1[b]) != hipSuccess) it_ms = -1.f;
    std::lock_guard<std::mutex> lk(S->mu);
    const double t = S->now_ms();
    if (it_ms >= 0.f) {
        const std::pair<double, double> m(S->load_at[b], (double)it_ms);
        if (S->meas.size() < 64)
            S->meas.push_back(m);
        else
            S->meas[S->meas_next++ % 64] = m;
        fit_model(S);
    }
    S->load_at[b] = 0.0;
    for (uint64_t id : S->fin_at[b]) {
        Req &R = S->reqs.at(id);
        if (const SchedReq *q = S->sched.find(id)) {
            // how late the prediction made at admission turned out
            const double e = t - q->pred_end;
            if (S->lateness.size() < 128)
                S->lateness.push_back(e);
            else
                S->lateness[S->late_next++ % 128] = e;
            if (S->lateness.size() >= 16) {
                std::vector<double> v = S->lateness;
                const size_t k = v.size() * 95 / 100;
                std::nth_element(v.begin(), v.begin() + k, v.end());
                S->model.margin_ms = std::max(v[k], 0.0);
            }
        }
        const PlanStats &p = *R.hp<PlanStats>(R.L.h_st);
        R.status = p.diverged ? MPPI_E_DIVERGED : MPPI_OK;
        if (!R.dev_io) {
            if (R.r.U_new) std::memcpy(R.r.U_new, R.hp<float>(R.L.h_U), (size_t)R.H * NU * sizeof(float));
            if (R.r.costs) std::memcpy(R.r.costs, R.hp<float>(R.L.h_cost), (size_t)R.K * sizeof(float));
        }
        if (R.r.stats) fill_stats(R, p, R.r.stats);
        R.iters = R.M;
        R.t_done = t;
        R.done = true;
        if (t > R.t_deadline) ++S->info.late;
        S->sched.release(id);
        R.d = R.h = nullptr;
        ++S->info.completed;
    }
    for (uint64_t id : S->drop_at[b]) {
        Req &R = S->reqs.at(id);
        const SchedReq *q = S->sched.find(id);
        R.iters = q ? q->m : 0;
        R.status = MPPI_E_CANCELLED;
        R.t_done = t;
        R.done = true;
        S->sched.release(id);
        R.d = R.h = nullptr;
        ++S->info.cancelled;
    }
    S->fin_at[b].clear();
    S->drop_at[b].clear();
    S->inflight[b] = false;
    S->cv_done.notify_all();
    return MPPI_OK;
}

// inputs of a newly admitted request -> its device slices
int stage(mppi_server *S, Req &R)
{
    hipStream_t s = S->s;
    PlanStats *hst = R.hp<PlanStats>(R.L.h_st);
    std::memset(hst, 0, sizeof *hst);
    hst->best = -1;
    HIPCHK(hipMemcpyAsync(R.dp<PlanStats>(R.L.st), hst, sizeof(PlanStats), hipMemcpyHostToDevice, s));
    const Cell *c = R.cp;
    const size_t nH = (size_t)R.H * NU * sizeof(float);
    auto in = [&](size_t doff, size_t hoff, const float *src, const std::vector<float> &copy, size_t bytes) -> int {
        if (R.dev_io) {
            HIPCHK(hipMemcpyAsync(R.d + doff, src, bytes, hipMemcpyDeviceToDevice, s));
        } else {
            std::memcpy(R.h + hoff, copy.data(), bytes);
            HIPCHK(hipMemcpyAsync(R.d + doff, R.h + hoff, bytes, hipMemcpyHostToDevice, s));
        }
        return MPPI_OK;
    };
    int rc;
    if (R.x0_from_cell)
        HIPCHK(hipMemcpyAsync(R.d + R.L.x0, c->x, NX * sizeof(float), hipMemcpyDeviceToDevice, s));
    else if ((rc = in(R.L.x0, R.L.h_x0, R.r.x0, R.x0, NX * sizeof(float))))
        return rc;
    if ((rc = in(R.L.sig, R.L.h_sig, R.r.sigma, R.sig, R.nsig * sizeof(float)))) return rc;
    if (R.nom_from_cell)
        HIPCHK(hipMemcpyAsync(R.d + R.L.nom, c->nu, nH, hipMemcpyDeviceToDevice, s));
    else if ((rc = in(R.L.nom, R.L.h_nom, R.r.nominal_U, R.nom, nH)))
        return rc;
    HIPCHK(hipMemcpyAsync(R.d + R.L.nu, R.d + R.L.nom, nH, hipMemcpyDeviceToDevice, s));
    return MPPI_OK;
}

int ensure_tab(mppi_server *S, int b, size_t bytes)
{
    if (S->tcap[b] >= bytes) return MPPI_OK;
    if (S->dtab[b]) HIPCHK(hipFree(S->dtab[b]));
    if (S->htab[b]) HIPCHK(hipHostFree(S->htab[b]));
    S->dtab[b] = S->htab[b] = nullptr;
    S->tcap[b] = 0;
    const size_t want = bytes * 2;
    if (hipMalloc(&S->dtab[b], want) != hipSuccess || hipHostMalloc(&S->htab[b], want) != hipSuccess)
        return fail(MPPI_E_NOMEM, "argument table allocation failed");
    S->tcap[b] = want;
    return MPPI_OK;
}

// One packed iteration over `act` into table buffer b; `fin` are the ones
// running their last iteration.
int launch_iteration(mppi_server *S, int b, const std::vector<Req *> &act, const std::vector<int> &m_of,
                     const std::vector<Req *> &fin)
{
    hipStream_t s = S->s;
    const int n = (int)act.size(), nf = (int)fin.size();
    // One rollout launch per group of requests that share the family of the
    // mapping they would run alone and the contact-list instantiation (n_cmax
    // up to 4, or up to 8), so a request's results and its cell's advance do
    // not depend on what else is in flight.
    auto group_of = [&](const Req *R) {
        return group_index(request_family(S->ctx, R->scene, R->K, S->o.flags), R->scene->host.n_cmax);
    };
    long grp_k[NGROUP] = {};
    for (Req *R : act) grp_k[group_of(R)] += R->K;
    int gmap[NGROUP];
    for (int g = 0; g < NGROUP; ++g)
        gmap[g] = family_launch_mapping(S->ctx, group_family(g), grp_k[g], S->o.flags);
    std::vector<int> gblk[NGROUP], gablk[NGROUP], ublk;
    for (int i = 0; i < n; ++i) {
        const int g = group_of(act[i]), per = samples_per_block(gmap[g]);
        const int nb = (act[i]->K + per - 1) / per;
        for (int q = 0; q < nb; ++q) { gblk[g].push_back(i); gblk[g].push_back(q); }
        for (int k = 0; k < act[i]->H; ++k) { ublk.push_back(i); ublk.push_back(k); }
    }
    // the plant advance of finished requests' cells: one sample each, in the
    // mapping family of the request (its own K decides, as when alone)
    std::vector<Req *> adv;
    for (Req *R : fin)
        if (R->cell >= 0 && R->advance > 0) {
            gablk[group_of(R)].push_back((int)adv.size());
            gablk[group_of(R)].push_back(0);
            adv.push_back(R);
        }
    int amap[NGROUP];
    for (int g = 0; g < NGROUP; ++g) amap[g] = family_launch_mapping(S->ctx, group_family(g), 1, S->o.flags);
    std::vector<int> blk, ablk;
    size_t goff[NGROUP], gaoff[NGROUP];
    for (int g = 0; g < NGROUP; ++g) {
        goff[g] = blk.size();
        blk.insert(blk.end(), gblk[g].begin(), gblk[g].end());
        gaoff[g] = ablk.size();
        ablk.insert(ablk.end(), gablk[g].begin(), gablk[g].end());
    }
    const int na = (int)adv.size();
    const size_t bytes = al(n * sizeof(RolloutArgs)) + al(n * sizeof(StatsArgs)) + al(n * sizeof(UpdateArgs)) +
                         al(nf * sizeof(FinishArgs)) + al(na * sizeof(RolloutArgs)) + al(blk.size() * sizeof(int)) +
                         al(ublk.size() * sizeof(int)) + al(ablk.size() * sizeof(int));
    int rc = ensure_tab(S, b, bytes);
    if (rc) return rc;
    char *h = (char *)S->htab[b], *d = (char *)S->dtab[b];
    size_t o = 0;
    auto take = [&](size_t sz) {
        const size_t r = o;
        o += al(sz);
        return r;
    };
    const size_t o_r = take(n * sizeof(RolloutArgs)), o_s = take(n * sizeof(StatsArgs)),
                 o_u = take(n * sizeof(UpdateArgs)), o_f = take(nf * sizeof(FinishArgs)),
                 o_a = take(na * sizeof(RolloutArgs)), o_b = take(blk.size() * sizeof(int)),
                 o_ub = take(ublk.size() * sizeof(int)), o_ab = take(ablk.size() * sizeof(int));
    RolloutArgs *hr = (RolloutArgs *)(h + o_r);
    StatsArgs *hs = (StatsArgs *)(h + o_s);
    UpdateArgs *hu = (UpdateArgs *)(h + o_u);
    FinishArgs *hf = (FinishArgs *)(h + o_f);
    RolloutArgs *ha = (RolloutArgs *)(h + o_a);
    for (int i = 0; i < n; ++i) {
        const Req &R = *act[i];
        const uint32_t k0 = (uint32_t)(R.r.opts.seed & 0xffffffffu), k1 = (uint32_t)(R.r.opts.seed >> 32);
        PlanStats *st = R.dp<PlanStats>(R.L.st);
        RolloutArgs ra = {};
        ra.md = R.scene->dev;
        ra.x0 = R.dp<float>(R.L.x0);
        ra.x0_shared = 1;
        ra.nu = R.dp<float>(R.L.nu);
        ra.sigma = R.dp<float>(R.L.sig);
        ra.sigma_per_step = R.sps ? 1 : 0;
        ra.key0 = k0;
        ra.key1 = k1;
        ra.m = m_of[i];
        ra.K = R.K;
        ra.H = R.H;
        ra.costs = R.dp<float>(R.L.cost);
        ra.counters = R.dp<int>(R.L.cnt);
        ra.diverged = &st->diverged;
        ra.dist = R.dp<float>(R.L.dist);
        hr[i] = ra;
        const int ne = (R.r.opts.n_elite <= 0 || R.r.opts.n_elite >= R.K) ? R.K : R.r.opts.n_elite;
        hs[i] = StatsArgs{R.dp<float>(R.L.cost), R.K, 1.0 / R.r.lambda, ne, R.dp<double>(R.L.w), st, m_of[i],
                          R.dp<int>(R.L.cnt)};
        hu[i] = UpdateArgs{R.dp<double>(R.L.w), R.K, R.H, R.dp<float>(R.L.nu), R.dp<float>(R.L.sig), ra.sigma_per_step,
                           R.scene->host.u_max, k0, k1, m_of[i], R.r.opts.eta, st, R.dp<float>(R.L.nu), nullptr};
    }
    for (int i = 0; i < nf; ++i) {
        const Req &R = *fin[i];
        hf[i] = FinishArgs{R.dp<PlanStats>(R.L.st), R.dp<float>(R.L.nom), R.dp<float>(R.L.nu),
                           (R.dev_io && R.r.U_new) ? R.r.U_new : nullptr,
                           R.cp ? R.cp->nu : nullptr, R.H, R.cp ? R.advance : 0};
    }
    for (int i = 0; i < na; ++i) {
        const Req &R = *adv[i];
        RolloutArgs ra = {};
        ra.md = R.scene->dev;
        ra.x0 = R.dp<float>(R.L.x0);
        ra.x0_shared = 1;
        ra.U = R.dp<float>(R.L.nu);  // the first `advance` rows of U_new
        ra.K = 1;
        ra.H = R.advance;
        ra.costs = R.dp<float>(R.L.adv_cost);
        ra.xout = R.cp->x;
        ra.dist = R.dp<float>(R.L.adv_dist);
        ha[i] = ra;
    }
    std::memcpy(h + o_b, blk.data(), blk.size() * sizeof(int));
    std::memcpy(h + o_ub, ublk.data(), ublk.size() * sizeof(int));
    std::memcpy(h + o_ab, ablk.data(), ablk.size() * sizeof(int));
    HIPCHK(hipMemcpyAsync(d, h, o, hipMemcpyHostToDevice, s));
    for (int g = 0; g < NGROUP; ++g)
        if (!gblk[g].empty())
            launch_rollout_batch((const RolloutArgs *)(d + o_r), (const int *)(d + o_b) + goff[g],
                                 (int)gblk[g].size() / 2, (g & 1) ? 8 : 4, -1, gmap[g], s);
    launch_stats_batch((const StatsArgs *)(d + o_s), n, -1, s);
    launch_update_batch((const UpdateArgs *)(d + o_u), (const int *)(d + o_ub), (int)ublk.size() / 2, -1, s);
    if (nf) launch_finish_batch((const FinishArgs *)(d + o_f), nf, s);
    for (int g = 0; g < NGROUP; ++g)
        if (!gablk[g].empty())
            launch_rollout_batch((const RolloutArgs *)(d + o_a), (const int *)(d + o_ab) + gaoff[g],
                                 (int)gablk[g].size() / 2, (g & 1) ? 8 : 4, 0, amap[g], s);
    HIPCHK(hipGetLastError());
    for (Req *R : fin) {
        const size_t nH = (size_t)R->H * NU * sizeof(float);
        if (R->dev_io) {
            if (R->r.costs)
                HIPCHK(hipMemcpyAsync(R->r.costs, R->d + R->L.cost, (size_t)R->K * sizeof(float),
                                      hipMemcpyDeviceToDevice, s));
        } else {
            if (R->r.U_new) HIPCHK(hipMemcpyAsync(R->h + R->L.h_U, R->d + R->L.nu, nH, hipMemcpyDeviceToHost, s));
            if (R->r.costs)
                HIPCHK(hipMemcpyAsync(R->h + R->L.h_cost, R->d + R->L.cost, (size_t)R->K * sizeof(float),
                                      hipMemcpyDeviceToHost, s));
        }
        HIPCHK(hipMemcpyAsync(R->h + R->L.h_st, R->d + R->L.st, sizeof(PlanStats), hipMemcpyDeviceToHost, s));
    }
    return MPPI_OK;
}

int worker_loop(mppi_server *S)
{
    int rc = set_device(S->ctx);
    if (rc) return rc;
    int b = 0;
    for (;;) {
        std::vector<Req *> admitted, act, fin;
        std::vector<int> m_of;
        std::vector<uint64_t> dropped;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            std::vector<uint64_t> shed;
            const double now = S->now_ms();
            // the iteration launched last pass (buffer b ^ 1) may still run
            for (uint64_t id : S->sched.admit(now, S->model, &shed, S->inflight[b ^ 1] ? 1 : 0)) {
                Req &R = S->reqs.at(id);
                const SchedReq *q = S->sched.find(id);
                R.d = S->dbase + q->dev_off;
                R.h = S->hbase + q->host_off;
                R.t_admit = now;
                admitted.push_back(&R);
            }
            for (uint64_t id : shed) {
                Req &R = S->reqs.at(id);
                R.done = true;
                R.status = MPPI_E_LATE;
                R.t_done = now;
                ++S->info.shed;
            }
            if (!shed.empty()) S->cv_done.notify_all();
            for (const SchedReq *q : S->sched.next_iteration(&dropped)) {
                Req &R = S->reqs.at(q->id);
                act.push_back(&R);
                m_of.push_back(q->m);
                if (q->m + 1 >= q->M) fin.push_back(&R);
            }
            S->info.mem_high_water = S->sched.dev().high_water();
        }
        for (Req *R : admitted)
            if ((rc = stage(S, *R))) return rc;
        if (act.empty()) {
            if (!dropped.empty()) {
                // cancelled requests whose last launches may still run
                HIPCHK(hipEventRecord(S->ev[b], S->s));
                S->drop_at[b] = dropped;
                S->inflight[b] = true;
            }
            if ((rc = retire(S, b ^ 1)) || (rc = retire(S, b))) return rc;
            std::unique_lock<std::mutex> lk(S->mu);
            if (S->sched.n_active() > 0) continue;
            if (S->sched.n_pending() > 0) {
                // nothing in flight holds memory any more; a request that
                // still cannot be admitted is blocked on its cell only
                continue;
            }
            if (S->stop) return MPPI_OK;
            S->cv_work.wait(lk, [&] { return S->stop || S->sched.n_pending() > 0 || S->sched.n_active() > 0; });
            continue;
        }
        HIPCHK(hipEventRecord(S->tev0[b], S->s));
        if ((rc = launch_iteration(S, b, act, m_of, fin))) return rc;
        HIPCHK(hipEventRecord(S->tev1[b], S->s));
        HIPCHK(hipEventRecord(S->ev[b], S->s));
        double load = 0.0;
        for (Req *R : act) load += (double)R->K * (double)R->H;
        S->load_at[b] = load;
        {
            std::lock_guard<std::mutex> lk(S->mu);
            std::vector<uint64_t> done = S->sched.advance();
            S->fin_at[b] = done;
            S->drop_at[b] = dropped;
            S->inflight[b] = true;
            ++S->info.iterations;
            S->info.request_iters += act.size();
            for (Req *R : act) S->info.env_steps += (uint64_t)R->K * (uint64_t)R->H;
        }
        if ((rc = retire(S, b ^ 1))) return rc;
        b ^= 1;
    }
}

void worker_main(mppi_server *S)
{
    const int rc = worker_loop(S);
    std::lock_guard<std::mutex> lk(S->mu);
    if (rc) {
        S->worker_rc = rc;
        S->worker_err = mppi_last_error();
        // fail everything still waiting
        for (auto &kv : S->reqs)
            if (!kv.second.done) {
                kv.second.done = true;
                kv.second.status = rc;
            }
    }
    S->cv_done.notify_all();
}

}  // namespace

extern "C" {

int mppi_server_create(mppi_ctx *ctx, const mppi_server_opts *opts, mppi_server **out)
{
    if (!ctx || !out) return fail(MPPI_E_INVAL, "NULL argument");
    *out = nullptr;
    mppi_server_opts o = opts ? *opts : mppi_server_opts{};
    if (o.mem_budget == 0) o.mem_budget = 1ull << 30;
    if (o.max_active <= 0) o.max_active = 256;
    if (o.max_pending <= 0) o.max_pending = 4096;
    if (o.max_active > 4096) return fail(MPPI_E_INVAL, "max_active above 4096");
    if (o.mem_budget < (1u << 20)) return fail(MPPI_E_INVAL, "mem_budget below 1 MiB");
    if (!(o.deadline_ms >= 0) || !(o.iter_base_ms >= 0) || !(o.iter_ms_per_menv >= 0) ||
        !std::isfinite(o.iter_base_ms) || !std::isfinite(o.iter_ms_per_menv))
        return fail(MPPI_E_INVAL, "deadline_ms and the iteration model must be finite and >= 0");
    int rc = set_device(ctx);
    if (rc) return rc;
    mppi_server *S = new mppi_server();
    S->ctx = ctx;
    S->o = o;
    S->t0 = std::chrono::steady_clock::now();
    // pinned staging: inputs, stats and host outputs; far smaller than the
    // device slices (no distance history, weights or counters)
    const size_t host_bytes = std::max<size_t>(o.mem_budget / 8, 16u << 20);
    bool ok = hipStreamCreateWithFlags(&S->s, hipStreamNonBlocking) == hipSuccess;
    ok = ok && hipMalloc((void **)&S->dbase, o.mem_budget) == hipSuccess;
    ok = ok && hipHostMalloc((void **)&S->hbase, host_bytes) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&S->ev[0], hipEventDisableTiming) == hipSuccess;
    ok = ok && hipEventCreateWithFlags(&S->ev[1], hipEventDisableTiming) == hipSuccess;
    for (int b = 0; b < 2; ++b) {
        ok = ok && hipEventCreate(&S->tev0[b]) == hipSuccess;
        ok = ok && hipEventCreate(&S->tev1[b]) == hipSuccess;
    }
    if (!ok) {
        if (S->dbase) (void)hipFree(S->dbase);
        if (S->hbase) (void)hipHostFree(S->hbase);
        if (S->s) (void)hipStreamDestroy(S->s);
        for (int b = 0; b < 2; ++b)
            for (hipEvent_t e : {S->ev[b], S->tev0[b], S->tev1[b]})
                if (e) (void)hipEventDestroy(e);
        delete S;
        return fail(MPPI_E_NOMEM, "server allocation failed");
    }
    S->model.base_ms = o.iter_base_ms;
    S->model.ms_per_work = o.iter_ms_per_menv * 1e-6;
    S->sched = Scheduler(o.mem_budget, host_bytes, o.max_active, o.max_pending);
    S->worker = std::thread(worker_main, S);
    *out = S;
    return MPPI_OK;
}

void mppi_server_destroy(mppi_server *S)
{
    if (!S) return;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        std::vector<uint64_t> ids;
        for (auto &kv : S->reqs)
            if (!kv.second.done) ids.push_back(kv.first);
        for (uint64_t id : ids) {
            if (S->sched.cancel(id) == 1) {
                Req &R = S->reqs.at(id);
                R.done = true;
                R.status = MPPI_E_CANCELLED;
            }
        }
        S->cv_work.notify_all();
    }
    if (S->worker.joinable()) S->worker.join();
    (void)hipSetDevice(S->ctx->device);
    (void)hipStreamSynchronize(S->s);
    for (auto &c : S->cells) {
        if (c->x) (void)hipFree(c->x);
        if (c->nu) (void)hipFree(c->nu);
    }
    for (int b = 0; b < 2; ++b) {
        if (S->dtab[b]) (void)hipFree(S->dtab[b]);
        if (S->htab[b]) (void)hipHostFree(S->htab[b]);
        if (S->ev[b]) (void)hipEventDestroy(S->ev[b]);
        if (S->tev0[b]) (void)hipEventDestroy(S->tev0[b]);
        if (S->tev1[b]) (void)hipEventDestroy(S->tev1[b]);
    }
    (void)hipFree(S->dbase);
    (void)hipHostFree(S->hbase);
    (void)hipStreamDestroy(S->s);
    delete S;
}

int mppi_cell_create(mppi_server *S, const mppi_scene *scene, int H, const float *x0, const float *nominal_U,
                     int *cell)
{
    if (!S || !scene || !x0 || !cell) return fail(MPPI_E_INVAL, "NULL argument");
    if (scene->ctx != S->ctx) return fail(MPPI_E_INVAL, "scene of another context");
    if (H < 1 || H > MPPI_MAX_H) return fail(MPPI_E_INVAL, "H=%d out of range", H);
    if (!all_finite(x0, NX) || (nominal_U && !all_finite(nominal_U, (size_t)H * NU)))
        return fail(MPPI_E_INVAL, "non-finite input");
    int rc = set_device(S->ctx);
    if (rc) return rc;
    auto cp = std::make_unique<Cell>();
    Cell &c = *cp;
    c.scene = scene;
    c.H = H;
    const size_t nH = (size_t)H * NU * sizeof(float);
    if (hipMalloc((void **)&c.x, NX * sizeof(float)) != hipSuccess || hipMalloc((void **)&c.nu, nH) != hipSuccess) {
        if (c.x) (void)hipFree(c.x);
        return fail(MPPI_E_NOMEM, "cell allocation failed");
    }
    std::vector<float> z((size_t)H * NU, 0.f);
    HIPCHK(hipMemcpy(c.x, x0, NX * sizeof(float), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c.nu, nominal_U ? nominal_U : z.data(), nH, hipMemcpyHostToDevice));
    std::lock_guard<std::mutex> lk(S->mu);
    S->cells.push_back(std::move(cp));
    *cell = (int)S->cells.size() - 1;
    return MPPI_OK;
}

int mppi_cell_read(mppi_server *S, int cell, float *x, float *nominal_U)
{
    if (!S) return fail(MPPI_E_INVAL, "NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    if (cell < 0 || cell >= (int)S->cells.size()) return fail(MPPI_E_INVAL, "unknown cell %d", cell);
    S->cv_done.wait(lk, [&] { return S->sched.cell_idle(cell) || S->worker_rc != MPPI_OK; });
    if (S->worker_rc) return fail(S->worker_rc, "server worker failed: %s", S->worker_err.c_str());
    const Cell c = *S->cells[cell];
    lk.unlock();
    int rc = set_device(S->ctx);
    if (rc) return rc;
    if (x) HIPCHK(hipMemcpy(x, c.x, NX * sizeof(float), hipMemcpyDeviceToHost));
    if (nominal_U) HIPCHK(hipMemcpy(nominal_U, c.nu, (size_t)c.H * NU * sizeof(float), hipMemcpyDeviceToHost));
    return MPPI_OK;
}

int mppi_submit(mppi_server *S, const mppi_request *req, int cell, int advance, unsigned flags, uint64_t *ticket)
{
    if (!S || !req || !ticket) return fail(MPPI_E_INVAL, "NULL argument");
    Req R;
    R.r = *req;
    R.cell = cell;
    R.K = req->K;
    R.M = req->opts.M;
    const Cell *c = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (cell >= (int)S->cells.size()) return fail(MPPI_E_INVAL, "unknown cell %d", cell);
        if (cell >= 0) c = S->cells[cell].get();
        if (S->worker_rc) return fail(S->worker_rc, "server worker failed: %s", S->worker_err.c_str());
        if (S->stop) return fail(MPPI_E_INVAL, "server is shutting down");
    }
    R.cp = (Cell *)c;
    if (c) {
        if (req->scene && req->scene != c->scene) return fail(MPPI_E_INVAL, "request scene differs from the cell's");
        if (req->H != 0 && req->H != c->H) return fail(MPPI_E_INVAL, "request H differs from the cell's");
        R.scene = c->scene;
        R.H = c->H;
        if (advance < 0 || advance > R.H) return fail(MPPI_E_INVAL, "advance %d outside [0, H]", advance);
        R.advance = advance;
        R.x0_from_cell = req->x0 == nullptr;
        R.nom_from_cell = req->nominal_U == nullptr;
        if (!req->sigma) return fail(MPPI_E_INVAL, "NULL sigma");
    } else {
        if (!req->scene || !req->x0 || !req->nominal_U || !req->sigma || !req->U_new)
            return fail(MPPI_E_INVAL, "NULL argument in a request without a cell");
        R.scene = req->scene;
        R.H = req->H;
    }
    if (R.scene->ctx != S->ctx) return fail(MPPI_E_INVAL, "scene of another context");
    int map_r;
    if (scene_mapping(S->ctx, R.scene, req->K, S->o.flags, &map_r)) return MPPI_E_INVAL;
    if (R.K < 1 || R.K > MPPI_MAX_K || R.H < 1 || R.H > MPPI_MAX_H) return fail(MPPI_E_INVAL, "K or H out of range");
    if (!(req->lambda > 0) || !std::isfinite(req->lambda) || R.M < 1 || R.M > 100000 || !std::isfinite(req->opts.eta))
        return fail(MPPI_E_INVAL, "bad lambda, M or eta");
    R.dev_io = req->opts.flags & MPPI_DEVICE_PTRS;
    R.sps = req->opts.flags & MPPI_SIGMA_PER_STEP;
    R.nsig = R.sps ? (size_t)R.H * NU : NU;
    const size_t nH = (size_t)R.H * NU;
    if (!R.dev_io) {
        if ((!R.x0_from_cell && !all_finite(req->x0, NX)) || (!R.nom_from_cell && !all_finite(req->nominal_U, nH)) ||
            !all_finite(req->sigma, R.nsig))
            return fail(MPPI_E_INVAL, "non-finite input");
        for (size_t q = 0; q < R.nsig; ++q)
            if (req->sigma[q] < 0) return fail(MPPI_E_INVAL, "sigma < 0");
        if (!R.x0_from_cell) R.x0.assign(req->x0, req->x0 + NX);
        if (!R.nom_from_cell) R.nom.assign(req->nominal_U, req->nominal_U + nH);
        R.sig.assign(req->sigma, req->sigma + R.nsig);
    }
    R.L = make_layout(R.K, R.H, R.nsig);
    std::lock_guard<std::mutex> lk(S->mu);
    R.id = S->next_id++;
    R.t_submit = S->now_ms();
    if (S->o.deadline_ms > 0) R.t_deadline = R.t_submit + S->o.deadline_ms;
    SchedReq q;
    q.id = R.id;
    q.cell = cell;
    q.M = R.M;
    q.deadline = R.t_deadline;
    q.work = (double)R.K * (double)R.H;
    q.dev_bytes = R.L.dev_total;
    q.host_bytes = R.L.host_total;
    std::vector<uint64_t> sup;
    const int e = S->sched.enqueue(q, (flags & MPPI_SUPERSEDE) != 0, &sup);
    for (uint64_t id : sup) {
        Req &O = S->reqs.at(id);
        O.done = true;
        O.status = MPPI_E_CANCELLED;
        O.t_done = R.t_submit;
        ++S->info.superseded;
    }
    if (!sup.empty()) S->cv_done.notify_all();
    if (e) {
        ++S->info.rejected;
        return fail(MPPI_E_BUSY, e == 1 ? "request queue full" : "request larger than the memory budget");
    }
    ++S->info.submitted;
    *ticket = R.id;
    S->reqs.emplace(R.id, std::move(R));
    S->cv_work.notify_one();
    return MPPI_OK;
}

int mppi_poll(mppi_server *S, uint64_t ticket, int timeout_ms, mppi_ticket_info *info)
{
    if (!S) return fail(MPPI_E_INVAL, "NULL server");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return fail(MPPI_E_INVAL, "unknown ticket %llu", (unsigned long long)ticket);
    if (!it->second.done && timeout_ms != 0) {
        auto pred = [&] { return S->reqs.at(ticket).done; };
        if (timeout_ms < 0)
            S->cv_done.wait(lk, pred);
        else
            S->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred);
        it = S->reqs.find(ticket);
    }
    Req &R = it->second;
    if (!R.done) return MPPI_PENDING;
    if (info) {
        info->status = R.status;
        info->iterations = R.iters;
        info->t_submit_ms = R.t_submit;
        info->t_admit_ms = R.t_admit;
        info->t_done_ms = R.t_done;
        info->t_deadline_ms = R.t_deadline;
    }
    S->sched.forget(ticket);
    S->reqs.erase(it);
    return MPPI_OK;
}

int mppi_cancel(mppi_server *S, uint64_t ticket)
{
    if (!S) return fail(MPPI_E_INVAL, "NULL server");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end() || it->second.done) return fail(MPPI_E_INVAL, "unknown or finished ticket");
    const int r = S->sched.cancel(ticket);
    if (r == 0) return fail(MPPI_E_INVAL, "request is finishing");
    if (r == 1) {
        it->second.done = true;
        it->second.status = MPPI_E_CANCELLED;
        it->second.t_done = S->now_ms();
        ++S->info.cancelled;
        S->cv_done.notify_all();
    }
    return MPPI_OK;
}

int mppi_server_query(mppi_server *S, mppi_server_info *info)
{
    if (!S || !info) return fail(MPPI_E_INVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    *info = S->info;
    info->active = S->sched.n_active();
    info->pending = S->sched.n_pending();
    info->mem_high_water = S->sched.dev().high_water();
    info->model_base_ms = S->model.base_ms;
    info->model_ms_per_menv = S->model.ms_per_work * 1e6;
    info->model_floor_ms = S->model.floor_ms;
    info->model_margin_ms = S->model.margin_ms;
    return MPPI_OK;
}

}  // extern "C"
