// Closed-loop ball transport: the receding-horizon executor around the
// planner (Alg. 1's output executed as the paper describes: the first steps
// of the best sequence averaged and run, the next plan warm-started), with
// the phase machine and termination rules of episode.h.  Host code over the
// library's own plan (optionally with the QP smoothing and the full
// covariance) and mppi_simulate.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "episode.h"
#include "internal.h"

using mppi_host::fail;

extern "C" int mppi_episode(mppi_ctx *ctx, const mppi_scene *pick, const mppi_scene *move, const float *x0, int K,
                            int H, double lambda, const float *sigma, const mppi_opts *opts,
                            const mppi_episode_opts *eo, const mppi_qp *qp, float *x_final, float *u_exec,
                            float *x_hist, mppi_episode_result *res, void *stream)
{
    using mppi::NU;
    using mppi::NX;
    if (!ctx || !pick || !move || !x0 || !sigma || !opts || !eo || !res) return fail(MPPI_E_INVAL, "NULL argument");
    if (pick->ctx != ctx || move->ctx != ctx) return fail(MPPI_E_INVAL, "scene belongs to another context");
    if (K < 1 || K > MPPI_MAX_K || H < 1 || H > MPPI_MAX_H) return fail(MPPI_E_INVAL, "K=%d or H=%d out of range", K, H);
    if (opts->flags & MPPI_DEVICE_PTRS) return fail(MPPI_E_INVAL, "mppi_episode takes host arrays");
    if (eo->n_avg < 1 || eo->n_avg > H || eo->n_exec < 1 || eo->n_exec > H)
        return fail(MPPI_E_INVAL, "n_avg=%d, n_exec=%d must be in 1..H", eo->n_avg, eo->n_exec);
    if (eo->max_replans < 0 || ((u_exec || x_hist) && eo->max_replans == 0))
        return fail(MPPI_E_INVAL, "max_replans must be >= 0 (> 0 with u_exec or x_hist)");
    const double tols[] = {eo->grasp_tol, eo->width_tol, eo->goal_tol, eo->t_max};
    for (double v : tols)
        if (!(v > 0) || !std::isfinite(v)) return fail(MPPI_E_INVAL, "tolerances and t_max must be finite and > 0");
    if (!std::isfinite(eo->lift_z) || !std::isfinite(eo->drop_z)) return fail(MPPI_E_INVAL, "non-finite heights");
    if (pick->desc.h != move->desc.h || pick->desc.n_sub != move->desc.n_sub)
        return fail(MPPI_E_INVAL, "pick and move scenes must share the time step");
    const double dt = move->desc.h * move->desc.n_sub;  // the control step, from the description (double)
    const int n = H * NU;
    const bool sps = opts->flags & MPPI_SIGMA_PER_STEP;
    std::vector<double> Sg, Sn;  // the full covariance carried between replans (use_cov)
    auto sig2 = [&](int i) {
        const double sg = sigma[sps ? i : i % NU];
        return sg * sg;
    };
    if (eo->use_cov) {
        if (n > MPPI_COV_MAX_N) return fail(MPPI_E_INVAL, "n = 14 H = %d above MPPI_COV_MAX_N", n);
        if (!(opts->eta > 0 && opts->eta <= 1)) return fail(MPPI_E_INVAL, "eta must be in (0, 1] with use_cov");
        if (!(eo->cov_eps >= 0) || !std::isfinite(eo->cov_eps)) return fail(MPPI_E_INVAL, "cov_eps must be >= 0");
        Sg.assign((size_t)n * n, 0.0);
        Sn.assign((size_t)n * n, 0.0);
        for (int i = 0; i < n; ++i) Sg[(size_t)i * n + i] = sig2(i);
    }
    const mppi::EpRule rule = {eo->grasp_tol, eo->width_tol, eo->goal_tol, eo->lift_z, eo->drop_z, eo->t_max};
    mppi::EpState es;
    std::vector<float> x(x0, x0 + NX), xo(NX), nom((size_t)H * NU, 0.f), unew((size_t)H * NU),
        ubest((size_t)H * NU), terms(mppi::NTERMS), u1(NU);
    std::vector<double> tcomp;
    mppi_opts o = *opts;
    o.flags &= ~(unsigned)(MPPI_SYNC | MPPI_TIME_KERNELS | MPPI_GRAPH);
    double t = 0.0, goal_min = INFINITY;
    int n_steps = 0, n_div = 0, r = 0;
    for (;; ++r) {
        if (eo->max_replans > 0 && r >= eo->max_replans) break;
        o.seed = opts->seed + (uint64_t)r;
        const mppi_scene *sc = es.phase == mppi::EP_PICK ? pick : move;
        mppi_stats ps;
        const auto t0 = std::chrono::steady_clock::now();
        mppi_cov cv = {Sg.data(), Sg.data(), eo->cov_eps, nullptr};
        int rc = mppi_host::plan_with(ctx, sc, x.data(), nom.data(), K, H, lambda, sigma, &o, qp,
                                      eo->use_cov ? &cv : nullptr, unew.data(), ubest.data(), nullptr, &ps,
                                      stream);
        tcomp.push_back(std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count());
        if (rc == MPPI_E_DIVERGED)
            ++n_div;
        else if (rc)
            return rc;
        for (int d = 0; d < NU; ++d) {
            double s = 0.0;
            for (int k = 0; k < eo->n_avg; ++k) s += ubest[(size_t)k * NU + d];
            u1[d] = (float)(s / eo->n_avg);
        }
        if (u_exec) std::copy(u1.begin(), u1.end(), u_exec + (size_t)r * NU);
        for (int s = 0; s < eo->n_exec; ++s) {
            rc = mppi_simulate(ctx, move, x.data(), 1, u1.data(), 1, 1, 0, nullptr, terms.data(), xo.data(), 0,
                               stream);
            if (rc) return rc;
            t += dt;
            ++n_steps;
            const mppi::EpObs ob = {t, terms[0], terms[1], std::sqrt(std::max(terms[2], 0.f)), xo[mppi::XPB + 2],
                                    (int)std::lround(terms[6])};
            goal_min = std::min(goal_min, (double)terms[0]);
            x = xo;
            if (mppi::ep_step(es, rule, ob) != mppi::EP_RUNNING) break;
        }
        if (x_hist) std::copy(x.begin(), x.end(), x_hist + (size_t)r * NX);
        if (es.status != mppi::EP_RUNNING) {
            ++r;
            break;
        }
        // warm start: the mean shifted by the executed steps, the last row repeated
        for (int k = 0; k < H; ++k) {
            const int src = std::min(k + eo->n_exec, H - 1);
            std::copy(unew.begin() + (size_t)src * NU, unew.begin() + (size_t)(src + 1) * NU, nom.begin() + (size_t)k * NU);
        }
        // and the covariance shifted alike: entries whose two steps stay inside
        // the horizon move up; the freed tail is diag(sigma^2)
        if (eo->use_cov) {
            const int sh = eo->n_exec * NU;
            for (int i = 0; i < n; ++i)
                for (int l = 0; l < n; ++l)
                    Sn[(size_t)i * n + l] = (i + sh < n && l + sh < n) ? Sg[(size_t)(i + sh) * n + l + sh]
                                                                        : (i == l ? sig2(i) : 0.0);
            Sg.swap(Sn);
        }
    }
    double mean = 0.0, mx = 0.0;
    for (double v : tcomp) {
        mean += v;
        mx = std::max(mx, v);
    }
    mean /= std::max<size_t>(tcomp.size(), 1);
    double var = 0.0;
    for (double v : tcomp) var += (v - mean) * (v - mean);
    var /= std::max<size_t>(tcomp.size(), 1);
    *res = mppi_episode_result{};
    res->status = es.status;
    res->phase = es.phase;
    res->n_replans = r;
    res->n_steps = n_steps;
    res->t_end = es.t_end >= 0 ? es.t_end : t;
    res->t_switch = es.t_switch;
    res->t_comp_mean_ms = mean;
    res->t_comp_std_ms = std::sqrt(var);
    res->t_comp_max_ms = mx;
    res->goal_dist_min = goal_min;
    for (int i = 0; i < 3; ++i) res->ball_final[i] = x[mppi::XPB + i];
    res->n_diverged = n_div;
    if (x_final) std::copy(x.begin(), x.end(), x_final);
    return MPPI_OK;
}
