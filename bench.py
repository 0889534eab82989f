"""Benchmark of the MPPI rollout hot path on one MI355X.

One step = one full MPPI plan (M iterations of sample -> rollout -> cost ->
weights -> update) of the ball-lift-past-obstacle workload: two 7-joint
arms, free ball, 3 static boxes, K=1024 samples, H=64 control steps of
5 x 0.002 s substeps, 10 iterations, synthetic seeded scene.  Inputs are
resident in HBM before timing; every plan is synchronous (its latency is
call -> U_new ready).

Prints one JSON line: env-steps/s (K*H per iteration), p50/p99 plan
latency, the roofline of the dominant kernel (rollout, FP32 VALU) and the
FP64 CPU oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rollout env-steps/s (K*H) + p50/p99 MPPI replan latency, batched vs plain"
PEAK_FP32 = 157.3e12          # MI355X FP32 vector peak (packed), FLOP/s
PEAK_FP32_NONPACKED = 78.6e12  # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
PEAK_FP64 = 78.6e12           # MI355X FP64 (vector and MFMA), FLOP/s
# vector instruction issue: one wave64 VALU instruction per SIMD every 4 cycles
# (16 lanes a cycle), 256 CU x 4 SIMD x 2.4 GHz / 4
PEAK_VALU_ISSUE = 256 * 4 * 2.4e9 / 4


def cpu_baseline(sc, pp, threads, min_s=10.0, max_plans=5):
    """The FP64 oracle's full plan of the same workload, repeated until at
    least min_s seconds of host work (bounded by max_plans)."""
    import numpy as np
    import oracle
    import workloads as W
    o = oracle.Oracle(sc)
    x0 = W.initial_state(sc)
    K, H, M = pp["K"], pp["H"], pp["M"]
    n, t0 = 0, time.perf_counter()
    while True:
        o.plan(x0, np.zeros((H, 14)), K, H, pp["lam"], pp["sigma"], M, pp["seed"], nthreads=threads)
        n += 1
        dt = time.perf_counter() - t0
        if dt >= min_s or n >= max_plans:
            break
    # one thread, on a bounded sample: the first 64 samples of the same plan
    K1, t1 = 64, time.perf_counter()
    o.plan(x0, np.zeros((H, 14)), K1, H, pp["lam"], pp["sigma"], M, pp["seed"], nthreads=1)
    dt1 = time.perf_counter() - t1
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return dict(value=n * M * K * H / dt, unit="env-steps/s", cores=threads, kind="oracle",
                sample=f"{n} full oracle plan(s) of the same workload (K={K}, H={H}, M={M}), FP64, "
                       f"{dt:.1f} s on {threads} threads", plan_ms=dt / n * 1e3, cpu_model=cpu,
                single_thread={"value": M * K1 * H / dt1, "unit": "env-steps/s",
                               "sample": f"one oracle plan with K={K1}, H={H}, M={M} on 1 thread, {dt1:.1f} s"})


def bench_packed(mp, ctx, steps, warmup, mapping, n_scenes=32):
    """Uneven batch of independently seeded scenes (K 256..4096, H 32..128,
    0..12 boxes, M=10): one mppi_plan_batch call per step against the plain
    form, the same requests planned one after another with mppi_plan."""
    import numpy as np
    import torch
    import workloads as W
    dev = torch.device("cuda:0")
    items = []
    for sc, pp in W.packed_scenes(n_scenes, 4):
        H, K = pp["H"], pp["K"]
        items.append(dict(scene=mp.Scene(ctx, sc), K=K, H=H, lam=pp["lam"], M=pp["M"], seed=pp["seed"],
                          x0=torch.tensor(W.initial_state(sc), dtype=torch.float32, device=dev),
                          nominal_U=torch.zeros((H, 14), dtype=torch.float32, device=dev),
                          sigma=torch.tensor(pp["sigma"], dtype=torch.float32, device=dev),
                          U_new=torch.zeros((H, 14), dtype=torch.float32, device=dev),
                          costs=torch.zeros(K, dtype=torch.float32, device=dev)))
    env = sum(it["M"] * it["K"] * it["H"] for it in items)

    def batched():
        mp.mppi_plan_batch(ctx, items, mapping=mapping)

    def plain():
        for it in items:
            mp.mppi_plan(ctx, it["scene"], it["x0"], it["nominal_U"], it["K"], it["H"], it["lam"], it["sigma"],
                         it["U_new"], it["costs"], M=it["M"], seed=it["seed"], mapping=mapping, want_stats=False,
                         sync=True)

    out = {"workload": f"{n_scenes} packed scenes: K 256..4096, H 32..128, 0..12 boxes, M=10, seeded",
           "env_steps_per_batch": env}
    for name, fn in (("batched", batched), ("plain", plain)):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        lat = []
        t0 = time.perf_counter()
        for _ in range(steps):
            a = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - a)
        el = time.perf_counter() - t0
        out[name] = {"env_steps_per_s": env * steps / el, "p50_ms": float(np.percentile(lat, 50) * 1e3),
                     "p99_ms": float(np.percentile(lat, 99) * 1e3), "steps": steps}
        print(json.dumps({"packed_leg": name, **out[name]}), file=sys.stderr, flush=True)
    out["speedup"] = out["batched"]["env_steps_per_s"] / out["plain"]["env_steps_per_s"]
    # roofline of the packed rollout launches: the work model over every
    # request's counters against the summed launch time (HIP events)
    from paper_2511_21264_amd.flops import rollout_flops
    sts = mp.mppi_plan_batch(ctx, items, mapping=mapping, time_kernels=True)
    flop = sum(rollout_flops(it["K"], it["H"], int(it["scene"].dict["n_sub"]), it["scene"].n_pairs,
                             it["scene"].n_cost_pairs, int(it["scene"].dict["n_pgs"]), st["contacts"] / it["M"],
                             st["np_tests"] / it["M"], st["box_tests"] / it["M"]) * it["M"]
               for it, st in zip(items, sts))
    t_roll = sts[0]["rollout_ms"] * 1e-3
    out["roofline"] = {"bound": "alu", "achieved": flop / t_roll / 1e12, "peak": PEAK_FP32 / 1e12,
                       "unit": "TFLOP/s", "frac": flop / t_roll / PEAK_FP32, "flop_per_batch": flop,
                       "rollout_ms_per_batch": t_roll * 1e3, "launches_per_batch": sts[0]["rollout_launches"]}
    # alone vs mix under the same flags: each request keeps its own mapping
    # family, so one packed call and the requests one by one agree bit for bit
    mp.mppi_plan_batch(ctx, items, mapping=mapping)
    torch.cuda.synchronize()
    mixed = [it["U_new"].clone() for it in items]
    for it in items:
        mp.mppi_plan(ctx, it["scene"], it["x0"], it["nominal_U"], it["K"], it["H"], it["lam"], it["sigma"],
                     it["U_new"], it["costs"], M=it["M"], seed=it["seed"], mapping=mapping, want_stats=False,
                     sync=True)
    torch.cuda.synchronize()
    diff = max(float((it["U_new"] - u).abs().max()) for it, u in zip(items, mixed))
    out["alone_equals_mix"] = {"mapping": mapping or "auto", "bit_identical": diff == 0.0, "max_abs_diff": diff}
    for it in items:
        it["scene"].close()
    return out


def bench_replan(mp, ctx, sc, pp, n=200, warmup=5, advance=2, mapping=None):
    """Receding-horizon latency on the main workload: each replan starts from
    the plant state the previous reply produced (its first `advance` controls
    executed in the GPU simulator) and from the previous plan shifted by
    `advance` steps; the latency is the plan call, U_new ready on return."""
    import numpy as np
    import torch
    import workloads as W
    dev = torch.device("cuda:0")
    scene = mp.Scene(ctx, sc)
    K, H, M = pp["K"], pp["H"], pp["M"]
    x = torch.tensor(W.initial_state(sc), dtype=torch.float32, device=dev)
    nom = torch.zeros((H, 14), dtype=torch.float32, device=dev)
    sig = torch.tensor(pp["sigma"], dtype=torch.float32, device=dev)
    Unew = torch.zeros((H, 14), dtype=torch.float32, device=dev)
    costs = torch.zeros(K, dtype=torch.float32, device=dev)
    xn = torch.zeros((1, x.numel()), dtype=torch.float32, device=dev)
    lat, over, cont = [], 0.0, 0.0
    cap = None
    for i in range(warmup + n):
        if i == warmup + n // 2:
            # contact-list truncation at a warm start (arms on the ball)
            cap = bench_contact_cap(mp, ctx, scene, sc, x, nom, sig, pp["seed"] + i)
        torch.cuda.synchronize()
        a = time.perf_counter()
        st = mp.mppi_plan(ctx, scene, x, nom, K, H, pp["lam"], sig, Unew, costs, M=M, seed=pp["seed"] + i,
                          mapping=mapping, sync=True)
        if i >= warmup:
            lat.append(time.perf_counter() - a)
            over += st["overflow"]
            cont += st["contacts"]
        # the executor: first `advance` controls in the simulator, plan shifted
        mp.mppi_simulate(ctx, scene, x.view(1, -1), Unew[:advance].reshape(1, advance, 14).contiguous(),
                         X_out=xn, mapping=mapping)
        x = xn.view(-1).clone()
        nom = torch.cat([Unew[advance:], Unew[-1:].expand(advance, 14)]).contiguous()
    scene.close()
    lat_ms = np.array(lat) * 1e3
    return {"workload": f"config 2, {n} warm-started replans (K={K}, H={H}, M={M}), plant advanced {advance} "
                        f"steps per reply in the GPU simulator, plan shifted by {advance}",
            "replans": n, "p50_ms": float(np.percentile(lat_ms, 50)), "p99_ms": float(np.percentile(lat_ms, 99)),
            "mean_ms": float(lat_ms.mean()), "env_steps_per_s": M * K * H / float(lat_ms.mean() * 1e-3),
            "full_contact_list_per_substep": over / (n * M * K * H * int(sc["n_sub"])),
            "contacts_per_substep": cont / (n * M * K * H * int(sc["n_sub"])), "contact_cap": cap}


def run_trace(mp, ctx, cells, scenes, trace, duration, max_active, mapping, deadline_ms=20.0, advance=2, model=None,
              M=None):
    """Replay an arrival trace against a server with a deadline: every arrival
    submits a warm-started cell request (state and nominal resident on the
    device, plant advanced by `advance` steps per reply, queued requests of
    the same cell superseded).  Misses: completed after the deadline, shed
    unrun (could not end in time), superseded, or unfinished at the end."""
    import numpy as np
    import torch
    import workloads as W
    dev = torch.device("cuda:0")
    base, slope = model if model else (0.0, 0.0)
    srv = mp.Server(ctx, mapping=mapping, max_active=max_active, max_pending=4096, mem_budget=8 << 30,
                    deadline_ms=deadline_ms, iter_base_ms=base, iter_ms_per_menv=slope)
    ids = [srv.cell(scenes[i], c["H"], W.initial_state(c["scene"]).astype(np.float32)) for i, c in enumerate(cells)]
    sig = [torch.full((14,), 0.3, dtype=torch.float32, device=dev) for _ in cells]
    torch.cuda.synchronize()
    out, n_sub = {}, [0] * len(cells)
    lat, status = [], {"ok": 0, "superseded": 0, "diverged": 0, "shed": 0, "late": 0}

    def account(r):
        if r["status"] == mp.E_CANCELLED:
            status["superseded"] += 1
        elif r["status"] == mp.E_LATE:
            status["shed"] += 1
        else:
            status["ok" if r["status"] == 0 else "diverged"] += 1
            lat.append(r["t_done_ms"] - r["t_submit_ms"])
            status["late"] += r["t_done_ms"] > r["t_deadline_ms"]

    last = [0.0]

    def collect():
        # every 2 ms at most: each poll takes the server's lock
        now = time.perf_counter()
        if now - last[0] < 0.002:
            return
        last[0] = now
        for t in list(out):
            r = srv.poll(t, 0)
            if r is not None:
                out.pop(t)
                account(r)

    t0 = time.perf_counter()
    for (ta, i) in trace:
        while time.perf_counter() - t0 < ta:
            collect()
            time.sleep(0.0005)
        c = cells[i]
        item = dict(K=c["K"], lam=0.1, sigma=sig[i], M=M or c["M"], seed=(i << 20) + n_sub[i])
        n_sub[i] += 1
        out[srv.submit(item, cell=ids[i], advance=advance, supersede=True, want_stats=False)] = i
    wall = time.perf_counter() - t0
    q = srv.query()
    # the trace is over: what is still queued or running ends on its own
    # (completed, late or shed against its deadline)
    unfinished = 0
    for t in list(out):
        account(srv.poll(t, -1))
        out.pop(t)
    srv.close()
    lat = np.array(lat) if lat else np.array([np.nan])
    n_req = len(trace)
    misses = status["late"] + status["shed"] + status["superseded"] + unfinished
    return {"requests": n_req, "completed": status["ok"] + status["diverged"], "late": status["late"],
            "shed": status["shed"], "superseded": status["superseded"], "unfinished_at_end": unfinished,
            "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "deadline_ms": deadline_ms, "miss_rate": misses / max(1, n_req),
            "env_steps_per_s": q["env_steps"] / wall, "wall_s": wall, "trace_s": duration,
            "packed_iterations": q["iterations"], "mean_active": q["request_iters"] / max(1, q["iterations"]),
            "max_active": max_active,
            "model": {"base_ms": q["model_base_ms"], "ms_per_million_env_steps": q["model_ms_per_menv"],
                      "floor_ms": q["model_floor_ms"], "margin_ms": q["model_margin_ms"]}}


def calibrate_server(mp, ctx, cells, scenes, M, mapping, loads=(1, 2, 4, 8, 16, 32)):
    """The packed-iteration model of a server (ms = base + slope * W / 1e6),
    fitted by the server itself to its own iterations while it serves
    bursts of 1..32 simultaneous requests of the cells' shape."""
    import numpy as np
    import torch
    import workloads as W
    dev = torch.device("cuda:0")
    srv = mp.Server(ctx, mapping=mapping, max_active=64, max_pending=4096, mem_budget=8 << 30)
    ids = [srv.cell(scenes[i], c["H"], W.initial_state(c["scene"]).astype(np.float32)) for i, c in enumerate(cells)]
    sig = torch.full((14,), 0.3, dtype=torch.float32, device=dev)
    models = []
    for n in loads:
        ts = [srv.submit(dict(K=cells[i]["K"], lam=0.1, sigma=sig, M=M, seed=7 + i), cell=ids[i], want_stats=False)
              for i in range(n)]
        for t in ts:
            srv.wait(t)
        q = srv.query()
        models.append((q["model_base_ms"], q["model_ms_per_menv"], q["model_floor_ms"]))
    srv.close()
    return models[-1]


def bench_serving(mp, ctx, duration, mapping, deadline_ms=20.0, search_s=10.0):
    """Serving workload: 64 cells (scene seeds 5000 + cell), Poisson arrivals
    at U[10, 50] Hz per cell, 20 ms deadline (the control period), served by
    the continuous-batching server with earliest-deadline-first admission
    against its iteration model (seeded by a calibration, then refitted to
    its own iterations).  Fixed cells (K=1024, H=64): the largest M whose
    plans meet the deadline at a light load (0.5 Hz per cell), then the
    highest arrival-rate scale that keeps the miss rate below 1 % (bisection
    on short traces, confirmed on a trace of `duration` seconds), with the
    utilization rho = offered env-steps/s over the packed capacity the
    model measures; the same trace through the plain form (one request at a
    time); and both shapes at the specified rates (rho > 1: misses are shed
    or late, and counted)."""
    import workloads as W
    res = {"deadline_ms": deadline_ms}
    fixed = W.serving_cells(64, "fixed")
    scenes = [mp.Scene(ctx, c["scene"]) for c in fixed]
    rates = [c["rate"] for c in fixed]
    mean_rate = sum(rates) / len(rates)

    def leg(name, scale, dur, M, max_active=64, seed=0, cells=fixed, scn=None):
        trace = W.poisson_trace([c["rate"] * scale for c in cells], dur, seed=seed)
        r = run_trace(mp, ctx, cells, scn or scenes, trace, dur, max_active, mapping, deadline_ms,
                      model=(model[2] or model[0], model[1]), M=M)
        off = sum(c["rate"] * scale * M * c["K"] * c["H"] for c in cells)
        r.update(rate_scale=scale, M=M, offered_env_steps_per_s=off, utilization=off / capacity,
                 mean_rate_per_cell_hz=sum(c["rate"] for c in cells) * scale / len(cells))
        print(json.dumps({"serving": name, **r}), file=sys.stderr, flush=True)
        return r

    model = calibrate_server(mp, ctx, fixed, scenes, 10, mapping)
    capacity = 1e9 / max(model[1], 1e-12)   # env-steps/s of large packed iterations
    res["iteration_model"] = {"base_ms": model[0], "ms_per_million_env_steps": model[1], "floor_ms": model[2],
                              "capacity_env_steps_per_s": capacity}
    light = 0.5 / mean_rate
    res["light_load"] = {}
    M_ok = None
    for M in (10, 8, 6, 5, 4, 3, 2):
        r = leg(f"light M={M}", light, search_s, M)
        res["light_load"][str(M)] = r
        if r["miss_rate"] < 0.01 and r["p99_ms"] < deadline_ms:
            M_ok = M
            break
    res["largest_M_meeting_deadline"] = M_ok
    if M_ok is not None:
        lo, hi = light, 1.0
        for _ in range(6):
            mid = (lo * hi) ** 0.5
            r = leg(f"search M={M_ok} scale={mid:.4f}", mid, search_s, M_ok, seed=11)
            if r["miss_rate"] < 0.01:
                lo = mid
            else:
                hi = mid
        # confirm on a long trace; a scale that fails there is halved (twice at most)
        for _ in range(3):
            r = leg(f"confirm M={M_ok} scale={lo:.4f}", lo, duration, M_ok, seed=12)
            if r["miss_rate"] < 0.01:
                break
            res.setdefault("confirm_failed", []).append(r)
            lo *= 0.5
        res["sustained"] = r
        res["sustained_plain"] = leg(f"plain M={M_ok}", lo, search_s, M_ok, max_active=1, seed=12)
    Ms = M_ok or 2
    res["spec_rates_fixed"] = leg(f"spec fixed M={Ms}", 1.0, search_s, Ms, seed=13)
    for s_ in scenes:
        s_.close()
    mixed = W.serving_cells(64, "mixed")
    mscenes = [mp.Scene(ctx, c["scene"]) for c in mixed]
    res["spec_rates_mixed"] = leg(f"spec mixed M={Ms}", 1.0, search_s, Ms, seed=14, cells=mixed, scn=mscenes)
    for s_ in mscenes:
        s_.close()
    res["workload"] = ("64 cells, scene seeds 5000+cell, Poisson arrivals U[10,50] Hz per cell (scaled by "
                       "rate_scale), warm start resident, plant advanced 2 steps per reply, stale queued requests "
                       "superseded; fixed: K=1024, H=64; mixed: K~U{256..4096}, H~U{32..128}")
    return res


def bench_qp(mp, ctx, sc, pp, config, plain_ms, n_launch=20, n_plan=5):
    """The QP smoothing of the samples (Alg. 1 projection step): the
    projection kernel alone on K sampled sequences of the main workload
    (one launch = K x 14 joint QPs, `iters` ADMM iterations each), and whole
    plans with the projection in every iteration against the plain plan."""
    import numpy as np
    import torch
    import workloads as W
    dev = torch.device("cuda:0")
    p = W.qp_params(config)
    K, H, M = pp["K"], pp["H"], pp["M"]
    scene = mp.Scene(ctx, sc)
    x0 = torch.tensor(W.initial_state(sc), dtype=torch.float32, device=dev)
    rng = np.random.default_rng(5)
    U = torch.tensor(rng.normal(0, float(pp["sigma"][0]), (K, H, 14)), dtype=torch.float32, device=dev)
    out = torch.empty_like(U)
    for _ in range(3):
        mp.mppi_project(ctx, scene, x0, U, out, p, x0_shared=True, sync=False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(n_launch):
        mp.mppi_project(ctx, scene, x0, U, out, p, x0_shared=True, sync=False)
    e1.record()
    torch.cuda.synchronize()
    launch_ms = e0.elapsed_time(e1) / n_launch
    # algorithmic flops: the product with (I + rho A^T A)^-1, 2 H^2 per joint
    # and iteration (the O(H) shuffles, scans and clips are not counted)
    flop = K * 14 * p["iters"] * 2.0 * H * H
    nom = torch.zeros((H, 14), dtype=torch.float32, device=dev)
    sig = torch.tensor(pp["sigma"], dtype=torch.float32, device=dev)
    Un = torch.zeros((H, 14), dtype=torch.float32, device=dev)
    costs = torch.zeros(K, dtype=torch.float32, device=dev)

    def plan():
        return mp.mppi_plan_qp(ctx, scene, x0, nom, K, H, pp["lam"], sig, p, Un, costs, M=M, seed=pp["seed"])

    for _ in range(2):
        plan()
    torch.cuda.synchronize()
    lat = []
    for _ in range(n_plan):
        a = time.perf_counter()
        st = plan()
        torch.cuda.synchronize()
        lat.append((time.perf_counter() - a) * 1e3)
    scene.close()
    return {
        "kernel": "project_kernel",
        "iters": p["iters"], "rho": p["rho"], "alpha": p["alpha"],
        "launch": f"K={K} samples x 14 joints, H={H}",
        "project_ms_per_launch": launch_ms,
        "project_flop_per_launch": flop,
        "project_tflops": flop / (launch_ms * 1e-3) / 1e12,
        "project_frac_fp32": flop / (launch_ms * 1e-3) / PEAK_FP32,
        "plan_qp_ms": float(np.median(lat)),
        "plan_ms": plain_ms,
        "plan_qp_env_steps_per_s": K * H * M / (float(np.median(lat)) * 1e-3),
        "ess": st["ess"], "c_min": st["c_min"],
    }


def bench_cov(mp, ctx, sc, pp, config, plain_ms, n_launch=20, n_plan=3):
    """Covariance adaptation and full-covariance sampling at the main
    workload's sizes (n = 14 H): each step of the path timed alone with
    algorithmic flops (the covariance update K n (n + 1) in FP64, the
    triangular sampling product K n (n + 1) in FP32, the Cholesky n^3 / 3
    in FP64), and whole plans with the full covariance against the plain
    plan (same K, H, M; eta and eps of the workload)."""
    import numpy as np
    import torch
    import workloads as W
    dev = torch.device("cuda:0")
    cp = W.cov_params(config)
    K, H, M = pp["K"], pp["H"], pp["M"]
    n = 14 * H
    rng = np.random.default_rng(9)
    U = torch.tensor(rng.normal(0, 0.3, (K, H, 14)), dtype=torch.float32, device=dev)
    w = torch.tensor(rng.exponential(1.0, K), dtype=torch.float64, device=dev)
    nu64 = torch.tensor(rng.normal(0, 0.1, n), dtype=torch.float64, device=dev)
    A = rng.normal(size=(n, n)) / np.sqrt(n)
    S = torch.tensor(0.09 * (A @ A.T + 0.1 * np.eye(n)), dtype=torch.float64, device=dev)
    S2 = torch.empty_like(S)
    L = torch.empty_like(S)
    nu = torch.zeros((H, 14), dtype=torch.float32, device=dev)
    Us = torch.empty_like(U)
    u_max = float(sc["u_max"])

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    upd_ms = timed(lambda: mp.mppi_cov_update(ctx, U, w, nu64, S, S2, cp["eta"], cp["eps"], sync=False), n_launch)
    chol_ms = timed(lambda: mp.mppi_cholesky(ctx, S, L), max(3, n_launch // 4))
    samp_ms = timed(lambda: mp.mppi_sample_full(ctx, nu, L, 1, 0, K, Us, u_max, sync=False), n_launch)
    f_upd = float(K) * n * (n + 1)
    f_samp = float(K) * n * (n + 1)
    f_chol = n ** 3 / 3.0
    scene = mp.Scene(ctx, sc)
    x0 = torch.tensor(W.initial_state(sc), dtype=torch.float32, device=dev)
    nom = torch.zeros((H, 14), dtype=torch.float32, device=dev)
    sig = torch.tensor(pp["sigma"], dtype=torch.float32, device=dev)
    Un = torch.zeros((H, 14), dtype=torch.float32, device=dev)
    costs = torch.zeros(K, dtype=torch.float32, device=dev)
    Sout = torch.zeros((n, n), dtype=torch.float64, device=dev)

    def plan():
        return mp.mppi_plan_cov(ctx, scene, x0, nom, K, H, pp["lam"], sig, Un, costs, eps=cp["eps"], Sigma_out=Sout,
                                M=M, seed=pp["seed"], eta=cp["eta"])

    plan()
    lat = []
    for _ in range(n_plan):
        a = time.perf_counter()
        st = plan()
        lat.append((time.perf_counter() - a) * 1e3)
    scene.close()
    return {
        "n": n, "eta": cp["eta"], "eps": cp["eps"],
        "cov_update_ms": upd_ms, "cov_update_flop": f_upd,
        "cov_update_frac_fp64": f_upd / (upd_ms * 1e-3) / PEAK_FP64,
        "cholesky_ms": chol_ms, "cholesky_flop": f_chol,
        "sample_full_ms": samp_ms, "sample_full_flop": f_samp,
        "sample_full_frac_fp32": f_samp / (samp_ms * 1e-3) / PEAK_FP32,
        "plan_cov_ms": float(np.median(lat)),
        "plan_ms": plain_ms,
        "plan_cov_env_steps_per_s": K * H * M / (float(np.median(lat)) * 1e-3),
        "ess": st["ess"], "c_min": st["c_min"],
        "note": "cholesky_ms is wall time of a call that synchronises (it reads back the pivot flag)",
    }


def bench_contact_cap(mp, ctx, scene, sc, x, nu, sig, seed, n=256):
    """How often the contact list is truncated: n sequences drawn around the
    plan's mean nu (as its last iteration draws them) are rolled out one
    substep per step from state x, and every substep's start state goes
    through the narrowphase of all candidate pairs; the active pairs per
    substep are counted without the cap."""
    import numpy as np
    import torch
    dev = torch.device("cuda:0")
    H, S = nu.shape[0], int(sc["n_sub"])
    U = torch.zeros((n, H, 14), device=dev)
    mp.mppi_sample(ctx, scene, nu.contiguous(), sig, seed, 0, n, U=U)
    Ur = U.repeat_interleave(S, dim=1).contiguous()
    traj = torch.zeros((n, H * S, 55), device=dev)
    mp.mppi_simulate(ctx, scene, x.view(1, -1), Ur, X_out=traj, x0_shared=True, n_sub=1, traj=True)
    starts = torch.cat([x.view(1, 1, -1).expand(n, 1, 55), traj[:, :-1]], dim=1).reshape(-1, 55).contiguous()
    counts = []
    for c0 in range(0, starts.shape[0], 32768):
        blk = starts[c0:c0 + 32768].contiguous()
        phi = torch.zeros((blk.shape[0], scene.n_pairs), device=dev)
        mp.mppi_narrowphase(ctx, scene, blk, phi)
        torch.cuda.synchronize()
        counts.append((phi < 0).sum(dim=1).cpu().numpy())
    cnt = np.concatenate(counts)
    cap = int(sc["n_cmax"])
    return {"substeps": int(cnt.size), "mean_active_pairs": float(cnt.mean()), "max_active_pairs": int(cnt.max()),
            "frac_over_cap": float((cnt > cap).mean()), "frac_over_8": float((cnt > 8).mean()),
            "frac_full_list": float((cnt >= cap).mean()), "n_cmax": cap,
            "sample": f"{n} sequences around the plan's mean, {H} steps x {S} substeps from the plan's start state"}


def bench_graph(mp, ctx, sc, pp, steps=20, warmup=3):
    """The plan's launch sequence captured as a HIP graph (MPPI_GRAPH) against
    eager launches, on the main workload and on the small one (K=64, H=20,
    M=5), where launch overhead is a larger share."""
    import numpy as np
    import torch
    import workloads as W
    dev = torch.device("cuda:0")
    out = {}
    for name, cfg in (("main", None), ("small", 1)):
        scx = sc if cfg is None else W.make_scene(cfg)
        ppx = pp if cfg is None else W.plan_params(cfg)
        K, H, M = ppx["K"], ppx["H"], ppx["M"]
        scene = mp.Scene(ctx, scx)
        x0 = torch.tensor(W.initial_state(scx), dtype=torch.float32, device=dev)
        nom = torch.zeros((H, 14), dtype=torch.float32, device=dev)
        sig = torch.tensor(ppx["sigma"], dtype=torch.float32, device=dev)
        U = torch.zeros((H, 14), dtype=torch.float32, device=dev)
        c = torch.zeros(K, dtype=torch.float32, device=dev)
        res = {"K": K, "H": H, "M": M}
        outs = {}
        for g in (False, True):
            lat = []
            for i in range(warmup + steps):
                torch.cuda.synchronize()
                a = time.perf_counter()
                mp.mppi_plan(ctx, scene, x0, nom, K, H, ppx["lam"], sig, U, c, M=M, seed=ppx["seed"], graph=g,
                             want_stats=False, sync=True)
                if i >= warmup:
                    lat.append(time.perf_counter() - a)
            outs[g] = U.clone()
            lat = np.array(lat) * 1e3
            res["graph" if g else "eager"] = {"p50_ms": float(np.percentile(lat, 50)),
                                              "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean())}
        res["speedup_p50"] = res["eager"]["p50_ms"] / res["graph"]["p50_ms"]
        res["bit_identical"] = bool(torch.equal(outs[False], outs[True]))
        out[name] = res
        scene.close()
    return out


def bench_plain(mp, ctx, sc, pp, batched_ms, steps=3):
    """The plain form of the survey's measurement: one launch per control step
    (state in device memory between launches, one sample per lane), no
    packing, no graph, one stream -- the same plan, bit-identical to the
    one-lane mapping -- against the batched form's plan time."""
    import numpy as np
    import torch
    import workloads as W
    dev = torch.device("cuda:0")
    K, H, M = pp["K"], pp["H"], pp["M"]
    scene = mp.Scene(ctx, sc)
    x0 = torch.tensor(W.initial_state(sc), dtype=torch.float32, device=dev)
    nom = torch.zeros((H, 14), dtype=torch.float32, device=dev)
    sig = torch.tensor(pp["sigma"], dtype=torch.float32, device=dev)
    U = torch.zeros((H, 14), dtype=torch.float32, device=dev)
    c = torch.zeros(K, dtype=torch.float32, device=dev)
    lat, roll = [], []
    for i in range(1 + steps):
        torch.cuda.synchronize()
        a = time.perf_counter()
        st = mp.mppi_plan(ctx, scene, x0, nom, K, H, pp["lam"], sig, U, c, M=M, seed=pp["seed"], per_step=True,
                          time_kernels=True)
        if i >= 1:
            lat.append(time.perf_counter() - a)
            roll.append(st["rollout_ms"])
    scene.close()
    lat = np.array(lat) * 1e3
    return {"form": "one rollout launch per control step (H x M launches per plan), one sample per lane, "
                    "state in HBM between launches, no graph",
            "launches_per_plan": H * M, "plans": steps, "p50_ms": float(np.percentile(lat, 50)),
            "mean_ms": float(lat.mean()), "env_steps_per_s": M * K * H / float(lat.mean() * 1e-3),
            "rollout_ms_per_plan": float(np.mean(roll)), "batched_over_plain": float(lat.mean() / batched_ms)}


def bench_occupancy(mp, ctx, Ks=(32768,), H=64, M=2):
    """Roofline at full occupancy: one plan of the main scene with K samples
    in the one-lane and the 16-lane team mappings, rollout time from HIP
    events, algorithmic flops from the work model and the launch's counters."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2511_21264_amd.flops import rollout_flops
    dev = torch.device("cuda:0")
    sc = W.make_scene(2)
    scene = mp.Scene(ctx, sc)
    out = {}
    for K in Ks:
        pp = W.plan_params(2, K=K, H=H, M=M)
        x0 = torch.tensor(W.initial_state(sc), dtype=torch.float32, device=dev)
        nom = torch.zeros((H, 14), dtype=torch.float32, device=dev)
        sig = torch.tensor(pp["sigma"], dtype=torch.float32, device=dev)
        U = torch.zeros((H, 14), dtype=torch.float32, device=dev)
        c = torch.zeros(K, dtype=torch.float32, device=dev)
        for mapping in ("lane", "team"):
            mp.mppi_plan(ctx, scene, x0, nom, K, H, pp["lam"], sig, U, c, M=M, seed=pp["seed"], mapping=mapping)
            st = mp.mppi_plan(ctx, scene, x0, nom, K, H, pp["lam"], sig, U, c, M=M, seed=pp["seed"],
                              mapping=mapping, time_kernels=True)
            f = rollout_flops(K, H, int(sc["n_sub"]), scene.n_pairs, scene.n_cost_pairs, int(sc["n_pgs"]),
                              st["contacts"] / M, st["np_tests"] / M, st["box_tests"] / M)
            t = st["rollout_ms"] / M * 1e-3
            out[f"K{K}_{mapping}"] = {"K": K, "H": H, "mapping": mapping, "avg_launch_ms": t * 1e3,
                                     "flop_per_launch": f, "achieved_tflops": f / t / 1e12,
                                     "frac": f / t / PEAK_FP32, "env_steps_per_s": K * H / t}
    scene.close()
    return out


def bench_tasks(mp, ctx, K=1024, H=64, M=10, plans=3, big_K=32768):
    """The tray-moving and hand-over phases (box-shaped object, the further
    task terms; one sample per lane): plan latency, rollout launch time,
    env-steps/s and the flop-model roofline fraction at the main workload's
    K, H and M, and at big_K samples (two iterations) for the fraction at
    full occupancy."""
    import numpy as np
    import torch
    import workloads as W
    from paper_2511_21264_amd.flops import rollout_flops
    dev = torch.device("cuda:0")
    out = {}
    for task, phase in (("tray", "pick"), ("tray", "move"), ("handover", "pick"), ("handover", "pass"),
                        ("handover", "place")):
        sc = W.task_scene(task, phase)
        scene = mp.Scene(ctx, sc)
        x0 = torch.tensor(W.initial_state(sc), dtype=torch.float32, device=dev)
        for k, m, n in ((K, M, plans), (big_K, 2, 1)):
            if k == big_K and (task, phase) != ("tray", "move"):
                continue
            pp = W.plan_params(2, K=k, H=H, M=m)
            nom = torch.zeros((H, 14), dtype=torch.float32, device=dev)
            sig = torch.tensor(pp["sigma"], dtype=torch.float32, device=dev)
            U = torch.zeros((H, 14), dtype=torch.float32, device=dev)
            c = torch.zeros(k, dtype=torch.float32, device=dev)
            mp.mppi_plan(ctx, scene, x0, nom, k, H, pp["lam"], sig, U, c, M=m, seed=pp["seed"])
            torch.cuda.synchronize()
            lat, roll, fl = [], [], []
            for _ in range(n):
                a = time.perf_counter()
                st = mp.mppi_plan(ctx, scene, x0, nom, k, H, pp["lam"], sig, U, c, M=m, seed=pp["seed"],
                                  time_kernels=True)
                lat.append(time.perf_counter() - a)
                roll.append(st["rollout_ms"] / m)
                fl.append(rollout_flops(k, H, int(sc["n_sub"]), scene.n_pairs, scene.n_cost_pairs, int(sc["n_pgs"]),
                                        st["contacts"] / m, st["np_tests"] / m, st["box_tests"] / m, obj_box=True,
                                        ext=True))
            t = float(np.mean(roll)) * 1e-3
            out[f"{task}_{phase}_K{k}"] = {
                "K": k, "H": H, "M": m, "plan_ms": float(np.median(lat)) * 1e3, "rollout_launch_ms": t * 1e3,
                "env_steps_per_s": m * k * H / float(np.median(lat)), "flop_per_launch": float(np.mean(fl)),
                "frac": float(np.mean(fl)) / t / PEAK_FP32,
                "contacts_per_substep": st["contacts"] / (m * k * H * int(sc["n_sub"])),
                "full_contact_list_per_substep": st["overflow"] / (m * k * H * int(sc["n_sub"])), "ess": st["ess"]}
        scene.close()
    return out


def bench_episode(mp, ctx, runs=((2, 8, "diag"), (2, 8, "qp"), (2, 8, "cov"), (3, 4, "diag"), (2, 8, "qp", 256),
                                 (2, 8, "qp", 512), (2, 8, "qp", 2048)), t_max=10.0):
    """Closed-loop ball transport (receding-horizon execution; pick and move
    phases; the experiments' success metric: collision, timeout or a fallen
    ball fail a run): for each (config, n, variant) the first n seeded scenes
    of the workload at its K and H, M warm-started iterations per replan with
    the elite set and learning rate of the executor settings; variant "diag"
    samples with the diagonal sigma, "qp" also smooths every sample by the
    QP of the workload, "cov" carries the full covariance (Sigma_M
    warm-started, the settings' variance floor); a fourth entry overrides
    K (the batch-size sweep of the closed loop).  Success rate, task time (simulated
    seconds to the goal) over the successes, and the compute time per replan
    pooled over every replan (mean, std)."""
    import numpy as np
    import workloads as W
    out = {}
    for run in runs:
        cfg, n, variant = run[:3]
        pp = W.plan_params(cfg)
        if len(run) > 3:
            pp["K"] = run[3]
        use_cov = variant == "cov"
        ep = W.episode_params(cfg, t_max=t_max, use_cov=int(use_cov))
        qp = W.qp_params(cfg) if variant == "qp" else None
        eta = ep["eta"]
        res = []
        for i in range(n):
            pk, mv = W.episode_scenes(cfg, i)
            spk, smv = mp.Scene(ctx, pk), mp.Scene(ctx, mv)
            r = mp.mppi_episode(ctx, spk, smv, W.initial_state(mv), pp["K"], pp["H"], pp["lam"], pp["sigma"], ep,
                                qp=qp, M=ep["M"], seed=1000 * cfg + i, eta=eta, n_elite=ep["n_elite"])
            spk.close()
            smv.close()
            res.append(r)
            print(json.dumps({"episode": cfg, "variant": variant, "scene": i, "outcome": r["outcome"], "t_end": r["t_end"],
                              "replans": r["n_replans"], "t_comp_mean_ms": r["t_comp_mean_ms"]}),
                  file=sys.stderr, flush=True)
        ok = [r for r in res if r["status"] == 1]
        nrep = np.array([r["n_replans"] for r in res], dtype=float)
        mu = np.array([r["t_comp_mean_ms"] for r in res])
        sd = np.array([r["t_comp_std_ms"] for r in res])
        m_all = float((nrep * mu).sum() / nrep.sum())
        v_all = float((nrep * (sd ** 2 + mu ** 2)).sum() / nrep.sum() - m_all ** 2)
        tt = np.array([r["t_end"] for r in ok])
        out[f"config{cfg}" + ("" if variant == "diag" else "_" + variant) + (f"_K{run[3]}" if len(run) > 3 else "")] = {
            "runs": n, "K": pp["K"], "H": pp["H"], "M_per_replan": ep["M"], "n_avg": ep["n_avg"],
            "n_elite": ep["n_elite"], "eta": eta, "covariance": {"eps": ep["cov_eps"]} if use_cov else None,
            "qp_smoothing": variant == "qp",
            "n_exec": ep["n_exec"], "t_max_s": t_max,
            "success_rate": len(ok) / n,
            "outcomes": {o: sum(r["outcome"] == o for r in res) for o in sorted({r["outcome"] for r in res})},
            "task_time_mean_s": float(tt.mean()) if len(tt) else None,
            "task_time_std_s": float(tt.std()) if len(tt) else None,
            "t_comp_mean_ms": m_all, "t_comp_std_ms": float(np.sqrt(max(v_all, 0.0))),
            "t_comp_max_ms": float(max(r["t_comp_max_ms"] for r in res)),
            "replans_total": int(nrep.sum()),
        }
    return out


def bench_precision(mp, ctx, n_check=16):
    """Precision study on the 8-box obstacle course (K=4096, H=100): FP32
    rollouts; weights, normaliser and weighted mean in FP64 (default) and in
    FP32, each against the FP64 oracle's update from the same GPU costs; and
    the GPU's FP32 rollout costs against the oracle's FP64 rollouts on the
    first n_check samples.  Rollouts are chaotic under contact, so the cost
    error is a statement about the world model's FP32 sensitivity."""
    import numpy as np
    import torch
    import oracle
    import workloads as W
    dev = torch.device("cuda:0")
    sc = W.make_scene(3)
    pp = W.plan_params(3)
    K, H = pp["K"], pp["H"]
    scene = mp.Scene(ctx, sc)
    o = oracle.Oracle(sc)
    x0 = W.initial_state(sc).astype(np.float32)
    sig = pp["sigma"].astype(np.float32)
    nom = np.zeros((H, 14), np.float32)
    U = torch.zeros((H, 14), device=dev)
    c = torch.zeros(K, device=dev)
    mp.mppi_plan(ctx, scene, torch.tensor(x0, device=dev), torch.tensor(nom, device=dev), K, H, pp["lam"],
                 torch.tensor(sig, device=dev), U, c, M=1, seed=pp["seed"])
    torch.cuda.synchronize()
    costs = c.cpu().numpy()
    Uo = o.sample(nom.astype(np.float64), sig.astype(np.float64), pp["seed"], K, 0)
    ref, _, ess = o.update(Uo, costs.astype(np.float64), pp["lam"], nom.astype(np.float64))
    res = {"workload": f"8-box obstacle course, K={K}, H={H}, first iteration from a zero nominal", "ess": ess}
    for fp32 in (False, True):
        out = torch.zeros((H, 14), device=dev)
        out64 = torch.zeros((H, 14), dtype=torch.float64, device=dev)
        mp.mppi_update(ctx, scene, c, torch.tensor(nom, device=dev), torch.tensor(sig, device=dev), pp["seed"], 0,
                       pp["lam"], out, out64, fp32_weights=fp32)
        torch.cuda.synchronize()
        err = np.abs(out64.cpu().numpy() - ref)
        res["fp32_weights" if fp32 else "fp64_weights"] = {"max_abs_err_nu": float(err.max()),
                                                          "rel_err_nu": float(err.max() / np.abs(ref).max())}
    co = o.rollout_batch(x0.astype(np.float64), Uo[:n_check])
    co = np.asarray(co[0] if isinstance(co, tuple) else co, dtype=np.float64)
    rel = np.abs(costs[:n_check] - co) / np.abs(co)
    res["rollout_cost_rel_err"] = {"samples": n_check, "median": float(np.median(rel)), "max": float(rel.max())}
    scene.close()
    return res


def traffic_per_launch(mapping, K, H, M):
    """HBM bytes per rollout launch from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, scaled by the copy calibration), or
    None when the kernel sources changed since the counters were taken or
    the summary is for another mapping or shape."""
    path = os.path.join(ROOT, "profiles", "rollout_traffic_c2.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("sources_sha256") != sources_hash() or rec.get("mapping") != mapping or \
            rec.get("K") != K or rec.get("H") != H:
        return None
    return rec["hbm_bytes_per_launch"]


def counter_flops_per_launch(mapping, K, H):
    """FP32 operations per rollout launch as the hardware counted them
    (SQ_INSTS_VALU_FLOPS_FP32 in the committed summary), under the same
    conditions as traffic_per_launch."""
    path = os.path.join(ROOT, "profiles", "rollout_traffic_c2.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("sources_sha256") != sources_hash() or rec.get("mapping") != mapping or \
            rec.get("K") != K or rec.get("H") != H:
        return None
    v = rec.get("valu_flops_fp32_per_dispatch")
    # the counter adds each issued wave instruction's FP32 operations once;
    # a wave instruction runs on 64 lanes
    return None if v is None else 64.0 * v


def counter_valu_insts_per_launch(mapping, K, H):
    """Wave-level VALU instructions per rollout launch (SQ_INSTS_VALU in the
    committed summary), under the same conditions as traffic_per_launch."""
    path = os.path.join(ROOT, "profiles", "rollout_traffic_c2.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("sources_sha256") != sources_hash() or rec.get("mapping") != mapping or \
            rec.get("K") != K or rec.get("H") != H:
        return None
    return rec.get("valu_insts_per_dispatch")


def sources_hash():
    import hashlib
    d = os.path.join(ROOT, "paper_2511_21264_amd", "csrc")
    h = hashlib.sha256()
    for f in sorted(os.listdir(d)):
        h.update(f.encode())
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()


# bench.py arguments of the profiled runs: the main workload alone (the
# rollout kernel's time, traffic and issued operations), and the QP and
# covariance legs (their kernels' times)
PROFILE_ARGS_MAIN = ("--steps 3 --warmup 1 --no-cpu-baseline --packed-steps 0 --serve-seconds 0 --no-precision "
                     "--replans 0 --no-qp --no-cov --no-extra")
PROFILE_ARGS_NEXT = ("--steps 1 --warmup 0 --no-cpu-baseline --packed-steps 0 --serve-seconds 0 --no-precision "
                     "--replans 0 --no-extra")
# launches that fill the chip, one workload per profiled process: the main
# scene at 32768 samples one per lane and 16 lanes per sample, the 32 packed
# scenes of the uneven-batch workload in one batch, and the tray's move phase
# at 32768 samples (the task form)
OCC_RUNS = {
    "lane32k": ("%rollout_kernel<4, false>%", "main scene, K=32768, H=64, one lane per sample"),
    "team32k": ("%rollout_team_kernel<4, 4, false>%", "main scene, K=32768, H=64, 16 lanes per sample"),
    "packed": ("%rollout_team_kernel<4, 4, false>%", "32 packed scenes (K 256..4096, H 32..128), one batch, team family"),
    "task32k": ("%rollout_kernel<8, true>%", "tray move phase, K=32768, H=64, task form"),
}


def occupancy_profile_run(which, meta_path):
    """One of OCC_RUNS for the profiler: a warm-up and a timed pass of the
    workload; writes the launch's algorithmic flops (work model over the
    library's counters) and launch time (HIP events) to meta_path."""
    import numpy as np
    import torch
    import paper_2511_21264_amd as mp
    import workloads as W
    from paper_2511_21264_amd.flops import rollout_flops
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = mp.Context(0)
    rec = {"run": which, "kernel_like": OCC_RUNS[which][0], "workload": OCC_RUNS[which][1]}
    if which == "packed":
        items = []
        for sc, pp in W.packed_scenes(32, 4):
            H, K = pp["H"], pp["K"]
            items.append(dict(scene=mp.Scene(ctx, sc), K=K, H=H, lam=pp["lam"], M=pp["M"], seed=pp["seed"],
                              x0=torch.tensor(W.initial_state(sc), dtype=torch.float32, device=dev),
                              nominal_U=torch.zeros((H, 14), dtype=torch.float32, device=dev),
                              sigma=torch.tensor(pp["sigma"], dtype=torch.float32, device=dev),
                              U_new=torch.zeros((H, 14), dtype=torch.float32, device=dev),
                              costs=torch.zeros(K, dtype=torch.float32, device=dev)))
        mp.mppi_plan_batch(ctx, items)
        sts = mp.mppi_plan_batch(ctx, items, time_kernels=True)
        torch.cuda.synchronize()
        flop = sum(rollout_flops(it["K"], it["H"], int(it["scene"].dict["n_sub"]), it["scene"].n_pairs,
                                 it["scene"].n_cost_pairs, int(it["scene"].dict["n_pgs"]), st["contacts"] / it["M"],
                                 st["np_tests"] / it["M"], st["box_tests"] / it["M"]) * it["M"]
                   for it, st in zip(items, sts))
        rec.update(launches=sts[0]["rollout_launches"], flop_per_launch=flop / sts[0]["rollout_launches"],
                   event_ms_per_launch=sts[0]["rollout_ms"] / sts[0]["rollout_launches"])
    else:
        K, H, M = 32768, 64, 2
        task = which == "task32k"
        sc = W.task_scene("tray", "move") if task else W.make_scene(2)
        scene = mp.Scene(ctx, sc)
        pp = W.plan_params(2, K=K, H=H, M=M)
        x0 = torch.tensor(W.initial_state(sc), dtype=torch.float32, device=dev)
        nom = torch.zeros((H, 14), dtype=torch.float32, device=dev)
        sig = torch.tensor(pp["sigma"], dtype=torch.float32, device=dev)
        U = torch.zeros((H, 14), dtype=torch.float32, device=dev)
        c = torch.zeros(K, dtype=torch.float32, device=dev)
        mapping = None if task else ("lane" if which == "lane32k" else "team")
        mp.mppi_plan(ctx, scene, x0, nom, K, H, pp["lam"], sig, U, c, M=M, seed=pp["seed"], mapping=mapping)
        st = mp.mppi_plan(ctx, scene, x0, nom, K, H, pp["lam"], sig, U, c, M=M, seed=pp["seed"], mapping=mapping,
                          time_kernels=True)
        torch.cuda.synchronize()
        rec.update(launches=M, flop_per_launch=rollout_flops(
            K, H, int(sc["n_sub"]), scene.n_pairs, scene.n_cost_pairs, int(sc["n_pgs"]), st["contacts"] / M,
            st["np_tests"] / M, st["box_tests"] / M, obj_box=task, ext=task), event_ms_per_launch=st["rollout_ms"] / M)
    os.makedirs(os.path.dirname(meta_path) or ".", exist_ok=True)
    json.dump(rec, open(meta_path, "w"), indent=1)
    print(json.dumps(rec), flush=True)


def occupancy_commands():
    out = []
    for w in OCC_RUNS:
        b = f"python3 bench.py --profile-run {w} --profile-meta gpurun_out/prof/occ_{w}.json"
        out += [f"rocprofv3 --kernel-trace --stats -d gpurun_out/prof/occ_{w}_trace -o run -- {b}",
                f"timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE SQ_INSTS_VALU SQ_INSTS_VALU_FLOPS_FP32 "
                f"-d gpurun_out/prof/occ_{w}_fetch -o run -- {b}",
                f"timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE -d gpurun_out/prof/occ_{w}_write -o run -- {b}"]
    return out + ["python3 bench.py --summarize-profiles gpurun_out/prof"]


def summarize_occupancy(base):
    """profiles/rollout_occupancy.md: the launches that fill the chip, each
    from its own profiled process (kernel time, HBM bytes, issued vector
    instructions) with the work model's flops from the same run."""
    import sqlite3
    import glob

    def db(sub):
        f = glob.glob(os.path.join(base, sub, "**", "*results.db"), recursive=True)
        return sqlite3.connect(f[0]) if f else None

    def cnt(sub, name, like):
        c = db(sub)
        if not c:
            return None
        return c.execute("select avg(value) from counters_collection where counter_name = ? and kernel_name like ?",
                         (name, like)).fetchone()[0]

    cf, cw = cnt("cfetch", "FETCH_SIZE", "%copyBuffer%"), cnt("cwrite", "WRITE_SIZE", "%copyBuffer%")
    if not cf or not cw:
        return
    copy_kib = (256 << 20) / 1024.0
    fs, ws = copy_kib / cf, copy_kib / cw
    rows = []
    for w, (like, desc) in OCC_RUNS.items():
        mf = os.path.join(base, f"occ_{w}.json")
        tr = db(f"occ_{w}_trace")
        if not tr or not os.path.exists(mf):
            continue
        meta = json.load(open(mf))
        r = tr.execute("select sum(total_calls), sum(total_duration) from top_kernels where name like ?",
                       (like,)).fetchone()
        if not r or not r[0]:
            continue
        avg_ms = r[1] / r[0] / 1e3
        fetch, write = cnt(f"occ_{w}_fetch", "FETCH_SIZE", like), cnt(f"occ_{w}_write", "WRITE_SIZE", like)
        vi, vf = cnt(f"occ_{w}_fetch", "SQ_INSTS_VALU", like), cnt(f"occ_{w}_fetch", "SQ_INSTS_VALU_FLOPS_FP32", like)
        fl = meta["flop_per_launch"]
        tf = fl / (avg_ms * 1e-3)
        hbm = (fetch * fs + write * ws) * 1024 if fetch is not None and write is not None else None
        rows.append(f"| {w} | {desc} | {like.strip('%')} | {r[0]} | {avg_ms:.3f} | {meta['event_ms_per_launch']:.3f} | "
                    f"{fl / 1e9:.1f} | {tf / 1e12:.2f} | {tf / PEAK_FP32:.4f} | "
                    f"{'' if hbm is None else f'{hbm / 1e6:.2f}'} | "
                    f"{'' if vi is None else f'{vi / 1e6:.0f}'} | "
                    f"{'' if vi is None else f'{vi / (avg_ms * 1e-3) / PEAK_VALU_ISSUE:.3f}'} | "
                    f"{'' if vf is None else f'{64 * vf / 1e9:.0f}'} |")
    md = ["# Rollout launches that fill the chip: kernel time, roofline fraction, HBM bytes, vector issue", "",
          "Commands (run from the repository root, TMPDIR=/tmp):", ""]
    md += [f"    {c}" for c in occupancy_commands()]
    md += ["", f"Kernel sources: sha256 {sources_hash()[:16]}.", "",
           "| run | workload | kernel | dispatches | avg ms (rocprofv3) | ms (HIP events, same run) | "
           "algorithmic GFLOP per launch | TFLOP/s | fraction of 157.3 TF | HBM MB per launch | "
           "wave64 VALU instructions per launch (M) | fraction of the issue peak | issued FP32 lane operations (G) |",
           "|---|---|---|---|---|---|---|---|---|---|---|---|---|"] + rows
    md += ["", "Flops from the work model (`paper_2511_21264_amd/flops.py`) over the library's contact and "
           "narrowphase counters of the same run; HBM bytes from FETCH_SIZE and WRITE_SIZE scaled by what the "
           "counters read for a 256 MiB device copy; the issue peak is one wave64 VALU instruction per SIMD every "
           "4 cycles at 2.4 GHz. The packed row averages the batch's team-family launches (one per iteration)."]
    open(os.path.join(ROOT, "profiles", "rollout_occupancy.md"), "w").write("\n".join(md) + "\n")
    print("\n".join(md))


# SQ counters of the rollout kernel, two passes of at most eight
STALL_PASS1 = ("SQ_WAVE_CYCLES SQ_BUSY_CYCLES SQ_WAIT_ANY SQ_WAIT_INST_ANY SQ_ACTIVE_INST_ANY SQ_ACTIVE_INST_VALU "
               "SQ_ACTIVE_INST_LDS SQ_ACTIVE_INST_SCA")
STALL_PASS2 = ("SQ_INSTS_VALU SQ_INSTS_SALU SQ_INSTS_LDS SQ_INSTS_SMEM SQ_WAIT_INST_LDS SQ_INSTS_BRANCH SQ_INSTS_VMEM "
               "SQ_WAVES")


def summarize_stalls(base, meta):
    """Where the rollout kernel's wave cycles go (SQ counters of the two
    stall passes) and its vector issue rate, against the launch time of the
    kernel trace taken with the same arguments."""
    import sqlite3
    import glob
    v = {}
    for sub in ("stall1", "stall2"):
        g = glob.glob(os.path.join(base, sub, "**", "*results.db"), recursive=True)
        if not g:
            return
        c = sqlite3.connect(g[0])
        for k, n, val, cnt in c.execute("select kernel_name, counter_name, avg(value), count(*) from counters_collection "
                                        "group by kernel_name, counter_name"):
            if "rollout_split" in k:
                v[n] = (val, cnt)
    g = glob.glob(os.path.join(base, "trace", "**", "*results.db"), recursive=True)
    if not g or "SQ_INSTS_VALU" not in v or "SQ_WAVE_CYCLES" not in v:
        return
    c = sqlite3.connect(g[0])
    avg_us = [a for n, a in c.execute("select name, average from top_kernels") if "rollout_split" in n][0]
    launch_s = avg_us * 1e-6
    waves = v["SQ_WAVES"][0]
    busy = v["SQ_BUSY_CYCLES"][0] / 32.0  # per shader engine: 8 XCDs x 4
    clk = busy / launch_s
    wc = v["SQ_WAVE_CYCLES"][0] * 4  # quad-cycles

    def share(n):
        return v[n][0] * 4 / wc
    valu = v["SQ_INSTS_VALU"][0]
    simd_cycles = valu * 4 / 1024
    md = ["# rollout_split_kernel<4, false>, K=1024, H=64 obstacle workload: where the wave cycles go (SQ counters)", "",
          "Commands (run from the repository root, TMPDIR=/tmp; two passes, at most eight SQ counters each):", ""]
    md += [f"    {c}" for c in meta["stall_commands"]]
    md += ["", f"Kernel sources: sha256 {sources_hash()[:16]} (the csrc tree as `bench.sources_hash` reads it). "
               f"Averages over {v['SQ_WAVES'][1]} dispatches;",
           f"launch time {avg_us / 1e3:.3f} ms from the kernel trace in `rollout_split_c2.md` (same sources, same "
           "arguments).", "",
           "| counter (per dispatch) | value | reading |", "|---|---|---|",
           f"| SQ_WAVES | {waves:.0f} | two waves per sample |",
           f"| SQ_BUSY_CYCLES | {v['SQ_BUSY_CYCLES'][0]:.4g} | summed over 32 shader engines: {busy / 1e6:.2f} M cycles "
           f"each, so the clock ran at {clk / 1e9:.2f} GHz over the {avg_us / 1e3:.3f} ms launch |",
           f"| SQ_WAVE_CYCLES | {v['SQ_WAVE_CYCLES'][0]:.4g} quad-cycles | {wc / waves / 1e6:.2f} M cycles per wave, "
           f"{wc / waves / busy:.0%} of the launch |",
           f"| SQ_ACTIVE_INST_ANY | {v['SQ_ACTIVE_INST_ANY'][0]:.4g} | {share('SQ_ACTIVE_INST_ANY'):.1%} of wave cycles "
           "working on an instruction |",
           f"| SQ_ACTIVE_INST_VALU | {v['SQ_ACTIVE_INST_VALU'][0]:.4g} | {share('SQ_ACTIVE_INST_VALU'):.1%} (one "
           "quad-cycle per VALU instruction) |",
           f"| SQ_ACTIVE_INST_SCA | {v['SQ_ACTIVE_INST_SCA'][0]:.4g} | {share('SQ_ACTIVE_INST_SCA'):.1%} scalar ALU and "
           "scalar memory |",
           f"| SQ_ACTIVE_INST_LDS | {v['SQ_ACTIVE_INST_LDS'][0]:.4g} | {share('SQ_ACTIVE_INST_LDS'):.1%} |",
           f"| SQ_WAIT_ANY | {v['SQ_WAIT_ANY'][0]:.4g} | {share('SQ_WAIT_ANY'):.1%} of wave cycles waiting "
           "(dependencies, barriers, memory) |",
           f"| SQ_WAIT_INST_ANY | {v['SQ_WAIT_INST_ANY'][0]:.4g} | {share('SQ_WAIT_INST_ANY'):.1%} waiting for issue |",
           f"| SQ_INSTS_VALU | {valu / 1e6:.1f} M | wave64 vector instructions |",
           f"| SQ_INSTS_SALU | {v['SQ_INSTS_SALU'][0] / 1e6:.1f} M | |",
           f"| SQ_INSTS_BRANCH | {v['SQ_INSTS_BRANCH'][0] / 1e6:.1f} M | |",
           f"| SQ_INSTS_LDS | {v['SQ_INSTS_LDS'][0] / 1e6:.1f} M | |",
           f"| SQ_INSTS_SMEM | {v['SQ_INSTS_SMEM'][0] / 1e6:.2f} M | scalar loads of the scene model |",
           f"| SQ_INSTS_VMEM | {v['SQ_INSTS_VMEM'][0] / 1e6:.2f} M | |",
           f"| SQ_WAIT_INST_LDS | {v['SQ_WAIT_INST_LDS'][0]:.4g} | |", "",
           f"Vector issue bound: {valu / 1e6:.0f} M wave64 VALU instructions at one per SIMD every 4 cycles occupy "
           f"each of the 1024 SIMDs for {simd_cycles / 1e6:.2f} M cycles = {simd_cycles / clk * 1e3:.2f} ms at the "
           f"measured {clk / 1e9:.2f} GHz, {simd_cycles / clk / launch_s:.0%} of the launch; against the 2.4 GHz issue "
           f"peak ({PEAK_VALU_ISSUE / 1e9:.1f} G wave instructions/s) the launch reaches {valu / launch_s / 1e9:.0f} G/s "
           f"= {valu / launch_s / PEAK_VALU_ISSUE:.0%}. The vector units are mostly busy: the gap to the FP32 peak is in "
           "what the instructions do (moves, selects, DPP broadcasts, integer and compare work, lanes idle under a "
           "mask or repeating a team's value), not in idle issue slots."]
    open(os.path.join(ROOT, "profiles", "rollout_stalls_c2.md"), "w").write("\n".join(md) + "\n")
    print("\n".join(md))


def profile_meta():
    b = f"python3 bench.py {PROFILE_ARGS_MAIN}"
    bn = f"python3 bench.py {PROFILE_ARGS_NEXT}"
    return {
        "title": "rollout_split_kernel<4, false> (two waves per sample), K=1024, H=64 obstacle workload: kernel time and "
                 "HBM traffic",
        "file": "rollout_split_c2.md", "mapping": "split", "K": 1024, "H": 64,
        "kernel_like": "%rollout_split_kernel<4, false>%", "calib_copy_bytes": 256 << 20,
        "commands": [
            f"rocprofv3 --kernel-trace --stats -d gpurun_out/prof/trace -o run -- {b}",
            f"timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE -d gpurun_out/prof/fetch -o run -- {b}",
            f"timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE -d gpurun_out/prof/write -o run -- {b}",
            f"timeout -s KILL 120 rocprofv3 --pmc SQ_INSTS_VALU_FLOPS_FP32 SQ_INSTS_VALU -d gpurun_out/prof/valu "
            f"-o run -- {b}",
            "timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE -d gpurun_out/prof/cfetch -o run -- python3 bench.py "
            "--calib-copy-mb 256",
            "timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE -d gpurun_out/prof/cwrite -o run -- python3 bench.py "
            "--calib-copy-mb 256",
            "python3 bench.py --summarize-profiles gpurun_out/prof",
        ],
        "stall_commands": [
            f"timeout -s KILL 90 rocprofv3 --pmc {STALL_PASS1} -d gpurun_out/prof/stall1 -o run -- {b}",
            f"timeout -s KILL 90 rocprofv3 --pmc {STALL_PASS2} -d gpurun_out/prof/stall2 -o run -- {b}",
            "python3 bench.py --summarize-profiles gpurun_out/prof",
        ],
        "next_commands": [
            f"rocprofv3 --kernel-trace --stats -d gpurun_out/prof/trace_next -o run -- {bn}",
            f"timeout -s KILL 120 rocprofv3 --pmc FETCH_SIZE -d gpurun_out/prof/fetch_next -o run -- {bn}",
            f"timeout -s KILL 120 rocprofv3 --pmc WRITE_SIZE -d gpurun_out/prof/write_next -o run -- {bn}",
            "python3 bench.py --summarize-profiles gpurun_out/prof",
        ],
    }


def summarize_next(base, meta):
    """Kernel times of the QP and covariance legs (K=1024, H=64: n = 896)
    with each kernel's algorithmic flops against its peak."""
    import sqlite3
    import glob
    f = glob.glob(os.path.join(base, "trace_next", "**", "*results.db"), recursive=True)
    if not f:
        return
    con = sqlite3.connect(f[0])
    rows = con.execute("select name, total_calls, total_duration, average from top_kernels "
                       "order by total_duration desc").fetchall()
    K, H, n, iters = 1024, 64, 896, 60
    model = {  # kernel -> (flops per launch, peak, label)
        "project_kernel": (K * 14 * iters * 2.0 * H * H, PEAK_FP32, "FP32 (product with P only)"),
        "cov_syrk_kernel": (float(K) * n * (n + 1), PEAK_FP64, "FP64 MFMA"),
        "sample_full_kernel": (float(K) * n * (n + 1), PEAK_FP32, "FP32 MFMA"),
    }
    # algorithmic HBM bytes per launch: inputs read once, outputs written once
    alg_bytes = {
        "project_kernel": K * H * 14 * 4 * 2 + H * (H + 4) * 4,   # samples in and out, P
        "cov_syrk_kernel": K * n * 4 + K * 8 + n * 8 + 2 * n * n * 8,  # samples, weights, mean, Sigma in and out
        "sample_full_kernel": 2 * K * n * 4 + n * n * 4 // 2,    # normals in, samples out, lower factor
        "chol_step_kernel": None, "chol_diag_kernel": None,
    }

    def counter_avg(sub, name):
        g = glob.glob(os.path.join(base, sub, "**", "*results.db"), recursive=True)
        if not g:
            return {}
        c = sqlite3.connect(g[0])
        rows = c.execute("select kernel_name, avg(value) from counters_collection where counter_name = ? "
                         "group by kernel_name", (name,)).fetchall()
        return {k.split("(")[0].replace("mppi::", "").replace("void ", ""): v for k, v in rows}

    fetch, write = counter_avg("fetch_next", "FETCH_SIZE"), counter_avg("write_next", "WRITE_SIZE")
    cf, cw = counter_avg("cfetch", "FETCH_SIZE"), counter_avg("cwrite", "WRITE_SIZE")
    copy_kib = (256 << 20) / 1024.0
    f_scale = copy_kib / cf["__amd_rocclr_copyBuffer"] if cf.get("__amd_rocclr_copyBuffer") else None
    w_scale = copy_kib / cw["__amd_rocclr_copyBuffer"] if cw.get("__amd_rocclr_copyBuffer") else None
    md = ["# QP smoothing and covariance kernels, K=1024, H=64 (n = 896): kernel time", "",
          "Commands (run from the repository root, TMPDIR=/tmp):", ""]
    md += [f"    {c}" for c in meta["next_commands"]]
    md += ["", "| kernel | calls | avg us | algorithmic GFLOP per launch | TFLOP/s | fraction of peak | "
               "HBM MB per launch (counters) | algorithmic MB |",
           "|---|---|---|---|---|---|---|---|"]
    for name, calls, tot, avg in rows:
        short = name.split("(")[0].replace("mppi::", "").replace("void ", "")
        short = short.split("<")[0] if short.startswith("project_kernel") else short
        if short.startswith(("rollout", "stats", "update", "reset", "at::", "__amd")):
            continue
        key = next((k for k in fetch if k.split("<")[0] == short), None)
        traffic = ""
        if key and f_scale and w_scale and key in write:
            traffic = f"{(fetch[key] * f_scale + write[key] * w_scale) * 1024 / 1e6:.2f}"
        ab = alg_bytes.get(short)
        ab = f"{ab / 1e6:.2f}" if ab else ""
        fl = model.get(short)
        if fl:
            tf = fl[0] / (avg * 1e-6) / 1e12
            md.append(f"| {short} | {calls} | {avg:.1f} | {fl[0] / 1e9:.2f} | {tf:.1f} | {tf * 1e12 / fl[1]:.3f} "
                      f"({fl[2]}) | {traffic} | {ab} |")
        else:
            md.append(f"| {short} | {calls} | {avg:.1f} | | | | {traffic} | {ab} |")
    md += ["", "The Cholesky of n = 896 is one `chol_diag_kernel` and 27 `chol_step_kernel` launches in sequence "
           "(n^3/3 = 0.24 GFLOP in FP64); its time is the chain of 896 column steps, not arithmetic.",
           "", "HBM bytes from FETCH_SIZE and WRITE_SIZE per dispatch, scaled by what the counters read for a "
           "256 MiB device copy (the calibration of the rollout profile); the QP and covariance legs include "
           "whole plans, so the averages mix launches of the plan sizes with the legs' own."]
    open(os.path.join(ROOT, "profiles", "qp_cov_kernels_c2.md"), "w").write("\n".join(md) + "\n")
    print("\n".join(md))


def summarize_profiles(base):
    """Turn rocprofv3 result folders (trace/, fetch/, write/, cfetch/,
    cwrite/, valu/, trace_next/ under `base`) into the profiles/ summaries:
    kernel-time tables, the counter-based HBM traffic and issued FP32
    operations per rollout launch."""
    import sqlite3
    import glob

    def db(sub):
        f = glob.glob(os.path.join(base, sub, "**", "*results.db"), recursive=True)
        return sqlite3.connect(f[0]) if f else None

    meta = profile_meta()
    summarize_next(base, meta)
    summarize_stalls(base, meta)
    summarize_occupancy(base)
    lines = []
    tr = db("trace")
    if tr:
        rows = tr.execute("select name, total_calls, total_duration, average, percentage from top_kernels "
                          "order by total_duration desc limit 12").fetchall()
        # rocprofv3 stores these durations in microseconds
        lines += ["| kernel | calls | total ms | avg ms | % |", "|---|---|---|---|---|"]
        for n, calls, tot, avg, pct in rows:
            lines.append(f"| {n[:90]} | {calls} | {tot / 1e3:.3f} | {avg / 1e3:.3f} | {pct:.2f} |")

    def counter(sub, name, like):
        c = db(sub)
        if not c:
            return None
        r = c.execute("select avg(value), count(*) from counters_collection where counter_name = ? and "
                      "kernel_name like ?", (name, like)).fetchone()
        return r

    like = meta["kernel_like"]
    fetch = counter("fetch", "FETCH_SIZE", like)
    write = counter("write", "WRITE_SIZE", like)
    cf = counter("cfetch", "FETCH_SIZE", "%copyBuffer%")
    cw = counter("cwrite", "WRITE_SIZE", "%copyBuffer%")
    rec = None
    if fetch and write and cf and cw and fetch[0] is not None and cf[0]:
        copy_kib = meta["calib_copy_bytes"] / 1024.0
        f_scale = copy_kib / cf[0]  # bytes the copy reads, over what the counter says
        w_scale = copy_kib / cw[0]
        hbm = fetch[0] * f_scale * 1024 + write[0] * w_scale * 1024
        rec = {"mapping": meta["mapping"], "K": meta["K"], "H": meta["H"], "kernel_like": like,
               "fetch_kib_per_dispatch": fetch[0], "write_kib_per_dispatch": write[0],
               "fetch_scale": f_scale, "write_scale": w_scale, "hbm_bytes_per_launch": hbm,
               "sources_sha256": sources_hash(), "commands": meta["commands"]}
        # FP32 operations the hardware counted (issued wave instructions, all 64 lanes)
        vf = counter("valu", "SQ_INSTS_VALU_FLOPS_FP32", like)
        vi = counter("valu", "SQ_INSTS_VALU", like)
        if vf and vf[0] is not None:
            rec["valu_flops_fp32_per_dispatch"] = vf[0]
            rec["valu_insts_per_dispatch"] = vi[0] if vi else None
        json.dump(rec, open(os.path.join(ROOT, "profiles", "rollout_traffic_c2.json"), "w"), indent=1)
    md = [f"# {meta['title']}", ""]
    md += ["Commands (run from the repository root, TMPDIR=/tmp):", ""]
    md += [f"    {c}" for c in meta["commands"]]
    md += ["", "## Kernel time (rocprofv3 --kernel-trace --stats)", ""] + lines
    if rec:
        md += ["", "## HBM traffic of the rollout kernel (per dispatch)", "",
               f"FETCH_SIZE {rec['fetch_kib_per_dispatch']:.1f} KiB x {rec['fetch_scale']:.3f}, "
               f"WRITE_SIZE {rec['write_kib_per_dispatch']:.1f} KiB x {rec['write_scale']:.3f} "
               f"(scale = bytes a {meta['calib_copy_bytes'] >> 20} MiB device copy moves / what the counter "
               f"reports for it) = {rec['hbm_bytes_per_launch'] / 1e6:.2f} MB per launch."]
        if rec.get("valu_flops_fp32_per_dispatch") is not None:
            md += ["", "## FP32 operations the hardware counted (per dispatch)", "",
                   f"SQ_INSTS_VALU_FLOPS_FP32 {rec['valu_flops_fp32_per_dispatch'] / 1e9:.2f} G "
                   f"(SQ_INSTS_VALU {rec['valu_insts_per_dispatch'] / 1e6:.2f} M wave instructions). The counter "
                   f"adds each issued wave instruction's FP32 operations once, so x 64 lanes = "
                   f"{64 * rec['valu_flops_fp32_per_dispatch'] / 1e9:.1f} G lane operations issued per launch, "
                   f"against the work model's algorithmic count: lanes that repeat a team's work or sit "
                   f"idle under a mask are in the issued figure."]
    open(os.path.join(ROOT, "profiles", meta["file"]), "w").write("\n".join(md) + "\n")
    print("\n".join(md))


def calib_copy(mb):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = mb * (1 << 20) // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"calib_copy_bytes_each_way": n * 4, "copies": 3}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--replans", type=int, default=200,
                    help="warm-started replans of the main workload for the receding-horizon latency (0: skip)")
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0)
    ap.add_argument("--mapping", default="auto", choices=["auto", "lane", "team", "wave", "split"])
    ap.add_argument("--packed-steps", type=int, default=2, help="steps of the packed-batch leg (0: skip)")
    ap.add_argument("--serve-seconds", type=float, default=30.0,
                    help="trace length of the sustained serving leg (0: skip serving)")
    ap.add_argument("--no-precision", dest="precision", action="store_false",
                    help="skip the FP64-vs-FP32 weights study on the 8-box workload")
    ap.add_argument("--no-qp", dest="qp", action="store_false",
                    help="skip the QP-smoothing leg (projection kernel and plans with the projection)")
    ap.add_argument("--no-cov", dest="cov", action="store_false",
                    help="skip the covariance-adaptation leg (its kernels alone and plans with the full covariance)")
    ap.add_argument("--episodes", action="store_true",
                    help="also run the closed-loop ball-transport runs (success rate, task and compute time)")
    ap.add_argument("--no-extra", dest="extra", action="store_false",
                    help="skip the graph, plain-form, full-occupancy and contact-cap legs")
    ap.add_argument("--profile-run", default="", choices=[""] + list(OCC_RUNS),
                    help="run one chip-filling workload for the profiler (see OCC_RUNS)")
    ap.add_argument("--profile-meta", default="gpurun_out/prof/occ.json")
    ap.add_argument("--summarize-profiles", default="",
                    help="read rocprofv3 result folders under this path and write the profiles/ summaries")
    args = ap.parse_args()
    if args.calib_copy_mb:
        calib_copy(args.calib_copy_mb)
        return
    if args.summarize_profiles:
        summarize_profiles(args.summarize_profiles)
        return
    if args.profile_run:
        occupancy_profile_run(args.profile_run, args.profile_meta)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only (no multi-GPU path); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2511_21264_amd as mp
    from paper_2511_21264_amd.flops import rollout_flops
    import workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    sc = W.make_scene(args.config)
    pp = W.plan_params(args.config)
    K, H, M = pp["K"], pp["H"], pp["M"]
    ctx = mp.Context(0)
    scene = mp.Scene(ctx, sc)
    x0 = torch.tensor(W.initial_state(sc), dtype=torch.float32, device=dev)
    nom = torch.zeros((H, 14), dtype=torch.float32, device=dev)
    sig = torch.tensor(pp["sigma"], dtype=torch.float32, device=dev)
    Unew = torch.zeros((H, 14), dtype=torch.float32, device=dev)
    costs = torch.zeros(K, dtype=torch.float32, device=dev)

    tuned = None
    if args.mapping == "auto":
        # the measured mapping for this K (the context keeps it for later calls)
        name, ms = mp.mppi_autotune(ctx, scene, W.initial_state(sc), pp["sigma"], K, H)
        tuned = {"K": K, "chosen": name, "rollout_ms": ms}
    mapping = None if args.mapping == "auto" else args.mapping
    used = tuned["chosen"] if tuned else args.mapping
    nc = 4 if int(sc["n_cmax"]) <= 4 else 8
    kernel_name = {"lane": f"rollout_kernel<{nc}, false>", "team": f"rollout_team_kernel<{nc}, 4, false>",
                   "wave": f"rollout_team_kernel<{nc}, 1, false>", "split": f"rollout_split_kernel<{nc}, false>"}[used]

    def plan():
        return mp.mppi_plan(ctx, scene, x0, nom, K, H, pp["lam"], sig, Unew, costs, M=M, seed=pp["seed"],
                            time_kernels=True, mapping=mapping)

    for _ in range(args.warmup):
        plan()
    torch.cuda.synchronize()
    lat, roll_ms, flops = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        st = plan()
        lat.append(time.perf_counter() - a)
        roll_ms.append(st["rollout_ms"] / M)
        flops.append(rollout_flops(K, H, int(sc["n_sub"]), scene.n_pairs, scene.n_cost_pairs, int(sc["n_pgs"]),
                                   st["contacts"] / M, st["np_tests"] / M, st["box_tests"] / M))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    env_steps = args.steps * M * K * H
    lat_ms = np.array(lat) * 1e3
    avg_launch_s = float(np.mean(roll_ms)) * 1e-3
    achieved = float(np.mean(flops)) / avg_launch_s
    cf_launch = counter_flops_per_launch(used, K, H)
    vi_launch = counter_valu_insts_per_launch(used, K, H)
    out = {
        "metric": METRIC,
        "value": env_steps / elapsed,
        "unit": "env-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"config {args.config}: ball lift past {sc['n_box']} boxes, K={K}, H={H}, "
                        f"{sc['n_sub']} x {sc['h']} s substeps, M={M} iterations, one plan per step",
            "K": K, "H": H, "M": M, "n_sub": int(sc["n_sub"]), "n_box": int(sc["n_box"]),
            "path": "batched: one rollout launch per iteration over all K samples, horizon loop inside the kernel",
        },
        "p50_ms": float(np.percentile(lat_ms, 50)),
        "p99_ms": float(np.percentile(lat_ms, 99)),
        "physics_substeps_per_s": env_steps * int(sc["n_sub"]) / elapsed,
        "roofline": {
            "kernel": kernel_name,
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP32 / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32,
            "traffic": traffic_per_launch(used, K, H, M),
            "peak_nonpacked": PEAK_FP32_NONPACKED / 1e12,
            "counter_flop_per_launch": cf_launch,
            "counter_achieved": None if cf_launch is None else cf_launch / avg_launch_s / 1e12,
            "counter_frac": None if cf_launch is None else cf_launch / avg_launch_s / PEAK_FP32,
            "avg_launch_ms": avg_launch_s * 1e3,
            "flop_per_launch": float(np.mean(flops)),
            # vector instruction issue (SQ_INSTS_VALU): what bounds this kernel in practice
            "valu_insts_per_launch": vi_launch,
            "valu_issue_achieved": None if vi_launch is None else vi_launch / avg_launch_s / 1e9,
            "valu_issue_peak": PEAK_VALU_ISSUE / 1e9,
            "valu_issue_unit": "G wave64 VALU instructions/s",
            "valu_issue_frac": None if vi_launch is None else vi_launch / avg_launch_s / PEAK_VALU_ISSUE,
        },
        "stats": {"ess": st["ess"], "c_min": st["c_min"], "contacts_per_substep":
                  st["contacts"] / (M * K * H * int(sc["n_sub"])),
                  "full_contact_list_per_substep": st["overflow"] / (M * K * H * int(sc["n_sub"]))},
        "mapping": used,
        "autotune": tuned,
    }
    if args.mapping == "auto" and (args.packed_steps > 0 or args.serve_seconds > 0):
        # size classes of single requests (256..4096 samples) and of packed
        # launches (up to 2^17 samples), measured once on this context
        sc5 = W.make_scene(4, 0)
        s5 = mp.Scene(ctx, sc5)
        out["autotune_classes"] = {}
        for c in range(8, 18):
            name, ms = mp.mppi_autotune(ctx, s5, W.initial_state(sc5), pp["sigma"], 1 << c, 16)
            out["autotune_classes"][str(1 << c)] = name
        s5.close()
    if args.extra:
        out["contact_cap_cold"] = bench_contact_cap(mp, ctx, scene, sc, x0, Unew.clone(), sig, pp["seed"])
        out["graph"] = bench_graph(mp, ctx, sc, pp)
        print(json.dumps({"graph": out["graph"]}), file=sys.stderr, flush=True)
        out["plain"] = bench_plain(mp, ctx, sc, pp, out["ms_per_step"])
        print(json.dumps({"plain": out["plain"]}), file=sys.stderr, flush=True)
        out["occupancy"] = bench_occupancy(mp, ctx)
        print(json.dumps({"occupancy": out["occupancy"]}), file=sys.stderr, flush=True)
        out["tasks"] = bench_tasks(mp, ctx)
        print(json.dumps({"tasks": out["tasks"]}), file=sys.stderr, flush=True)
    if args.replans > 0:
        out["replan"] = bench_replan(mp, ctx, sc, pp, n=args.replans, mapping=mapping)
        print(json.dumps({"replan": out["replan"]}), file=sys.stderr, flush=True)
    if args.qp:
        out["qp"] = bench_qp(mp, ctx, sc, pp, args.config, out["ms_per_step"])
        print(json.dumps({"qp": out["qp"]}), file=sys.stderr, flush=True)
    if args.cov:
        out["cov"] = bench_cov(mp, ctx, sc, pp, args.config, out["ms_per_step"])
        print(json.dumps({"cov": out["cov"]}), file=sys.stderr, flush=True)
    if args.episodes:
        out["episode"] = bench_episode(mp, ctx)
        print(json.dumps({"episode": out["episode"]}), file=sys.stderr, flush=True)
    if args.packed_steps > 0:
        out["packed"] = bench_packed(mp, ctx, args.packed_steps, 1, mapping)
    if args.serve_seconds > 0:
        out["serving"] = bench_serving(mp, ctx, args.serve_seconds, mapping)
    if args.precision:
        out["precision"] = bench_precision(mp, ctx)
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        out["cpu_baseline"] = cpu_baseline(sc, pp, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
