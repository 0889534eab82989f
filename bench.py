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
    return dict(value=n * M * K * H / dt, unit="env-steps/s", cores=threads, kind="oracle",
                sample=f"{n} full oracle plan(s) of the same workload (K={K}, H={H}, M={M}), FP64, "
                       f"{dt:.1f} s on {threads} threads", plan_ms=dt / n * 1e3)


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
    for it in items:
        it["scene"].close()
    return out


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
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calib-copy-mb", type=int, default=0)
    ap.add_argument("--mapping", default="auto", choices=["auto", "lane", "team"])
    ap.add_argument("--packed-steps", type=int, default=2, help="steps of the packed-batch leg (0: skip)")
    args = ap.parse_args()
    if args.calib_copy_mb:
        calib_copy(args.calib_copy_mb)
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

    def plan():
        return mp.mppi_plan(ctx, scene, x0, nom, K, H, pp["lam"], sig, Unew, costs, M=M, seed=pp["seed"],
                            time_kernels=True, mapping=args.mapping)

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
            "kernel": "rollout_kernel",
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP32 / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32,
            "traffic": None,
            "peak_nonpacked": PEAK_FP32_NONPACKED / 1e12,
            "avg_launch_ms": avg_launch_s * 1e3,
            "flop_per_launch": float(np.mean(flops)),
        },
        "stats": {"ess": st["ess"], "c_min": st["c_min"], "contacts_per_substep":
                  st["contacts"] / (M * K * H * int(sc["n_sub"]))},
    }
    if args.packed_steps > 0:
        out["packed"] = bench_packed(mp, ctx, args.packed_steps, 1, args.mapping)
    if not args.no_cpu_baseline:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        out["cpu_baseline"] = cpu_baseline(sc, pp, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
