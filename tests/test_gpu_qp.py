"""GPU parity of the QP smoothing (Alg. 1 sampling step, Eqs. proj_cost and
proj_bounds with r = 0..3) through the C ABI against the FP64 oracle's ADMM
on the same inputs and the same iteration count.

Tolerance: the projection is a fixed number of over-relaxed ADMM iterations,
each a contraction-like map.  The kernel evaluates the v-update as
v~ + rho P A^T (z - w - A v~), so FP32 rounding acts on the correction, not
on terms of the size of the prefix-sum rows; a float32 emulation of that
order stays within 2e-6 rad/s of the FP64 iteration at H = 64 over 60
iterations, and the tests allow 2e-5 (ten times that).
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
ATOL = 2e-5


@pytest.fixture(scope="module")
def mp():
    import paper_2511_21264_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


@pytest.fixture(scope="module")
def ctx(mp):
    c = mp.Context(0)
    yield c
    c.close()


@pytest.fixture(scope="module")
def qpo():
    from oracle import qp
    return qp


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


def _inputs(sc, K, H, seed, spread=0.3):
    rng = np.random.default_rng(seed)
    U = rng.normal(0, spread, (K, H, 14)) + 0.3 * np.sin(np.arange(H) * 0.2)[None, :, None]
    X0 = np.repeat(W.initial_state(sc)[None], K, axis=0)
    # commanded start positions near the position bounds, so r = 0 binds too
    X0[:, 28:42] += rng.uniform(-1.4, 1.4, (K, 14))
    return U.astype(np.float32), X0.astype(np.float32)


def _oracle(qpo, sc, U, X0, p):
    dt = sc["h"] * sc["n_sub"]
    return qpo.project_sequences(U.astype(np.float64), X0[:, 28:42].astype(np.float64), dt, float(sc["u_max"]),
                                 np.asarray(p["pos_lo"], dtype=np.float32).astype(np.float64),
                                 np.asarray(p["pos_hi"], dtype=np.float32).astype(np.float64),
                                 p["acc_max"], p["jerk_max"], p["rho"], p["iters"], p["alpha"])


@pytest.mark.parametrize("K,H", [(8, 64), (5, 17), (3, 3), (2, 2), (4, 1), (4, 65), (6, 100), (3, 128)])
def test_project_matches_oracle(mp, ctx, qpo, K, H):
    sc = W.make_scene(2)
    scene = mp.Scene(ctx, sc)
    p = W.qp_params(2)
    U, X0 = _inputs(sc, K, H, 100 + H)
    out = torch.zeros((K, H, 14), device=DEV)
    mp.mppi_project(ctx, scene, T(X0), T(U), out, p)
    torch.cuda.synchronize()
    ref = _oracle(qpo, sc, U, X0, p)
    got = out.cpu().numpy()
    err = np.abs(got - ref).max()
    print(f"project K={K} H={H}: max |gpu - oracle| {err:.2e}, max |u| {np.abs(got).max():.3f}")
    assert err < ATOL
    assert np.all(np.abs(got) <= float(sc["u_max"]) * (1 + 1e-6))
    scene.close()


def test_project_full_size_launch_on_sampled_sequences(mp, ctx, qpo):
    """The launch the bench times (K = 1024 samples, H = 64, the workload's
    settings): 24 sampled sequences (every joint) against the oracle, and
    the velocity box on every output."""
    sc = W.make_scene(2)
    scene = mp.Scene(ctx, sc)
    p = W.qp_params(2)
    K, H = 1024, 64
    U, X0 = _inputs(sc, K, H, 2024)
    out = torch.zeros((K, H, 14), device=DEV)
    mp.mppi_project(ctx, scene, T(X0), T(U), out, p)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    idx = np.random.default_rng(5).choice(K, 24, replace=False)
    ref = _oracle(qpo, sc, U[idx], X0[idx], p)
    err = np.abs(got[idx] - ref).max()
    print(f"project K={K} H={H} (24 sampled): max |gpu - oracle| {err:.2e}")
    assert err < ATOL
    assert np.all(np.abs(got) <= float(sc["u_max"]) * (1 + 1e-6))
    scene.close()


def test_project_two_steps_per_lane_full_size_sampled(mp, ctx, qpo):
    """The 8-box workload's sizes (K = 4096, H = 100: two horizon steps per
    lane): 12 sampled sequences against the oracle."""
    sc = W.make_scene(3)
    scene = mp.Scene(ctx, sc)
    p = W.qp_params(3)
    K, H = 4096, 100
    U, X0 = _inputs(sc, K, H, 3100)
    out = torch.zeros((K, H, 14), device=DEV)
    mp.mppi_project(ctx, scene, T(X0), T(U), out, p)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    idx = np.random.default_rng(6).choice(K, 12, replace=False)
    ref = _oracle(qpo, sc, U[idx], X0[idx], p)
    err = np.abs(got[idx] - ref).max()
    print(f"project K={K} H={H} (12 sampled): max |gpu - oracle| {err:.2e}")
    assert err < ATOL
    assert np.all(np.abs(got) <= float(sc["u_max"]) * (1 + 1e-6))
    scene.close()


def test_project_feasible_sequences_are_kept(mp, ctx):
    sc = W.make_scene(2)
    scene = mp.Scene(ctx, sc)
    p = W.qp_params(2)
    K, H = 4, 64
    U = np.repeat((0.2 * np.sin(np.arange(H) * 0.05))[None, :, None], K, axis=0).repeat(14, axis=2)
    X0 = np.repeat(W.initial_state(sc)[None], K, axis=0).astype(np.float32)
    out = torch.zeros((K, H, 14), device=DEV)
    mp.mppi_project(ctx, scene, T(X0), T(U), out, p)
    torch.cuda.synchronize()
    assert np.abs(out.cpu().numpy() - U).max() < ATOL
    scene.close()


def test_project_in_place_shared_state_and_host_arrays(mp, ctx, qpo):
    sc = W.make_scene(2)
    scene = mp.Scene(ctx, sc)
    p = W.qp_params(2)
    K, H = 6, 32
    U, X0 = _inputs(sc, K, H, 7)
    x0 = X0[0]
    ref = _oracle(qpo, sc, U, np.repeat(x0[None], K, axis=0), p)
    # device, in place, one shared start state
    Ud = T(U)
    mp.mppi_project(ctx, scene, T(x0), Ud, Ud, p, x0_shared=True)
    torch.cuda.synchronize()
    assert np.abs(Ud.cpu().numpy() - ref).max() < ATOL
    # host arrays
    out = np.zeros_like(U)
    mp.mppi_project(ctx, scene, x0, U, out, p, x0_shared=True)
    assert np.abs(out - ref).max() < ATOL
    scene.close()


def test_project_rejects_bad_arguments(mp, ctx):
    sc = W.make_scene(2)
    scene = mp.Scene(ctx, sc)
    p = W.qp_params(2)
    x0 = W.initial_state(sc).astype(np.float32)
    for bad in (dict(iters=0), dict(rho=0.0), dict(alpha=2.0), dict(acc_max=-1.0)):
        with pytest.raises(mp.MppiError):
            mp.mppi_project(ctx, scene, x0, np.zeros((2, 8, 14), np.float32), np.zeros((2, 8, 14), np.float32),
                            {**p, **bad}, x0_shared=True)
    with pytest.raises(mp.MppiError):  # longer than the kernel's two steps per lane
        mp.mppi_project(ctx, scene, x0, np.zeros((1, 129, 14), np.float32), np.zeros((1, 129, 14), np.float32), p,
                        x0_shared=True)
    lo = np.array(p["pos_lo"])
    with pytest.raises(mp.MppiError):
        mp.mppi_project(ctx, scene, x0, np.zeros((1, 8, 14), np.float32), np.zeros((1, 8, 14), np.float32),
                        {**p, "pos_hi": lo}, x0_shared=True)
    scene.close()


def test_plan_qp_against_oracle(mp, ctx, qpo):
    """Alg. 1 with the QP smoothing at the small workload (K=64, H=20, 5
    iterations): every iteration's samples nu + sigma z are projected, rolled
    out and averaged; the oracle composes its noise, ADMM, FP64 rollouts and
    update in the same order."""
    import oracle as oracle_mod
    sc = W.make_scene(1)
    scene = mp.Scene(ctx, sc)
    o = oracle_mod.Oracle(sc)
    pp = W.plan_params(1)
    p = W.qp_params(1)
    K, H, M = pp["K"], pp["H"], pp["M"]
    x0 = W.initial_state(sc).astype(np.float32)
    sig = pp["sigma"].astype(np.float32)
    Unew = torch.zeros((H, 14), device=DEV)
    costs = torch.zeros(K, device=DEV)
    st = mp.mppi_plan_qp(ctx, scene, T(x0), torch.zeros((H, 14), device=DEV), K, H, pp["lam"], T(sig), p, Unew,
                         costs, M=M, seed=pp["seed"])
    torch.cuda.synchronize()
    nu = np.zeros((H, 14))
    X0 = np.repeat(x0[None].astype(np.float64), K, axis=0)
    for m in range(M):
        z = o.noise(pp["seed"], K, H, m)
        Ut = nu.astype(np.float32).astype(np.float64)[None] + sig.astype(np.float64)[None, None] * z
        U = _oracle(qpo, sc, Ut, X0, p)
        c = o.rollout_batch(x0.astype(np.float64), U)
        c = c[0] if isinstance(c, tuple) else c
        nu, nf, ess = o.update(U, c, pp["lam"], nu)
    cg = costs.cpu().numpy()
    rel = np.abs(cg - c) / np.abs(c)
    dU = np.abs(Unew.cpu().numpy() - nu).max()
    print(f"c1 plan with QP: cost rel err median {np.median(rel):.2e} max {rel.max():.2e}; |dU_new|max {dU:.2e}; "
          f"ess {st['ess']:.2f} (oracle {ess:.2f})")
    assert st["rc"] == 0
    assert np.median(rel) < 1e-3
    assert dU < 0.05 * pp["sigma"][0]
    scene.close()
