"""Contexts on the GPU: calls on one context that name different streams run
in call order (they share the context's scratch buffers), and the cached
plan graphs follow the scene they were captured for, not the address its
model happened to occupy."""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


@pytest.fixture(scope="module")
def mp():
    import paper_2511_21264_amd as m
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    m.lib()
    return m


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


def _inputs(sc, H, seed):
    rng = np.random.default_rng(seed)
    x0 = W.random_states(sc, 1, seed=seed, spread=0.1)[0]
    nom = rng.uniform(-0.3, 0.3, (H, 14))
    return T(x0), T(nom)


def test_calls_on_two_streams_run_in_call_order(mp):
    """Plan A is enqueued on one stream and returns at once; plan B and the
    autotuner follow on other streams without any synchronisation.  They
    stage their inputs into the same scratch buffers A is still reading, so
    A's and B's results equal the same plans run one after the other only if
    each call waits for the context's previous one."""
    sc = W.make_scene(2)
    K, H, M = 4096, 32, 2
    pp = W.plan_params(2, K=K, H=H, M=M)
    sig = T(pp["sigma"])
    xa, na = _inputs(sc, H, 1)
    xb, nb = _inputs(sc, H, 2)
    ref = mp.Context(0)
    rscene = mp.Scene(ref, sc)
    want = []
    for x, n in ((xa, na), (xb, nb), (xa, nb)):
        U = torch.zeros((H, 14), device=DEV)
        c = torch.zeros(K, device=DEV)
        mp.mppi_plan(ref, rscene, x, n, K, H, pp["lam"], sig, U, c, M=M, seed=pp["seed"], mapping="split", sync=True)
        torch.cuda.synchronize()
        want.append((U, c))
    ctx = mp.Context(0)
    scene = mp.Scene(ctx, sc)
    s1, s2, s3 = torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()
    got = [(torch.zeros((H, 14), device=DEV), torch.zeros(K, device=DEV)) for _ in range(3)]
    torch.cuda.synchronize()
    for rep in range(3):
        for (x, n), (U, c), s in zip(((xa, na), (xb, nb), (xa, nb)), got, (s1, s2, s3)):
            mp.mppi_plan(ctx, scene, x, n, K, H, pp["lam"], sig, U, c, M=M, seed=pp["seed"], mapping="split",
                         want_stats=False, stream=s.cuda_stream)
        torch.cuda.synchronize()
        for (U, c), (Uw, cw) in zip(got, want):
            assert torch.equal(U, Uw) and torch.equal(c, cw), f"repeat {rep}"
    # the autotuner reuses the same scratch on a stream of its own
    U, c = got[0]
    U.zero_()
    torch.cuda.synchronize()
    mp.mppi_plan(ctx, scene, xa, na, K, H, pp["lam"], sig, U, c, M=M, seed=pp["seed"], mapping="split",
                 want_stats=False, stream=s1.cuda_stream)
    mp.mppi_autotune(ctx, scene, W.initial_state(sc), pp["sigma"], 2048, 8)
    torch.cuda.synchronize()
    assert torch.equal(U, want[0][0]) and torch.equal(c, want[0][1])
    scene.close()
    ctx.close()
    rscene.close()
    ref.close()


def test_graph_cache_follows_the_scene_not_its_address(mp):
    """A graph captured for one scene is not replayed for a scene created
    after it was destroyed, even at the same model address: the velocity
    bound baked into the update nodes is the new scene's."""
    ctx = mp.Context(0)
    K, H, M = 256, 8, 3
    pp = W.plan_params(2, K=K, H=H, M=M)
    sig = T(pp["sigma"])
    x0, nom = _inputs(W.make_scene(2), H, 5)
    U = torch.zeros((H, 14), device=DEV)
    c = torch.zeros(K, device=DEV)
    for u_max in (1.5, 0.4, 0.9):
        scene = mp.Scene(ctx, W.make_scene(2, u_max=u_max))
        mp.mppi_plan(ctx, scene, x0, nom, K, H, pp["lam"], sig, U, c, M=M, seed=pp["seed"], graph=True, sync=True)
        torch.cuda.synchronize()
        Ug = U.clone()
        Ue = torch.zeros_like(U)
        mp.mppi_plan(ctx, scene, x0, nom, K, H, pp["lam"], sig, Ue, torch.zeros_like(c), M=M, seed=pp["seed"],
                     sync=True)
        torch.cuda.synchronize()
        assert torch.equal(Ug, Ue), u_max
        assert float(Ug.abs().max()) <= u_max + 1e-6
        scene.close()
    ctx.close()
