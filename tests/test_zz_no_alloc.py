"""The allocation-free plan (mppi_plan_noalloc) through the C ABI: its
results equal mppi_plan's bit for bit on two calls in a row (the second
smaller, so the static working array holds the first call's contents), free
device memory does not change across each of its calls, and calls beyond
the array's size are rejected."""
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


def _case(sc, K, H, M, seed, task=False):
    pp = W.plan_params(2, K=K, H=H, M=M, seed=seed)
    x0 = T(W.initial_state(sc) if task else W.random_states(sc, 1, seed=seed, spread=0.1)[0])
    nom = T(np.random.default_rng(seed).uniform(-0.3, 0.3, (H, 14)))
    return pp, x0, nom


@pytest.mark.parametrize("scene_kind,mapping", [("ball", None), ("ball", "lane"), ("tray", None)])
def test_noalloc_plan_equals_plan_twice(mp, scene_kind, mapping):
    """Ball scenes in the default and the one-lane mapping; the tray-moving
    phase (box object, further cost terms) in its default task form."""
    ctx = mp.Context(0)
    task = scene_kind == "tray"
    sc = W.task_scene("tray", "move") if task else W.make_scene(2)
    scene = mp.Scene(ctx, sc)
    cases = [(1024, 64, 3, 11), (300, 17, 2, 12)]   # the second call smaller than the first
    # warm-up: kernels loaded and the context's own buffers grown by mppi_plan
    outs = []
    for K, H, M, seed in cases:
        pp, x0, nom = _case(sc, K, H, M, seed, task)
        U = torch.zeros((H, 14), device=DEV)
        c = torch.zeros(K, device=DEV)
        st = mp.mppi_plan(ctx, scene, x0, nom, K, H, pp["lam"], T(pp["sigma"]), U, c, M=M, seed=pp["seed"],
                          mapping=mapping)
        torch.cuda.synchronize()
        outs.append((pp, x0, nom, U, c, st))
    got = []
    for (K, H, M, seed), (pp, x0, nom, U, c, st) in zip(cases, outs):
        U2 = torch.full((H, 14), 7.0, device=DEV)
        c2 = torch.full((K,), 7.0, device=DEV)
        sig = T(pp["sigma"])
        torch.cuda.synchronize()
        free_b = torch.cuda.mem_get_info()[0]
        st2 = mp.mppi_plan_noalloc(ctx, scene, x0, nom, K, H, pp["lam"], sig, U2, c2, M=M, seed=pp["seed"],
                                   mapping=mapping)
        torch.cuda.synchronize()
        assert torch.cuda.mem_get_info()[0] == free_b
        got.append((U2, c2, st2))
    for (U2, c2, st2), (pp, x0, nom, U, c, st) in zip(got, outs):
        assert st2["rc"] == 0 and st["rc"] == 0
        assert torch.equal(U2, U) and torch.equal(c2, c)
        for k in ("best", "ess", "c_min", "cmin_iter", "contacts", "np_tests", "overflow"):
            assert st2[k] == st[k], k
    # without a costs array (the costs go to the static array), asynchronous
    K, H, M, seed = cases[1]
    pp, x0, nom, U, c, st = outs[1]
    U3 = torch.zeros((H, 14), device=DEV)
    assert mp.mppi_plan_noalloc(ctx, scene, x0, nom, K, H, pp["lam"], T(pp["sigma"]), U3, None, M=M, seed=pp["seed"],
                                mapping=mapping, want_stats=False) is None
    torch.cuda.synchronize()
    assert torch.equal(U3, U)
    scene.close()
    ctx.close()


def test_noalloc_rejects_sizes_beyond_the_array(mp):
    ctx = mp.Context(0)
    sc = W.make_scene(2)
    scene = mp.Scene(ctx, sc)
    K, H = 40000, 64
    pp, x0, nom = _case(sc, 64, H, 1, 3)
    U = torch.zeros((H, 14), device=DEV)
    with pytest.raises(mp.MppiError) as e:
        mp.mppi_plan_noalloc(ctx, scene, x0, nom, K, H, pp["lam"], T(pp["sigma"]), U, torch.zeros(K, device=DEV))
    assert e.value.code == mp.E_INVAL and "MPPI_NOALLOC_SCRATCH_BYTES" in str(e.value)
    with pytest.raises(ValueError):
        mp.mppi_plan_noalloc(ctx, scene, x0.cpu().numpy(), nom.cpu().numpy(), 64, H, pp["lam"],
                             pp["sigma"].astype(np.float32), np.zeros((H, 14), np.float32))
    scene.close()
    ctx.close()
