"""Serving loop on the GPU: requests served by continuous batching equal the
same plans run alone (bit for bit, pinned mapping); cells keep the plant
state and the warm-start nominal on the device across requests; queue
limits, cancellation and supersession."""
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


@pytest.fixture(scope="module")
def ctx(mp):
    c = mp.Context(0)
    yield c
    c.close()


def T(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


def _plan_alone(mp, ctx, it, mapping):
    U = torch.zeros((it["H"], 14), device=DEV)
    c = torch.zeros(it["K"], device=DEV)
    st = mp.mppi_plan(ctx, it["scene"], it["x0"], it["nominal_U"], it["K"], it["H"], it["lam"], it["sigma"], U, c,
                      M=it["M"], seed=it["seed"], eta=it.get("eta", 1.0), n_elite=it.get("n_elite", 0),
                      sigma_per_step=it.get("sigma_per_step", False), mapping=mapping)
    torch.cuda.synchronize()
    return U, c, st


def _items(mp, ctx, shapes, base=0):
    out = []
    for i, (K, H, M) in enumerate(shapes):
        sc = W.make_scene(4, base + i)
        pp = W.plan_params(4, K=K, H=H, M=M, seed=7000 + base + i)
        out.append(dict(scene=mp.Scene(ctx, sc), x0=T(W.initial_state(sc)), K=K, H=H, lam=pp["lam"],
                        sigma=T(pp["sigma"]), M=M, seed=pp["seed"],
                        nominal_U=T(np.random.default_rng(base + i).uniform(-0.2, 0.2, (H, 14))),
                        n_elite=16 if i == 2 else 0, eta=0.7 if i == 3 else 1.0,
                        U_new=torch.zeros((H, 14), device=DEV), costs=torch.zeros(K, device=DEV)))
    return out


@pytest.mark.parametrize("mapping", ["team", "lane", "wave", "split", None])
def test_served_requests_equal_plans_alone(mp, ctx, mapping):
    """Served requests equal the same plans alone bit for bit, with a pinned
    mapping and under default flags (None), where one request is large
    enough to run one sample per lane alone while the others run in the
    team family."""
    shapes = [(70, 6, 3), (5, 4, 1), (130, 9, 4), (33, 3, 2), (64, 5, 6), (200, 7, 2)]
    if mapping is None:
        shapes.append((33000, 3, 2))
    items = _items(mp, ctx, shapes)
    srv = mp.Server(ctx, mapping=mapping)
    tickets = [srv.submit(it) for it in items]
    res = [srv.wait(t) for t in tickets]
    q = srv.query()
    srv.close()
    assert q["completed"] == len(items) and q["iterations"] >= 6
    # the requests shared launches: fewer packed iterations than request iterations
    assert q["request_iters"] == sum(it["M"] for it in items) and q["iterations"] < q["request_iters"]
    for it, r in zip(items, res):
        U, c, st = _plan_alone(mp, ctx, it, mapping)
        assert r["status"] == 0 and r["iterations"] == it["M"]
        assert torch.equal(U, it["U_new"]) and torch.equal(c, it["costs"])
        assert r["stats"]["best"] == st["best"] and r["stats"]["ess"] == st["ess"]
        assert r["stats"]["cmin_iter"] == st["cmin_iter"]
        assert r["t_submit_ms"] <= r["t_admit_ms"] <= r["t_done_ms"]
    for it in items:
        it["scene"].close()


def test_served_host_pointer_requests(mp, ctx):
    items = _items(mp, ctx, [(40, 5, 2), (17, 3, 3)], base=10)
    host = []
    for it in items:
        h = dict(it)
        for k in ("x0", "nominal_U", "sigma"):
            h[k] = it[k].cpu().numpy()
        h["U_new"] = np.zeros((it["H"], 14), np.float32)
        h["costs"] = np.zeros(it["K"], np.float32)
        host.append(h)
    srv = mp.Server(ctx, mapping="team")
    ts = [srv.submit(h) for h in host]
    for t in ts:
        assert srv.wait(t)["status"] == 0
    srv.close()
    for it, h in zip(items, host):
        U, c, _ = _plan_alone(mp, ctx, it, "team")
        assert np.array_equal(U.cpu().numpy(), h["U_new"]) and np.array_equal(c.cpu().numpy(), h["costs"])
        it["scene"].close()


def _shift(U, s):
    H = U.shape[0]
    idx = np.minimum(np.arange(H) + s, H - 1)
    return U[idx]


def _chain_alone(mp, ctx, scene, x0, nom, reqs, mapping):
    """The cell protocol replayed with single calls: plan, advance the state
    by `adv` steps of U_new, shift the nominal."""
    x = T(x0)
    nu = T(nom)
    outs = []
    for (K, M, seed, adv, sigma, lam) in reqs:
        H = nu.shape[0]
        U = torch.zeros((H, 14), device=DEV)
        c = torch.zeros(K, device=DEV)
        mp.mppi_plan(ctx, scene, x, nu, K, H, lam, T(sigma), U, c, M=M, seed=seed, mapping=mapping)
        torch.cuda.synchronize()
        outs.append((U.clone(), c.clone()))
        if adv > 0:
            xo = torch.zeros((1, 55), device=DEV)
            mp.mppi_simulate(ctx, scene, x, U[:adv].contiguous().reshape(1, adv, 14), X_out=xo, x0_shared=True,
                             mapping=mapping)
            torch.cuda.synchronize()
            x = xo[0].clone()
        nu = T(_shift(U.cpu().numpy(), adv))
    return x.cpu().numpy(), nu.cpu().numpy(), outs


def test_cell_warm_start_chain(mp, ctx):
    sc = W.make_scene(4, 3)
    scene = mp.Scene(ctx, sc)
    H = 8
    x0 = W.initial_state(sc).astype(np.float32)
    nom0 = np.random.default_rng(3).uniform(-0.1, 0.1, (H, 14)).astype(np.float32)
    pp = W.plan_params(4, K=48, H=H, M=2)
    reqs = [(48, 2, 11, 2, pp["sigma"], pp["lam"]), (48, 3, 12, 1, pp["sigma"], pp["lam"]),
            (20, 1, 13, 0, pp["sigma"], pp["lam"]), (48, 2, 14, 3, pp["sigma"], pp["lam"])]
    srv = mp.Server(ctx, mapping="team")
    cell = srv.cell(scene, H, x0, nom0)
    got = []
    for (K, M, seed, adv, sigma, lam) in reqs:
        it = dict(K=K, lam=lam, sigma=T(sigma), M=M, seed=seed, U_new=torch.zeros((H, 14), device=DEV),
                  costs=torch.zeros(K, device=DEV))
        t = srv.submit(it, cell=cell, advance=adv)
        got.append((t, it))
    for t, it in got:
        assert srv.wait(t)["status"] == 0
    x_srv, nu_srv = srv.cell_read(cell, H)
    srv.close()
    x_ref, nu_ref, outs = _chain_alone(mp, ctx, scene, x0, nom0, reqs, "team")
    for (t, it), (U, c) in zip(got, outs):
        assert torch.equal(it["U_new"], U) and torch.equal(it["costs"], c)
    assert np.array_equal(x_srv, x_ref)
    assert np.array_equal(nu_srv, nu_ref)
    assert not np.array_equal(x_srv, x0)  # the plant moved
    scene.close()


def test_many_cells_in_the_mix_equal_alone(mp, ctx):
    """12 cells with different scenes, K and H; three rounds of requests
    submitted back to back so that they overlap on the device; each cell's
    results equal its own chain replayed alone."""
    rng = np.random.default_rng(21)
    cells = []
    srv = mp.Server(ctx, mapping="team", max_active=8)
    for i in range(12):
        sc = W.make_scene(4, 20 + i)
        H = int(rng.integers(3, 12))
        scene = mp.Scene(ctx, sc)
        x0 = W.initial_state(sc).astype(np.float32)
        pp = W.plan_params(4, K=16, H=H, M=2)
        reqs = [(int(rng.integers(8, 150)), int(rng.integers(1, 4)), 100 * i + r, int(rng.integers(0, 3)),
                 pp["sigma"], pp["lam"]) for r in range(3)]
        cid = srv.cell(scene, H, x0)
        cells.append(dict(scene=scene, H=H, x0=x0, reqs=reqs, cell=cid, got=[]))
    for r in range(3):
        for c in cells:
            K, M, seed, adv, sigma, lam = c["reqs"][r]
            it = dict(K=K, lam=lam, sigma=T(sigma), M=M, seed=seed, U_new=torch.zeros((c["H"], 14), device=DEV),
                      costs=torch.zeros(K, device=DEV))
            c["got"].append((srv.submit(it, cell=c["cell"], advance=adv), it))
    for c in cells:
        for t, _ in c["got"]:
            assert srv.wait(t)["status"] == 0
        c["x"], c["nu"] = srv.cell_read(c["cell"], c["H"])
    q = srv.query()
    srv.close()
    assert q["completed"] == 36
    for c in cells:
        x_ref, nu_ref, outs = _chain_alone(mp, ctx, c["scene"], c["x0"], np.zeros((c["H"], 14), np.float32),
                                           c["reqs"], "team")
        for (t, it), (U, cc) in zip(c["got"], outs):
            assert torch.equal(it["U_new"], U) and torch.equal(it["costs"], cc)
        assert np.array_equal(c["x"], x_ref) and np.array_equal(c["nu"], nu_ref)
        c["scene"].close()


def test_cancel_supersede_limits(mp, ctx):
    sc = W.make_scene(4, 1)
    scene = mp.Scene(ctx, sc)
    H = 16
    pp = W.plan_params(4, K=512, H=H, M=10)
    srv = mp.Server(ctx, mapping="team", max_active=1, max_pending=3, mem_budget=64 << 20)
    cell = srv.cell(scene, H, W.initial_state(sc).astype(np.float32))

    def item(K=512, M=10, seed=1):
        return dict(K=K, lam=pp["lam"], sigma=T(pp["sigma"]), M=M, seed=seed)

    a = srv.submit(item(seed=1), cell=cell, advance=1)
    b = srv.submit(item(seed=2), cell=cell, advance=1)
    c = srv.submit(item(seed=3), cell=cell, advance=1, supersede=True)  # replaces b (queued)
    d = srv.submit(item(seed=4), cell=cell, advance=1)
    rb = srv.poll(b)
    assert rb is not None and rb["status"] == mp.E_CANCELLED and rb["iterations"] == 0
    srv.cancel(d)  # queued: dropped at once
    rd = srv.poll(d)
    assert rd["status"] == mp.E_CANCELLED
    with pytest.raises(mp.MppiError):
        srv.poll(d)  # released
    # queue limit: c plus three more fill max_pending=3 (a may be running)
    extra = []
    with pytest.raises(mp.MppiError) as e:
        for s in range(10):
            extra.append(srv.submit(item(seed=10 + s), cell=cell))
    assert e.value.code == mp.E_BUSY
    # a request that can never fit the memory budget is refused at once
    with pytest.raises(mp.MppiError) as e:
        srv.submit(dict(item(K=1 << 16, M=1), scene=scene, H=H, x0=T(W.initial_state(sc)),
                        nominal_U=torch.zeros((H, 14), device=DEV), U_new=torch.zeros((H, 14), device=DEV)))
    assert e.value.code == mp.E_BUSY
    assert srv.wait(a)["status"] == 0
    rc = srv.wait(c)
    assert rc["status"] == 0 and rc["iterations"] == 10
    for t in extra:
        r = srv.wait(t)
        assert r["status"] == 0
    # cancelling a running request stops it at an iteration boundary
    long = srv.submit(item(M=60, seed=99), cell=cell)
    import time
    t_end = time.time() + 10
    while srv.query()["active"] == 0 and srv.query()["pending"] > 0 and time.time() < t_end:
        time.sleep(0.001)
    try:
        srv.cancel(long)
        r = srv.wait(long)
        assert r["status"] == mp.E_CANCELLED and r["iterations"] < 60
    except mp.MppiError:  # it finished first
        assert srv.wait(long)["status"] == 0
    q = srv.query()
    assert q["superseded"] == 1 and q["rejected"] >= 2
    with pytest.raises(mp.MppiError):
        srv.cancel(123456)
    srv.close()
    scene.close()


def test_destroy_with_work_in_flight(mp, ctx):
    items = _items(mp, ctx, [(256, 16, 5)] * 6, base=40)
    srv = mp.Server(ctx, mapping="team", max_active=2)
    for it in items:
        srv.submit(it)
    srv.close()  # cancels the queue, drains what runs, joins the worker
    for it in items:
        it["scene"].close()


def test_deadlines_shed_order_and_results(mp, ctx):
    """With a deadline, a request that cannot end in time even alone under the
    iteration model is shed unrun (MPPI_E_LATE); the others run, carry their
    deadline, and equal their plans alone bit for bit; the server fits its
    own iteration model when none is given."""
    items = _items(mp, ctx, [(64, 6, 2), (40, 5, 3), (80, 4, 2)], base=40)
    # 10 ms per packed iteration predicted: M = 20 needs 210 ms > 100 ms
    big = _items(mp, ctx, [(32, 4, 20)], base=50)[0]
    srv = mp.Server(ctx, mapping="team", deadline_ms=100.0, iter_base_ms=10.0)
    t_big = srv.submit(big)
    ts = [srv.submit(it) for it in items]
    r_big = srv.wait(t_big)
    assert r_big["status"] == mp.E_LATE and r_big["iterations"] == 0
    res = [srv.wait(t) for t in ts]
    q = srv.query()
    srv.close()
    assert q["shed"] == 1 and q["completed"] == len(items)
    for it, r in zip(items, res):
        assert r["status"] == 0
        assert r["t_deadline_ms"] == pytest.approx(r["t_submit_ms"] + 100.0)
        U, c, _ = _plan_alone(mp, ctx, it, "team")
        assert torch.equal(U, it["U_new"]) and torch.equal(c, it["costs"])
    # no model given: the server measures its iterations and fits one
    srv = mp.Server(ctx, mapping="team", deadline_ms=1e6)
    for rep in range(3):
        for it in items:
            srv.wait(srv.submit(it))
    q = srv.query()
    srv.close()
    assert q["iterations"] >= 8 and q["model_floor_ms"] > 0 and q["late"] == 0 and q["shed"] == 0
    for it in items + [big]:
        it["scene"].close()
