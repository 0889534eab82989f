"""GPU parity on the obstacle scenes: the collision cost against boxes, the
contact solve with more than four contacts, truncation of the contact list
at n_cmax, and the packed-batch scene parameters (12 boxes, small and large
balls), each against the FP64 oracle on the same inputs, in every
sample-to-lane mapping.

Eq. collision_cost is evaluated on the arm-box and arm-arm signed distances
(saturated at m_c) of rollouts that start with arm geoms inside m_c of a box,
some of them penetrating; the states are seeded and found with the oracle's
narrowphase (no GPU value enters an input or an expected value).
"""
import numpy as np
import pytest

import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"
MAPPINGS = ["lane", "team", "wave", "split"]
# one group per body and kind: each arm's joint positions, velocities and PD
# targets; the ball's centre, orientation, linear and angular velocity
GROUPS = [(0, 7), (7, 14), (14, 21), (21, 28), (28, 35), (35, 42), (42, 45), (45, 49), (49, 52), (52, 55)]


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


def T(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def _scales(want, r_ball):
    """Largest magnitude of each group of `want` (over every leading axis):
    contact impulses act through a body's whole inverse inertia, so the
    rounding error of one joint velocity follows its arm's largest velocity,
    and the ball's spin error follows its linear velocity over its radius."""
    out = []
    for a, b in GROUPS:
        scale = max(np.abs(want[..., a:b]).max(), 1e-3)
        if a == 52:
            scale = max(scale, np.abs(want[..., 49:52]).max() / r_ball)
        out.append(scale)
    return out


def _close(got, want, rtol, r_ball, what=""):
    """|got - want| <= rtol * scale per body and kind of coordinate."""
    for (a, b), scale in zip(GROUPS, _scales(want, r_ball)):
        err = np.abs(got[..., a:b] - want[..., a:b]).max()
        assert err <= rtol * scale, (what, a, b, err, scale)


# scene cases: the 3-box and 8-box workloads, and packed-batch scenes with
# 12 boxes and the extreme ball radii and masses of that workload
SCENES = {
    "c2": (2, 0, {}),
    "c3": (3, 0, {}),
    "c4_r06": (4, 3, dict(n_box=12, ball_r=0.06, ball_m=0.2)),
    "c4_r14": (4, 5, dict(n_box=12, ball_r=0.14, ball_m=1.0)),
}
SEEDS = {"c2": 101, "c3": 102, "c4_r06": 103, "c4_r14": 104}
_ORACLE_ROLLOUTS = {}


def _scene(name, **extra):
    cfg, idx, kw = SCENES[name]
    return W.make_scene(cfg, idx, **kw, **extra)


def _near_box_states(o, sc, n, seed, min_neg):
    """Seeded states whose arm geoms lie within m_c of a box (at least
    `min_neg` of them penetrating one), every pair deeper than -1 cm
    excluded, joint velocities moderate; the ball flies far from everything
    (a ball resting on the table keeps a contact at |phi| ~ 1e-6, where
    FP32 and FP64 may disagree on whether it is active)."""
    rng = np.random.default_rng(seed)
    nb = int(sc["n_box"])
    out, neg = [], 0
    while len(out) < n:
        x = W.initial_state(sc)
        x[42:45] = [0.0, 3.0, 2.0]
        x[0:14] = np.asarray(sc["q_home"]) + rng.uniform(-1.3, 1.3, 14)
        x[28:42] = x[0:14]
        x[14:28] = rng.uniform(-1.0, 1.0, 14)
        d = o.cost_dist(x)[:14 * nb]
        if not (-0.01 < d.min() < sc["m_c"]):
            continue
        if o.narrow_all(x)[0].min() < -0.01:
            continue
        is_neg = d.min() < 0
        if not is_neg and len(out) - neg >= n - min_neg:
            continue
        out.append(x)
        neg += is_neg
    return np.array(out)


def _flip_margin(o, sc, x0, U):
    """Smallest |phi| of every pair at every substep's start state, and
    smallest |d| of the unsaturated cost distances at every control step, of
    the oracle's rollout: a contact or an indicator can switch between FP32
    and FP64 only when one of them is near zero."""
    x = x0.copy()
    m_phi, m_d = np.inf, np.inf
    for k in range(U.shape[0]):
        for _ in range(int(sc["n_sub"])):
            phi = o.narrow_all(x)[0]
            m_phi = min(m_phi, np.abs(phi).min())
            x, _ = o.substep(x, U[k])
        d = o.cost_dist(x)
        d = d[d < sc["m_c"]]
        if d.size:
            m_d = min(m_d, np.abs(d).min())
    return m_phi, m_d


@pytest.mark.parametrize("mapping", MAPPINGS)
@pytest.mark.parametrize("name", list(SCENES))
def test_collision_cost_terms_on_box_scenes(mp, ctx, oracle_mod, name, mapping):
    """Every cost term (goal, eef-obj, distance, planar, smoothness, barrier,
    indicator) of H = 6 rollouts from states near and inside the boxes, per
    sample, against the oracle; n = 250 samples span several workgroups and
    a ragged tail, so the [pair][sample] history of the distances is laid
    out at a stride other than one workgroup."""
    sc = _scene(name)
    o = oracle_mod.Oracle(sc)
    scene = mp.Scene(ctx, sc)
    n, H = 250, 6
    X = f32(_near_box_states(o, sc, n, seed=SEEDS[name], min_neg=n // 3)).astype(np.float32)
    U = np.random.default_rng(7).uniform(-1.5, 1.5, (n, H, 14)).astype(np.float32)
    if name not in _ORACLE_ROLLOUTS:  # the same inputs in every mapping: compute the oracle's side once
        _ORACLE_ROLLOUTS[name] = [(o.rollout(f32(X[i]), f32(U[i]), want_traj=True),
                                   _flip_margin(o, sc, f32(X[i]), f32(U[i]))) for i in range(n)]
    costs = torch.zeros(n, device=DEV)
    terms = torch.zeros((n, mp.NTERMS), device=DEV)
    Xo = torch.zeros((n, H, 55), device=DEV)
    mp.mppi_simulate(ctx, scene, T(X), T(U), costs=costs, terms=terms, X_out=Xo, traj=True, mapping=mapping)
    torch.cuda.synchronize()
    tg, cg, xg = terms.cpu().numpy().astype(np.float64), costs.cpu().numpy(), Xo.cpu().numpy().astype(np.float64)
    kept, n_ind, n_bar = 0, 0.0, 0
    worst = np.zeros(mp.NTERMS)
    for i in range(n):
        (c, tm, traj), (m_phi, m_d) = _ORACLE_ROLLOUTS[name][i]
        if m_phi < 2e-5 or m_d < 2e-5:
            continue  # a contact or indicator near its switching point
        kept += 1
        _close(xg[i], traj, 1e-4, sc["ball_r"], f"sample {i}")
        rel = np.abs(tg[i] - tm) / np.maximum(np.abs(tm), 1e-3)
        worst = np.maximum(worst, rel)
        assert np.all(rel[:5] < 1e-4), (i, tg[i], tm)
        assert abs(tg[i, 5] - tm[5]) < 1e-4 * max(1.0, tm[5]), (i, tg[i, 5], tm[5])
        assert tg[i, 6] == tm[6], (i, tg[i, 6], tm[6])
        assert abs(cg[i] - c) <= 1e-4 * abs(c)
        n_ind += tm[6]
        n_bar += tm[5] > 0
    print(f"{name} {mapping}: {kept}/{n} samples clear of switching points; worst term rel err {worst}; "
          f"indicator total {n_ind:.0f}, samples with a barrier {n_bar}")
    assert kept >= 0.7 * n
    assert n_ind >= 10 and n_bar >= 5   # the penetration and barrier branches are exercised
    scene.close()


def _many_contact_states(o, sc, n, lo, hi, seed, iters=1200):
    """Seeded hill climb over arm configurations and the ball position for
    states whose uncapped contact lists hold lo..hi active pairs (every pair
    shallower than 1.2 cm)."""
    rng = np.random.default_rng(seed)
    out = []

    def score(x):
        phi = o.narrow_all(x)[0]
        return -1 if phi.min() < -0.012 else int((phi < 0).sum())

    for _ in range(40 * n):
        x = W.initial_state(sc)
        x[44] = sc["ball_r"] - 0.003
        x[0:14] = np.asarray(sc["q_home"]) + rng.uniform(-1.0, 1.0, 14)
        s = score(x)
        for _ in range(iters):
            y = x.copy()
            y[0:14] += rng.normal(0, 0.05, 14)
            y[42:45] += rng.normal(0, 0.01, 3)
            sy = score(y)
            if sy >= s:
                x, s = y, sy
            if s >= hi:
                break
        if lo <= s <= hi:
            x[28:42] = x[0:14]
            x[14:28] = rng.uniform(-0.3, 0.3, 14)
            x[49:55] = rng.uniform(-0.1, 0.1, 6)
            out.append(x)
            if len(out) == n:
                break
    assert len(out) == n, f"found {len(out)} states with {lo}..{hi} contacts"
    return np.array(out)


@pytest.fixture(scope="module")
def contact_rich(oracle_mod):
    """States of the 8-box workload with 5..8 active contact pairs."""
    sc = _scene("c3", n_cmax=16)
    o = oracle_mod.Oracle(sc)
    return f32(_many_contact_states(o, sc, 12, 5, 8, seed=11)).astype(np.float32)


def _substep_case(mp, ctx, oracle_mod, sc, X, mapping, rtol=1e-5):
    scene = mp.Scene(ctx, sc)
    o = oracle_mod.Oracle(sc)
    n = len(X)
    U = np.random.default_rng(5).uniform(-1.0, 1.0, (n, 1, 14)).astype(np.float32)
    ncon = []
    for nsub in (1, int(sc["n_sub"])):
        Xo = torch.zeros((n, 55), device=DEV)
        mp.mppi_simulate(ctx, scene, T(X), T(U), X_out=Xo, n_sub=nsub, mapping=mapping)
        torch.cuda.synchronize()
        got = Xo.cpu().numpy().astype(np.float64)
        want = np.zeros_like(got)
        for i in range(n):
            x = f32(X[i])
            for s in range(nsub):
                if s == 0:
                    ncon.append(len(o.contacts(x, cap=64)[0]))
                x, _ = o.substep(x, f32(U[i, 0]))
            want[i] = x
        # the bound over the case (scale: the group's largest value over all
        # states), and each state against its own scales within 5x the bound
        # (one control step carries each substep's rounding into the next:
        # twice the bound; deep, truncated contact lists with arm velocities
        # of 5 rad/s reach 1.02e-5 there in the lane mapping's impulse-space
        # sweeps)
        tol = rtol if nsub == 1 else 2 * rtol
        _close(got, want, tol, sc["ball_r"], f"n_sub {nsub}")
        for i in range(n):
            _close(got[i], want[i], 5 * tol, sc["ball_r"], f"n_sub {nsub} state {i}")
    scene.close()
    return ncon


@pytest.mark.parametrize("mapping", MAPPINGS)
def test_eight_contact_solve_against_oracle(mp, ctx, oracle_mod, contact_rich, mapping):
    """n_cmax = 8 (the 8-contact instantiations of every mapping): states with
    5..8 active pairs, one substep within 1e-5 and one control step within
    2e-5 of each body's scale."""
    sc = _scene("c3", n_cmax=8)
    ncon = _substep_case(mp, ctx, oracle_mod, sc, contact_rich, mapping)
    assert min(ncon[:len(contact_rich)]) >= 5 and max(ncon[:len(contact_rich)]) <= 8


@pytest.mark.parametrize("mapping", MAPPINGS)
@pytest.mark.parametrize("cap", [4, 3, 5])
def test_contact_list_truncated_in_canonical_order(mp, ctx, oracle_mod, contact_rich, mapping, cap):
    """More active pairs than n_cmax: both sides keep the first n_cmax in the
    canonical pair order (ball-table, ball-pads, ball-links, ball-boxes,
    arm-table, arm-boxes, arm-arm) and drop the rest; keeping any other
    subset changes the impulses and fails the 1e-5 bound."""
    sc = _scene("c3", n_cmax=cap)
    o = oracle_mod.Oracle(_scene("c3", n_cmax=16))
    ga, gb = o.pairs()
    over = [i for i, x in enumerate(contact_rich) if len(o.contacts(f32(x), cap=64)[0]) > cap]
    assert len(over) >= 4
    X = contact_rich[over]
    # the truncated lists differ from a list ordered any other way: the dropped
    # pairs carry impulses of their own when the cap is lifted
    _substep_case(mp, ctx, oracle_mod, sc, X, mapping)
    full = oracle_mod.Oracle(_scene("c3", n_cmax=8))
    capped = oracle_mod.Oracle(sc)
    u = np.zeros(14)
    diff = [np.abs(full.substep(f32(x), u)[0] - capped.substep(f32(x), u)[0]).max() for x in X]
    assert max(diff) > 1e-3


@pytest.mark.parametrize("mapping", MAPPINGS)
@pytest.mark.parametrize("name", ["c4_r06", "c4_r14"])
def test_packed_scene_parameters_one_substep(mp, ctx, oracle_mod, name, mapping):
    """A 12-box packed-batch scene with the smallest and the largest ball
    (r = 0.06 m, 0.2 kg; r = 0.14 m, 1.0 kg): one substep and one control
    step from near-box states and from states with the ball pressed into
    the table under a pad, against the oracle."""
    sc = _scene(name)
    o = oracle_mod.Oracle(sc)
    X = _near_box_states(o, sc, 40, seed=3, min_neg=10)
    rng = np.random.default_rng(4)
    B = np.tile(W.initial_state(sc), (30, 1))
    B[:, 44] = sc["ball_r"] - rng.uniform(0.0, 0.004, 30)
    B[:, 0:7] += np.array([0, 0.35, 0, 0.2, 0, 0.25, 0]) * rng.uniform(0.8, 1.2, (30, 1))
    B[:, 14:28] = rng.uniform(-0.3, 0.3, (30, 14))
    B[:, 28:42] = B[:, 0:14]
    B[:, 49:55] = rng.uniform(-0.1, 0.1, (30, 6))
    X = f32(np.concatenate([X, B])).astype(np.float32)
    ncon = _substep_case(mp, ctx, oracle_mod, sc, X, mapping)
    assert np.mean(np.array(ncon) > 0) > 0.4
