"""Oracle pins: ball-task cost terms (Sec. IV-B), the collision cost
(Eq. collision_cost) on scripted distances, and the MPPI update
(Eqs. mean_update, s_formula) against a brute-force weighted mean in
50-digit decimal arithmetic and its invariants.
"""
import math
from decimal import Decimal, getcontext

import numpy as np
import pytest

import workloads as W


def test_stage_terms_worked_example(oracle_mod):
    """Both arms straight up: pads at (-+0.55, 0, 1.06) exactly."""
    sc = W.make_scene(2)
    o = oracle_mod.Oracle(sc)
    x = W.initial_state(sc)
    x[0:14] = 0.0
    x[42:45] = [0.1, 0.2, 0.3]
    t = o.stage_terms(x)
    goal = np.array([0.0, 0.5, 0.3])
    assert t[0] == pytest.approx(math.sqrt(0.1 ** 2 + 0.3 ** 2 + 0.0 ** 2), abs=1e-14)
    eps = 0.3 * 0.1
    # midpoint (0, 0, 1.06) vs ball - (0, 0, eps) = (0.1, 0.2, 0.27)
    assert t[1] == pytest.approx(math.sqrt(0.1 ** 2 + 0.2 ** 2 + (1.06 - 0.27) ** 2), abs=1e-14)
    l_ball = 2 * math.sqrt((0.1 + 0.04) ** 2 - eps ** 2)
    assert t[2] == pytest.approx((1.1 - l_ball) ** 2, abs=1e-14)
    assert t[3] == pytest.approx(0.0, abs=1e-15)
    assert o.model()["l_ball"] == pytest.approx(l_ball, abs=1e-15)
    # planar term: shift arm 2's base yaw so its pad leaves the xz plane
    x[7] = 0.3    # arm 2 joint 1 (yaw) rotates the upright arm about its own axis: pad unchanged
    assert o.stage_terms(x)[3] == pytest.approx(0.0, abs=1e-14)
    x[8] = 0.5    # arm 2 pitches: with yaw 0.3 its pad moves off y = 0
    _, o1, _, _ = o.fk(1, x[7:14])
    t = o.stage_terms(x)
    assert t[3] == pytest.approx(math.hypot(o1[-1][1], o1[-1][2] - 1.06), abs=1e-14)


def test_collision_cost_scripted(oracle_mod):
    O = oracle_mod.Oracle
    g = 0.5
    # one pair approaching: d = 0.05, 0.01, -0.01, 0.02
    d = np.array([[0.05], [0.01], [-0.01], [0.02]])
    bar, ind = O.collision_cost(d, g)
    # barrier terms max(-d_{k+1} + 0.5 d_k, 0): 0.015, 0.015, 0 (-0.02-0.005<0)
    assert bar == pytest.approx(0.015 + 0.015 + 0.0, abs=1e-15)
    assert ind == 1.0
    # two pairs, the second always saturated far away -> contributes nothing
    d2 = np.concatenate([d, np.full((4, 1), 0.05)], axis=1)
    assert O.collision_cost(d2, g) == pytest.approx((bar, ind))
    # gamma -> 1: barrier reduces to max(-d_{k+1}, 0)
    bar1, _ = O.collision_cost(d, 0.999999999)
    assert bar1 == pytest.approx(0.01, abs=1e-9)


def test_cost_dist_saturation_and_consistency(oracle_mod):
    sc = W.make_scene(3)
    o = oracle_mod.Oracle(sc)
    X = W.random_states(sc, 10, seed=3, spread=1.0)
    nd = 14 * sc["n_box"] + 49
    for x in X:
        d = o.cost_dist(x)
        phi, _, _ = o.narrow_all(x)
        assert len(d) == nd
        assert np.allclose(d, np.minimum(phi[-nd:], sc["m_c"]), atol=0.0)


def test_rollout_cost_composition(oracle_mod):
    sc = W.make_scene(2)
    o = oracle_mod.Oracle(sc)
    x0 = W.initial_state(sc)
    H = 6
    U = np.zeros((H, 14))
    U[3:, 2] = 0.4        # one jump of 0.4 in joint 3 at k = 3
    U[5, 9] = -0.3        # and one of 0.3 at k = 5
    c, terms = o.rollout(x0, U)
    assert terms[4] == pytest.approx(0.4 ** 2 + 0.3 ** 2, abs=1e-15)
    w = [sc["w_goal"], sc["w_eo"], sc["w_l"], sc["w_yz"], sc["w_s"], sc["w_c"], sc["w_c"]]
    assert np.all(terms[7:] == 0.0)   # the further task terms are off in a ball scene
    assert c == pytest.approx(float(np.dot(w, terms[:7])), rel=1e-15)
    # the per-step terms are the stage terms of the trajectory
    c2, terms2, traj = o.rollout(x0, U, want_traj=True)
    st = np.array([o.stage_terms(x) for x in traj]).sum(axis=0)
    assert np.allclose(terms2[:4], st, rtol=1e-14)
    # non-finite rollout -> +inf
    xbad = x0.copy()
    xbad[14] = np.nan
    cb, _ = o.rollout(xbad, U)
    assert cb == np.inf


def _brute_update(U, c, lam, nu, eta):
    getcontext().prec = 50
    w = [(-Decimal(float(cj)) / Decimal(float(lam))).exp() for cj in c]
    Z = sum(w)
    out = np.zeros_like(nu)
    for idx in np.ndindex(nu.shape):
        s = sum(wj * Decimal(float(U[j][idx])) for j, wj in enumerate(w))
        out[idx] = float((1 - Decimal(eta)) * Decimal(float(nu[idx])) + Decimal(eta) * s / Z)
    return out


def test_update_matches_brute_force_weighted_mean(oracle_mod):
    O = oracle_mod.Oracle
    rng = np.random.default_rng(20)
    for trial in range(5):
        K, H = 3, 2
        U = rng.uniform(-1.5, 1.5, size=(K, H, 14))
        c = rng.uniform(20.0, 21.0, K)          # unshifted exp(-c/lambda) ~ e^-200: fine in 50 digits
        nu = rng.uniform(-1, 1, size=(H, 14))
        for lam, eta in ((0.1, 1.0), (0.5, 0.3)):
            out, nf, ess = O.update(U, c, lam, nu, eta)
            assert nf == K
            assert np.allclose(out, _brute_update(U, c, lam, nu, eta), rtol=1e-12, atol=1e-14)


def test_update_invariants(oracle_mod):
    O = oracle_mod.Oracle
    rng = np.random.default_rng(21)
    K, H = 9, 4
    U = rng.uniform(-1, 1, size=(K, H, 14))
    c = rng.uniform(0, 3, K)
    nu = rng.uniform(-1, 1, size=(H, 14))
    base, _, _ = O.update(U, c, 0.7, nu)
    assert np.allclose(O.update(U, c + 123.0, 0.7, nu)[0], base, rtol=1e-12)     # cost shift
    perm = rng.permutation(K)
    assert np.allclose(O.update(U[perm], c[perm], 0.7, nu)[0], base, rtol=1e-12)  # permutation
    assert np.allclose(O.update(U, c, 1e9, nu)[0], U.mean(axis=0), atol=1e-8)     # lambda -> inf
    assert np.allclose(O.update(U, c, 1e-6, nu)[0], U[np.argmin(c)], atol=1e-12)  # lambda -> 0
    assert np.allclose(O.update(U, c, 0.7, nu, eta=0.0)[0], nu, atol=0)            # eta = 0
    same = np.repeat(U[:1], K, axis=0)
    assert np.allclose(O.update(same, c, 0.7, nu)[0], U[0], rtol=1e-13)            # identical samples
    assert np.allclose(O.update(U, c, 0.7, nu, n_elite=1)[0], U[np.argmin(c)], atol=0)  # one elite
    # elite set of 3: equals the update over the 3 lowest costs only
    idx = np.argsort(c, kind="stable")[:3]
    assert np.allclose(O.update(U, c, 0.7, nu, n_elite=3)[0], O.update(U[idx], c[idx], 0.7, nu)[0], rtol=1e-13)
    # non-finite costs get weight 0
    c2 = c.copy()
    c2[[1, 4]] = np.inf
    keep = [j for j in range(K) if j not in (1, 4)]
    assert np.allclose(O.update(U, c2, 0.7, nu)[0], O.update(U[keep], c[keep], 0.7, nu)[0], rtol=1e-13)
    out, nf, _ = O.update(U, np.full(K, np.inf), 0.7, nu)
    assert nf == 0 and np.array_equal(out, nu)
    # effective sample size: 1 for lambda -> 0, K for lambda -> inf
    assert O.update(U, c, 1e-6, nu)[2] == pytest.approx(1.0)
    assert O.update(U, c, 1e9, nu)[2] == pytest.approx(K, rel=1e-6)


def test_plan_is_composition_of_steps(oracle_mod):
    sc = W.make_scene(1)
    o = oracle_mod.Oracle(sc)
    x0 = W.initial_state(sc)
    K, H, M = 8, 5, 2
    sig = np.full(14, 0.3)
    nom = np.zeros((H, 14))
    r = o.plan(x0, nom, K, H, 0.1, sig, M, seed=11, nthreads=2)
    nu = nom
    for m in range(M):
        U = o.sample(nu, sig, 11, K, m)
        c = o.rollout_batch(x0, U, nthreads=2)
        nu, _, _ = o.update(U, c, 0.1, nu)
    assert r["rc"] == 0
    assert np.allclose(r["nu"], nu, rtol=0, atol=0)
    assert np.allclose(r["costs"], c, rtol=0, atol=0)
    assert r["best"] == int(np.argmin(c))
    # all samples non-finite -> error and nominal returned
    xb = x0.copy()
    xb[14] = np.nan
    r2 = o.plan(xb, nom + 0.1, K, H, 0.1, sig, 1, seed=11, nthreads=2)
    assert r2["rc"] == -4 and np.array_equal(r2["nu"], nom + 0.1)
