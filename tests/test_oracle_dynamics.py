"""Oracle pins for the world model f (Eq. state_evol): closed forms and
invariants of the substep (free flight, a resting drop, rolling friction,
energy behaviour, and projected Gauss-Seidel against an exact LCP solve).
"""
import itertools
import math

import numpy as np
import pytest

import workloads as W


def far_ball_state(sc, p, v=(0, 0, 0), w=(0, 0, 0)):
    x = W.initial_state(sc)
    x[42:45] = p
    x[49:52] = v
    x[52:55] = w
    return x


def test_ballistic_flight_discrete_closed_form(oracle_mod):
    sc = W.make_scene(2)
    o = oracle_mod.Oracle(sc)
    h, g = sc["h"], sc["g"]
    p0, v0, w0 = np.array([0.1, 0.6, 1.2]), np.array([0.3, -0.2, 1.0]), np.array([0.5, -1.0, 2.0])
    x = far_ball_state(sc, p0, v0, w0)
    u = np.zeros(14)
    n = 150
    for _ in range(n):
        x, nc = o.substep(x, u)
        assert nc == 0
    # semi-implicit Euler: v_n = v0 - n g h, p_n = p0 + n h v0 - g h^2 n (n + 1) / 2
    want_p = p0 + n * h * v0 - np.array([0, 0, g * h * h * n * (n + 1) / 2])
    want_v = v0 - np.array([0, 0, n * g * h])
    assert np.allclose(x[42:45], want_p, rtol=1e-12, atol=1e-14)
    assert np.allclose(x[49:52], want_v, rtol=1e-12, atol=1e-14)
    assert np.allclose(x[52:55], w0)
    # constant spin: n steps of exp(h w / 2) compose to exp(n h w / 2)
    th = n * h * w0
    a = np.linalg.norm(th)
    want_q = np.concatenate([[math.cos(a / 2)], math.sin(a / 2) * th / a])
    assert np.allclose(x[45:49], want_q, atol=1e-12)
    # arms at rest at their PD target under gravity compensation stay put
    assert np.allclose(x[0:14], sc["q_home"], atol=0.0)


def _rest_penetration(sc):
    """Steady state of one ball-plane contact: v+ = 0 needs 4 f = m g h; the
    converged soft LCP row gives R f = kappa pen / h with
    A_ee = (1 + mu^2)/m + mu^2 rho^2 / I, rho = r - pen/2 (lever arm of the
    midpoint contact).  Solved by fixed-point iteration."""
    m, g, h, r = sc["ball_m"], sc["g"], sc["h"], sc["ball_r"]
    mu, kap, er = sc["mu"], sc["kappa"], sc["eps_r"]
    I = 0.4 * m * r * r
    f = m * g * h / 4.0
    pen = 0.0
    for _ in range(100):
        rho = r - pen / 2
        Aee = (1 + mu * mu) / m + mu * mu * rho * rho / I
        pen = er * Aee * f * h / kap
    return pen


def test_drop_comes_to_rest_at_closed_form_depth(oracle_mod):
    # many sweeps: the four pyramid rows have a near-null direction (x pair
    # minus y pair cancels in force and torque) that only R regularises, so
    # Gauss-Seidel converges slowly there; the closed form assumes convergence
    sc = W.make_scene(2, n_pgs=3000)
    o = oracle_mod.Oracle(sc)
    x = far_ball_state(sc, [0.0, 0.6, 0.3])
    u = np.zeros(14)
    for _ in range(1500):
        x, _ = o.substep(x, u)
    pen = _rest_penetration(sc)
    assert x[44] == pytest.approx(sc["ball_r"] - pen, abs=1e-10)
    assert np.allclose(x[49:55], 0.0, atol=1e-9)
    assert np.allclose(x[42:44], [0.0, 0.6], atol=1e-12)


def test_sliding_ball_rolls_at_five_sevenths(oracle_mod):
    sc = W.make_scene(2, n_pgs=3000)
    o = oracle_mod.Oracle(sc)
    pen = _rest_penetration(sc)
    v0 = 0.5
    x = far_ball_state(sc, [0.0, 0.6, sc["ball_r"] - pen], v=[v0, 0, 0])
    u = np.zeros(14)
    for _ in range(250):
        x, _ = o.substep(x, u)
    vx, wy = x[49], x[53]
    assert vx == pytest.approx(5.0 / 7.0 * v0, rel=2e-3)
    rho = sc["ball_r"] - pen / 2
    assert vx == pytest.approx(wy * rho, rel=1e-6)   # rolling without slip at the contact point
    assert abs(x[50]) < 1e-12 and abs(x[52]) < 1e-12


def _arm_energy(o, x, md, sc):
    E = 0.0
    for a in range(2):
        q, qd = x[7 * a:7 * a + 7], x[14 + 7 * a:21 + 7 * a]
        M = o.mass_matrix(a, q) + sc["armature"] * np.eye(7)
        _, _, _, c = o.fk(a, q)
        E += 0.5 * qd @ M @ qd + sc["g"] * np.sum(md["m"][a] * c[:, 2])
    return E


def test_energy_error_first_order_without_contacts(oracle_mod):
    """Contacts, damping and actuation off, gravity on: the energy error of the
    semi-implicit step over a fixed time halves when h halves."""
    devs = []
    for h in (1e-3, 5e-4):
        sc = W.make_scene(2, h=h, kp=0.0, kd=0.0, damp=0.0, gravcomp=0, n_cmax=0)
        o = oracle_mod.Oracle(sc)
        md = o.model()
        x = W.initial_state(sc)
        rng = np.random.default_rng(7)
        x[0:14] += rng.uniform(-0.5, 0.5, 14)
        x[14:28] = rng.uniform(-1.0, 1.0, 14)
        x[28:42] = x[0:14]
        E0 = _arm_energy(o, x, md, sc)
        dev = 0.0
        for _ in range(int(round(0.4 / h))):
            x, _ = o.substep(x, np.zeros(14))
            dev = max(dev, abs(_arm_energy(o, x, md, sc) - E0))
        devs.append(dev)
    assert devs[0] / devs[1] == pytest.approx(2.0, rel=0.15)
    assert devs[0] < 0.05 * abs(E0)


def _lcp_exact(A, b):
    """Unique solution of f >= 0, A f + b >= 0, f.(A f + b) = 0 (A SPD) by
    enumerating active sets."""
    m = len(b)
    for mask in itertools.product([0, 1], repeat=m):
        S = [i for i in range(m) if mask[i]]
        f = np.zeros(m)
        if S:
            f[S] = np.linalg.solve(A[np.ix_(S, S)], -b[S])
        w = A @ f + b
        if np.all(f >= -1e-12) and np.all(w >= -1e-10):
            return f
    raise AssertionError("no LCP solution")


def test_pgs_converges_to_exact_lcp(oracle_mod):
    sc = W.make_scene(1, n_pgs=3000)
    o = oracle_mod.Oracle(sc)
    x = W.initial_state(sc)
    x[44] = 0.095                        # ball pressed into the table
    x[0:7] += [0, 0.35, 0, 0.2, 0, 0.25, 0]  # arm 1 pushes its pad into the ball
    x[14:28] = 0.3
    A, b, f, vf = o.lcp(x, np.full(14, 0.5))
    m = len(b)
    assert 8 <= m <= 12
    AR = A + np.diag(sc["eps_r"] * np.diag(A))
    assert np.allclose(A, A.T, atol=1e-12)
    assert np.linalg.eigvalsh(AR).min() > 0
    fx = _lcp_exact(AR, b)
    assert np.allclose(f, fx, rtol=1e-6, atol=1e-9)
    w = AR @ f + b
    assert np.all(f >= 0) and np.all(w >= -1e-8) and abs(f @ w) < 1e-9
