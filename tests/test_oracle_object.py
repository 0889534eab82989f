"""Oracle pins for the box-shaped free object (the tray of Sec. IV-A, the cube
of Sec. IV-C) and the further task-cost terms of Sec. IV: the box's inertia
against grid integration, quaternion conversions, the box's narrowphase
against brute force (dense sampling and bounded least squares), the
separating-axis depth against a search over many directions, the
gyroscopic step against torque-free rigid-body invariants, a box coming to
rest flat on the table, and each further cost term on hand-built states.
"""
import math

import numpy as np
import pytest
from scipy.optimize import lsq_linear, minimize
from scipy.spatial.transform import Rotation

import workloads as W


def _quat(rot):
    x, y, z, w = rot.as_quat()
    return np.array([w, x, y, z])


def _R(q):
    return Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()


@pytest.fixture(scope="module")
def tray(oracle_mod):
    return oracle_mod.Oracle(W.task_scene("tray", "pick"))


def test_box_inertia_numeric(oracle_mod):
    sc = W.task_scene("tray", "pick")
    o = oracle_mod.Oracle(sc)
    # the model's principal inertias through the rest of the model: a spin
    # about body axis i has energy I_i w^2 / 2; compare with a grid integral
    h, m = np.array(sc["obj_h"]), sc["ball_m"]
    n = 60
    g = [(np.arange(n) + 0.5) / n * 2 * h[i] - h[i] for i in range(3)]
    X, Y, Z = np.meshgrid(*g, indexing="ij")
    rho = m / (8 * h.prod())
    dv = 8 * h.prod() / n ** 3
    I_num = rho * dv * np.array([np.sum(Y ** 2 + Z ** 2), np.sum(X ** 2 + Z ** 2), np.sum(X ** 2 + Y ** 2)])
    # free spin about each body axis from the identity pose: the angular
    # velocity is unchanged (principal axis) and an impulse-free step keeps it
    x = W.initial_state(sc)
    x[42:45] = [0.0, 2.0, 2.0]
    for i in range(3):
        xx = x.copy()
        xx[52 + i] = 3.0
        xn, _ = o.substep(xx, np.zeros(14))
        assert np.allclose(xn[52:55], xx[52:55], atol=1e-14)
    # the grid integral against the closed form the oracle uses (m (b^2 + c^2) / 3 for half extents)
    I_cf = m / 3 * np.array([h[1] ** 2 + h[2] ** 2, h[0] ** 2 + h[2] ** 2, h[0] ** 2 + h[1] ** 2])
    assert np.allclose(I_num, I_cf, rtol=2e-3)


def test_quaternion_round_trip(oracle_mod):
    rng = np.random.default_rng(1)
    for _ in range(50):
        q = rng.normal(size=4)
        q /= np.linalg.norm(q)
        R, qb = oracle_mod.Oracle.quat_R(q)
        assert np.allclose(R, _R(q), atol=1e-14)
        assert np.allclose(R @ R.T, np.eye(3), atol=1e-14) and np.isclose(np.linalg.det(R), 1.0)
        assert np.allclose(qb * np.sign(qb @ q), q, atol=1e-13)


def _box_frame(xo):
    return np.asarray(xo[:3]), _R(xo[3:7])


def _box_sd_brute(xo, h, p):
    """Signed distance of point p to the oriented box: outside by bounded least
    squares in the box frame, inside the least face distance."""
    c, R = _box_frame(xo)
    l = R.T @ (p - c)
    if np.all(np.abs(l) <= h):
        return -np.min(h - np.abs(l))
    r = lsq_linear(np.eye(3), l, bounds=(-h, h))
    return np.linalg.norm(l - r.x)


def _random_pose(rng, c_spread=0.0):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    return np.concatenate([rng.uniform(-c_spread, c_spread, 3), q])


def test_box_object_against_sphere_and_capsule(tray):
    h = np.array(tray.scene["obj_h"])
    rng = np.random.default_rng(2)
    for _ in range(40):
        xo = _random_pose(rng, 0.1)
        # sphere
        x = xo[:3] + rng.uniform(-0.2, 0.2, 3)
        r = 0.04
        phi, n, p = tray.obj_prim(xo, 0, x, x, r)
        assert phi == pytest.approx(_box_sd_brute(xo, h, x) - r, abs=1e-9)
        # the normal points from the sphere towards the box, the point sits between the surfaces
        assert np.linalg.norm(n) == pytest.approx(1.0)
        if phi > 1e-3:
            assert n @ (xo[:3] - x) > 0
        # capsule: the least signed distance over the segment, by a fine scan plus refinement
        a, b = xo[:3] + rng.uniform(-0.3, 0.3, 3), xo[:3] + rng.uniform(-0.3, 0.3, 3)
        ts = np.linspace(0, 1, 2001)
        sd = [_box_sd_brute(xo, h, a + t * (b - a)) for t in ts[::50]]
        t0 = ts[::50][int(np.argmin(sd))]
        res = minimize(lambda t: _box_sd_brute(xo, h, a + float(np.clip(t[0], 0, 1)) * (b - a)), [t0],
                       method="Nelder-Mead", options=dict(xatol=1e-10, fatol=1e-12))
        best = min(min(sd), res.fun)
        phi_c, _, _ = tray.obj_prim(xo, 1, a, b, 0.05)
        assert phi_c == pytest.approx(best - 0.05, abs=2e-6)


def test_box_object_against_table_vertices(tray):
    h = np.array(tray.scene["obj_h"])
    rng = np.random.default_rng(3)
    for _ in range(20):
        xo = _random_pose(rng, 0.05)
        c, R = _box_frame(xo)
        verts = [c + R @ (np.array([1 if k & 1 else -1, 1 if k & 2 else -1, 1 if k & 4 else -1]) * h)
                 for k in range(8)]
        low = min(verts, key=lambda v: v[2])
        phi, n, p = tray.obj_prim(xo, 2, np.zeros(3))
        assert phi == pytest.approx(low[2], abs=1e-14)
        assert np.allclose(n, [0, 0, 1]) and np.allclose(p, [low[0], low[1], 0.5 * low[2]], atol=1e-14)


def test_box_object_against_static_box_separating_axes(tray):
    """Overlapping boxes: phi is minus the least overlap over every direction
    (20000 random directions never go below the separating-axis value, and a
    local search from the best of them reaches it); apart: 0 < phi <= the
    boxes' true distance (a small QP)."""
    h = np.array(tray.scene["obj_h"])
    rng = np.random.default_rng(4)
    dirs = rng.normal(size=(20000, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    n_over = n_apart = 0
    for _ in range(30):
        xo = _random_pose(rng, 0.0)
        cb = rng.uniform(-0.3, 0.3, 3)
        hb = rng.uniform(0.05, 0.15, 3)
        phi, n, p = tray.obj_prim(xo, 3, cb, hb)
        R = _R(xo[3:])
        d = xo[:3] - cb
        overlap = (np.abs(dirs @ R) @ h) + (np.abs(dirs) @ hb) - np.abs(dirs @ d)
        assert n @ d >= -1e-12  # turned towards the object
        if phi < 0:
            n_over += 1
            assert overlap.min() >= -phi - 1e-12

            def ov(v):
                v = v / np.linalg.norm(v)
                return np.abs(v @ R) @ h + np.abs(v) @ hb - abs(v @ d)
            best = min(minimize(ov, dirs[i], method="Nelder-Mead",
                                options=dict(xatol=1e-12, fatol=1e-14, maxiter=4000)).fun
                       for i in np.argsort(overlap)[:20])
            assert -phi - 1e-12 <= best <= -phi + 1e-7
        else:
            n_apart += 1
            # true distance: min |a - b| with a in the object, b in the box
            def f(z):
                a = xo[:3] + R @ z[:3]
                return np.sum((a - z[3:]) ** 2)
            res = minimize(f, np.concatenate([np.zeros(3), cb]), method="L-BFGS-B",
                           bounds=[(-h[i], h[i]) for i in range(3)] + [(cb[i] - hb[i], cb[i] + hb[i]) for i in range(3)])
            assert 0 <= phi <= math.sqrt(res.fun) + 1e-6
    assert n_over >= 5 and n_apart >= 5


def _box_state(sc, p, q, v=(0, 0, 0), w=(0, 0, 0)):
    x = W.initial_state(sc)
    x[42:45], x[45:49], x[49:52], x[52:55] = p, q, v, w
    return x


def _momentum(sc, md_I, x):
    R = _R(x[45:49])
    return R @ np.diag(md_I) @ R.T @ x[52:55]


def test_gyroscopic_step_conserves_momentum_to_first_order(oracle_mod):
    """Torque-free spin of the box in free flight: the world angular momentum
    R I R^T w drifts only by the explicit step's error, which halves with h
    (first order); energy likewise; the centre follows the ballistic closed form."""
    drifts = []
    for h in (1e-3, 5e-4):
        sc = W.task_scene("tray", "pick", h=h, n_cmax=0)
        o = oracle_mod.Oracle(sc)
        hh, m = np.array(sc["obj_h"]), sc["ball_m"]
        I = m / 3 * np.array([hh[1] ** 2 + hh[2] ** 2, hh[0] ** 2 + hh[2] ** 2, hh[0] ** 2 + hh[1] ** 2])
        x = _box_state(sc, [0.0, 2.0, 5.0], [1.0, 0, 0, 0], w=[2.0, 0.3, 1.0])
        L0 = _momentum(sc, I, x)
        E0 = 0.5 * x[52:55] @ _R(x[45:49]) @ np.diag(I) @ _R(x[45:49]).T @ x[52:55]
        dL = dE = 0.0
        for _ in range(int(round(0.2 / h))):
            x, nc = o.substep(x, np.zeros(14))
            assert nc == 0
            dL = max(dL, np.linalg.norm(_momentum(sc, I, x) - L0))
            R = _R(x[45:49])
            dE = max(dE, abs(0.5 * x[52:55] @ R @ np.diag(I) @ R.T @ x[52:55] - E0))
        drifts.append((dL, dE))
    assert drifts[0][0] / drifts[1][0] == pytest.approx(2.0, rel=0.15)
    assert drifts[0][0] < 0.05 * np.linalg.norm(L0)


def test_box_comes_to_rest_flat_on_the_table(oracle_mod):
    sc = W.task_scene("tray", "pick", n_pgs=200)
    o = oracle_mod.Oracle(sc)
    hh = np.array(sc["obj_h"])
    x = _box_state(sc, [0.0, 0.6, hh[2] + 0.02], [1.0, 0, 0, 0])
    ncs = []
    for _ in range(1500):
        x, nc = o.substep(x, np.zeros(14))
        ncs.append(nc)
    assert ncs[-1] == 4                              # four bottom vertices
    assert np.all(np.abs(x[49:55]) < 1e-5)           # at rest (from 0.6 m/s at impact)
    assert np.allclose(x[45:49], [1, 0, 0, 0], atol=1e-5)  # level
    assert hh[2] - 2e-3 < x[44] < hh[2]
    assert np.allclose(x[42:44], [0.0, 0.6], atol=1e-5)


def test_further_cost_terms_worked(oracle_mod):
    """Terms 7..16 on hand-built states: joint deviation, vertical alignment,
    the relative-velocity summand (pad velocities by finite differences of
    the kinematics), per-arm position and x targets, and the orientation
    terms against targets rotated by known angles."""
    sc = W.task_scene("tray", "pick")
    rng = np.random.default_rng(5)
    x = W.initial_state(sc)
    x[0:14] = np.asarray(sc["q_home"]) + rng.uniform(-0.4, 0.4, 14)
    x[14:28] = rng.uniform(-1, 1, 14)
    o0 = oracle_mod.Oracle(sc)
    R1, org1, _, _ = o0.fk(0, x[0:7])
    R2, org2, _, _ = o0.fk(1, x[7:14])
    p = [org1[7], org2[7]]
    Rp = [R1[6], R2[6]]
    alpha = [0.7, 2.3]
    axis = [np.array([1.0, 2.0, -0.5]), np.array([-0.3, 0.1, 1.0])]
    targets = []
    for a in range(2):
        qa = _quat(Rotation.from_matrix(Rp[a]) * Rotation.from_rotvec(alpha[a] * axis[a] / np.linalg.norm(axis[a])))
        targets.append(qa)
    q_obj = np.array([0.9, 0.1, -0.3, 0.2])
    q_obj /= np.linalg.norm(q_obj)
    x[45:49] = q_obj
    orot = _quat(Rotation.from_quat([q_obj[1], q_obj[2], q_obj[3], q_obj[0]]) * Rotation.from_rotvec([0, 0.4, 0]))
    apos = np.array([[0.1, 0.2, 0.3], [-0.2, 0.1, 0.05]])
    sc.update(apos=apos, ax_t=np.array([0.05, -0.1]), arot=np.array(targets), orot=orot)
    o = oracle_mod.Oracle(sc)
    t = o.ext_terms(x)
    assert t[0] == pytest.approx(np.linalg.norm(x[0:14] - sc["q_home"]), rel=1e-14)
    assert t[1] == pytest.approx(abs(p[0][2] - p[1][2]), rel=1e-14)
    eps = 1e-6
    v = []
    for a in range(2):
        q, qd = x[7 * a:7 * a + 7], x[14 + 7 * a:21 + 7 * a]
        v.append((o.fk(a, q + eps * qd)[1][7] - o.fk(a, q - eps * qd)[1][7]) / (2 * eps))
    assert t[2] == pytest.approx(((p[0] - p[1]) @ (v[0] - v[1])) ** 2, rel=1e-6)
    for a in range(2):
        assert t[3 + a] == pytest.approx(np.linalg.norm(p[a] - apos[a]), rel=1e-14)
        assert t[5 + a] == pytest.approx(abs(p[a][0] - sc["ax_t"][a]), rel=1e-14)
        assert t[7 + a] == pytest.approx(alpha[a], abs=1e-9)
    assert t[9] == pytest.approx(0.4, abs=1e-9)


def test_rollout_total_with_further_terms(oracle_mod):
    """The rollout's total is the weighted sum of all 17 terms, term 9 the root
    of its summed squares; with ext off terms 7..16 stay zero."""
    sc = W.task_scene("handover", "pass")
    o = oracle_mod.Oracle(sc)
    x0 = W.initial_state(sc)
    U = np.random.default_rng(6).uniform(-0.5, 0.5, (4, 14))
    c, terms, traj = o.rollout(x0, U, want_traj=True)
    summ = sum(o.ext_terms(traj[k])[2] for k in range(4))
    assert terms[9] == pytest.approx(math.sqrt(summ), rel=1e-12)
    for i, j in ((7, 0), (8, 1), (12, 5), (13, 6), (14, 7), (15, 8), (16, 9)):
        assert terms[i] == pytest.approx(sum(o.ext_terms(traj[k])[j] for k in range(4)), rel=1e-12)
    w = [sc["w_goal"], sc["w_eo"], sc["w_l"], sc["w_yz"], sc["w_s"], sc["w_c"], sc["w_c"], sc["w_home"],
         sc["w_vert"], sc["w_relv"], *sc["w_apos"], *sc["w_ax"], *sc["w_arot"], sc["w_orot"]]
    assert c == pytest.approx(float(np.dot(w, terms)), rel=1e-13)
    off = oracle_mod.Oracle(dict(sc, ext=0))
    _, t0 = off.rollout(x0, U)
    assert np.all(t0[7:] == 0)
