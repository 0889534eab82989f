"""Oracle pins for the actuated substep and the contact-point Jacobian.

The world model of Eq. state_evol is a reading (PD actuators on an
integrated position target, linearly implicit damping, four pyramid-edge
rows per contact).  These tests rebuild one contact-free substep from pieces
that are pinned elsewhere by other means -- the mass matrix as the Hessian of
the kinetic energy computed from finite differences of the kinematics, the
bias forces from the inverse dynamics (pinned against the potential gradient
and Lagrange's equations), numpy's dense solve -- and check the Jacobian of
a point fixed to each body against the finite-difference velocity of that
point.  A sign error in the damping terms, the position target advanced at
the wrong time, a dropped torque clamp, a missing diagonal term, a wrong
link range in the arm Jacobian or a wrong side of a contact pair each fail
one of them.
"""
import numpy as np
import pytest

import workloads as W


def _kinetic(o, arm, q, qd, md, eps=1e-6):
    """T = 1/2 sum (m |v_c|^2 + w^T I w) with velocities from central
    differences of the forward kinematics along qd."""
    Rp, _, _, cp = o.fk(arm, q + eps * qd)
    Rm, _, _, cm = o.fk(arm, q - eps * qd)
    R0, _, _, _ = o.fk(arm, q)
    T = 0.0
    for i in range(7):
        v = (cp[i] - cm[i]) / (2 * eps)
        W_ = ((Rp[i] - Rm[i]) / (2 * eps)) @ R0[i].T
        w = np.array([W_[2, 1], W_[0, 2], W_[1, 0]])
        Ib = np.diag([md["Ix"][arm][i], md["Ix"][arm][i], md["Iz"][arm][i]])
        T += 0.5 * (md["m"][arm][i] * v @ v + w @ (R0[i] @ Ib @ R0[i].T) @ w)
    return T


def _mass_from_energy(o, arm, q, md):
    E = np.eye(7)
    M = np.zeros((7, 7))
    Ti = [_kinetic(o, arm, q, E[i], md) for i in range(7)]
    for i in range(7):
        M[i, i] = 2 * Ti[i]
        for j in range(i):
            M[i, j] = M[j, i] = _kinetic(o, arm, q, E[i] + E[j], md) - Ti[i] - Ti[j]
    return M


def _expected_substep(o, sc, md, x, u):
    """One contact-free substep of the arms, assembled independently:
    q_des' = q_des + h u; tau = clamp(Kp (q_des' - q) + Kd (u - qd), +-tau_max);
    (M + diag(a + h (Kd + b))) dqd = h (tau - b qd - c); q' = q + h (qd + dqd)."""
    h = sc["h"]
    q, qd, qdes = x[0:14], x[14:28], x[28:42]
    qdes_n = qdes + h * u
    qn, qdn = np.zeros(14), np.zeros(14)
    for a in range(2):
        s = slice(7 * a, 7 * a + 7)
        M = _mass_from_energy(o, a, q[s], md)
        c = o.rnea(a, q[s], qd[s], np.zeros(7), gravity=0 if sc["gravcomp"] else 1)
        tau = np.clip(sc["kp"] * (qdes_n[s] - q[s]) + sc["kd"] * (u[s] - qd[s]), -sc["tau_max"], sc["tau_max"])
        Mt = M + np.diag(np.full(7, sc["armature"] + h * (sc["kd"] + sc["damp"])))
        dqd = np.linalg.solve(Mt, h * (tau - sc["damp"] * qd[s] - c))
        qdn[s] = qd[s] + dqd
        qn[s] = q[s] + h * qdn[s]
    return qn, qdn, qdes_n


def _free_arm_state(sc, rng, sat=False):
    x = W.initial_state(sc)
    x[42:45] = [0.0, 2.0, 1.5]            # ball far from everything
    x[0:14] = np.asarray(sc["q_home"]) + rng.uniform(-0.3, 0.3, 14)
    x[14:28] = rng.uniform(-1.0, 1.0, 14)
    x[28:42] = x[0:14] + rng.uniform(-0.05, 0.05, 14)
    if sat:  # position errors of +-2 rad: Kp e = 200 N m exceeds tau_max on these joints
        x[28:42][[1, 3, 8, 12]] = x[0:14][[1, 3, 8, 12]] + np.array([2.0, -2.0, 2.0, -2.0])
    return x


@pytest.mark.parametrize("cfg,gravcomp,sat", [(1, 1, False), (1, 0, False), (2, 0, False), (1, 1, True),
                                              (2, 1, True)])
def test_pd_substep_against_independent_solve(oracle_mod, cfg, gravcomp, sat):
    sc = W.make_scene(cfg, gravcomp=gravcomp, n_cmax=0)
    o = oracle_mod.Oracle(sc)
    md = o.model()
    rng = np.random.default_rng(10 + cfg + 2 * gravcomp + 4 * sat)
    for _ in range(3):
        x = _free_arm_state(sc, rng, sat)
        u = rng.uniform(-1.5, 1.5, 14)
        if sat:
            tau = sc["kp"] * (x[28:42] + sc["h"] * u - x[0:14]) + sc["kd"] * (u - x[14:28])
            assert np.sum(np.abs(tau) > sc["tau_max"]) >= 4
        xn, nc = o.substep(x, u)
        assert nc == 0
        qn, qdn, qdesn = _expected_substep(o, sc, md, x, u)
        assert np.array_equal(xn[28:42], qdesn)
        # the energy Hessian is accurate to ~1e-7 relative; the step itself is
        # O(h tau / M) ~ 1e-2..1, so these bounds see every term
        assert np.allclose(xn[14:28], qdn, rtol=0, atol=2e-6), np.abs(xn[14:28] - qdn).max()
        assert np.allclose(xn[0:14], qn, rtol=0, atol=2e-8)


def test_pd_terms_are_visible(oracle_mod):
    """The bounds above resolve each term: perturbing one reading of the
    actuator by the planted mistakes it guards against moves qd' by far more
    than the tolerance."""
    sc = W.make_scene(1, gravcomp=1, n_cmax=0)
    o = oracle_mod.Oracle(sc)
    md = o.model()
    rng = np.random.default_rng(3)
    x = _free_arm_state(sc, rng)
    u = rng.uniform(-1.5, 1.5, 14)
    h = sc["h"]
    q, qd, qdes = x[0:14], x[14:28], x[28:42]
    base = _expected_substep(o, sc, md, x, u)[1]
    # the position target advanced after the torque: the Kp h u term missing
    M = _mass_from_energy(o, 0, q[:7], md) + np.diag(np.full(7, sc["armature"] + h * (sc["kd"] + sc["damp"])))
    d_late = np.linalg.solve(M, h * sc["kp"] * h * u[:7])
    assert np.abs(d_late).max() > 100 * 2e-6
    # a flipped Kd sign changes the torque by 2 Kd (u - qd)
    d_kd = np.linalg.solve(M, h * 2 * sc["kd"] * (u[:7] - qd[:7]))
    assert np.abs(d_kd).max() > 100 * 2e-6
    assert np.isfinite(base).all()


def _rodrigues(w, t):
    th = np.linalg.norm(w) * t
    if th == 0:
        return np.eye(3)
    k = w / np.linalg.norm(w)
    Kx = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(th) * Kx + (1 - np.cos(th)) * Kx @ Kx


def _point_velocity_fd(o, x, vel, gid, p, eps=1e-6):
    """Velocity of the point p rigidly attached to geom gid when the state
    moves with generalised velocity vel (20: arm joints, ball v, ball w), by
    central differences of the body's pose (arm geom g rides on link g, the
    pad (g = 6) on the last link; the ball rotates about its centre)."""
    if gid == 0:
        c = x[42:45]
        r = p - c
        pp = c + eps * vel[14:17] + _rodrigues(vel[17:20], eps) @ r
        pm = c - eps * vel[14:17] + _rodrigues(vel[17:20], -eps) @ r
        return (pp - pm) / (2 * eps)
    if 2 <= gid < 16:
        arm, g = (gid - 2) // 7, (gid - 2) % 7
        q = x[7 * arm:7 * arm + 7]
        qd = vel[7 * arm:7 * arm + 7]
        R0, o0, _, _ = o.fk(arm, q)
        loc = R0[g].T @ (p - o0[g])
        Rp, op, _, _ = o.fk(arm, q + eps * qd)
        Rm, om, _, _ = o.fk(arm, q - eps * qd)
        return ((op[g] + Rp[g] @ loc) - (om[g] + Rm[g] @ loc)) / (2 * eps)
    return np.zeros(3)  # table and boxes are static


def test_point_jacobian_matches_fd_velocity(oracle_mod):
    sc = W.make_scene(2)
    o = oracle_mod.Oracle(sc)
    rng = np.random.default_rng(21)
    for _ in range(4):
        x = W.initial_state(sc)
        x[0:14] = rng.uniform(-1.5, 1.5, 14)
        x[45:49] = rng.normal(size=4)
        x[45:49] /= np.linalg.norm(x[45:49])
        vel = rng.uniform(-1.0, 1.0, 20)
        for gid in [0] + list(range(2, 16)):
            p = rng.uniform(-0.8, 0.8, 3) + np.array([0, 0, 0.4])
            J = o.point_jac(x, gid, p)
            v_fd = _point_velocity_fd(o, x, vel, gid, p)
            assert np.allclose(J @ vel, v_fd, rtol=0, atol=1e-8), (gid, J @ vel, v_fd)
            # only the body's own coordinates move the point
            if gid == 0:
                assert np.all(J[:, :14] == 0)
            else:
                arm, g = (gid - 2) // 7, (gid - 2) % 7
                cols = [7 * arm + j for j in range(g + 1)]
                mask = np.ones(20, bool)
                mask[cols] = False
                assert np.all(J[:, mask] == 0)
        for gid in (1, 16, 18):
            assert np.all(o.point_jac(x, gid, rng.uniform(-1, 1, 3)) == 0)


def _contact_states(sc, o, rng, want, tries=4000):
    """Random arm configurations (and a pressed ball) whose contact lists hold
    the pair kinds in `want` (names of the canonical pair groups)."""
    ga, gb = o.pairs()
    found = {}
    for _ in range(tries):
        x = W.initial_state(sc)
        x[0:14] = np.asarray(sc["q_home"]) + rng.uniform(-1.2, 1.2, 14)
        x[44] = sc["ball_r"] - 0.004
        pair, phi, n, p = o.contacts(x)
        for c in range(len(pair)):
            a, b = ga[pair[c]], gb[pair[c]]
            kind = ("ball" if a == 0 else "arm") + "-" + (
                "table" if b == 1 else "box" if b >= 16 else "ball" if b == 0 else "arm")
            if kind in want and kind not in found:
                found[kind] = x.copy()
        if len(found) == len(want):
            break
    return found


def test_contact_rows_are_relative_velocity_along_edges(oracle_mod):
    """Each contact's four rows are e_r . (v_A(p) - v_B(p)) at the free
    velocity minus the Baumgarte bias: their sum is 4 n . dv - 4 kappa pen / h
    and their differences 2 mu t . dv, with dv from finite differences of the
    two bodies' poses (A is the first geom of the canonical pair)."""
    sc = W.make_scene(2, n_cmax=16)
    o = oracle_mod.Oracle(sc)
    ga, gb = o.pairs()
    rng = np.random.default_rng(5)
    states = _contact_states(sc, o, rng, {"ball-table", "arm-ball", "arm-table", "arm-box", "arm-arm"})
    assert {"ball-table", "arm-box", "arm-arm"} <= set(states), sorted(states)
    h, kap, mu = sc["h"], sc["kappa"], sc["mu"]
    n_checked = 0
    for kind, x in states.items():
        x = x.copy()
        x[14:28] = rng.uniform(-1.0, 1.0, 14)
        x[49:55] = rng.uniform(-0.5, 0.5, 6)
        u = rng.uniform(-1.0, 1.0, 14)
        A, b, f, vf = o.lcp(x, u)
        pair, phi, n, p = o.contacts(x, cap=16)
        assert len(b) == 4 * len(pair)
        for c in range(len(pair)):
            dv = _point_velocity_fd(o, x, vf, ga[pair[c]], p[c]) - _point_velocity_fd(o, x, vf, gb[pair[c]], p[c])
            t1, t2 = o.tangents(n[c])
            pen = max(-phi[c], 0.0)
            rows = b[4 * c:4 * c + 4]
            assert rows.sum() == pytest.approx(4 * n[c] @ dv - 4 * kap * pen / h, abs=1e-7)
            assert rows[0] - rows[1] == pytest.approx(2 * mu * t1 @ dv, abs=1e-7)
            assert rows[2] - rows[3] == pytest.approx(2 * mu * t2 @ dv, abs=1e-7)
            n_checked += 1
    assert n_checked >= 5
