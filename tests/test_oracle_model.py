"""Oracle pins: kinematics, link inertias, mass matrix and inverse dynamics.

The paper's world model is MuJoCo (Eq. state_evol, Sec. V-A); the arm model
is a reading.  Each oracle function is pinned to something other than
itself: closed-form poses, numeric integration of the capsule, the kinetic
energy Hessian, the potential-energy gradient and Lagrange's equations.
"""
import numpy as np
import pytest

import workloads as W


@pytest.fixture(scope="module")
def o(oracle_mod):
    return oracle_mod.Oracle(W.make_scene(2))


def test_fk_straight_and_planar(o):
    sc = o.scene
    L = sc["link_len"]
    R, org, a, c = o.fk(0, np.zeros(7))
    assert np.allclose(org[-1], [-0.55, 0, L.sum()], atol=1e-14)
    # only the pitch joints (local y) non-zero: planar chain in the xz plane
    q = np.array([0, 0.3, 0, -0.7, 0, 0.4, 0])
    R, org, a, c = o.fk(0, q)
    ang = np.cumsum(q)  # pitch angles accumulate (joints 2, 4, 6)
    p = np.array([-0.55, 0.0, 0.0])
    for i in range(7):
        p = p + L[i] * np.array([np.sin(ang[i]), 0.0, np.cos(ang[i])])
        assert np.allclose(org[i + 1], p, atol=1e-14)
    # arm 2 is arm 1 mirrored through x = 0 (base yaw pi) for identical q
    q = np.array([0.2, 0.5, -0.3, 1.1, 0.4, -0.6, 0.9])
    _, o0, _, _ = o.fk(0, q)
    _, o1, _, _ = o.fk(1, q)
    assert np.allclose(o1[:, 0], -o0[:, 0]) and np.allclose(o1[:, 1], -o0[:, 1]) and np.allclose(o1[:, 2], o0[:, 2])


def test_fk_rotations_orthonormal_and_lengths(o):
    rng = np.random.default_rng(1)
    for _ in range(5):
        q = rng.uniform(-np.pi, np.pi, 7)
        R, org, a, c = o.fk(1, q)
        for i in range(7):
            assert np.allclose(R[i] @ R[i].T, np.eye(3), atol=1e-13)
            assert np.isclose(np.linalg.det(R[i]), 1.0)
            assert np.isclose(np.linalg.norm(org[i + 1] - org[i]), o.scene["link_len"][i])
            assert np.allclose(c[i], 0.5 * (org[i] + org[i + 1]))
            assert np.isclose(np.linalg.norm(a[i]), 1.0)


def _capsule_grid(rho, L, r, n=160):
    """Brute force: midpoint grid over the capsule's box, count cells inside."""
    xs = (np.arange(n) + 0.5) / n * 2 * r - r
    zs = (np.arange(3 * n) + 0.5) / (3 * n) * (L + 2 * r) - r
    X, Y, Z = np.meshgrid(xs, xs, zs, indexing="ij")
    Zc = np.clip(Z, 0, L)
    inside = X ** 2 + Y ** 2 + (Z - Zc) ** 2 <= r * r
    dv = (2 * r / n) ** 2 * ((L + 2 * r) / (3 * n))
    m = rho * inside.sum() * dv
    zc = Z - L / 2
    Ix = rho * dv * np.sum(inside * (Y ** 2 + zc ** 2))
    Iz = rho * dv * np.sum(inside * (X ** 2 + Y ** 2))
    return m, Ix, Iz


def test_capsule_inertia_numeric(o):
    md = o.model()
    for i in (1, 6):
        m, Ix, Iz = _capsule_grid(o.scene["density"][0][i], o.scene["link_len"][i], o.scene["link_rad"][i])
        assert np.isclose(md["m"][0][i], m, rtol=3e-3)
        assert np.isclose(md["Ix"][0][i], Ix, rtol=5e-3)
        assert np.isclose(md["Iz"][0][i], Iz, rtol=5e-3)
    r, mb = o.scene["ball_r"], o.scene["ball_m"]
    assert np.isclose(md["ball_I"], 0.4 * mb * r * r)


def _kinetic(o, arm, q, qd, md, eps=1e-6):
    """T = 1/2 sum (m |v_c|^2 + w^T I w), velocities from finite differences of FK."""
    Rp, _, _, cp = o.fk(arm, q + eps * qd)
    Rm, _, _, cm = o.fk(arm, q - eps * qd)
    R0, _, _, _ = o.fk(arm, q)
    T = 0.0
    for i in range(7):
        v = (cp[i] - cm[i]) / (2 * eps)
        Rd = (Rp[i] - Rm[i]) / (2 * eps)
        W = Rd @ R0[i].T
        w = np.array([W[2, 1], W[0, 2], W[1, 0]])
        Ib = np.diag([md["Ix"][arm][i], md["Ix"][arm][i], md["Iz"][arm][i]])
        Iw = R0[i] @ Ib @ R0[i].T
        T += 0.5 * (md["m"][arm][i] * v @ v + w @ Iw @ w)
    return T


def test_mass_matrix_is_kinetic_energy_hessian(o):
    md = o.model()
    rng = np.random.default_rng(2)
    for arm in (0, 1):
        q = rng.uniform(-2, 2, 7)
        M = o.mass_matrix(arm, q)
        E = np.eye(7)
        Mh = np.zeros((7, 7))
        for i in range(7):
            Mh[i, i] = 2 * _kinetic(o, arm, q, E[i], md)
            for j in range(i):
                v = _kinetic(o, arm, q, E[i] + E[j], md) - _kinetic(o, arm, q, E[i], md) - _kinetic(o, arm, q, E[j], md)
                Mh[i, j] = Mh[j, i] = v
        assert np.allclose(M, M.T, atol=1e-15)
        assert np.allclose(M, Mh, rtol=1e-6, atol=1e-9)
        assert np.linalg.eigvalsh(M).min() > 0.0


def test_gravity_torque_is_potential_gradient(o):
    md = o.model()
    g = o.scene["g"]

    def V(q):
        _, _, _, c = o.fk(0, q)
        return g * np.sum(md["m"][0] * c[:, 2])

    q = np.array([0.3, -0.4, 0.8, 1.2, -0.5, 0.7, 0.1])
    tau = o.rnea(0, q, np.zeros(7), np.zeros(7), gravity=1)
    eps = 1e-6
    grad = np.array([(V(q + eps * e) - V(q - eps * e)) / (2 * eps) for e in np.eye(7)])
    assert np.allclose(tau, grad, rtol=1e-6, atol=1e-8)


def test_rnea_acceleration_part_is_mass_matrix(o):
    q = np.array([-0.2, 0.9, 0.1, -1.0, 0.6, 0.3, -0.8])
    M = o.mass_matrix(1, q)
    for j in range(7):
        col = o.rnea(1, q, np.zeros(7), np.eye(7)[j], gravity=0)
        assert np.allclose(col, M[:, j], rtol=1e-12, atol=1e-14)


def test_rnea_round_trip(o):
    rng = np.random.default_rng(3)
    q, qd, qdd = rng.uniform(-2, 2, 7), rng.uniform(-2, 2, 7), rng.uniform(-3, 3, 7)
    tau = o.rnea(0, q, qd, qdd, gravity=1)
    bias = o.rnea(0, q, qd, np.zeros(7), gravity=1)
    M = o.mass_matrix(0, q)
    assert np.allclose(np.linalg.solve(M, tau - bias), qdd, rtol=1e-10, atol=1e-10)


def test_coriolis_from_lagrange_equations(o):
    """c_i = sum_jk (dM_ij/dq_k - 1/2 dM_jk/dq_i) qd_j qd_k, dM by finite differences."""
    rng = np.random.default_rng(4)
    q, qd = rng.uniform(-2, 2, 7), rng.uniform(-2, 2, 7)
    eps = 1e-6
    dM = np.zeros((7, 7, 7))  # dM[k] = dM/dq_k
    for k in range(7):
        e = np.eye(7)[k]
        dM[k] = (o.mass_matrix(0, q + eps * e) - o.mass_matrix(0, q - eps * e)) / (2 * eps)
    c_lag = np.einsum("kij,j,k->i", dM, qd, qd) - 0.5 * np.einsum("ijk,j,k->i", dM, qd, qd)
    c = o.rnea(0, q, qd, np.zeros(7), gravity=0)
    assert np.allclose(c, c_lag, rtol=1e-6, atol=1e-8)
    # power balance qd^T c = 1/2 qd^T Mdot qd
    Mdot = np.einsum("kij,k->ij", dM, qd)
    assert np.isclose(qd @ c, 0.5 * qd @ Mdot @ qd, rtol=1e-6)
    # quadratic in qd
    assert np.allclose(o.rnea(0, q, 2 * qd, np.zeros(7), gravity=0), 4 * c, rtol=1e-12)


def test_cholesky_matches_numpy(oracle_mod):
    rng = np.random.default_rng(5)
    A = rng.normal(size=(7, 7))
    A = A @ A.T + 0.1 * np.eye(7)
    L = oracle_mod.Oracle.cholesky(A)
    assert np.allclose(L, np.linalg.cholesky(A), rtol=1e-12, atol=1e-14)
    B = -np.eye(3)
    assert oracle_mod.Oracle.cholesky(B) is None
