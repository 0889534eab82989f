"""Oracle pins: Philox noise, Gaussian draws and the velocity-box projection.

Alg. 1 draws n sequences from N(nu_m, Sigma_m) and projects them with the QP
of Eqs. proj_cost/proj_bounds; with only velocity bounds that QP is the
Euclidean projection onto a box.
"""
import os

import numpy as np
import pytest
from scipy import optimize, stats

import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


def test_philox_known_answers(oracle_mod):
    for ctr, key, want in _kat():
        got = oracle_mod.Oracle.philox(ctr, key)
        assert [int(g) for g in got] == want


def test_normals_statistics(oracle_mod):
    z = oracle_mod.Oracle.noise(seed=12345, K=2000, H=40, m=3).reshape(-1, 14)
    flat = z.ravel()
    assert abs(flat.mean()) < 5e-3
    assert abs(flat.var() - 1.0) < 5e-3
    ks = stats.kstest(flat[:200000], "norm")
    assert ks.pvalue > 1e-3
    c = np.corrcoef(z.T)
    off = c[~np.eye(14, dtype=bool)]
    assert np.max(np.abs(off)) < 0.01


def test_noise_streams_distinct_and_deterministic(oracle_mod):
    O = oracle_mod.Oracle
    a = O.noise(7, 4, 3, 0)
    b = O.noise(7, 4, 3, 1)
    c = O.noise(8, 4, 3, 0)
    assert np.array_equal(a, O.noise(7, 4, 3, 0))
    assert not np.allclose(a, b) and not np.allclose(a, c)
    # the stream of sample j does not depend on K
    assert np.array_equal(O.noise(7, 10, 3, 0)[:4], a)


def test_projection_is_box_qp(oracle_mod):
    """clamp(nu + sigma z) equals the QP argmin 1/2 ||u - u~||^2 s.t. |u| <= u_max."""
    sc = W.make_scene(1)
    o = oracle_mod.Oracle(sc)
    H, K = 3, 5
    rng = np.random.default_rng(0)
    nu = rng.uniform(-1.5, 1.5, size=(H, 14))
    sigma = np.full(14, 1.2)
    U = o.sample(nu, sigma, seed=99, K=K, m=2)
    z = oracle_mod.Oracle.noise(99, K, H, 2)
    for j in range(K):
        raw = (nu + sigma * z[j]).ravel()
        qp = optimize.lsq_linear(np.eye(raw.size), raw, bounds=(-sc["u_max"], sc["u_max"]),
                                 method="bvls", tol=1e-14)
        assert np.allclose(U[j].ravel(), qp.x, atol=1e-12)
    assert np.any(np.abs(U) == sc["u_max"])  # some samples were projected


def test_sigma_per_step(oracle_mod):
    sc = W.make_scene(1)
    o = oracle_mod.Oracle(sc)
    H = 4
    nu = np.zeros((H, 14))
    sig = np.zeros((H, 14))
    sig[2] = 0.5
    U = o.sample(nu, sig, seed=3, K=2, m=0)
    assert np.all(U[:, [0, 1, 3]] == 0.0)
    assert np.all(U[:, 2] != 0.0)
