"""Oracle pins: narrowphase primitives, the capsule-box minimiser, pair table,
broadphase and the contact list, against brute force.

The collision cost (Eq. collision_cost) consumes signed distances; the
world model consumes contacts.  Primitive types: 0 sphere, 1 capsule,
2 plane z = 0, 3 axis-aligned box.
"""
import numpy as np
import pytest
from scipy import optimize

import workloads as W

SPH, CAP, PLANE, BOX = 0, 1, 2, 3


def box_sdf(P, c, h):
    """Textbook signed distance of points P (n,3) to an axis-aligned box."""
    q = np.abs(P - c) - h
    out = np.linalg.norm(np.maximum(q, 0.0), axis=-1)
    ins = np.minimum(np.max(q, axis=-1), 0.0)
    return out + ins


def seg_pts(A0, A1, t):
    return A0[None, :] + t[:, None] * (A1 - A0)[None, :]


def brute_core_dist(ta, A0, A1, tb, B0, B1, n=2001):
    """min distance between two cores (point or segment), grid + local refine."""
    ts = np.linspace(0, 1, n) if ta == CAP else np.zeros(1)
    us = np.linspace(0, 1, n) if tb == CAP else np.zeros(1)
    PA = seg_pts(A0, A1, ts)
    PB = seg_pts(B0, B1, us)
    best = np.inf
    bi = (0, 0)
    for i in range(0, len(PA), 1):
        d = np.linalg.norm(PB - PA[i], axis=1)
        j = int(np.argmin(d))
        if d[j] < best:
            best, bi = d[j], (i, j)

    def f(x):
        s = np.clip(x[0], 0, 1) if ta == CAP else 0.0
        t = np.clip(x[1], 0, 1) if tb == CAP else 0.0
        return np.linalg.norm(A0 + s * (A1 - A0) - B0 - t * (B1 - B0))

    r = optimize.minimize(f, [ts[bi[0]], us[bi[1]]], method="Nelder-Mead",
                          options=dict(xatol=1e-12, fatol=1e-14, maxiter=4000))
    return min(best, r.fun)


def random_seg(rng, center, L=0.3):
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    a = center + rng.uniform(-0.1, 0.1, 3)
    return a, a + L * rng.uniform(0.3, 1.0) * d


def check_surface_points(ta, A0, A1, ra, tb, B0, B1, rb, phi, n, p):
    """sA = p + phi n / 2 lies on A's surface, sB = p - phi n / 2 on B's."""
    assert np.isclose(np.linalg.norm(n), 1.0, atol=1e-12)
    sA, sB = p + 0.5 * phi * n, p - 0.5 * phi * n

    def surf_dist(t, X0, X1, r, x):
        if t == PLANE:
            return x[2]
        if t == BOX:
            return box_sdf(x[None, :], X0, X1)[0]
        if t == SPH:
            return np.linalg.norm(x - X0) - r
        D = X1 - X0
        s = np.clip((x - X0) @ D / (D @ D), 0, 1)
        return np.linalg.norm(x - X0 - s * D) - r

    assert abs(surf_dist(ta, A0, A1, ra, sA)) < 1e-9
    assert abs(surf_dist(tb, B0, B1, rb, sB)) < 1e-9


def test_sphere_capsule_pairs_vs_brute_force(oracle_mod):
    O = oracle_mod.Oracle
    rng = np.random.default_rng(10)
    for trial in range(40):
        ta, tb = rng.choice([SPH, CAP]), rng.choice([SPH, CAP])
        A0, A1 = random_seg(rng, np.zeros(3))
        B0, B1 = random_seg(rng, rng.uniform(-0.15, 0.15, 3))
        if ta == SPH:
            A1 = A0.copy()
        if tb == SPH:
            B1 = B0.copy()
        ra, rb = rng.uniform(0.02, 0.08, 2)
        phi, n, p = O.prim(ta, A0, A1, ra, tb, B0, B1, rb)
        want = brute_core_dist(ta, A0, A1, tb, B0, B1) - ra - rb
        assert phi == pytest.approx(want, abs=1e-8), (trial, ta, tb)
        check_surface_points(ta, A0, A1, ra, tb, B0, B1, rb, phi, n, p)
        # swap symmetry: same phi and point, opposite normal
        phi2, n2, p2 = O.prim(tb, B0, B1, rb, ta, A0, A1, ra)
        assert phi2 == pytest.approx(phi, abs=1e-12)
        assert np.allclose(n2, -n, atol=1e-9) and np.allclose(p2, p, atol=1e-12)


def test_plane_contacts(oracle_mod):
    O = oracle_mod.Oracle
    z = np.zeros(3)
    phi, n, p = O.prim(SPH, np.array([0.1, 0.2, 0.03]), z, 0.05, PLANE, z, z, 0.0)
    assert phi == pytest.approx(-0.02) and np.allclose(n, [0, 0, 1]) and np.allclose(p, [0.1, 0.2, -0.01])
    # capsule: the deeper end touches
    A0, A1 = np.array([0.0, 0.0, 0.2]), np.array([0.3, 0.0, 0.01])
    phi, n, p = O.prim(CAP, A0, A1, 0.04, PLANE, z, z, 0.0)
    assert phi == pytest.approx(0.01 - 0.04)
    assert np.allclose(p, [0.3, 0.0, 0.5 * (0.01 - 0.04)])


def test_sphere_box_vs_projection(oracle_mod):
    O = oracle_mod.Oracle
    rng = np.random.default_rng(11)
    for trial in range(60):
        c = rng.uniform(-0.2, 0.2, 3)
        h = rng.uniform(0.05, 0.15, 3)
        x = c + rng.uniform(-0.3, 0.3, 3)
        r = rng.uniform(0.02, 0.06)
        phi, n, p = O.prim(SPH, x, x, r, BOX, c, h, 0.0)
        inside = np.all(np.abs(x - c) <= h)
        if inside:
            want = -np.min(h - np.abs(x - c))
        else:  # Euclidean projection onto the box by a bounded least-squares solver
            sol = optimize.lsq_linear(np.eye(3), x, bounds=(c - h, c + h), method="bvls", tol=1e-15)
            want = np.linalg.norm(x - sol.x)
        assert phi == pytest.approx(want - r, abs=1e-10)
        check_surface_points(SPH, x, x, r, BOX, c, h, 0.0, phi, n, p)


def test_capsule_box_minimiser_vs_brute_force(oracle_mod):
    O = oracle_mod.Oracle
    rng = np.random.default_rng(12)
    ts = np.linspace(0.0, 1.0, 200001)
    for trial in range(60):
        c = rng.uniform(-0.1, 0.1, 3)
        h = rng.uniform(0.05, 0.15, 3)
        A, B = random_seg(rng, c + rng.uniform(-0.25, 0.25, 3), L=0.35)
        t = O.seg_box_tstar(A, B, c, h)
        g = box_sdf(seg_pts(A, B, ts), c, h)
        i0 = int(np.argmin(g))
        ref = optimize.minimize_scalar(lambda u: box_sdf(seg_pts(A, B, np.array([u])), c, h)[0],
                                       bounds=(ts[max(i0 - 2, 0)], ts[min(i0 + 2, len(ts) - 1)]),
                                       method="bounded", options=dict(xatol=1e-15))
        gmin = min(g.min(), ref.fun)
        gt = box_sdf(seg_pts(A, B, np.array([t])), c, h)[0]
        assert gt <= gmin + 1e-12, trial
        # unique minimiser: t agrees with the brute-force location
        near = ts[g <= g.min() + 1e-9]
        if near.max() - near.min() < 1e-3:
            assert abs(t - ts[np.argmin(g)]) < 2e-3
        r = 0.04
        phi, n, p = O.prim(CAP, A, B, r, BOX, c, h, 0.0)
        # the oracle's point is attained (phi = sdf at t* - r) and is at least
        # as deep as every brute-force sample, so it is the minimum
        assert phi == pytest.approx(gt - r, abs=1e-12)
        assert gt <= gmin + 1e-12 and gt >= gmin - 1e-6


def test_capsule_box_flat_interval_midpoint(oracle_mod):
    """Segment parallel to a face: the minimising interval's midpoint."""
    O = oracle_mod.Oracle
    c, h = np.zeros(3), np.array([0.1, 0.1, 0.1])
    A, B = np.array([-0.3, 0.0, 0.15]), np.array([0.05, 0.0, 0.15])
    # distance 0.05 over t with x in [-0.1, 0.05] -> t in [0.5714.., 1]
    t = O.seg_box_tstar(A, B, c, h)
    t_lo = (-0.1 + 0.3) / 0.35
    assert t == pytest.approx(0.5 * (t_lo + 1.0), abs=1e-12)


def test_tangent_basis(oracle_mod):
    rng = np.random.default_rng(13)
    for _ in range(50):
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        t1, t2 = oracle_mod.Oracle.tangents(n)
        B = np.stack([t1, t2, n])
        assert np.allclose(B @ B.T, np.eye(3), atol=1e-12)
        assert np.isclose(np.linalg.det(B), 1.0)


def test_pair_table_canonical(oracle_mod):
    sc = W.make_scene(2)
    o = oracle_mod.Oracle(sc)
    ga, gb = o.pairs()
    nb = sc["n_box"]
    assert len(ga) == 76 + 15 * nb
    pairs = list(zip(ga.tolist(), gb.tolist()))
    assert len(set(pairs)) == len(pairs)
    assert pairs[0] == (0, 1)                     # ball-table
    assert pairs[1:3] == [(0, 8), (0, 15)]        # ball-pads
    for a, b in pairs:                            # no same-arm pair, no static-static
        if 2 <= a < 16 and 2 <= b < 16:
            assert (a - 2) // 7 != (b - 2) // 7
        assert a in range(0, 16)
    assert (2, 1) not in pairs and (9, 1) not in pairs  # base links never against the table
    # cost pairs are the tail: arm-box then arm-arm
    nd = 14 * nb + 49
    tail = pairs[-nd:]
    assert all(2 <= a < 16 and (b >= 16 or 9 <= b < 16) for a, b in tail)


def test_broadphase_conservative_and_exact(oracle_mod):
    sc = W.make_scene(3)
    o = oracle_mod.Oracle(sc)
    X = W.random_states(sc, 30, seed=5, spread=1.2)
    ga, gb = o.pairs()
    rng = np.random.default_rng(0)
    for x in X:
        lo, hi = o.aabbs(x)
        flags = o.broadphase(lo.astype(np.float32), hi.astype(np.float32))
        phi, _, _ = o.narrow_all(x)
        assert np.all(flags[phi < 0] == 1)   # every contact survives the cull
        # AABB containment: sampled surface points of each geom lie inside its box
        for g in range(2, 16):
            R_, org, _, _ = o.fk((g - 2) // 7, x[0:7] if g < 9 else x[7:14])
            k = (g - 2) % 7
            if k < 6:
                P = seg_pts(org[k], org[k + 1], rng.uniform(0, 1, 50))
                r = sc["link_rad"][k]
            else:
                P = org[7][None, :]
                r = sc["pad_rad"]
            d = rng.normal(size=(len(P), 3))
            S = P + r * d / np.linalg.norm(d, axis=1, keepdims=True)
            assert np.all(S >= lo[g] - 1e-12) and np.all(S <= hi[g] + 1e-12)
        # exact: a flag equals a direct interval-overlap check in float64
        l32, h32 = lo.astype(np.float32).astype(np.float64), hi.astype(np.float32).astype(np.float64)
        direct = np.all((l32[ga] <= h32[gb]) & (l32[gb] <= h32[ga]), axis=1).astype(np.int32)
        assert np.array_equal(flags, direct)


def test_contacts_order_and_cap(oracle_mod):
    sc = W.make_scene(2)
    o = oracle_mod.Oracle(sc)
    x = W.initial_state(sc)
    x[44] = 0.08          # ball pressed into the table
    x[0:7] += np.array([0, 0.3, 0, 0.3, 0, 0.3, 0])   # arm 1 leans in
    phi, _, _ = o.narrow_all(x)
    pair, cphi, _, _ = o.contacts(x)
    want = np.nonzero(phi < 0)[0]
    assert np.array_equal(pair, want) and len(want) >= 2
    pair2, _, _, _ = o.contacts(x, cap=1)
    assert np.array_equal(pair2, want[:1])
