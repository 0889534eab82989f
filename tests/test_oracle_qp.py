"""Pins of the oracle's QP smoothing (Alg. 1 sampling step, Eqs. proj_cost and
proj_bounds with r = 0..3): the stacked operator against the definitions of
differences and prefix sums, a feasible sequence as a fixed point, the
velocity-only case against its closed form (the clamp), the optimiser
against a brute-force enumeration of active sets, and the ADMM iteration
against the optimum it converges to."""
import itertools

import numpy as np
import pytest

from oracle import qp
import workloads as W

DT, UMAX = 0.01, 1.0


def test_operator_rows_are_identity_differences_and_prefix_sums():
    rng = np.random.default_rng(0)
    H = 9
    v = rng.normal(size=H)
    Av = qp.operators(H) @ v
    np.testing.assert_allclose(Av[:H], v, rtol=0, atol=1e-15)
    np.testing.assert_allclose(Av[H:2 * H - 1], np.diff(v), rtol=0, atol=1e-15)
    np.testing.assert_allclose(Av[2 * H - 1:3 * H - 3], np.diff(v, 2), rtol=0, atol=1e-14)
    np.testing.assert_allclose(Av[3 * H - 3:], np.cumsum(v), rtol=0, atol=1e-14)


def test_feasible_sequence_is_a_fixed_point():
    H = 32
    vt = 0.3 * np.sin(np.arange(H) * 0.05)  # slow: every bound inactive
    lo, hi = -1.0, 1.0
    assert qp.violation(vt, 0.0, DT, UMAX, lo, hi, 4.0, 60.0) == 0.0
    for iters in (1, 7, 60):
        v = qp.project_admm(vt, 0.0, DT, UMAX, lo, hi, 4.0, 60.0, rho=3.0, iters=iters, alpha=1.6)
        np.testing.assert_allclose(v, vt, rtol=0, atol=1e-12)


def test_velocity_box_alone_is_the_clamp():
    rng = np.random.default_rng(1)
    H = 12
    vt = rng.normal(0, 1.2, H)
    args = (0.0, DT, UMAX, -1e6, 1e6, 1e9, 1e12)  # only |v| <= u_max can bind
    np.testing.assert_allclose(qp.project_exact(vt, *args), np.clip(vt, -UMAX, UMAX), rtol=0, atol=1e-7)
    v = qp.project_admm(vt, *args, rho=1.0, iters=2000)
    np.testing.assert_allclose(v, np.clip(vt, -UMAX, UMAX), rtol=0, atol=1e-9)


def _enumerate_projection(vt, lo, hi, A):
    """Projection onto {lo <= A v <= hi} by trying every active set: each
    constraint at its lower bound, at its upper bound, or free; the best
    feasible stationary point is the optimum."""
    H = vt.size
    best, best_f = None, np.inf
    m = A.shape[0]
    for states in itertools.product((0, 1, 2), repeat=m):
        act = [i for i in range(m) if states[i]]
        if len(act) > H:
            continue
        if act:
            Aa = A[act]
            ba = np.array([lo[i] if states[i] == 1 else hi[i] for i in act])
            # min |v - vt|^2 s.t. Aa v = ba (least-norm correction)
            try:
                lam = np.linalg.solve(Aa @ Aa.T, Aa @ vt - ba)
            except np.linalg.LinAlgError:
                continue
            v = vt - Aa.T @ lam
        else:
            v = vt.copy()
        Av = A @ v
        if np.all(Av >= lo - 1e-12) and np.all(Av <= hi + 1e-12):
            f = np.sum((v - vt) ** 2)
            if f < best_f:
                best, best_f = v, f
    return best


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_optimiser_equals_active_set_enumeration(seed):
    rng = np.random.default_rng(10 + seed)
    H = 3
    vt = rng.normal(0, 0.8, H)
    args = (0.1, DT, UMAX, -0.2, 0.2, 20.0, 1500.0)  # every bound family can bind at this scale
    lo, hi = qp.bounds(*args[:1], DT, UMAX, -0.2, 0.2, 20.0, 1500.0, H)
    ref = _enumerate_projection(vt, lo, hi, qp.operators(H))
    assert ref is not None
    np.testing.assert_allclose(qp.project_exact(vt, *args), ref, rtol=0, atol=1e-7)


def test_admm_converges_to_the_projection():
    rng = np.random.default_rng(3)
    H = 16
    p = W.qp_params(2)
    for trial in range(3):
        vt = 0.2 * np.sin(np.arange(H) * 0.3 + trial) + rng.normal(0, 0.3, H)
        args = (0.0, DT, UMAX, -0.05, 0.05, p["acc_max"], p["jerk_max"])
        ex = qp.project_exact(vt, *args)
        assert qp.violation(ex, *args) < 1e-9
        errs = [np.abs(qp.project_admm(vt, *args, rho=p["rho"], iters=n, alpha=p["alpha"]) - ex).max()
                for n in (30, 300, 3000)]
        assert errs[2] < 1e-5
        assert errs[2] < errs[1] <= errs[0] + 1e-12


def test_production_settings_on_sampled_sequences():
    """With the workload's settings (60 over-relaxed ADMM iterations) the
    result is within a few hundredths of the projection on noisy H = 64
    samples, and every bound holds to within a few thousandths; the velocity
    box holds exactly."""
    rng = np.random.default_rng(4)
    H = 64
    p = W.qp_params(2)
    for trial in range(2):
        vt = rng.normal(0, 0.3, H)
        args = (0.0, DT, UMAX, -0.5, 0.5, p["acc_max"], p["jerk_max"])
        v = qp.project_admm(vt, *args, rho=p["rho"], iters=p["iters"], alpha=p["alpha"])
        ex = qp.project_exact(vt, *args)
        assert np.abs(v - ex).max() < 0.05
        assert qp.violation(v, *args) < 0.01
        assert np.all(np.abs(v) <= UMAX)
        # smoothing: the projected sequence's steps are far smaller than the noise's
        assert np.abs(np.diff(v)).max() < 0.2 * np.abs(np.diff(vt)).max()


def test_single_step_is_the_clamp_to_both_intervals():
    """H = 1: no difference rows exist, and the velocity row and the one
    position row bound the same scalar, so the projection is the clamp to
    the intersection of [-u_max, u_max] and [(pos_lo - q0)/dt, (pos_hi - q0)/dt]."""
    q0, lo_p, hi_p = 0.3, 0.29, 0.305
    lo, hi = qp.bounds(q0, DT, UMAX, lo_p, hi_p, 4.0, 60.0, 1)
    assert lo.shape == hi.shape == (2,)
    for vt in (-2.0, -0.7, 0.2, 0.45, 3.0):
        ref = min(max(vt, -UMAX, (lo_p - q0) / DT), UMAX, (hi_p - q0) / DT)
        args = (q0, DT, UMAX, lo_p, hi_p, 4.0, 60.0)
        assert abs(qp.project_exact(np.array([vt]), *args)[0] - ref) < 1e-7
        assert abs(qp.project_admm(np.array([vt]), *args, rho=1.0, iters=500)[0] - ref) < 1e-9
