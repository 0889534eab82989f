"""QP smoothing of sampled joint-velocity sequences -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and `bench.py`'s `cpu_baseline` leg
may import this module; the product library never loads it.

Alg. 1 (sampling step, then "QP based smoothing") projects every sampled
sequence onto the set of Eq. proj_bounds, the bounds on the r-th derivative
of each joint's trajectory for r = 0..3, with the least-squares objective of
Eq. proj_cost.  The paper gives neither the discretisation, the bound values
nor the solver; the readings here (also listed with the design notes):

* Each joint is its own QP over the horizon (objective and bounds separate
  per joint): the H control-step velocities v_0..v_{H-1} of one joint.
* r = 0: the commanded position after step k, q_des0 + dt * (v_0 + .. + v_k),
  stays in [pos_lo, pos_hi]; dt = n_sub * h is the control step and q_des0
  the commanded position of the start state.
* r = 1: |v_k| <= u_max (the sampling box of the velocity-only projection).
* r = 2: |v_k - v_{k-1}| <= acc_max * dt for k = 1..H-1; r = 3:
  |v_k - 2 v_{k-1} + v_{k-2}| <= jerk_max * dt^2 for k = 2..H-1 (differences
  within the sequence: the start state carries no commanded-velocity history).
* Solver: ADMM (Boyd et al., 2011, with over-relaxation alpha) on
  min 1/2 |v - vt|^2 s.t. l <= A v <= u with the stacked operator
  A = [I; D1; D2; L] (identity, first and second differences, prefix sums;
  every row in velocity units, so one penalty rho suits all):
      v  <- (I + rho A^T A)^-1 (vt + rho A^T (z - w))
      a  <- alpha A v + (1 - alpha) z
      z' <- clip(a + w, l, u)
      w  <- w + a - z',  z <- z'
  from z = clip(A vt, l, u), w = 0, for a fixed number of iterations; the
  result is v clipped to the velocity box (so r = 1 holds exactly).  A
  fixed iteration count leaves the other bounds approximately satisfied.

`project_exact` solves the same QP to optimality with a general solver; it
is the pin that the ADMM iteration is converging to the projection.
"""
from __future__ import annotations

import numpy as np


def operators(H: int):
    """The stacked constraint operator A (rows: H identity, H-1 first
    differences, H-2 second differences, H prefix sums) as a dense matrix."""
    I = np.eye(H)
    D1 = (np.eye(H) - np.eye(H, k=-1))[1:]
    D2 = (np.eye(H) - 2 * np.eye(H, k=-1) + np.eye(H, k=-2))[2:]
    L = np.tril(np.ones((H, H)))
    return np.vstack([I, D1, D2, L])


def bounds(q0, dt, u_max, pos_lo, pos_hi, acc_max, jerk_max, H):
    """Lower and upper bounds of A v for one joint (q0: commanded start position)."""
    n1, n2 = max(H - 1, 0), max(H - 2, 0)  # difference rows exist only for k >= 1 and k >= 2
    lo = np.concatenate([np.full(H, -u_max), np.full(n1, -acc_max * dt), np.full(n2, -jerk_max * dt * dt),
                         np.full(H, (pos_lo - q0) / dt)])
    hi = np.concatenate([np.full(H, u_max), np.full(n1, acc_max * dt), np.full(n2, jerk_max * dt * dt),
                         np.full(H, (pos_hi - q0) / dt)])
    return lo, hi


def system_inverse(H: int, rho: float):
    """(I + rho A^T A)^-1, the same matrix for every joint and sample."""
    A = operators(H)
    return np.linalg.inv(np.eye(H) + rho * A.T @ A)


def project_admm(vt, q0, dt, u_max, pos_lo, pos_hi, acc_max, jerk_max, rho, iters, alpha=1.0):
    """ADMM projection of one joint's sequence vt[H] (the steps in the module
    docstring, in that order); returns v[H]."""
    vt = np.asarray(vt, dtype=np.float64)
    H = vt.size
    A = operators(H)
    P = system_inverse(H, rho)
    lo, hi = bounds(q0, dt, u_max, pos_lo, pos_hi, acc_max, jerk_max, H)
    z = np.clip(A @ vt, lo, hi)
    w = np.zeros_like(z)
    v = vt.copy()
    for _ in range(iters):
        v = P @ (vt + rho * A.T @ (z - w))
        a = alpha * (A @ v) + (1.0 - alpha) * z
        zn = np.clip(a + w, lo, hi)
        w = w + a - zn
        z = zn
    return np.clip(v, -u_max, u_max)


def project_sequences(U, q_des0, dt, u_max, pos_lo, pos_hi, acc_max, jerk_max, rho, iters, alpha=1.0):
    """Project U[K, H, 14] joint by joint; q_des0[K, 14] (or [14]) are the
    commanded start positions.  Returns a new [K, H, 14] array."""
    U = np.asarray(U, dtype=np.float64)
    K, H, nu = U.shape
    q = np.broadcast_to(np.asarray(q_des0, dtype=np.float64), (K, nu))
    out = np.empty_like(U)
    for j in range(K):
        for d in range(nu):
            out[j, :, d] = project_admm(U[j, :, d], q[j, d], dt, u_max, pos_lo[d], pos_hi[d], acc_max, jerk_max,
                                        rho, iters, alpha)
    return out


def project_exact(vt, q0, dt, u_max, pos_lo, pos_hi, acc_max, jerk_max):
    """The projection itself: min 1/2 |v - vt|^2 s.t. l <= A v <= u, solved
    to optimality with SciPy's SLSQP (small H only)."""
    from scipy.optimize import minimize
    vt = np.asarray(vt, dtype=np.float64)
    H = vt.size
    A = operators(H)
    lo, hi = bounds(q0, dt, u_max, pos_lo, pos_hi, acc_max, jerk_max, H)
    cons = [{"type": "ineq", "fun": lambda v: A @ v - lo, "jac": lambda v: A},
            {"type": "ineq", "fun": lambda v: hi - A @ v, "jac": lambda v: -A}]
    x0 = np.clip(vt, -u_max, u_max)
    r = minimize(lambda v: 0.5 * np.sum((v - vt) ** 2), x0, jac=lambda v: v - vt, constraints=cons, method="SLSQP",
                 options={"ftol": 1e-14, "maxiter": 1000})
    if not r.success:
        raise RuntimeError(r.message)
    return r.x


def violation(v, q0, dt, u_max, pos_lo, pos_hi, acc_max, jerk_max):
    """Largest bound violation of A v (0 when feasible)."""
    v = np.asarray(v, dtype=np.float64)
    A = operators(v.size)
    lo, hi = bounds(q0, dt, u_max, pos_lo, pos_hi, acc_max, jerk_max, v.size)
    Av = A @ v
    return float(max(np.max(lo - Av), np.max(Av - hi), 0.0))
