"""Closed-loop ball transport -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and `bench.py`'s `cpu_baseline` leg
may import this module; the product library never loads it.

The receding-horizon execution the paper describes after Alg. 1: each
replan returns the best sequence of its final iteration together with the
mean; the first few steps of the best sequence are averaged and executed,
and the next replan is warm-started with the mean.  The ball task runs in a
pick phase (no object-to-target term) and a move phase (every term); a run
fails on a collision, on a timeout or when the ball falls (the experiments'
success metric).  Readings (the same ones the design notes list): the grasp
is detected from the pad midpoint's distance to the grasp point and the pad
distance's error; the ball has fallen when, in the move phase and after it
was lifted above lift_z, it is below drop_z; checks after every executed
control step in the order collision, phase rule, timeout; the warm start is
the mean shifted by the executed steps with its last row repeated; plan
seeds are seed + replan index; with the full covariance, Sigma_M is
shifted like the mean and the freed tail is diag(sigma^2).  FP64
throughout, on the C oracle.
"""
from __future__ import annotations

import numpy as np

RUNNING, SUCCESS, COLLISION, TIMEOUT, FELL = 0, 1, -1, -2, -3
PICK, MOVE = 0, 1


class Rules:
    """Phase and outcome after each executed control step."""

    def __init__(self, grasp_tol, width_tol, goal_tol, lift_z, drop_z, t_max):
        self.grasp_tol, self.width_tol, self.goal_tol = grasp_tol, width_tol, goal_tol
        self.lift_z, self.drop_z, self.t_max = lift_z, drop_z, t_max
        self.phase, self.status, self.lifted = PICK, RUNNING, False
        self.t_switch, self.t_end = -1.0, -1.0

    def observe(self, t, goal_dist, grasp_dist, width_err, ball_z, penetrations):
        if self.status != RUNNING:
            return self.status
        if penetrations > 0:
            self.status = COLLISION
        elif self.phase == PICK:
            if grasp_dist < self.grasp_tol and width_err < self.width_tol:
                self.phase, self.t_switch = MOVE, t
        else:
            self.lifted = self.lifted or ball_z > self.lift_z
            if self.lifted and ball_z < self.drop_z:
                self.status = FELL
            elif goal_dist < self.goal_tol:
                self.status = SUCCESS
        if self.status == RUNNING and t >= self.t_max:
            self.status = TIMEOUT
        if self.status != RUNNING:
            self.t_end = t
        return self.status


def best_sequence(o, x, nominal, K, H, lam, sigma, M, seed, eta=1.0, n_elite=None):
    """(nu_M, best sequence of the final iteration): the lowest-cost sample of
    iteration M - 1, drawn around that iteration's mean."""
    r = o.plan(x, nominal, K, H, lam, sigma, M, seed, eta=eta, n_elite=n_elite)
    nu_prev = np.asarray(nominal, dtype=np.float64).reshape(H, 14) if M == 1 else \
        o.plan(x, nominal, K, H, lam, sigma, M - 1, seed, eta=eta, n_elite=n_elite)["nu"]
    if r["best"] < 0:
        return r["nu"], nu_prev
    return r["nu"], o.sample(nu_prev, sigma, seed, K, M - 1)[r["best"]]


def shift_sigma(S, sigma, H, n_exec):
    """Warm start of the full covariance: the entries whose two steps stay
    inside the horizon move up by the executed steps; the freed tail is
    diag(sigma^2) with no cross-covariance."""
    from oracle import cov
    D = cov.diagonal_sigma(sigma, H)
    n = 14 * H
    sh = 14 * n_exec
    out = D.copy()
    if sh < n:
        out[:n - sh, :n - sh] = S[sh:, sh:]
    return out


def best_sequence_cov(o, x, nominal, K, H, lam, Sigma, M, seed, eta, eps, u_max, n_elite=None):
    """(nu_M, best sequence of the final iteration, Sigma_M) of the plan with
    the full covariance."""
    from oracle import cov
    r = cov.plan(o, x, nominal, K, H, lam, Sigma, M, seed, eta, eps, u_max, n_elite=n_elite)
    c = np.asarray(r["costs"], dtype=np.float64)
    fin = np.isfinite(c)
    best = int(np.flatnonzero(fin)[np.argmin(c[fin])]) if fin.any() else -1
    ub = r["U"][best] if best >= 0 else r["nu"]
    return r["nu"], np.asarray(ub).reshape(H, 14), r["Sigma"]


def best_sequence_qp(o, x, nominal, K, H, lam, sigma, M, seed, eta, n_elite, project):
    """(nu_M, best sequence of the final iteration) of the plan whose samples
    nu + sigma z are smoothed by `project` before their rollouts."""
    from oracle import cov
    nu = np.asarray(nominal, dtype=np.float64).reshape(H, 14).copy()
    sig = np.broadcast_to(np.asarray(sigma, dtype=np.float64).reshape(-1, 14), (H, 14))
    U = c = None
    for m in range(M):
        U = project(nu[None] + sig[None] * o.noise(seed, K, H, m))
        c = o.rollout_batch(x, U)
        c = c[0] if isinstance(c, tuple) else c
        w = cov.weights(c, lam, n_elite)
        nu = cov.mean_update(U, w, nu, eta).reshape(H, 14)
    c = np.asarray(c, dtype=np.float64)
    fin = np.isfinite(c)
    best = int(np.flatnonzero(fin)[np.argmin(c[fin])]) if fin.any() else -1
    return nu, (U[best] if best >= 0 else nu)


def run(o_pick, o_move, x0, K, H, lam, sigma, M, seed, ep, eta=1.0, n_elite=None, max_replans=None, project=None):
    """One closed-loop run; ep: the executor settings (n_avg, n_exec,
    tolerances, heights, t_max; use_cov and cov_eps for the plan with the
    full covariance, warm-started with Sigma_M shifted like the mean);
    project(U, x): the QP smoothing of a replan's samples from state x.
    Returns the outcome, the executed commands and the state after each
    replan's execution."""
    rules = Rules(ep["grasp_tol"], ep["width_tol"], ep["goal_tol"], ep["lift_z"], ep["drop_z"], ep["t_max"])
    dt = o_move.scene["h"] * o_move.scene["n_sub"]
    x = np.asarray(x0, dtype=np.float64).copy()
    nom = np.zeros((H, 14))
    use_cov = bool(ep.get("use_cov", 0))
    if use_cov:
        from oracle import cov
        S = cov.diagonal_sigma(sigma, H)
    t, u_exec, x_hist = 0.0, [], []
    r = 0
    while max_replans is None or r < max_replans:
        o = o_pick if rules.phase == PICK else o_move
        if use_cov:
            nu, ub, S = best_sequence_cov(o, x, nom, K, H, lam, S, M, seed + r, eta, ep["cov_eps"],
                                          float(o_move.scene["u_max"]), n_elite)
        elif project is not None:
            nu, ub = best_sequence_qp(o, x, nom, K, H, lam, sigma, M, seed + r, eta, n_elite,
                                      lambda U, x=x: project(U, x))
        else:
            nu, ub = best_sequence(o, x, nom, K, H, lam, sigma, M, seed + r, eta, n_elite)
        u = ub[:ep["n_avg"]].mean(axis=0)
        u_exec.append(u)
        for _ in range(ep["n_exec"]):
            _, terms, traj = o_move.rollout(x, u[None, :], want_traj=True)
            x = traj[0]
            t += dt
            rules.observe(t, terms[0], terms[1], np.sqrt(max(terms[2], 0.0)), x[44], int(round(terms[6])))
            if rules.status != RUNNING:
                break
        x_hist.append(x.copy())
        r += 1
        if rules.status != RUNNING:
            break
        nom = np.concatenate([nu[ep["n_exec"]:], np.repeat(nu[-1:], min(ep["n_exec"], H), axis=0)])[:H]
        if use_cov:
            S = shift_sigma(S, sigma, H, ep["n_exec"])
    return dict(status=rules.status, phase=rules.phase, t_end=rules.t_end if rules.t_end >= 0 else t,
                t_switch=rules.t_switch, n_replans=r, u_exec=np.array(u_exec), x_hist=np.array(x_hist))
