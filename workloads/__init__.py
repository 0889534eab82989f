"""Seeded synthetic inputs for the bimanual MPPI hot path.

This module only *generates data*: scene descriptions (robot geometry,
inertia densities, obstacles, goal), initial states and plan parameters.
It holds none of the method's arithmetic (no kinematics, dynamics,
contact, cost or MPPI update); both the FP64 oracle and the HIP library
consume the plain dictionaries it returns and marshal them on their own.

The scenes stand in for the paper's PerAct2-derived ball-lifting task
(Sec. IV-B; experimental setup in Sec. V-A): two serial 7-joint arms
facing each other along x, a free ball on a table plane, static
axis-aligned boxes and a goal position for the ball.  The paper uses
MuJoCo models of two UR5e arms that are not available here; the synthetic
arms below (capsule links, seeded uniform densities) replace them.

Recipe (seeds fixed):
  * scene seed = 1000*config + index, numpy PCG64;
  * link densities ~ U[800, 1200] kg/m^3 per link per arm;
  * boxes: half extents ~ U[0.05, 0.15] per axis, centre x, y ~ U[-0.5, 0.5],
    resting on the table (z = half height), rejection-sampled clear of the
    arm/ball corridor at home pose, of the goal and of each other;
  * noise seed = 0xC0FFEE + config.
"""
from __future__ import annotations

import math

import numpy as np

# ---------------------------------------------------------------------------
# Fixed robot description (synthetic 7-joint arm, capsule links).
# Joint axes in link-local frames: 0 = x, 1 = y, 2 = z.
ARM_AXES = (2, 1, 2, 1, 2, 1, 2)
LINK_LEN = (0.15, 0.25, 0.10, 0.25, 0.10, 0.15, 0.06)
LINK_RAD = (0.05, 0.05, 0.05, 0.05, 0.04, 0.04, 0.04)
PAD_RAD = 0.04
BASE_POS = ((-0.55, 0.0, 0.0), (0.55, 0.0, 0.0))
# base yaw given as (cos, sin) so both consumers see exact values
BASE_CS = ((1.0, 0.0), (-1.0, 0.0))
# Home pose (same joint values for both arms; arm 2 is mirrored by its base
# yaw).  Chosen by hand so that each pad sits ~5 cm outside a 0.1 m ball at
# the origin, at ball-centre height.
Q_HOME_ARM = (0.0, -0.093, 0.0, 2.46, 0.0, -0.012, 0.0)

MAX_BOXES = 16
STATE_DIM = 55  # q[14] qd[14] qdes[14] pb[3] quat[4] vb[3] wb[3]
NU = 14

# physics defaults (readings of the paper's unstated world model)
PHYSICS = dict(
    kp=100.0, kd=20.0, damp=0.5, armature=0.1, tau_max=150.0,
    gravcomp=1, g=9.81,
    mu=1.0, kappa=0.2, eps_r=0.01, n_pgs=20, n_cmax=4,
    u_max=1.5,
)
COST = dict(
    w_goal=1.0, w_eo=1.0, w_l=10.0, w_yz=1.0, w_s=0.01, w_c=10.0,
    gamma=0.5, m_c=0.05, eps_frac=0.3,
)
# the free object (a ball unless a task scene makes it a box) and the further
# task-cost terms (off unless a task scene turns them on)
EXTRA = dict(
    obj_box=0, obj_h=np.zeros(3), ext=0, l_target=0.0,
    w_home=0.0, w_vert=0.0, w_relv=0.0, w_orot=0.0,
    w_apos=np.zeros(2), w_ax=np.zeros(2), w_arot=np.zeros(2),
    apos=np.zeros((2, 3)), ax_t=np.zeros(2), arot=np.array([[1.0, 0, 0, 0], [1.0, 0, 0, 0]]),
    orot=np.array([1.0, 0, 0, 0]),
)
# task objects: the tray (held along x between the pads) and the cube
TRAY_H, TRAY_M = (0.12, 0.10, 0.015), 0.4
CUBE_H, CUBE_M = (0.03, 0.03, 0.03), 0.1

# arm / ball corridor at home pose (xy rectangle boxes must stay clear of)
_CORRIDOR = (-0.65, 0.65, -0.12, 0.12)


def _box_ok(c, hh, boxes, goal, ball_r, clear=0.05):
    x0, x1, y0, y1 = _CORRIDOR
    # footprint vs corridor (expanded by `clear`)
    if (c[0] + hh[0] + clear > x0 and c[0] - hh[0] - clear < x1 and
            c[1] + hh[1] + clear > y0 and c[1] - hh[1] - clear < y1):
        return False
    # goal clearance: the goal point, grown by ball radius + clear, outside box
    g = np.asarray(goal)
    if np.all(np.abs(g - c) < hh + ball_r + clear):
        return False
    for (c2, h2) in boxes:
        if np.all(np.abs(c[:2] - c2[:2]) < hh[:2] + h2[:2] + 0.02):
            return False
    return True


def _sample_boxes(rng, n, goal, ball_r):
    boxes = []
    shrink = 1.0
    tries = 0
    while len(boxes) < n:
        hh = rng.uniform(0.05, 0.15, size=3) * shrink
        c = np.array([rng.uniform(-0.5, 0.5), rng.uniform(-0.5, 0.5), 0.0])
        c[2] = hh[2]
        if _box_ok(c, hh, boxes, goal, ball_r):
            boxes.append((c, hh))
        tries += 1
        if tries % 300 == 0:
            shrink *= 0.9
        if tries > 20000:
            raise RuntimeError("box placement failed")
    return boxes


def make_scene(config: int, index: int = 0, *, n_box=None, ball_r=None,
               ball_m=None, goal=None, h=None, n_sub=None, **overrides):
    """Seeded scene description for workload `config` (1..5), scene `index`.

    Returns a plain dict of Python floats / lists / numpy arrays.
    """
    rng = np.random.Generator(np.random.PCG64(1000 * config + index))
    density = rng.uniform(800.0, 1200.0, size=(2, 7))
    if config in (1, 2, 3):
        r, m = 0.1, 0.5
        nb = {1: 0, 2: 3, 3: 8}[config]
        hh, ns = (0.01, 2) if config == 1 else (0.002, 5)
        if config == 1:
            g = (0.0, 0.0, r + 0.3)
        elif config == 2:
            g = (0.0, 0.5, 0.3)
        else:
            ang = rng.uniform(-0.5, 0.5) + (math.pi / 2 if rng.uniform() < 0.5 else -math.pi / 2)
            g = (0.8 * math.cos(ang), 0.8 * math.sin(ang), 0.25)
    else:
        r = rng.uniform(0.06, 0.14)
        m = rng.uniform(0.2, 1.0)
        nb = int(rng.integers(0, 13))
        hh, ns = 0.002, 5
        ang = rng.uniform(-0.5, 0.5) + (math.pi / 2 if rng.uniform() < 0.5 else -math.pi / 2)
        dist = rng.uniform(0.3, 0.8)
        g = (dist * math.cos(ang), dist * math.sin(ang), rng.uniform(0.15, 0.35))
    if n_box is not None:
        nb = n_box
    if ball_r is not None:
        r = ball_r
    if ball_m is not None:
        m = ball_m
    if goal is not None:
        g = tuple(goal)
    if h is not None:
        hh = h
    if n_sub is not None:
        ns = n_sub
    boxes = _sample_boxes(rng, nb, g, r) if nb > 0 else []
    scene = dict(
        base_pos=np.array(BASE_POS, dtype=np.float64),
        base_cs=np.array(BASE_CS, dtype=np.float64),
        axes=np.array(ARM_AXES, dtype=np.int32),
        link_len=np.array(LINK_LEN, dtype=np.float64),
        link_rad=np.array(LINK_RAD, dtype=np.float64),
        density=density,
        pad_rad=PAD_RAD,
        ball_r=float(r), ball_m=float(m),
        ball_p0=np.array([0.0, 0.0, float(r)]),
        n_box=len(boxes),
        box_c=np.array([b[0] for b in boxes], dtype=np.float64).reshape(-1, 3),
        box_h=np.array([b[1] for b in boxes], dtype=np.float64).reshape(-1, 3),
        goal=np.array(g, dtype=np.float64),
        h=float(hh), n_sub=int(ns),
        q_home=np.array(Q_HOME_ARM * 2, dtype=np.float64),
    )
    scene.update(PHYSICS)
    scene.update(COST)
    scene.update({k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in EXTRA.items()})
    for k, v in overrides.items():
        if k not in scene:
            raise KeyError(k)
        scene[k] = v
    return scene


def initial_state(scene) -> np.ndarray:
    """x0 = home pose at rest, PD target = home, ball at rest on the table."""
    x = np.zeros(STATE_DIM, dtype=np.float64)
    x[0:14] = scene["q_home"]
    x[28:42] = scene["q_home"]
    x[42:45] = scene["ball_p0"]
    x[45] = 1.0  # quaternion (w, x, y, z)
    return x


PLAN = {
    1: dict(K=64, H=20, M=5, lam=0.1, sigma=0.3),
    2: dict(K=1024, H=64, M=10, lam=0.1, sigma=0.3),
    3: dict(K=4096, H=100, M=10, lam=0.1, sigma=0.3),
}


def plan_params(config: int, **overrides):
    """Plan parameters (K, H, M, lambda, sigma[14], eta, n_elite, seed)."""
    if config in PLAN:
        p = dict(PLAN[config])
    else:
        p = dict(K=1024, H=64, M=10, lam=0.1, sigma=0.3)
    p.update(eta=1.0, n_elite=p["K"], seed=0xC0FFEE + config)
    p.update(overrides)
    p["sigma"] = np.full(NU, float(p["sigma"])) if np.ndim(p["sigma"]) == 0 else np.asarray(p["sigma"], dtype=np.float64)
    return p


def packed_scenes(n=32, config=4):
    """Uneven batch: n independent scenes with K ~ U{256..4096}, H ~ U{32..128}."""
    out = []
    for i in range(n):
        sc = make_scene(config, i)
        rng = np.random.Generator(np.random.PCG64(77_000 + 1000 * config + i))
        K = int(rng.integers(256, 4097))
        H = int(rng.integers(32, 129))
        out.append((sc, plan_params(config, K=K, H=H, M=10, seed=(0xC0FFEE + config) * 1000 + i)))
    return out


def random_states(scene, n, seed, spread=0.3, vel=0.5):
    """Random perturbed states near home (for single-step parity tests)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    X = np.tile(initial_state(scene), (n, 1))
    X[:, 0:14] += rng.uniform(-spread, spread, size=(n, 14))
    X[:, 14:28] = rng.uniform(-vel, vel, size=(n, 14))
    X[:, 28:42] = X[:, 0:14] + rng.uniform(-0.05, 0.05, size=(n, 14))
    X[:, 42:45] += rng.uniform(-0.02, 0.02, size=(n, 3)) * np.array([1, 1, 0.5])
    q = rng.normal(size=(n, 4))
    X[:, 45:49] = q / np.linalg.norm(q, axis=1, keepdims=True)
    X[:, 49:52] = rng.uniform(-0.2, 0.2, size=(n, 3))
    X[:, 52:55] = rng.uniform(-1.0, 1.0, size=(n, 3))
    return X


def random_controls(n, H, seed, scale=1.0):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(-scale, scale, size=(n, H, NU))


def serving_cells(n=64, shape="mixed"):
    """Cells of the serving workload: cell i is scene make_scene(5, i) with a
    per-cell request rate ~ U[10, 50] Hz.  shape "mixed": K ~ U{256..4096},
    H ~ U{32..128} per cell (seeded); shape "fixed": K=1024, H=64."""
    out = []
    for i in range(n):
        rng = np.random.Generator(np.random.PCG64(55_000 + i))
        K = int(rng.integers(256, 4097))
        H = int(rng.integers(32, 129))
        rate = float(rng.uniform(10.0, 50.0))
        if shape == "fixed":
            K, H = 1024, 64
        out.append(dict(scene=make_scene(5, i), K=K, H=H, rate=rate, M=10))
    return out


def poisson_trace(rates, duration, seed=0):
    """Merged Poisson arrivals: list of (time_s, cell) sorted by time, cell i
    arriving at rates[i] per second over [0, duration)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ev = []
    for i, r in enumerate(rates):
        if r <= 0:
            continue
        t = rng.exponential(1.0 / r)
        while t < duration:
            ev.append((t, i))
            t += rng.exponential(1.0 / r)
    ev.sort()
    return ev


def qp_params(config: int = 2, **overrides):
    """Bounds and solver settings of the QP smoothing of sampled sequences:
    commanded joint positions within 1.5 rad of the home pose, velocity box
    from the scene (u_max), acceleration and jerk limits, ADMM penalty,
    over-relaxation and iteration count."""
    home = np.array(Q_HOME_ARM * 2, dtype=np.float64)
    p = dict(pos_lo=home - 1.5, pos_hi=home + 1.5, acc_max=4.0, jerk_max=60.0, rho=3.0, alpha=1.6, iters=60)
    p.update(overrides)
    return p


def cov_params(config: int = 2, **overrides):
    """Settings of the plan with covariance adaptation: the learning rate eta
    shared by the mean and covariance updates, and eps, the variance added
    to the diagonal after each covariance update ((rad/s)^2; 1e-4 is a
    standard deviation of 0.01 rad/s against the sampling sigma of 0.3)."""
    p = dict(eta=0.5, eps=1e-4)
    p.update(overrides)
    return p


def episode_scenes(config: int = 2, index: int = 0, **overrides):
    """The two cost configurations of the closed-loop ball task (Sec. IV-B
    phases): pick, without the object-to-target term (w_goal = 0), and move,
    with every term; same world, same physics."""
    move = make_scene(config, index, **overrides)
    pick = dict(move)
    pick["w_goal"] = 0.0
    return pick, move


def episode_params(config: int = 2, **overrides):
    """Executor settings of the closed-loop ball task: the first n_avg steps
    of the best sequence averaged and run for n_exec control steps per
    replan; grasp detected within 3 cm of the grasp point and 2 cm of the
    pad distance; success within 5 cm of the goal; the ball counts as lifted
    5 cm above its resting height and as fallen back below 1 cm above it;
    timeout t_max (the experiments use 120 s; shorter here); iterations M
    per warm-started replan; the elite set n_elite and learning rate eta of
    each replan; cov_eps, the variance floor of the covariance update when
    the full covariance is carried between replans (0.01 (rad/s)^2: a
    standard deviation of 0.1 against the sampling sigma of 0.3)."""
    sc = make_scene(config)
    r = float(sc["ball_r"])
    p = dict(n_avg=2, n_exec=2, max_replans=0, grasp_tol=0.03, width_tol=0.02, goal_tol=0.05,
             lift_z=r + 0.05, drop_z=r + 0.01, t_max=10.0, M=3, n_elite=32, eta=0.8, use_cov=0, cov_eps=0.01)
    p.update(overrides)
    return p


def _rot(axis, ang):
    """Unit quaternion (w, x, y, z) of a rotation by ang about a unit axis."""
    a = np.asarray(axis, dtype=np.float64)
    a = a / np.linalg.norm(a)
    return np.concatenate([[math.cos(ang / 2)], math.sin(ang / 2) * a])


def task_scene(task, phase, index=0, **overrides):
    """Scenes of the tray-moving task (Sec. IV-A; phases "pick", "move") and
    of the hand-over task (Sec. IV-C; phases "pick", "pass", "place") on the
    3-box workload's world: the free object is a box (the tray of half
    extents TRAY_H, mass TRAY_M, resting on the table at the origin; the
    cube of CUBE_H, CUBE_M, resting in front of arm 1) and the cost is the
    task's total with the phase's weights and targets (the paper switches
    w_pick / w_move, and the hand-over's per-arm phase weights, by phase).
    Weights are hand-set, as in the paper; the end-effector orientation
    targets are fixed quaternions (the synthetic arms' pads are spheres, so
    their orientation is a cost target only)."""
    base = make_scene(2, index)
    pad = PAD_RAD
    q_tilt = [_rot((0, 1, 0), 0.5 * math.pi), _rot((0, 1, 0), -0.5 * math.pi)]
    common = dict(ext=1, w_goal=0.0, w_eo=0.0, w_l=0.0, w_yz=0.0, w_s=0.01, w_c=10.0, w_home=0.1, n_cmax=8)
    if task == "tray":
        h = np.array(TRAY_H)
        grasp = np.array([[-(h[0] + pad), 0.0, h[2]], [h[0] + pad, 0.0, h[2]]])
        sc = dict(base, obj_box=1, obj_h=h, ball_m=TRAY_M, ball_r=float(h[2]), ball_p0=np.array([0.0, 0.0, h[2]]),
                  goal=np.array([0.0, 0.3, 0.25]), l_target=2.0 * (h[0] + pad), orot=np.array([1.0, 0, 0, 0]),
                  w_vert=1.0, w_relv=1.0, **common)
        if phase == "pick":     # w_pick = 1: C_p,pick (1/2 per arm), C_r,pick (1/2 per arm)
            sc.update(apos=grasp, w_apos=np.array([0.5, 0.5]), arot=np.array(q_tilt), w_arot=np.array([0.05, 0.05]))
        elif phase == "move":   # w_move = 1: C_l, C_p,tray (term 0), C_r,tray, C_r,move (1/2 per arm)
            sc.update(w_l=10.0, w_goal=1.0, w_orot=1.0, arot=np.array(q_tilt), w_arot=np.array([0.05, 0.05]))
        else:
            raise ValueError(phase)
    elif task == "handover":
        h = np.array(CUBE_H)
        p_obj = np.array([-0.25, 0.0, h[2]])
        target = np.array([0.3, 0.1, 0.15])
        sc = dict(base, obj_box=1, obj_h=h, ball_m=CUBE_M, ball_r=float(h[2]), ball_p0=p_obj, goal=target, **common)
        eps = float(base["eps_frac"]) * float(h[2])
        q_phase = {"pick": _rot((0, 1, 0), 0.5 * math.pi), "pass": _rot((1, 0, 0), 0.5 * math.pi),
                   "place": _rot((0, 1, 0), -0.5 * math.pi)}[phase]
        sc.update(arot=np.array([q_phase, q_phase]))
        if phase == "pick":     # arm 1 picks: C_p,1^pick, C_r,1^pick
            sc.update(apos=np.array([p_obj + [0, 0, eps], p_obj + [0, 0, eps]]), w_apos=np.array([1.0, 0.0]),
                      w_arot=np.array([0.1, 0.0]))
        elif phase == "pass":   # both arms to the pass line, aligned in yz: C_p^pass, w_pass C_yz
            sc.update(ax_t=np.array([-0.05, 0.05]), w_ax=np.array([1.0, 1.0]), w_yz=1.0,
                      w_arot=np.array([0.1, 0.1]))
        elif phase == "place":  # arm 2 places: C_p,2^place
            sc.update(apos=np.array([target, target]), w_apos=np.array([0.0, 1.0]), w_arot=np.array([0.0, 0.1]))
        else:
            raise ValueError(phase)
    else:
        raise ValueError(task)
    sc.update(overrides)
    return sc
