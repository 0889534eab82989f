"""FP64 CPU oracle of the bimanual MPPI hot path -- TEST INFRASTRUCTURE ONLY.

Only `tests/`, `__graft_entry__.smoke()` and the `cpu_baseline` leg of
`bench.py` may import this package.  The product library never loads it and
shares no code with it; both only consume the plain scene dictionaries of
`workloads`.

The C sources under `oracle/src` are plain FP64 loops written from the
paper (arXiv 2511.21264): Alg. 1 (sampling, projection, rollouts, cost,
elite set, update), Eqs. proj_cost/proj_bounds (velocity box -> clamp),
Eqs. mean_update/s_formula, Eq. collision_cost and the Sec. IV-B ball-task
costs.  The paper's world model (MuJoCo) fixes no physics, so the rigid-body
world is a set of readings documented in `oracle/src/*.c` headers.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle.so")
_SOURCES = ["philox.c", "model.c", "collide.c", "object.c", "step.c", "cost.c", "plan.c"]
NTERMS = 17

MAXBOX = 16
NX = 55


def build(verbose=False):
    """Compile the oracle (gcc, -O2, OpenMP) into oracle/_build/liboracle.so."""
    os.makedirs(_BUILD, exist_ok=True)
    srcs = [os.path.join(_HERE, "src", f) for f in _SOURCES]
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-march=native",
           "-ffp-contract=off", "-o", _LIB_PATH + ".tmp"] + srcs + ["-lm"]
    subprocess.run(cmd, check=True, capture_output=not verbose)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


class OScene(C.Structure):
    _fields_ = [
        ("base_pos", C.c_double * 6),
        ("base_cs", C.c_double * 4),
        ("axes", C.c_int * 7),
        ("link_len", C.c_double * 7),
        ("link_rad", C.c_double * 7),
        ("density", C.c_double * 14),
        ("pad_rad", C.c_double),
        ("ball_r", C.c_double), ("ball_m", C.c_double), ("ball_p0", C.c_double * 3),
        ("n_box", C.c_int),
        ("box_c", C.c_double * (3 * MAXBOX)),
        ("box_h", C.c_double * (3 * MAXBOX)),
        ("goal", C.c_double * 3),
        ("h", C.c_double), ("n_sub", C.c_int),
        ("kp", C.c_double), ("kd", C.c_double), ("damp", C.c_double),
        ("armature", C.c_double), ("tau_max", C.c_double),
        ("gravcomp", C.c_int), ("g", C.c_double),
        ("mu", C.c_double), ("kappa", C.c_double), ("eps_r", C.c_double),
        ("n_pgs", C.c_int), ("n_cmax", C.c_int),
        ("u_max", C.c_double),
        ("w_goal", C.c_double), ("w_eo", C.c_double), ("w_l", C.c_double), ("w_yz", C.c_double),
        ("w_s", C.c_double), ("w_c", C.c_double), ("gamma", C.c_double), ("m_c", C.c_double),
        ("eps_frac", C.c_double),
        ("obj_box", C.c_int), ("obj_h", C.c_double * 3),
        ("ext", C.c_int), ("l_target", C.c_double), ("q_home", C.c_double * 14),
        ("w_home", C.c_double), ("w_vert", C.c_double), ("w_relv", C.c_double), ("w_orot", C.c_double),
        ("w_apos", C.c_double * 2), ("w_ax", C.c_double * 2), ("w_arot", C.c_double * 2),
        ("apos", C.c_double * 6), ("ax_t", C.c_double * 2), ("arot", C.c_double * 8), ("orot", C.c_double * 4),
    ]


def _fill(arr, vals):
    vals = np.asarray(vals, dtype=np.float64).ravel()
    for i, v in enumerate(vals):
        arr[i] = float(v)


def make_oscene(sc: dict) -> OScene:
    s = OScene()
    _fill(s.base_pos, sc["base_pos"])
    _fill(s.base_cs, sc["base_cs"])
    for i, a in enumerate(sc["axes"]):
        s.axes[i] = int(a)
    _fill(s.link_len, sc["link_len"])
    _fill(s.link_rad, sc["link_rad"])
    _fill(s.density, sc["density"])
    s.pad_rad = sc["pad_rad"]
    s.ball_r, s.ball_m = sc["ball_r"], sc["ball_m"]
    _fill(s.ball_p0, sc["ball_p0"])
    nb = int(sc["n_box"])
    if nb > MAXBOX:
        raise ValueError("too many boxes")
    s.n_box = nb
    if nb:
        _fill(s.box_c, sc["box_c"])
        _fill(s.box_h, sc["box_h"])
    _fill(s.goal, sc["goal"])
    s.h, s.n_sub = sc["h"], int(sc["n_sub"])
    for k in ("kp", "kd", "damp", "armature", "tau_max", "g", "mu", "kappa", "eps_r", "u_max",
              "w_goal", "w_eo", "w_l", "w_yz", "w_s", "w_c", "gamma", "m_c", "eps_frac"):
        setattr(s, k, float(sc[k]))
    s.gravcomp = int(sc["gravcomp"])
    s.n_pgs = int(sc["n_pgs"])
    s.n_cmax = int(sc["n_cmax"])
    # the free object's shape and the further task-cost terms (defaults: a ball, terms off)
    s.obj_box = int(sc.get("obj_box", 0))
    _fill(s.obj_h, sc.get("obj_h", (0.0, 0.0, 0.0)))
    s.ext = int(sc.get("ext", 0))
    s.l_target = float(sc.get("l_target", 0.0))
    _fill(s.q_home, sc.get("q_home", np.zeros(14)))
    for k in ("w_home", "w_vert", "w_relv", "w_orot"):
        setattr(s, k, float(sc.get(k, 0.0)))
    for k in ("w_apos", "w_ax", "w_arot", "ax_t"):
        _fill(getattr(s, k), sc.get(k, (0.0, 0.0)))
    _fill(s.apos, sc.get("apos", np.zeros((2, 3))))
    _fill(s.arot, sc.get("arot", ((1.0, 0, 0, 0), (1.0, 0, 0, 0))))
    _fill(s.orot, sc.get("orot", (1.0, 0, 0, 0)))
    return s


_lib = None

_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_F = np.ctypeslib.ndpointer(dtype=np.float32, flags="C_CONTIGUOUS")
_I = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_U32 = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_S = C.POINTER(OScene)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        sig = {
            "oracle_philox": (None, [_U32, _U32, _U32]),
            "oracle_noise": (None, [C.c_uint64, C.c_int, C.c_int, C.c_int, _D]),
            "oracle_fk": (None, [_S, C.c_int, _D, _D, _D, _D, _D]),
            "oracle_model": (None, [_S, _D, _D, _D, _D]),
            "oracle_mass_matrix": (None, [_S, C.c_int, _D, _D]),
            "oracle_rnea": (None, [_S, C.c_int, _D, _D, _D, C.c_int, _D]),
            "oracle_cholesky": (C.c_int, [C.c_int, _D, _D]),
            "oracle_num_pairs": (C.c_int, [_S]),
            "oracle_pairs": (None, [_S, _I, _I]),
            "oracle_narrow_all": (None, [_S, _D, _D, _D, _D]),
            "oracle_aabbs": (None, [_S, _D, _D, _D]),
            "oracle_broadphase": (None, [_S, _F, _F, C.c_float, _I]),
            "oracle_seg_box_tstar": (C.c_double, [_D, _D, _D, _D]),
            "oracle_prim": (None, [C.c_int, _D, _D, C.c_double, C.c_int, _D, _D, C.c_double, _D]),
            "oracle_collision_cost": (None, [_D, C.c_int, C.c_int, C.c_double, _D]),
            "oracle_contacts": (None, [_S, _D, C.c_int, C.POINTER(C.c_int), _I, _D, _D, _D]),
            "oracle_substep": (None, [_S, _D, _D, _D, C.POINTER(C.c_int)]),
            "oracle_tangents": (None, [_D, _D, _D]),
            "oracle_lcp": (C.c_int, [_S, _D, _D, _D, _D, _D, _D]),
            "oracle_point_jac": (None, [_S, _D, C.c_int, _D, _D]),
            "oracle_obj_prim": (None, [_S, _D, C.c_int, _D, _D, C.c_double, _D]),
            "oracle_quat_R": (None, [_D, _D, _D]),
            "oracle_ext_terms": (None, [_S, _D, _D]),
            "oracle_rollout": (C.c_double, [_S, _D, _D, C.c_int, C.c_void_p, C.c_void_p]),
            "oracle_stage_terms": (None, [_S, _D, _D]),
            "oracle_cost_dist": (None, [_S, _D, _D]),
            "oracle_num_cost_pairs": (C.c_int, [_S]),
            "oracle_rollout_batch": (None, [_S, _D, _D, C.c_int, C.c_int, _D, C.c_void_p, C.c_int]),
            "oracle_sample": (None, [_S, _D, _D, C.c_int, C.c_uint64, C.c_int, C.c_int, C.c_int, _D]),
            "oracle_update": (C.c_int, [_D, _D, C.c_int, C.c_int, C.c_double, C.c_double, C.c_int, _D, _D,
                                        C.POINTER(C.c_double), C.POINTER(C.c_double)]),
            "oracle_plan": (C.c_int, [_S, _D, _D, C.c_int, C.c_int, C.c_double, _D, C.c_int, C.c_int,
                                      C.c_uint64, C.c_double, C.c_int, _D, _D, C.POINTER(C.c_int), _D,
                                      C.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _d(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


class Oracle:
    """Thin ctypes front-end over liboracle for one scene."""

    def __init__(self, scene: dict):
        self.scene = scene
        self.s = make_oscene(scene)
        self.L = lib()
        self.ps = C.byref(self.s)

    # -- noise ---------------------------------------------------------
    @staticmethod
    def philox(ctr, key):
        out = np.zeros(4, dtype=np.uint32)
        lib().oracle_philox(np.asarray(ctr, dtype=np.uint32), np.asarray(key, dtype=np.uint32), out)
        return out

    @staticmethod
    def noise(seed, K, H, m):
        z = np.zeros((K, H, 14))
        lib().oracle_noise(C.c_uint64(seed), K, H, m, z)
        return z

    # -- model ---------------------------------------------------------
    def model(self):
        m, Ix, Iz, ex = np.zeros(14), np.zeros(14), np.zeros(14), np.zeros(3)
        self.L.oracle_model(self.ps, m, Ix, Iz, ex)
        return dict(m=m.reshape(2, 7), Ix=Ix.reshape(2, 7), Iz=Iz.reshape(2, 7), ball_I=ex[0], eps=ex[1],
                    l_ball=ex[2])

    def fk(self, arm, q7):
        R, o, a, c = np.zeros(63), np.zeros(24), np.zeros(21), np.zeros(21)
        self.L.oracle_fk(self.ps, arm, _d(q7), R, o, a, c)
        return R.reshape(7, 3, 3), o.reshape(8, 3), a.reshape(7, 3), c.reshape(7, 3)

    def mass_matrix(self, arm, q7):
        M = np.zeros(49)
        self.L.oracle_mass_matrix(self.ps, arm, _d(q7), M)
        return M.reshape(7, 7)

    def rnea(self, arm, q7, qd, qdd, gravity):
        tau = np.zeros(7)
        self.L.oracle_rnea(self.ps, arm, _d(q7), _d(qd), _d(qdd), int(gravity), tau)
        return tau

    @staticmethod
    def cholesky(A):
        A = _d(A)
        n = A.shape[0]
        L = np.zeros((n, n))
        ok = lib().oracle_cholesky(n, A, L)
        return L if ok else None

    # -- collision -----------------------------------------------------
    def num_pairs(self):
        return self.L.oracle_num_pairs(self.ps)

    def pairs(self):
        n = self.num_pairs()
        ga, gb = np.zeros(n, dtype=np.int32), np.zeros(n, dtype=np.int32)
        self.L.oracle_pairs(self.ps, ga, gb)
        return ga, gb

    def narrow_all(self, x):
        n = self.num_pairs()
        phi, nrm, p = np.zeros(n), np.zeros(3 * n), np.zeros(3 * n)
        self.L.oracle_narrow_all(self.ps, _d(x), phi, nrm, p)
        return phi, nrm.reshape(n, 3), p.reshape(n, 3)

    def aabbs(self, x):
        ng = 16 + int(self.scene["n_box"])
        lo, hi = np.zeros(3 * ng), np.zeros(3 * ng)
        self.L.oracle_aabbs(self.ps, _d(x), lo, hi)
        return lo.reshape(ng, 3), hi.reshape(ng, 3)

    def broadphase(self, lo32, hi32, margin=0.0):
        n = self.num_pairs()
        flags = np.zeros(n, dtype=np.int32)
        self.L.oracle_broadphase(self.ps, np.ascontiguousarray(lo32, dtype=np.float32).ravel(),
                                 np.ascontiguousarray(hi32, dtype=np.float32).ravel(), C.c_float(margin), flags)
        return flags

    @staticmethod
    def seg_box_tstar(A, B, c, h):
        return lib().oracle_seg_box_tstar(_d(A), _d(B), _d(c), _d(h))

    @staticmethod
    def prim(ta, A0, A1, ra, tb, B0, B1, rb):
        """Narrowphase between two primitives (0 sphere, 1 capsule, 2 plane, 3 box)."""
        out = np.zeros(7)
        lib().oracle_prim(int(ta), _d(A0), _d(A1), float(ra), int(tb), _d(B0), _d(B1), float(rb), out)
        return out[0], out[1:4], out[4:7]

    @staticmethod
    def collision_cost(d, gamma):
        d = _d(d)
        H, B = d.shape
        out = np.zeros(2)
        lib().oracle_collision_cost(d, H, B, float(gamma), out)
        return out[0], out[1]

    def contacts(self, x, cap=64):
        n = C.c_int(0)
        pair = np.zeros(64, dtype=np.int32)
        phi, nrm, p = np.zeros(64), np.zeros(192), np.zeros(192)
        self.L.oracle_contacts(self.ps, _d(x), cap, C.byref(n), pair, phi, nrm, p)
        k = n.value
        return pair[:k], phi[:k], nrm.reshape(64, 3)[:k], p.reshape(64, 3)[:k]

    # -- dynamics ------------------------------------------------------
    def substep(self, x, u):
        xn = np.zeros(NX)
        nc = C.c_int(0)
        self.L.oracle_substep(self.ps, _d(x), _d(u), xn, C.byref(nc))
        return xn, nc.value

    def step(self, x, u):
        for _ in range(int(self.scene["n_sub"])):
            x, _ = self.substep(x, u)
        return x

    @staticmethod
    def tangents(n):
        t1, t2 = np.zeros(3), np.zeros(3)
        lib().oracle_tangents(_d(n), t1, t2)
        return t1, t2

    def point_jac(self, x, gid, p):
        """3 x 20 Jacobian of a point p rigidly attached to geom gid (global
        geom ids: 0 ball, 1 table, 2 + 7 arm + g arm geoms, 16 + b boxes)."""
        J = np.zeros(60)
        self.L.oracle_point_jac(self.ps, _d(x), int(gid), _d(p), J)
        return J.reshape(3, 20)

    def lcp(self, x, u):
        A, b, f, vf = np.zeros(64 * 64), np.zeros(64), np.zeros(64), np.zeros(20)
        m = self.L.oracle_lcp(self.ps, _d(x), _d(u), A, b, f, vf)
        return A[: m * m].reshape(m, m), b[:m], f[:m], vf

    # -- cost / rollout --------------------------------------------------
    def stage_terms(self, x):
        t = np.zeros(4)
        self.L.oracle_stage_terms(self.ps, _d(x), t)
        return t

    def cost_dist(self, x):
        n = self.L.oracle_num_cost_pairs(self.ps)
        d = np.zeros(max(n, 1))
        self.L.oracle_cost_dist(self.ps, _d(x), d)
        return d[:n]

    def obj_prim(self, xo, tb, B0, B1=None, rb=0.0):
        """The box object (state xo: centre, quaternion) against a primitive of
        type tb (0 sphere, 1 capsule, 2 plane, 3 axis-aligned box): phi, n, p."""
        out = np.zeros(7)
        B1 = B0 if B1 is None else B1
        self.L.oracle_obj_prim(self.ps, _d(xo), int(tb), _d(B0), _d(B1), float(rb), out)
        return out[0], out[1:4], out[4:7]

    def ext_terms(self, x):
        """The further task-cost terms 7..16 at state x (term 9 as its squared
        summand ((p1 - p2) . (p1' - p2'))^2)."""
        t = np.zeros(10)
        self.L.oracle_ext_terms(self.ps, _d(x), t)
        return t

    @staticmethod
    def quat_R(q):
        """Rotation matrix of a unit quaternion (w, x, y, z), and the quaternion
        recovered from it."""
        R, qb = np.zeros(9), np.zeros(4)
        lib().oracle_quat_R(_d(q), R, qb)
        return R.reshape(3, 3), qb

    def rollout(self, x0, U, want_traj=False):
        U = _d(U)
        H = U.shape[0]
        terms = np.zeros(NTERMS)
        traj = np.zeros((H, NX)) if want_traj else None
        c = self.L.oracle_rollout(self.ps, _d(x0), U, H,
                                  traj.ctypes.data_as(C.c_void_p) if want_traj else None,
                                  terms.ctypes.data_as(C.c_void_p))
        return (c, terms, traj) if want_traj else (c, terms)

    def rollout_batch(self, x0, U, nthreads=None, want_final=False):
        U = _d(U)
        n, H = U.shape[0], U.shape[1]
        costs = np.zeros(n)
        fin = np.zeros((n, NX)) if want_final else None
        self.L.oracle_rollout_batch(self.ps, _d(x0), U, n, H, costs,
                                    fin.ctypes.data_as(C.c_void_p) if want_final else None,
                                    nthreads or os.cpu_count())
        return (costs, fin) if want_final else costs

    # -- MPPI ------------------------------------------------------------
    def sample(self, nu, sigma, seed, K, m):
        nu = _d(nu)
        H = nu.shape[0]
        sigma = _d(sigma)
        per_step = int(sigma.size == H * 14 and sigma.size != 14)
        U = np.zeros((K, H, 14))
        self.L.oracle_sample(self.ps, nu, sigma, per_step, C.c_uint64(seed), K, H, m, U)
        return U

    @staticmethod
    def update(U, costs, lam, nu, eta=1.0, n_elite=None):
        U = _d(U)
        K, H = U.shape[0], U.shape[1]
        out = np.zeros((H, 14))
        ws, ess = C.c_double(0), C.c_double(0)
        nf = lib().oracle_update(U, _d(costs), K, H, float(lam), float(eta), int(n_elite or K), _d(nu), out,
                                 C.byref(ws), C.byref(ess))
        return out, nf, ess.value

    def plan(self, x0, nominal, K, H, lam, sigma, M, seed, eta=1.0, n_elite=None, nthreads=None):
        nominal = _d(nominal).reshape(H, 14)
        sigma = _d(sigma)
        per_step = int(sigma.size == H * 14 and sigma.size != 14)
        nu = np.zeros((H, 14))
        costs = np.zeros(K)
        best = C.c_int(-1)
        cmin = np.zeros(M)
        rc = self.L.oracle_plan(self.ps, _d(x0), nominal, K, H, float(lam), sigma, per_step, M, C.c_uint64(seed),
                                float(eta), int(n_elite or K), nu, costs, C.byref(best), cmin,
                                int(nthreads or os.cpu_count()))
        return dict(rc=rc, nu=nu, costs=costs, best=best.value, cmin_iter=cmin)
