"""Python binding of the MI355X MPPI rollout library (libmppi.so, C ABI in include/mppi.h).

Argument marshalling only: every stage of the hot path (noise, projection,
rollout, cost, weights, update) runs in the HIP kernels of the library.
Arrays are torch tensors on the GPU (passed as device pointers, launched on
the current torch stream) or numpy arrays (staged by the library).  The
library must be built (``__graft_entry__.build()``); there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os
import weakref

import numpy as np

from ._build import LIB_PATH, build  # noqa: F401

NU = 14
NX = 55
MAX_BOXES = 16

OK, E_INVAL, E_NOMEM, E_MODEL, E_DIVERGED, E_DEVICE, E_BUSY, E_CANCELLED = 0, -1, -2, -3, -4, -5, -6, -7
E_NOTPD = -8
E_LATE = -9
COV_MAX_N = 3584
PENDING = 1
DEVICE_PTRS, SIGMA_PER_STEP, SYNC, TIME_KERNELS, TRAJ, MAP_LANE, MAP_TEAM, SUPERSEDE = 1, 2, 4, 8, 16, 32, 64, 128
MAP_WAVE, FP32_WEIGHTS, GRAPH, MAP_SPLIT, PER_STEP = 256, 512, 1024, 2048, 4096
_MAPS = {None: 0, "auto": 0, "lane": MAP_LANE, "team": MAP_TEAM, "wave": MAP_WAVE, "split": MAP_SPLIT}


class MppiError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"mppi error {code}: {msg}")
        self.code = code


class SceneDesc(C.Structure):
    _fields_ = [
        ("base_pos", C.c_double * 6),
        ("base_cs", C.c_double * 4),
        ("axes", C.c_int * 7),
        ("link_len", C.c_double * 7),
        ("link_rad", C.c_double * 7),
        ("density", C.c_double * 14),
        ("pad_rad", C.c_double),
        ("ball_r", C.c_double), ("ball_m", C.c_double),
        ("n_box", C.c_int),
        ("box_c", C.c_double * (3 * MAX_BOXES)),
        ("box_h", C.c_double * (3 * MAX_BOXES)),
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


NTERMS = 17


class Opts(C.Structure):
    _fields_ = [("M", C.c_int), ("seed", C.c_uint64), ("eta", C.c_double), ("n_elite", C.c_int),
                ("flags", C.c_uint)]


class QP(C.Structure):
    """mppi_qp: bounds and solver settings of the QP smoothing."""
    _fields_ = [("pos_lo", C.c_double * 14), ("pos_hi", C.c_double * 14), ("acc_max", C.c_double),
                ("jerk_max", C.c_double), ("rho", C.c_double), ("alpha", C.c_double), ("iters", C.c_int)]


def make_qp(params):
    """An mppi_qp from a dict with pos_lo[14], pos_hi[14], acc_max, jerk_max, rho, alpha, iters."""
    q = QP()
    for d in range(14):
        q.pos_lo[d] = float(params["pos_lo"][d])
        q.pos_hi[d] = float(params["pos_hi"][d])
    q.acc_max, q.jerk_max = float(params["acc_max"]), float(params["jerk_max"])
    q.rho, q.alpha, q.iters = float(params["rho"]), float(params["alpha"]), int(params["iters"])
    return q


class Cov(C.Structure):
    _fields_ = [("Sigma0", C.c_void_p), ("Sigma_out", C.c_void_p), ("eps", C.c_double), ("U_best", C.c_void_p)]


class EpisodeOpts(C.Structure):
    _fields_ = [("n_avg", C.c_int), ("n_exec", C.c_int), ("max_replans", C.c_int), ("use_cov", C.c_int),
                ("grasp_tol", C.c_double), ("width_tol", C.c_double), ("goal_tol", C.c_double),
                ("lift_z", C.c_double), ("drop_z", C.c_double), ("t_max", C.c_double), ("cov_eps", C.c_double)]


class EpisodeResult(C.Structure):
    _fields_ = [("status", C.c_int), ("phase", C.c_int), ("n_replans", C.c_int), ("n_steps", C.c_int),
                ("t_end", C.c_double), ("t_switch", C.c_double), ("t_comp_mean_ms", C.c_double),
                ("t_comp_std_ms", C.c_double), ("t_comp_max_ms", C.c_double), ("goal_dist_min", C.c_double),
                ("ball_final", C.c_double * 3), ("n_diverged", C.c_int), ("pad2", C.c_int)]

    def as_dict(self):
        d = {f: getattr(self, f) for f, _ in self._fields_ if not f.startswith("pad")}
        d["ball_final"] = list(self.ball_final)
        return d


EPISODE_STATUS = {1: "success", -1: "collision", -2: "timeout", -3: "ball fell", 0: "replan cap"}


class Stats(C.Structure):
    _fields_ = [
        ("ess", C.c_double), ("c_min", C.c_double), ("best", C.c_int), ("n_nonfinite", C.c_int),
        ("diverged", C.c_int), ("iterations", C.c_int), ("cmin_iter", C.c_double * 64),
        ("contacts", C.c_double), ("np_tests", C.c_double), ("box_tests", C.c_double),
        ("overflow", C.c_double), ("rollout_ms", C.c_float), ("rollout_launches", C.c_int),
    ]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "cmin_iter"}
        d["cmin_iter"] = list(self.cmin_iter[: max(0, min(64, self.iterations))])
        return d


class Request(C.Structure):
    _fields_ = [
        ("scene", C.c_void_p), ("x0", C.c_void_p), ("nominal_U", C.c_void_p), ("K", C.c_int), ("H", C.c_int),
        ("lam", C.c_double), ("sigma", C.c_void_p), ("opts", Opts), ("U_new", C.c_void_p), ("costs", C.c_void_p),
        ("stats", C.POINTER(Stats)), ("status", C.c_int),
    ]


class ServerOpts(C.Structure):
    _fields_ = [("mem_budget", C.c_uint64), ("max_active", C.c_int), ("max_pending", C.c_int), ("flags", C.c_uint),
                ("deadline_ms", C.c_double), ("iter_base_ms", C.c_double), ("iter_ms_per_menv", C.c_double)]


class TicketInfo(C.Structure):
    _fields_ = [("status", C.c_int), ("iterations", C.c_int), ("t_submit_ms", C.c_double),
                ("t_admit_ms", C.c_double), ("t_done_ms", C.c_double), ("t_deadline_ms", C.c_double)]


class ServerInfo(C.Structure):
    _fields_ = [("submitted", C.c_uint64), ("completed", C.c_uint64), ("cancelled", C.c_uint64),
                ("superseded", C.c_uint64), ("rejected", C.c_uint64), ("iterations", C.c_uint64),
                ("request_iters", C.c_uint64), ("env_steps", C.c_uint64), ("mem_high_water", C.c_uint64),
                ("active", C.c_int), ("pending", C.c_int), ("shed", C.c_uint64), ("late", C.c_uint64),
                ("model_base_ms", C.c_double), ("model_ms_per_menv", C.c_double), ("model_floor_ms", C.c_double),
                ("model_margin_ms", C.c_double)]


_lib = None
_P = C.c_void_p


def lib():
    """Load libmppi.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library missing: {LIB_PATH} (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        sig = {
            "mppi_ctx_create": (C.c_int, [C.c_int, C.POINTER(_P)]),
            "mppi_ctx_destroy": (None, [_P]),
            "mppi_last_error": (C.c_char_p, []),
            "mppi_scene_create": (C.c_int, [_P, C.POINTER(SceneDesc), C.POINTER(_P)]),
            "mppi_scene_destroy": (None, [_P]),
            "mppi_scene_num_pairs": (C.c_int, [_P, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
            "mppi_plan": (C.c_int, [_P, _P, _P, _P, C.c_int, C.c_int, C.c_double, _P, C.POINTER(Opts), _P, _P,
                                    C.POINTER(Stats), _P]),
            "mppi_plan_noalloc": (C.c_int, [_P, _P, _P, _P, C.c_int, C.c_int, C.c_double, _P, C.POINTER(Opts), _P,
                                            _P, C.POINTER(Stats), _P]),
            "mppi_simulate": (C.c_int, [_P, _P, _P, C.c_int, _P, C.c_int, C.c_int, C.c_int, _P, _P, _P, C.c_uint,
                                        _P]),
            "mppi_plan_batch": (C.c_int, [_P, C.c_int, C.POINTER(Request), C.c_uint, _P]),
            "mppi_server_create": (C.c_int, [_P, C.POINTER(ServerOpts), C.POINTER(_P)]),
            "mppi_server_destroy": (None, [_P]),
            "mppi_cell_create": (C.c_int, [_P, _P, C.c_int, _P, _P, C.POINTER(C.c_int)]),
            "mppi_cell_read": (C.c_int, [_P, C.c_int, _P, _P]),
            "mppi_submit": (C.c_int, [_P, C.POINTER(Request), C.c_int, C.c_int, C.c_uint, C.POINTER(C.c_uint64)]),
            "mppi_poll": (C.c_int, [_P, C.c_uint64, C.c_int, C.POINTER(TicketInfo)]),
            "mppi_cancel": (C.c_int, [_P, C.c_uint64]),
            "mppi_server_query": (C.c_int, [_P, C.POINTER(ServerInfo)]),
            "mppi_sample": (C.c_int, [_P, _P, _P, _P, C.c_uint64, C.c_int, C.c_int, C.c_int, _P, _P, _P, C.c_uint,
                                      _P]),
            "mppi_update": (C.c_int, [_P, _P, _P, _P, _P, C.c_uint64, C.c_int, C.c_int, C.c_int, C.c_double,
                                      C.c_double, C.c_int, _P, _P, _P, C.POINTER(Stats), C.c_uint, _P]),
            "mppi_autotune": (C.c_int, [_P, _P, _P, _P, C.c_int, C.c_int, C.POINTER(C.c_int), _P]),
            "mppi_project": (C.c_int, [_P, _P, _P, C.c_int, _P, _P, C.c_int, C.c_int, C.POINTER(QP), C.c_uint, _P]),
            "mppi_plan_qp": (C.c_int, [_P, _P, _P, _P, C.c_int, C.c_int, C.c_double, _P, C.POINTER(Opts),
                                       C.POINTER(QP), _P, _P, C.POINTER(Stats), _P]),
            "mppi_cov_update": (C.c_int, [_P, _P, _P, _P, _P, C.c_double, C.c_double, _P, C.c_int, C.c_int,
                                          C.c_uint, _P]),
            "mppi_cholesky": (C.c_int, [_P, _P, _P, C.c_int, C.c_uint, _P]),
            "mppi_sample_full": (C.c_int, [_P, _P, _P, C.c_uint64, C.c_int, C.c_int, C.c_int, C.c_float, _P,
                                           C.c_uint, _P]),
            "mppi_plan_cov": (C.c_int, [_P, _P, _P, _P, C.c_int, C.c_int, C.c_double, _P, C.POINTER(Opts),
                                        C.POINTER(Cov), C.POINTER(QP), _P, _P, C.POINTER(Stats), _P]),
            "mppi_plan_best": (C.c_int, [_P, _P, _P, _P, C.c_int, C.c_int, C.c_double, _P, C.POINTER(Opts), _P, _P,
                                         _P, C.POINTER(Stats), _P]),
            "mppi_episode": (C.c_int, [_P, _P, _P, _P, C.c_int, C.c_int, C.c_double, _P, C.POINTER(Opts),
                                       C.POINTER(EpisodeOpts), C.POINTER(QP), _P, _P, _P, C.POINTER(EpisodeResult),
                                       _P]),
            "mppi_broadphase": (C.c_int, [_P, _P, _P, _P, C.c_int, C.c_float, _P, C.c_uint, _P]),
            "mppi_narrowphase": (C.c_int, [_P, _P, _P, C.c_int, _P, _P, _P, _P, _P, C.c_uint, _P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise MppiError(rc, lib().mppi_last_error().decode())
    return rc


def _fill(arr, vals):
    vals = np.asarray(vals, dtype=np.float64).ravel()
    for i, v in enumerate(vals):
        arr[i] = float(v)


def scene_desc(sc: dict) -> SceneDesc:
    """Marshal a scene dictionary (see workloads.make_scene) into mppi_scene_desc."""
    d = SceneDesc()
    _fill(d.base_pos, sc["base_pos"])
    _fill(d.base_cs, sc["base_cs"])
    for i, a in enumerate(sc["axes"]):
        d.axes[i] = int(a)
    _fill(d.link_len, sc["link_len"])
    _fill(d.link_rad, sc["link_rad"])
    _fill(d.density, sc["density"])
    d.pad_rad = float(sc["pad_rad"])
    d.ball_r, d.ball_m = float(sc["ball_r"]), float(sc["ball_m"])
    d.n_box = int(sc["n_box"])
    if d.n_box > MAX_BOXES:
        raise ValueError("too many boxes")
    if d.n_box:
        _fill(d.box_c, sc["box_c"])
        _fill(d.box_h, sc["box_h"])
    _fill(d.goal, sc["goal"])
    d.h, d.n_sub = float(sc["h"]), int(sc["n_sub"])
    for k in ("kp", "kd", "damp", "armature", "tau_max", "g", "mu", "kappa", "eps_r", "u_max",
              "w_goal", "w_eo", "w_l", "w_yz", "w_s", "w_c", "gamma", "m_c", "eps_frac"):
        setattr(d, k, float(sc[k]))
    d.gravcomp = int(sc["gravcomp"])
    d.n_pgs = int(sc["n_pgs"])
    d.n_cmax = int(sc["n_cmax"])
    # the free object's shape and the further task-cost terms (defaults: a ball, terms off)
    d.obj_box = int(sc.get("obj_box", 0))
    _fill(d.obj_h, sc.get("obj_h", (0.0, 0.0, 0.0)))
    d.ext = int(sc.get("ext", 0))
    d.l_target = float(sc.get("l_target", 0.0))
    _fill(d.q_home, sc.get("q_home", np.zeros(14)))
    for k in ("w_home", "w_vert", "w_relv", "w_orot"):
        setattr(d, k, float(sc.get(k, 0.0)))
    for k in ("w_apos", "w_ax", "w_arot", "ax_t"):
        _fill(getattr(d, k), sc.get(k, (0.0, 0.0)))
    _fill(d.apos, sc.get("apos", np.zeros((2, 3))))
    _fill(d.arot, sc.get("arot", ((1.0, 0, 0, 0), (1.0, 0, 0, 0))))
    _fill(d.orot, sc.get("orot", (1.0, 0, 0, 0)))
    return d


def _is_dev(a):
    try:
        import torch
        return isinstance(a, torch.Tensor) and a.is_cuda
    except ImportError:  # pragma: no cover
        return False


def _ptr(a, dtype):
    """(pointer, on_device) of a contiguous array of `dtype` (numpy dtype)."""
    if a is None:
        return None, None
    if _is_dev(a):
        import torch
        tdt = {np.float32: torch.float32, np.float64: torch.float64, np.int32: torch.int32,
               np.uint32: torch.int32}[dtype]
        if a.dtype != tdt and not (dtype is np.uint32 and a.dtype == torch.int32):
            raise TypeError(f"expected {tdt}, got {a.dtype}")
        if not a.is_contiguous():
            raise ValueError("device arrays must be contiguous")
        return a.data_ptr(), True
    if not (isinstance(a, np.ndarray) and a.dtype == dtype and a.flags["C_CONTIGUOUS"]):
        raise TypeError(f"expected a C-contiguous numpy array of {np.dtype(dtype)}")
    return a.ctypes.data, False


def _ptrs(specs):
    """Marshal [(array, dtype)] that must all live on the same side."""
    out, side = [], None
    for a, dt in specs:
        p, dev = _ptr(a, dt)
        if p is not None:
            if side is None:
                side = dev
            elif side != dev:
                raise ValueError("mixing device and host arrays in one call")
        out.append(p)
    return out, bool(side)


def _stream(dev, stream):
    if stream is not None:
        return stream
    if dev:
        import torch
        return torch.cuda.current_stream().cuda_stream
    return None


class Context:
    """A device context.  Closing it first closes the servers, then the
    scenes made on it that are still open (their handles die with it)."""

    def __init__(self, device: int = 0):
        self._h = _P()
        _check(lib().mppi_ctx_create(device, C.byref(self._h)))
        self.device = device
        self._servers = weakref.WeakSet()
        self._scenes = weakref.WeakSet()

    def close(self):
        if self._h:
            for srv in list(self._servers):
                srv.close()
            for sc in list(self._scenes):
                sc.close()
            lib().mppi_ctx_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Scene:
    def __init__(self, ctx: Context, scene: dict):
        self.ctx = ctx
        self.dict = scene
        self.desc = scene_desc(scene)
        self._h = _P()
        _check(lib().mppi_scene_create(ctx._h, C.byref(self.desc), C.byref(self._h)))
        ctx._scenes.add(self)
        a, b = C.c_int(0), C.c_int(0)
        _check(lib().mppi_scene_num_pairs(self._h, C.byref(a), C.byref(b)))
        self.n_pairs, self.n_cost_pairs = a.value, b.value
        self.n_geoms = 16 + int(scene["n_box"])

    def close(self):
        if self._h:
            lib().mppi_scene_destroy(self._h)
            self._h = _P()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mppi_plan_noalloc(ctx, scene, x0, nominal_U, K, H, lam, sigma, U_new, costs=None, *, M=1, seed=0, eta=1.0,
                      n_elite=0, sigma_per_step=False, want_stats=True, sync=False, stream=None, mapping=None,
                      fp32_weights=False):
    """mppi_plan whose working memory is the library's static device array
    (no device allocation); every array must be a torch tensor on the GPU."""
    (px0, pnom, psig, pU, pc), dev = _ptrs([(x0, np.float32), (nominal_U, np.float32), (sigma, np.float32),
                                             (U_new, np.float32), (costs, np.float32)])
    if not dev:
        raise ValueError("mppi_plan_noalloc takes device arrays")
    flags = DEVICE_PTRS | (SIGMA_PER_STEP if sigma_per_step else 0) | (SYNC if sync else 0) | _MAPS[mapping] | \
        (FP32_WEIGHTS if fp32_weights else 0)
    o = Opts(int(M), int(seed) & 0xFFFFFFFFFFFFFFFF, float(eta), int(n_elite), flags)
    st = Stats()
    rc = lib().mppi_plan_noalloc(ctx._h, scene._h, px0, pnom, int(K), int(H), float(lam), psig, C.byref(o), pU, pc,
                                 C.byref(st) if want_stats else None, _stream(dev, stream))
    if rc == E_DIVERGED:
        d = st.as_dict()
        d["rc"] = rc
        return d
    _check(rc)
    if want_stats:
        d = st.as_dict()
        d["rc"] = rc
        return d
    return None


def mppi_plan(ctx, scene, x0, nominal_U, K, H, lam, sigma, U_new, costs=None, *, M=1, seed=0, eta=1.0,
              n_elite=0, sigma_per_step=False, time_kernels=False, want_stats=True, sync=False, stream=None,
              mapping=None, fp32_weights=False, graph=False, per_step=False):
    """One plan (Alg. 1).  Arrays: x0[55], nominal_U[H,14], sigma[14] or [H,14],
    U_new[H,14] (out), costs[K] (out).  mapping: None/"auto", "lane", "team",
    "wave" or "split"; per_step: the plain form (one launch per control step).
    Returns a stats dict (or None)."""
    (px0, pnom, psig, pU, pc), dev = _ptrs([(x0, np.float32), (nominal_U, np.float32), (sigma, np.float32),
                                             (U_new, np.float32), (costs, np.float32)])
    flags = (DEVICE_PTRS if dev else 0) | (SIGMA_PER_STEP if sigma_per_step else 0) | \
            (TIME_KERNELS if time_kernels else 0) | (SYNC if sync else 0) | _MAPS[mapping] | \
            (FP32_WEIGHTS if fp32_weights else 0) | (GRAPH if graph else 0) | (PER_STEP if per_step else 0)
    o = Opts(int(M), int(seed) & 0xFFFFFFFFFFFFFFFF, float(eta), int(n_elite), flags)
    st = Stats()
    rc = lib().mppi_plan(ctx._h, scene._h, px0, pnom, int(K), int(H), float(lam), psig, C.byref(o), pU, pc,
                         C.byref(st) if want_stats else None, _stream(dev, stream))
    if rc == E_DIVERGED:
        d = st.as_dict()
        d["rc"] = rc
        return d
    _check(rc)
    if want_stats:
        d = st.as_dict()
        d["rc"] = rc
        return d
    return None


def mppi_plan_qp(ctx, scene, x0, nominal_U, K, H, lam, sigma, qp, U_new, costs=None, *, M=1, seed=0, eta=1.0,
                 n_elite=0, sigma_per_step=False, time_kernels=False, want_stats=True, sync=False, stream=None,
                 mapping=None, fp32_weights=False):
    """mppi_plan with the QP smoothing of every sample; qp: a dict for make_qp
    or a QP structure.  Returns a stats dict (or None)."""
    q = qp if isinstance(qp, QP) else make_qp(qp)
    (px0, pnom, psig, pU, pc), dev = _ptrs([(x0, np.float32), (nominal_U, np.float32), (sigma, np.float32),
                                             (U_new, np.float32), (costs, np.float32)])
    flags = (DEVICE_PTRS if dev else 0) | (SIGMA_PER_STEP if sigma_per_step else 0) | \
            (TIME_KERNELS if time_kernels else 0) | (SYNC if sync else 0) | _MAPS[mapping] | \
            (FP32_WEIGHTS if fp32_weights else 0)
    o = Opts(int(M), int(seed) & 0xFFFFFFFFFFFFFFFF, float(eta), int(n_elite), flags)
    st = Stats()
    rc = lib().mppi_plan_qp(ctx._h, scene._h, px0, pnom, int(K), int(H), float(lam), psig, C.byref(o), C.byref(q),
                            pU, pc, C.byref(st) if want_stats else None, _stream(dev, stream))
    if rc == E_DIVERGED:
        d = st.as_dict()
        d["rc"] = rc
        return d
    _check(rc)
    if want_stats:
        d = st.as_dict()
        d["rc"] = rc
        return d
    return None


def mppi_plan_best(ctx, scene, x0, nominal_U, K, H, lam, sigma, U_new, U_best, costs=None, *, M=1, seed=0, eta=1.0,
                   n_elite=0, sigma_per_step=False, want_stats=True, sync=False, stream=None, mapping=None):
    """mppi_plan that also returns the best sequence of the final iteration
    in U_best[H, 14].  Returns a stats dict (or None)."""
    (px0, pnom, psig, pU, pB, pc), dev = _ptrs([(x0, np.float32), (nominal_U, np.float32), (sigma, np.float32),
                                                 (U_new, np.float32), (U_best, np.float32), (costs, np.float32)])
    flags = (DEVICE_PTRS if dev else 0) | (SIGMA_PER_STEP if sigma_per_step else 0) | (SYNC if sync else 0) | \
        _MAPS[mapping]
    o = Opts(int(M), int(seed) & 0xFFFFFFFFFFFFFFFF, float(eta), int(n_elite), flags)
    st = Stats()
    rc = lib().mppi_plan_best(ctx._h, scene._h, px0, pnom, int(K), int(H), float(lam), psig, C.byref(o), pU, pB, pc,
                              C.byref(st) if want_stats else None, _stream(dev, stream))
    if rc == E_DIVERGED:
        d = st.as_dict()
        d["rc"] = rc
        return d
    _check(rc)
    if want_stats:
        d = st.as_dict()
        d["rc"] = rc
        return d
    return None


def make_episode_opts(params):
    """An mppi_episode_opts from a dict (see workloads.episode_params)."""
    e = EpisodeOpts()
    for f, _ in EpisodeOpts._fields_:
        if f in ("use_cov", "cov_eps"):
            setattr(e, f, params.get(f, 0))
        else:
            setattr(e, f, params[f])
    return e


def mppi_episode(ctx, pick, move, x0, K, H, lam, sigma, eo, *, qp=None, M=1, seed=0, eta=1.0, n_elite=0,
                 sigma_per_step=False, mapping=None, record=False, stream=None):
    """Closed-loop run of the ball task (host arrays).  eo: dict or
    EpisodeOpts; qp: dict or QP for the smoothing of every replan's samples.
    Returns the result dict, with x_final and, when `record`, u_exec[n_replans,
    14] and x_hist[n_replans, NX] (needs max_replans > 0)."""
    e = eo if isinstance(eo, EpisodeOpts) else make_episode_opts(eo)
    q = None if qp is None else (qp if isinstance(qp, QP) else make_qp(qp))
    x0 = np.ascontiguousarray(x0, dtype=np.float32)
    sigma = np.ascontiguousarray(sigma, dtype=np.float32)
    xf = np.zeros(NX, np.float32)
    ue = np.zeros((max(e.max_replans, 1), 14), np.float32) if record else None
    xh = np.zeros((max(e.max_replans, 1), NX), np.float32) if record else None
    flags = (SIGMA_PER_STEP if sigma_per_step else 0) | _MAPS[mapping]
    o = Opts(int(M), int(seed) & 0xFFFFFFFFFFFFFFFF, float(eta), int(n_elite), flags)
    r = EpisodeResult()
    _check(lib().mppi_episode(ctx._h, pick._h, move._h, x0.ctypes.data, int(K), int(H), float(lam),
                              sigma.ctypes.data, C.byref(o), C.byref(e), C.byref(q) if q is not None else None,
                              xf.ctypes.data,
                              ue.ctypes.data if record else None, xh.ctypes.data if record else None, C.byref(r),
                              stream))
    d = r.as_dict()
    d["outcome"] = EPISODE_STATUS.get(d["status"], "?")
    d["x_final"] = xf
    if record:
        d["u_exec"] = ue[:r.n_replans]
        d["x_hist"] = xh[:r.n_replans]
    return d


def mppi_plan_cov(ctx, scene, x0, nominal_U, K, H, lam, sigma, U_new, costs=None, *, eps=0.0, Sigma0=None,
                  Sigma_out=None, U_best=None, qp=None, M=1, seed=0, eta=1.0, n_elite=0, sigma_per_step=False,
                  want_stats=True, stream=None, mapping=None):
    """mppi_plan with the full covariance over the sequence (Sigma0[n, n] or
    None for diag(sigma^2); Sigma_out[n, n] receives Sigma_M), optionally
    with the QP smoothing (qp: dict or QP).  Synchronises.  Returns a stats
    dict."""
    q = None if qp is None else (qp if isinstance(qp, QP) else make_qp(qp))
    (px0, pnom, psig, pU, pc, pS0, pSo, pB), dev = _ptrs([(x0, np.float32), (nominal_U, np.float32),
                                                          (sigma, np.float32), (U_new, np.float32),
                                                          (costs, np.float32), (Sigma0, np.float64),
                                                          (Sigma_out, np.float64), (U_best, np.float32)])
    flags = (DEVICE_PTRS if dev else 0) | (SIGMA_PER_STEP if sigma_per_step else 0) | _MAPS[mapping]
    o = Opts(int(M), int(seed) & 0xFFFFFFFFFFFFFFFF, float(eta), int(n_elite), flags)
    cv = Cov(pS0, pSo, float(eps), pB)
    st = Stats()
    rc = lib().mppi_plan_cov(ctx._h, scene._h, px0, pnom, int(K), int(H), float(lam), psig, C.byref(o), C.byref(cv),
                             C.byref(q) if q is not None else None, pU, pc, C.byref(st) if want_stats else None,
                             _stream(dev, stream))
    if rc == E_DIVERGED:
        d = st.as_dict()
        d["rc"] = rc
        return d
    _check(rc)
    if want_stats:
        d = st.as_dict()
        d["rc"] = rc
        return d
    return None


def mppi_cov_update(ctx, U, w, nu_new, Sigma_in, Sigma_out, eta, eps=0.0, *, sync=True, stream=None):
    """Sigma_out = (1 - eta) Sigma_in + eta Delta Sigma + eps I from the samples
    U[K, n] (or [K, H, 14]), weights w[K] and the updated mean nu_new[n]."""
    K = U.shape[0]
    n = int(np.prod(U.shape[1:]))
    (pU, pw, pnu, pSi, pSo), dev = _ptrs([(U, np.float32), (w, np.float64), (nu_new, np.float64),
                                           (Sigma_in, np.float64), (Sigma_out, np.float64)])
    flags = (DEVICE_PTRS if dev else 0) | (SYNC if sync else 0)
    _check(lib().mppi_cov_update(ctx._h, pU, pw, pnu, pSi, float(eta), float(eps), pSo, int(K), n, flags,
                                 _stream(dev, stream)))


def mppi_cholesky(ctx, Sigma, L, *, stream=None):
    """L (lower, upper zeroed) with L L^T = Sigma; raises MppiError(E_NOTPD)
    when a pivot is not positive."""
    n = Sigma.shape[0]
    (pS, pL), dev = _ptrs([(Sigma, np.float64), (L, np.float64)])
    _check(lib().mppi_cholesky(ctx._h, pS, pL, int(n), DEVICE_PTRS if dev else 0, _stream(dev, stream)))


def mppi_sample_full(ctx, nu, L, seed, m, K, U, u_max, *, sync=True, stream=None):
    """U[K, H, 14] = clip(nu + L z_j, +-u_max) for iteration m of `seed`."""
    H = nu.shape[0]
    (pnu, pL, pU), dev = _ptrs([(nu, np.float32), (L, np.float64), (U, np.float32)])
    flags = (DEVICE_PTRS if dev else 0) | (SYNC if sync else 0)
    _check(lib().mppi_sample_full(ctx._h, pnu, pL, int(seed) & 0xFFFFFFFFFFFFFFFF, int(m), int(K), int(H),
                                  float(u_max), pU, flags, _stream(dev, stream)))


def mppi_project(ctx, scene, X0, U_in, U_out, qp, *, x0_shared=False, sync=True, stream=None):
    """QP smoothing of U_in[K,H,14] into U_out[K,H,14] from the start states
    X0[K,55] (or one shared state)."""
    q = qp if isinstance(qp, QP) else make_qp(qp)
    (px0, pin, pout), dev = _ptrs([(X0, np.float32), (U_in, np.float32), (U_out, np.float32)])
    K, H = U_in.shape[0], U_in.shape[1]
    flags = (DEVICE_PTRS if dev else 0) | (SYNC if sync else 0)
    _check(lib().mppi_project(ctx._h, scene._h, px0, int(bool(x0_shared)), pin, pout, int(K), int(H), C.byref(q),
                              flags, _stream(dev, stream)))


def mppi_simulate(ctx, scene, X0, U, costs=None, terms=None, X_out=None, *, x0_shared=False, n_sub=0, traj=False,
                  sync=True, stream=None, mapping=None):
    """Roll out explicit controls U[n,H,14] from X0[n,55] (or one shared state)."""
    (px0, pU, pc, pt, px), dev = _ptrs([(X0, np.float32), (U, np.float32), (costs, np.float32),
                                        (terms, np.float32), (X_out, np.float32)])
    n, H = U.shape[0], U.shape[1]
    flags = (DEVICE_PTRS if dev else 0) | (TRAJ if traj else 0) | (SYNC if sync else 0) | _MAPS[mapping]
    _check(lib().mppi_simulate(ctx._h, scene._h, px0, int(bool(x0_shared)), pU, int(n), int(H), int(n_sub), pc, pt,
                               px, flags, _stream(dev, stream)))


def mppi_sample(ctx, scene, nu, sigma, seed, m, K, U=None, z=None, words=None, *, sigma_per_step=False, sync=True,
                stream=None):
    (pnu, psig, pU, pz, pw), dev = _ptrs([(nu, np.float32), (sigma, np.float32), (U, np.float32),
                                          (z, np.float32), (words, np.uint32)])
    H = nu.shape[0]
    flags = (DEVICE_PTRS if dev else 0) | (SIGMA_PER_STEP if sigma_per_step else 0) | (SYNC if sync else 0)
    _check(lib().mppi_sample(ctx._h, scene._h, pnu, psig, int(seed) & 0xFFFFFFFFFFFFFFFF, int(m), int(K), int(H),
                             pU, pz, pw, flags, _stream(dev, stream)))


def mppi_update(ctx, scene, costs, nu_in, sigma, seed, m, lam, nu_out, nu_out64=None, weights=None, *, eta=1.0,
                n_elite=0, sigma_per_step=False, stream=None, fp32_weights=False):
    (pc, pnu, psig, po), dev = _ptrs([(costs, np.float32), (nu_in, np.float32), (sigma, np.float32),
                                      (nu_out, np.float32)])
    (po64, pw), dev2 = _ptrs([(nu_out64, np.float64), (weights, np.float64)])
    if (nu_out64 is not None or weights is not None) and dev2 != dev:
        raise ValueError("mixing device and host arrays in one call")
    K, H = costs.shape[0], nu_in.shape[0]
    flags = (DEVICE_PTRS if dev else 0) | (SIGMA_PER_STEP if sigma_per_step else 0) | \
        (FP32_WEIGHTS if fp32_weights else 0)
    st = Stats()
    rc = lib().mppi_update(ctx._h, scene._h, pc, pnu, psig, int(seed) & 0xFFFFFFFFFFFFFFFF, int(m), int(K), int(H),
                           float(lam), float(eta), int(n_elite), po, po64, pw, C.byref(st), flags,
                           _stream(dev, stream))
    if rc not in (OK, E_DIVERGED):
        _check(rc)
    d = st.as_dict()
    d["rc"] = rc
    return d


def mppi_broadphase(ctx, scene, lo, hi, flags_out, margin=0.0, *, sync=True, stream=None):
    (plo, phi, pf), dev = _ptrs([(lo, np.float32), (hi, np.float32), (flags_out, np.int32)])
    n = lo.shape[0]
    flags = (DEVICE_PTRS if dev else 0) | (SYNC if sync else 0)
    _check(lib().mppi_broadphase(ctx._h, scene._h, plo, phi, int(n), float(margin), pf, flags,
                                 _stream(dev, stream)))


def mppi_narrowphase(ctx, scene, X, phi, normal=None, point=None, lo=None, hi=None, *, sync=True, stream=None):
    (pX, pphi, pn, pp, plo, phi_), dev = _ptrs([(X, np.float32), (phi, np.float32), (normal, np.float32),
                                                (point, np.float32), (lo, np.float32), (hi, np.float32)])
    flags = (DEVICE_PTRS if dev else 0) | (SYNC if sync else 0)
    _check(lib().mppi_narrowphase(ctx._h, scene._h, pX, int(X.shape[0]), pphi, pn, pp, plo, phi_, flags,
                                  _stream(dev, stream)))


def mppi_plan_batch(ctx, items, *, mapping=None, time_kernels=False, stream=None):
    """Packed uneven batch.  `items`: list of dicts with keys scene (Scene),
    x0, nominal_U, K, H, lam, sigma, U_new, costs (optional), M, seed, eta,
    n_elite, sigma_per_step.  Returns one stats dict (with "status") per item."""
    n = len(items)
    reqs = (Request * n)()
    stats = [Stats() for _ in range(n)]
    side = None
    for i, it in enumerate(items):
        (px0, pnom, psig, pU, pc), dev = _ptrs([(it["x0"], np.float32), (it["nominal_U"], np.float32),
                                                 (it["sigma"], np.float32), (it["U_new"], np.float32),
                                                 (it.get("costs"), np.float32)])
        if side is None:
            side = dev
        elif side != dev:
            raise ValueError("mixing device and host arrays in one batch")
        r = reqs[i]
        r.scene = it["scene"]._h
        r.x0, r.nominal_U, r.sigma, r.U_new, r.costs = px0, pnom, psig, pU, pc
        r.K, r.H, r.lam = int(it["K"]), int(it["H"]), float(it["lam"])
        r.opts = Opts(int(it.get("M", 1)), int(it.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF, float(it.get("eta", 1.0)),
                      int(it.get("n_elite", 0)), SIGMA_PER_STEP if it.get("sigma_per_step") else 0)
        r.stats = C.pointer(stats[i])
    flags = (DEVICE_PTRS if side else 0) | (TIME_KERNELS if time_kernels else 0) | _MAPS[mapping]
    _check(lib().mppi_plan_batch(ctx._h, n, reqs, flags, _stream(bool(side), stream)))
    out = []
    for i in range(n):
        d = stats[i].as_dict()
        d["status"] = reqs[i].status
        out.append(d)
    return out


def _request(it, dev_flag):
    """mppi_request of one item dict (see mppi_plan_batch); returns (Request, keep-alive list)."""
    (px0, pnom, psig, pU, pc), dev = _ptrs([(it.get("x0"), np.float32), (it.get("nominal_U"), np.float32),
                                             (it["sigma"], np.float32), (it.get("U_new"), np.float32),
                                             (it.get("costs"), np.float32)])
    r = Request()
    sc = it.get("scene")
    r.scene = sc._h if sc is not None else None
    r.x0, r.nominal_U, r.sigma, r.U_new, r.costs = px0, pnom, psig, pU, pc
    r.K, r.H, r.lam = int(it["K"]), int(it.get("H", 0)), float(it["lam"])
    fl = (SIGMA_PER_STEP if it.get("sigma_per_step") else 0) | (DEVICE_PTRS if dev else 0)
    r.opts = Opts(int(it.get("M", 1)), int(it.get("seed", 0)) & 0xFFFFFFFFFFFFFFFF, float(it.get("eta", 1.0)),
                  int(it.get("n_elite", 0)), fl)
    return r, dev


class Server:
    """Continuous-batching replanning server (mppi_server_* / mppi_submit / mppi_poll / mppi_cancel).
    Output arrays and stats of a request are kept alive here until it is polled done."""

    def __init__(self, ctx, mem_budget=0, max_active=0, max_pending=0, mapping=None, deadline_ms=0.0,
                 iter_base_ms=0.0, iter_ms_per_menv=0.0):
        self.ctx = ctx
        self._h = _P()
        o = ServerOpts(int(mem_budget), int(max_active), int(max_pending), _MAPS[mapping], float(deadline_ms),
                       float(iter_base_ms), float(iter_ms_per_menv))
        _check(lib().mppi_server_create(ctx._h, C.byref(o), C.byref(self._h)))
        ctx._servers.add(self)
        self._keep = {}

    def close(self):
        if self._h:
            lib().mppi_server_destroy(self._h)
            self._h = _P()
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def cell(self, scene, H, x0, nominal_U=None):
        x0 = np.ascontiguousarray(x0, dtype=np.float32)
        nom = None if nominal_U is None else np.ascontiguousarray(nominal_U, dtype=np.float32)
        c = C.c_int(-1)
        _check(lib().mppi_cell_create(self._h, scene._h, int(H), x0.ctypes.data,
                                      None if nom is None else nom.ctypes.data, C.byref(c)))
        return c.value

    def cell_read(self, cell, H):
        x = np.zeros(NX, np.float32)
        nu = np.zeros((H, NU), np.float32)
        _check(lib().mppi_cell_read(self._h, int(cell), x.ctypes.data, nu.ctypes.data))
        return x, nu

    def submit(self, item, cell=-1, advance=0, supersede=False, want_stats=True):
        """item: dict as for mppi_plan_batch (x0 / nominal_U may be omitted for cell requests)."""
        r, _ = _request(item, None)
        st = Stats() if want_stats else None
        r.stats = C.pointer(st) if st is not None else None
        t = C.c_uint64(0)
        _check(lib().mppi_submit(self._h, C.byref(r), int(cell), int(advance), SUPERSEDE if supersede else 0,
                                 C.byref(t)))
        self._keep[t.value] = (item, st, r)
        return t.value

    def poll(self, ticket, timeout_ms=0):
        """None while pending; else a dict with status, iterations, times and stats."""
        info = TicketInfo()
        rc = lib().mppi_poll(self._h, C.c_uint64(ticket), int(timeout_ms), C.byref(info))
        if rc == PENDING:
            return None
        _check(rc)
        item, st, _ = self._keep.pop(ticket, (None, None, None))
        d = {k: getattr(info, k) for k, _ in info._fields_}
        if st is not None:
            d["stats"] = st.as_dict()
        return d

    def wait(self, ticket):
        return self.poll(ticket, timeout_ms=-1)

    def cancel(self, ticket):
        _check(lib().mppi_cancel(self._h, C.c_uint64(ticket)))

    def query(self):
        i = ServerInfo()
        _check(lib().mppi_server_query(self._h, C.byref(i)))
        return {k: getattr(i, k) for k, _ in i._fields_}


_MAP_NAMES = {MAP_LANE: "lane", MAP_TEAM: "team", MAP_WAVE: "wave", MAP_SPLIT: "split"}


def mppi_autotune(ctx, scene, x0, sigma, K, H):
    """Time the lane, team, wave and split mappings on one rollout launch; the
    context remembers the fastest for K's size class.  Returns (name, ms dict)."""
    x0 = np.ascontiguousarray(x0, dtype=np.float32)
    sigma = np.ascontiguousarray(np.broadcast_to(np.asarray(sigma, dtype=np.float32), (14,)))
    m = C.c_int(0)
    ms = (C.c_float * 4)()
    _check(lib().mppi_autotune(ctx._h, scene._h, x0.ctypes.data, sigma.ctypes.data, int(K), int(H), C.byref(m),
                               ms))
    return _MAP_NAMES[m.value], {"lane": ms[0], "team": ms[1], "wave": ms[2], "split": ms[3]}
