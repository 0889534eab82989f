"""The closed-loop executor's phase machine and termination rules
(csrc/episode.h, compiled for the CPU) against the oracle's own
implementation of the same readings (oracle/episode.py) on scripted and
random observation sequences: identical status, phase and switch/end times
at every step."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

from oracle import episode as oe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RULE = (0.03, 0.02, 0.05, 0.15, 0.11, 2.0)  # grasp, width, goal tolerances, lift, drop heights, t_max


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    d = tmp_path_factory.mktemp("ep")
    so = str(d / "ep.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-I",
                    os.path.join(ROOT, "paper_2511_21264_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "episode_shim.cpp"), "-o", so], check=True)
    L = C.CDLL(so)
    L.ep_run.argtypes = [C.c_int, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
    return L


def _both(L, obs):
    n = len(obs)
    obs = np.ascontiguousarray(obs, dtype=np.float64)
    st, ph, tm = np.zeros(n, np.int32), np.zeros(n, np.int32), np.zeros(2)
    L.ep_run(n, obs.ctypes.data, np.array(RULE).ctypes.data, st.ctypes.data, ph.ctypes.data, tm.ctypes.data)
    R = oe.Rules(*RULE)
    st2 = [R.observe(*o[:5], int(o[5])) for o in obs]
    ph2 = []
    R = oe.Rules(*RULE)
    for o in obs:
        R.observe(*o[:5], int(o[5]))
        ph2.append(R.phase)
    return (st, ph, tm), (np.array(st2), np.array(ph2), np.array([R.t_switch, R.t_end]))


def _seq(t, goal, grasp, width, z, pen):
    return np.stack([t, goal, grasp, width, z, pen], axis=1)


def test_scripted_success_after_grasp_and_lift(shim):
    n = 80
    t = 0.02 * np.arange(1, n + 1)
    grasp = np.maximum(0.1 - 0.2 * t, 0.0)   # the pads close on the grasp point by t = 0.5
    z = np.where(t > 0.5, 0.1 + (t - 0.5), 0.1)  # lifted after the switch
    goal = np.maximum(0.5 - np.maximum(t - 0.5, 0) * 1.2, 0.0)
    (st, ph, tm), (st2, ph2, tm2) = _both(shim, _seq(t, goal, grasp, np.full(n, 0.01), z, np.zeros(n)))
    assert np.array_equal(st, st2) and np.array_equal(ph, ph2) and np.array_equal(tm, tm2)
    assert st[-1] == oe.SUCCESS and 0 < tm[0] < tm[1]


def test_scripted_fall_collision_and_timeout(shim):
    n = 150
    t = 0.02 * np.arange(1, n + 1)
    z = np.where(t < 0.6, 0.1 + t * 0.2, 0.05)   # lifted, then back on the table
    (st, ph, tm), (st2, ph2, tm2) = _both(shim, _seq(t, np.full(n, 0.4), np.zeros(n), np.zeros(n), z, np.zeros(n)))
    assert np.array_equal(st, st2) and np.array_equal(tm, tm2) and st[-1] == oe.FELL
    pen = np.zeros(n)
    pen[17] = 1
    (st, ph, tm), (st2, ph2, tm2) = _both(shim, _seq(t, np.full(n, 0.4), np.full(n, 0.5), np.ones(n), np.full(n, 0.1),
                                                     pen))
    assert np.array_equal(st, st2) and st[-1] == oe.COLLISION and tm[1] == t[17]
    (st, ph, tm), (st2, ph2, tm2) = _both(shim, _seq(t, np.full(n, 0.4), np.full(n, 0.5), np.ones(n), np.full(n, 0.1),
                                                     np.zeros(n)))
    assert np.array_equal(st, st2) and st[-1] == oe.TIMEOUT and tm[1] == t[np.argmax(t >= RULE[5])]


@pytest.mark.parametrize("seed", range(20))
def test_random_sequences_agree(shim, seed):
    rng = np.random.default_rng(seed)
    n = 200
    t = np.cumsum(rng.uniform(0.005, 0.02, n))
    obs = _seq(t, rng.uniform(0, 0.2, n), rng.uniform(0, 0.08, n), rng.uniform(0, 0.05, n),
               rng.uniform(0.05, 0.25, n), (rng.random(n) < 0.01).astype(float))
    (st, ph, tm), (st2, ph2, tm2) = _both(shim, obs)
    assert np.array_equal(st, st2) and np.array_equal(ph, ph2) and np.array_equal(tm, tm2)
