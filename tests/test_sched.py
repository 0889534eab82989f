"""Host logic of the serving loop (csrc/sched.h), on the CPU: the first-fit
arena against a brute-force byte map, and the admission rules of the
scheduler (FIFO, per-cell order, memory admission without overtaking,
active-slot limit, cancellation, supersession, release; with deadlines:
earliest deadline first, admission only when the iteration model predicts
the request and every active one on time, shedding of requests that cannot
finish in time even alone)."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
U64 = C.c_uint64


@pytest.fixture(scope="module")
def S(tmp_path_factory):
    d = tmp_path_factory.mktemp("sched")
    so = str(d / "libsched.so")
    subprocess.run(["g++", "-O1", "-std=c++17", "-shared", "-fPIC", "-I",
                    os.path.join(ROOT, "paper_2511_21264_amd", "csrc"),
                    os.path.join(ROOT, "tests", "native", "sched_shim.cpp"), "-o", so], check=True)
    L = C.CDLL(so)
    sig = {
        "arena_new": (C.c_void_p, [U64]), "arena_free": (None, [C.c_void_p]),
        "arena_alloc": (C.c_int64, [C.c_void_p, U64]), "arena_release": (C.c_int, [C.c_void_p, U64]),
        "arena_used": (U64, [C.c_void_p]), "arena_largest": (U64, [C.c_void_p]),
        "arena_nfree": (U64, [C.c_void_p]), "arena_high": (U64, [C.c_void_p]),
        "sched_new": (C.c_void_p, [U64, U64, C.c_int, C.c_int]), "sched_free": (None, [C.c_void_p]),
        "sched_enqueue": (C.c_int, [C.c_void_p, U64, C.c_int, C.c_int, U64, U64, C.c_int, C.POINTER(U64),
                                    C.POINTER(C.c_int)]),
        "sched_admit": (C.c_int, [C.c_void_p, C.POINTER(U64)]),
        "sched_enqueue_dl": (C.c_int, [C.c_void_p, U64, C.c_int, C.c_int, U64, C.c_double, C.c_double]),
        "sched_admit_dl": (C.c_int, [C.c_void_p, C.c_double, C.c_double, C.c_double, C.c_double, C.c_int,
                                     C.POINTER(U64), C.POINTER(U64), C.POINTER(C.c_int)]),
        "sched_cancel": (C.c_int, [C.c_void_p, U64]),
        "sched_next": (C.c_int, [C.c_void_p, C.POINTER(U64), C.POINTER(C.c_int), C.POINTER(U64),
                                 C.POINTER(C.c_int)]),
        "sched_advance": (C.c_int, [C.c_void_p, C.POINTER(U64)]),
        "sched_release": (C.c_int, [C.c_void_p, U64]), "sched_forget": (None, [C.c_void_p, U64]),
        "sched_cell_idle": (C.c_int, [C.c_void_p, C.c_int]),
        "sched_counts": (C.c_int, [C.c_void_p, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(U64),
                                   C.POINTER(U64)]),
    }
    for n, (r, a) in sig.items():
        f = getattr(L, n)
        f.restype, f.argtypes = r, a
    return L


class Sched:
    def __init__(self, L, dev, host, max_active, max_pending):
        self.L, self.h = L, L.sched_new(dev, host, max_active, max_pending)
        self.buf = (U64 * 4096)()
        self.buf2 = (U64 * 4096)()
        self.ms = (C.c_int * 4096)()

    def enqueue(self, id, cell, M, dev, host=256, supersede=False):
        n = C.c_int(0)
        rc = self.L.sched_enqueue(self.h, id, cell, M, dev, host, int(supersede), self.buf, C.byref(n))
        return rc, [self.buf[i] for i in range(n.value)]

    def admit(self):
        n = self.L.sched_admit(self.h, self.buf)
        return [self.buf[i] for i in range(n)]

    def enqueue_dl(self, id, cell, M, deadline, work, dev=1000):
        return self.L.sched_enqueue_dl(self.h, id, cell, M, dev, float(deadline), float(work))

    def admit_dl(self, now, base, slope, floor=0.0, extra=1):
        ns = C.c_int(0)
        n = self.L.sched_admit_dl(self.h, float(now), float(base), float(slope), float(floor), int(extra), self.buf,
                                  self.buf2, C.byref(ns))
        return [self.buf[i] for i in range(n)], [self.buf2[i] for i in range(ns.value)]

    def next(self):
        nd = C.c_int(0)
        n = self.L.sched_next(self.h, self.buf, self.ms, self.buf2, C.byref(nd))
        return [(self.buf[i], self.ms[i]) for i in range(n)], [self.buf2[i] for i in range(nd.value)]

    def advance(self):
        n = self.L.sched_advance(self.h, self.buf)
        return [self.buf[i] for i in range(n)]

    def counts(self):
        a, p, d, h = C.c_int(), C.c_int(), U64(), U64()
        self.L.sched_counts(self.h, C.byref(a), C.byref(p), C.byref(d), C.byref(h))
        return a.value, p.value, d.value, h.value

    def close(self):
        self.L.sched_free(self.h)


def test_arena_against_brute_force_byte_map(S):
    """Random alloc/release sequences: blocks never overlap, stay inside the
    arena and are 256-aligned; a request fails only when no free run of the
    rounded size exists; released space is merged (one free range when empty)."""
    cap = 1 << 16
    rng = np.random.default_rng(5)
    a = S.arena_new(cap)
    used = np.zeros(cap // 256, bool)  # 256-byte granules
    live = {}
    for step in range(3000):
        if live and rng.random() < 0.45:
            off = list(live)[rng.integers(len(live))]
            n = live.pop(off)
            assert S.arena_release(a, off) == 1
            used[off // 256:(off + n) // 256] = False
        else:
            req = int(rng.integers(1, 6000))
            n = (req + 255) // 256 * 256
            off = S.arena_alloc(a, req)
            g = n // 256
            # does any run of g free granules exist?
            free_run, best = 0, 0
            for u in used:
                free_run = 0 if u else free_run + 1
                best = max(best, free_run)
            if off < 0:
                assert best < g, "allocation failed although a free run exists"
            else:
                assert off % 256 == 0 and off + n <= cap
                assert not used[off // 256:off // 256 + g].any(), "overlap"
                # first fit: no lower free run of g granules
                run = 0
                for i in range(off // 256):
                    run = 0 if used[i] else run + 1
                    assert run < g, "not first fit"
                used[off // 256:off // 256 + g] = True
                live[off] = n
        assert S.arena_used(a) == used.sum() * 256
    for off in list(live):
        assert S.arena_release(a, off) == 1
    assert S.arena_used(a) == 0 and S.arena_nfree(a) == 1 and S.arena_largest(a) == cap
    assert S.arena_release(a, 12345) == 0
    assert S.arena_high(a) <= cap
    S.arena_free(a)


def test_fifo_per_cell_order_and_slot_limit(S):
    s = Sched(S, 1 << 20, 1 << 20, max_active=3, max_pending=100)
    # ids 1..6: cells 0,0,1,2,1,3
    for i, cell in zip(range(1, 7), [0, 0, 1, 2, 1, 3]):
        assert s.enqueue(i, cell, M=2, dev=1000)[0] == 0
    # admission: FIFO, skipping requests whose cell is busy, up to 3 slots
    assert s.admit() == [1, 3, 4]
    act, drop = s.next()
    assert act == [(1, 0), (3, 0), (4, 0)] and drop == []
    assert s.advance() == []
    assert s.admit() == []  # slots full
    act, _ = s.next()
    assert [m for _, m in act] == [1, 1, 1]
    assert s.advance() == [1, 3, 4]
    # cell 0's second request and cell 1's second now admissible; 6 too
    assert s.admit() == [2, 5, 6]
    for i in (1, 3, 4):
        assert S.sched_release(s.h, i) == 1
    assert s.counts()[:2] == (3, 0)
    s.close()


def test_memory_admission_without_overtaking(S):
    s = Sched(S, 10_000, 1 << 20, max_active=10, max_pending=10)
    assert s.enqueue(1, -1, 1, 6000)[0] == 0
    assert s.enqueue(2, -1, 1, 6000)[0] == 0   # does not fit beside 1
    assert s.enqueue(3, -1, 1, 1000)[0] == 0   # would fit, but must not overtake 2
    assert s.enqueue(4, -1, 1, 20_000)[0] == 2  # never fits: rejected at once
    assert s.admit() == [1]
    assert s.admit() == []
    s.next()
    assert s.advance() == [1]
    assert s.admit() == []  # 1's memory is held until release
    assert S.sched_release(s.h, 1) == 1
    assert s.admit() == [2, 3]
    s.close()


def test_queue_limit_cancel_and_supersede(S):
    s = Sched(S, 1 << 20, 1 << 20, max_active=1, max_pending=3)
    assert s.enqueue(1, 7, 3, 100)[0] == 0
    assert s.admit() == [1]
    for i in (2, 3, 4):
        assert s.enqueue(i, 7, 3, 100)[0] == 0
    assert s.enqueue(5, 8, 3, 100)[0] == 1  # queue full
    # supersede: the new request of cell 7 replaces the queued ones (not the running one)
    rc, sup = s.enqueue(6, 7, 3, 100, supersede=True)
    assert rc == 0 and sup == [2, 3, 4]
    assert s.counts()[:2] == (1, 1)
    # cancel: queued -> 1, running -> 2 (dropped at the next boundary), unknown -> 0
    assert S.sched_cancel(s.h, 6) == 1
    assert S.sched_cancel(s.h, 1) == 2
    assert S.sched_cancel(s.h, 99) == 0
    act, drop = s.next()
    assert act == [] and drop == [1]
    assert S.sched_cell_idle(s.h, 7) == 0  # 1 still holds memory (in flight)
    assert S.sched_release(s.h, 1) == 1
    for i in (2, 3, 4, 6):
        S.sched_forget(s.h, i)
    assert S.sched_cell_idle(s.h, 7) == 1
    assert s.counts() == (0, 0, 0, 0)
    s.close()


def test_random_workload_invariants(S):
    """Random submissions, cancellations and iterations: every request runs
    its M iterations in order exactly once unless cancelled, a cell never has
    two requests active, slots and memory limits always hold, and nothing
    starves."""
    rng = np.random.default_rng(11)
    dev_cap = 50_000
    s = Sched(S, dev_cap, 1 << 20, max_active=4, max_pending=1000)
    M = {}
    seen = {}
    cell_of = {}
    nid = 1
    done, cancelled = set(), set()
    inflight = []
    for it in range(400):
        for _ in range(rng.integers(0, 3)):
            cell = int(rng.integers(0, 5))
            M[nid] = int(rng.integers(1, 5))
            cell_of[nid] = cell
            rc, _ = s.enqueue(nid, cell, M[nid], int(rng.integers(1000, 20000)))
            assert rc == 0
            nid += 1
        if rng.random() < 0.05 and nid > 1:
            v = int(rng.integers(1, nid))
            if v not in done and v not in cancelled:
                r = S.sched_cancel(s.h, v)
                if r == 1:
                    cancelled.add(v)
                    S.sched_forget(s.h, v)
                elif r == 2:
                    cancelled.add(v)
        for rid in inflight:  # previous iteration's finishing requests complete
            assert S.sched_release(s.h, rid) == 1
        inflight = []
        s.admit()
        act, drop = s.next()
        inflight += drop
        a, p, d, _ = s.counts()
        assert a <= 4 and d <= dev_cap
        cells = [cell_of[i] for i, _ in act]
        assert len(cells) == len(set(cells)), "two requests of one cell active"
        for i, m in act:
            assert seen.get(i, 0) == m, "iterations out of order"
            seen[i] = m + 1
        fin = s.advance()
        for i in fin:
            assert seen[i] == M[i]
            done.add(i)
        inflight += fin
    # drain
    for _ in range(200):
        for rid in inflight:
            S.sched_release(s.h, rid)
        inflight = []
        s.admit()
        act, drop = s.next()
        inflight += drop
        for i, m in act:
            assert seen.get(i, 0) == m
            seen[i] = m + 1
        for i in s.advance():
            done.add(i)
            inflight.append(i)
    assert s.counts()[:2] == (0, 0)
    for i in range(1, nid):
        assert (i in done) != (i in cancelled) or (i in cancelled and i not in done)
        if i not in cancelled:
            assert i in done and seen[i] == M[i]
    s.close()


INF = float("inf")


def test_earliest_deadline_first(S):
    s = Sched(S, 1 << 20, 1 << 20, max_active=1, max_pending=100)
    for i, dl in zip((1, 2, 3, 4), (30.0, 10.0, INF, 20.0)):
        assert s.enqueue_dl(i, i, 2, dl, 100) == 0
    order = []
    for _ in range(4):
        adm, shed = s.admit_dl(0.0, 0.0, 0.0)
        assert shed == [] and len(adm) == 1
        order += adm
        s.next()
        s.next()
        s.advance()
        s.next()
        for f in s.advance():
            assert S.sched_release(s.h, f) == 1
    assert order == [2, 4, 1, 3]   # by deadline; no deadline last
    s.close()


def test_shed_requests_that_cannot_finish_even_alone(S):
    """A request whose M iterations (plus the one in flight) at its own load
    end after its deadline is shed; one that fits is admitted; a request
    already past its deadline is shed even with no time model."""
    s = Sched(S, 1 << 20, 1 << 20, max_active=8, max_pending=100)
    assert s.enqueue_dl(1, 0, 10, 15.0, 100) == 0     # (10 + 1) x 2 ms = 22 > 15
    assert s.enqueue_dl(2, 1, 10, 25.0, 100) == 0     # 22 <= 25
    adm, shed = s.admit_dl(0.0, 2.0, 0.0)
    assert shed == [1] and adm == [2]
    assert s.enqueue_dl(3, 2, 1, 5.0, 100) == 0
    adm, shed = s.admit_dl(6.0, 0.0, 0.0)            # zero model: only past deadlines shed
    assert shed == [3] and adm == []
    s.close()


def test_admission_keeps_active_requests_on_time(S):
    """Admitting a large request would stretch every packed iteration and make
    an active request late: it waits (and nothing overtakes it) until the
    active one has finished, then it is admitted."""
    s = Sched(S, 1 << 20, 1 << 20, max_active=8, max_pending=100)
    base, slope = 1.0, 0.01                           # T(W) = 1 + 0.01 W ms
    assert s.enqueue_dl(1, 0, 5, 30.0, 100) == 0      # alone: 6 x 2 = 12 <= 30
    assert s.admit_dl(0.0, base, slope) == ([1], [])
    assert s.enqueue_dl(2, 1, 5, 100.0, 1000) == 0    # with 1: T = 12, 1 would end at 72 > 30
    assert s.enqueue_dl(3, 2, 1, 200.0, 10) == 0      # later deadline: must not overtake 2
    assert s.admit_dl(0.0, base, slope) == ([], [])
    for _ in range(5):
        s.next()
        fin = s.advance()
    assert fin == [1]
    assert S.sched_release(s.h, 1) == 1
    adm, shed = s.admit_dl(10.0, base, slope)         # 2 alone: 10 + 6 x 11 = 76 <= 100
    assert shed == [] and adm == [2, 3]
    s.close()


def test_deadlines_keep_per_cell_order(S):
    """A cell's later request with an earlier deadline still waits for the
    cell's earlier one."""
    s = Sched(S, 1 << 20, 1 << 20, max_active=8, max_pending=100)
    assert s.enqueue_dl(1, 4, 1, 50.0, 10) == 0
    assert s.enqueue_dl(2, 4, 1, 10.0, 10) == 0
    assert s.enqueue_dl(3, 5, 1, 20.0, 10) == 0
    assert s.admit_dl(0.0, 0.0, 0.0) == ([3, 1], [])
    s.next()
    assert sorted(s.advance()) == [1, 3]
    assert s.admit_dl(0.0, 0.0, 0.0) == ([2], [])
    s.close()


def test_random_deadline_workload_predictions_hold(S):
    """Random arrivals against a server whose iterations take exactly the
    model's time: every admitted request finishes by its deadline (the
    admission test is exact for that model), every request is either
    finished or shed, and shedding happens only to requests that could not
    finish in time even alone at the moment they were shed."""
    rng = np.random.default_rng(3)
    base, slope = 0.5, 0.002
    s = Sched(S, 1 << 24, 1 << 24, max_active=16, max_pending=10000)
    t, nid = 0.0, 1
    info = {}
    active_work = {}
    finished, shed_all = {}, set()
    for step in range(600):
        for _ in range(rng.poisson(0.6)):
            M, work = int(rng.integers(1, 6)), float(rng.integers(50, 800))
            dl = t + float(rng.uniform(5.0, 40.0))
            assert s.enqueue_dl(nid, int(rng.integers(0, 40)), M, dl, work) == 0
            info[nid] = (M, work, dl)
            nid += 1
        adm, shed = s.admit_dl(t, base, slope)
        for i in shed:
            M, work, dl = info[i]
            assert t + (M + 1) * (base + slope * work) > dl
            shed_all.add(i)
        for i in adm:
            active_work[i] = info[i][1]
        act, _ = s.next()
        W = sum(active_work[i] for i, _ in act)
        if act:
            t += base + slope * W      # the iteration takes the model's time
        else:
            t += 0.5
        for i in s.advance():
            finished[i] = t
            active_work.pop(i)
            assert S.sched_release(s.h, i) == 1
    for i, tf in finished.items():
        # the in-flight iteration the admission budgets for is not simulated
        # here, so every finish is strictly within the deadline
        assert tf <= info[i][2] + 1e-9, (i, tf, info[i])
    assert len(finished) > 100 and len(shed_all) > 0
    s.close()


def test_iteration_floor_and_work_in_flight(S):
    """The model's floor bounds small loads from below; with nothing in
    flight a request waits for no earlier iteration."""
    s = Sched(S, 1 << 20, 1 << 20, max_active=8, max_pending=100)
    # floor 3 ms beats 1 + 0.001 * 100 ms: M = 5 needs 5 x 3 = 15 ms, plus 3 in flight
    assert s.enqueue_dl(1, 0, 5, 16.0, 100) == 0
    assert s.admit_dl(0.0, 1.0, 0.001, floor=3.0, extra=1) == ([], [1])
    assert s.enqueue_dl(2, 1, 5, 16.0, 100) == 0
    assert s.admit_dl(0.0, 1.0, 0.001, floor=3.0, extra=0) == ([2], [])
    s.close()
