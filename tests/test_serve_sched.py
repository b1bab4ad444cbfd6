"""Host-side tests of the serving scheduler (admission by memory footprint in
arrival order, packing by kind, stream rotation, completion, deadline
accounting, errors), driven through a stand-in executor compiled with g++."""
import ctypes as C
import os
import random
import subprocess
import threading

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OK, EINVAL, ENOMEM, EAGAIN, EDEVICE, ENOTFOUND = 0, -1, -2, -3, -4, -5


class Timing(C.Structure):
    _fields_ = [("arrive", C.c_double), ("admit", C.c_double), ("start", C.c_double),
                ("done", C.c_double), ("missed", C.c_int32), ("reserved", C.c_int32)]


@pytest.fixture(scope="module")
def F(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("fake") / "libservefake.so")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-shared", "-fPIC", "-pthread",
                    "-I", os.path.join(ROOT, "include"),
                    "-I", os.path.join(ROOT, "paper_2604_27193_amd", "csrc"),
                    os.path.join(ROOT, "tests", "serve_fake.cpp"), "-o", out], check=True)
    L = C.CDLL(out)
    vp, u64, i64 = C.c_void_p, C.c_uint64, C.c_int64
    L.arena_new.restype = vp
    L.arena_new.argtypes = [u64]
    L.arena_delete.argtypes = [vp]
    L.arena_alloc.restype = i64
    L.arena_alloc.argtypes = [vp, u64]
    L.arena_release.argtypes = [vp, i64]
    L.arena_state.argtypes = [vp, C.POINTER(u64)]
    L.fake_create.restype = vp
    L.fake_create.argtypes = [u64, C.c_int, C.c_int, C.c_int, C.c_int, i64, u64, C.c_int]
    L.fake_destroy.argtypes = [vp]
    L.fake_submit.argtypes = [vp, i64, C.c_int, C.c_int, C.c_double, C.POINTER(u64)]
    L.fake_poll.argtypes = [vp, u64, C.POINTER(i64), C.POINTER(Timing)]
    for f in ("fake_step", "fake_launches", "fake_start", "fake_wait_idle", "fake_stop",
              "fake_drain", "fake_fail_next"):
        getattr(L, f).argtypes = [vp]
    L.fake_complete.argtypes = [vp, C.c_int]
    L.fake_tick.argtypes = [vp, C.c_int, C.POINTER(u64), C.c_int]
    L.fake_counters.argtypes = [vp, C.POINTER(u64)]
    return L


class Sched:
    """Scheduler with a stand-in executor; 1 byte per sample unless stated."""

    def __init__(self, F, arena=1000, slots=8, streams=1, tick_us=0, queue=100,
                 max_tick=10**6, per=1, auto_polls=-1):
        self.F = F
        self.h = F.fake_create(arena, slots, streams, tick_us, queue, max_tick, per, auto_polls)

    def submit(self, n, integrator=0, obstacle=1, deadline=10.0):
        t = C.c_uint64()
        rc = self.F.fake_submit(self.h, n, integrator, obstacle, deadline, C.byref(t))
        return rc, t.value

    def poll(self, ticket):
        out = (C.c_int64 * 3)()
        tm = Timing()
        rc = self.F.fake_poll(self.h, ticket, out, C.byref(tm))
        return rc, list(out), tm

    def step(self):
        return self.F.fake_step(self.h)

    def complete(self, stream=0):
        self.F.fake_complete(self.h, stream)

    def tick(self, stream=0):
        buf = (C.c_uint64 * 4096)()
        n = self.F.fake_tick(self.h, stream, buf, 4096)
        return list(buf[:n])

    def counters(self):
        out = (C.c_uint64 * 10)()
        self.F.fake_counters(self.h, out)
        keys = ("submitted", "completed", "failed", "missed", "ticks", "queued", "admitted",
                "running", "in_use", "peak")
        return dict(zip(keys, list(out)))

    def close(self):
        self.F.fake_destroy(self.h)


# ---------------------------------------------------------------------------
# arena
# ---------------------------------------------------------------------------

def arena_state(F, a):
    out = (C.c_uint64 * 4)()
    F.arena_state(a, out)
    return list(out)


def test_arena_first_fit_alignment_and_coalescing(F):
    a = F.arena_new(4096)
    x = F.arena_alloc(a, 1)        # rounds to 256
    y = F.arena_alloc(a, 300)      # 512
    z = F.arena_alloc(a, 256)
    assert (x, y, z) == (0, 256, 768)
    assert arena_state(F, a)[0] == 1024
    assert F.arena_release(a, y) == 1
    assert F.arena_release(a, y) == 0       # double free is refused
    assert F.arena_alloc(a, 200) == 256     # first fit reuses the hole
    assert F.arena_release(a, 256) == 1
    assert F.arena_release(a, x) == 1
    assert F.arena_release(a, z) == 1
    in_use, peak, largest, nfree = arena_state(F, a)
    assert (in_use, largest, nfree) == (0, 4096, 1)   # everything coalesced
    assert peak == 1024
    assert F.arena_alloc(a, 4097) == -1
    assert F.arena_alloc(a, 4096) == 0
    assert F.arena_alloc(a, 1) == -1
    F.arena_delete(a)


def test_arena_random_against_interval_model(F):
    rng = random.Random(7)
    cap = 256 * 200
    a = F.arena_new(cap)
    live = {}
    for _ in range(3000):
        if live and rng.random() < 0.45:
            off = rng.choice(list(live))
            assert F.arena_release(a, off) == 1
            del live[off]
        else:
            b = rng.randint(1, 256 * 12)
            off = F.arena_alloc(a, b)
            need = (b + 255) // 256 * 256
            if off < 0:
                # refusal only when no gap of that size exists
                ends = sorted((o, o + n) for o, n in live.items())
                gaps, cur = [], 0
                for s, e in ends:
                    gaps.append(s - cur)
                    cur = e
                gaps.append(cap - cur)
                assert max(gaps) < need
                continue
            assert off % 256 == 0 and off + need <= cap
            for o, n in live.items():
                assert off + need <= o or o + n <= off, "overlap"
            live[off] = need
        assert arena_state(F, a)[0] == sum(live.values())
    for off in list(live):
        F.arena_release(a, off)
    assert arena_state(F, a)[2:] == [cap, 1]
    F.arena_delete(a)


# ---------------------------------------------------------------------------
# scheduler
# ---------------------------------------------------------------------------

def test_admission_by_footprint_in_arrival_order(F):
    s = Sched(F, arena=1024, slots=8)
    t = [s.submit(n)[1] for n in (512, 512, 256)]
    s.step()
    assert s.tick() == t[:2]                 # both fit, one launch
    c = s.counters()
    assert (c["running"], c["queued"], c["in_use"]) == (2, 1, 1024)
    assert s.poll(t[0])[0] == EAGAIN
    s.step()                                  # nothing frees: the third waits
    assert s.counters()["queued"] == 1
    s.complete()
    s.step()
    rc, out, tm = s.poll(t[0])
    assert rc == OK and out[:2] == [512, t[0]]
    assert tm.arrive <= tm.admit <= tm.start <= tm.done
    assert s.poll(t[0])[0] == ENOTFOUND       # collected once
    assert s.tick() == [t[2]]                 # admitted and launched after the release
    s.complete()
    s.step()
    assert s.poll(t[2])[0] == OK
    assert s.poll(t[1])[0] == OK
    c = s.counters()
    assert (c["completed"], c["failed"], c["in_use"], c["peak"]) == (3, 0, 0, 1024)
    s.close()


def test_no_overtaking_of_a_large_request(F):
    s = Sched(F, arena=1024, slots=8)
    a = s.submit(768)[1]
    b = s.submit(512)[1]          # does not fit next to a
    c = s.submit(256)[1]          # would fit, but must not overtake b
    s.step()
    assert s.tick() == [a]
    assert s.counters()["queued"] == 2
    s.complete()
    s.step()
    assert s.tick() == [b, c]
    s.close()


def test_slots_limit_requests_in_flight(F):
    s = Sched(F, arena=10**6, slots=3)
    ts = [s.submit(10)[1] for _ in range(5)]
    s.step()
    assert s.tick() == ts[:3]
    s.complete()
    s.step()
    assert s.tick() == ts[3:]
    s.close()


def test_errors(F):
    s = Sched(F, arena=1024, queue=2, max_tick=600)
    assert s.submit(2000)[0] == ENOMEM       # larger than the arena
    assert s.submit(700)[0] == ENOMEM        # larger than a launch
    assert s.submit(10, integrator=1)[0] == EINVAL
    assert s.submit(0)[0] == EINVAL
    assert s.submit(10)[0] == OK and s.submit(10)[0] == OK
    assert s.submit(10)[0] == EAGAIN         # queue full
    assert s.poll(999)[0] == ENOTFOUND
    assert s.counters()["submitted"] == 2
    s.close()


def test_packing_by_kind_and_launch_size(F):
    s = Sched(F, arena=10**6, slots=16, streams=1, max_tick=300)
    a = s.submit(100, obstacle=1)[1]
    b = s.submit(100, obstacle=2)[1]
    c = s.submit(150, obstacle=1)[1]
    d = s.submit(100, obstacle=1)[1]
    s.step()
    assert s.tick() == [a, c]                 # same kind, up to 300 samples
    s.complete()
    s.step()
    assert s.tick() == [b]                    # the oldest admitted sets the kind
    s.complete()
    s.step()
    assert s.tick() == [d]
    s.close()


def test_streams_overlap_and_rotate(F):
    s = Sched(F, arena=10**6, slots=16, streams=2, tick_us=0)
    a = s.submit(10)[1]
    s.step()
    b = s.submit(10)[1]
    s.step()
    c = s.submit(10)[1]
    s.step()
    assert s.tick(0) == [a] and s.tick(1) == [b]
    assert s.counters()["admitted"] == 1      # both streams busy: c waits
    s.complete(1)
    s.step()
    assert s.tick(1) == [c]
    rc, out, _ = s.poll(b)
    assert rc == OK and out[2] == 1           # finished on stream 1
    s.close()


def test_packing_window_while_busy(F):
    s = Sched(F, arena=10**6, slots=16, streams=2, tick_us=10**6)
    a = s.submit(10)[1]
    s.step()
    assert s.tick(0) == [a]                   # idle device: launch at once
    b = s.submit(10)[1]
    c = s.submit(10)[1]
    s.step()
    assert s.tick(1) == []                    # busy: wait for more within the window
    assert s.counters()["admitted"] == 2
    s.complete(0)
    s.step()                                  # idle again: go
    assert s.tick(0) == [b, c]
    s.close()


def test_deadline_accounting(F):
    s = Sched(F, arena=10**6)
    a = s.submit(10, deadline=1e-9)[1]
    b = s.submit(10, deadline=100.0)[1]
    s.step()
    s.complete()
    s.step()
    assert s.poll(a)[2].missed == 1
    assert s.poll(b)[2].missed == 0
    assert s.counters()["missed"] == 1
    s.close()


def test_launch_failure_releases_and_reports(F):
    s = Sched(F, arena=1024)
    F.fake_fail_next(s.h)
    a = s.submit(500)[1]
    s.step()
    rc, _, _ = s.poll(a)
    assert rc == EDEVICE
    c = s.counters()
    assert (c["failed"], c["completed"], c["in_use"], c["running"]) == (1, 1, 0, 0)
    b = s.submit(900)[1]                       # the memory is free again
    s.step()
    assert s.tick() == [b]
    s.close()


def test_threaded_worker_many_clients(F):
    s = Sched(F, arena=4000, slots=6, streams=3, tick_us=100, queue=10**5, auto_polls=3)
    F.fake_start(s.h)
    rng = random.Random(3)
    sizes = [rng.choice((100, 400, 1500)) for _ in range(600)]
    tickets = [None] * len(sizes)

    def client(k0):
        for k in range(k0, len(sizes), 4):
            rc, t = s.submit(sizes[k])
            assert rc == OK
            tickets[k] = t

    th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
    for t in th:
        t.start()
    for t in th:
        t.join()
    F.fake_wait_idle(s.h)
    for k, t in enumerate(tickets):
        rc, out, tm = s.poll(t)
        assert rc == OK and out[0] == sizes[k] and out[1] == t
        assert tm.arrive <= tm.admit <= tm.start <= tm.done
    c = s.counters()
    assert c["completed"] == len(sizes) and c["in_use"] == 0 and c["peak"] <= 4000
    F.fake_stop(s.h)
    s.close()
