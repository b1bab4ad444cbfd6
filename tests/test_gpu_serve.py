"""GPU tests of the serving path: every request's statistics equal those of
the same scenario rolled out and reduced alone (bit for bit), whatever else
shared its launch; the FP64 statistics match the reference; admission by
footprint holds under a small arena; refusals are reported."""
import threading

import numpy as np
import pytest

from paper_2604_27193_amd import workloads as W

pytestmark = pytest.mark.gpu

RISK = (0.05, 0.01, 0.001)
MQ = (0.0, 0.01, 0.5)
GRID = (30.0, 130.0, 64)


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2604_27193_amd import binding
    binding.lib()
    return binding


def alone(B, d, precision):
    out = B.rollout(d, precision=precision)
    return B.reduce(out, risk=RISK, margin_q=MQ, grid=GRID)


def same(a, b):
    for k in a:
        if isinstance(a[k], np.ndarray):
            assert np.array_equal(a[k], b[k]), k
        elif isinstance(a[k], float) and np.isnan(a[k]):
            assert np.isnan(b[k]), k
        else:
            assert a[k] == b[k], (k, a[k], b[k])


def mixed_requests(n_req, seed=11, sizes=(3000, 12000, 40000)):
    reqs = W.serving_stream(rate=1000.0, duration=10.0, seed=seed, sizes=sizes,
                            probs=(0.5, 0.3, 0.2))
    return [d for _, d, _ in reqs[:n_req]]


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_requests_equal_alone_in_the_mix(B, prec):
    scns = mixed_requests(24)
    with B.Server(256 << 20, precision=prec, max_slots=32, n_streams=3, tick_us=500,
                  max_tick_samples=1 << 18, risk=RISK, margin_q=MQ, grid=GRID) as srv:
        tickets = [srv.submit(d) for d in scns]
        got = [srv.wait(t) for t in tickets]
        info = srv.info()
    assert info["completed"] == len(scns) and info["failed"] == 0
    assert info["ticks"] < len(scns)          # requests shared launches
    for d, (st, tm) in zip(scns, got):
        same(alone(B, d, prec), st)
        assert tm["arrive"] <= tm["admit"] <= tm["start"] <= tm["done"]


def test_served_statistics_match_reference(B, orc):
    d = W.single(5000, seed=3, scenario_id=9)
    with B.Server(64 << 20, max_slots=4, n_streams=1, max_tick_samples=1 << 16,
                  risk=RISK, margin_q=MQ, grid=GRID) as srv:
        st, _ = srv.wait(srv.submit(d))
    ref = orc.reduce(orc.run(d), risk=RISK, margin_q=MQ, grid=GRID)
    for k in ("n", "n_collide", "n_stop", "n_impact", "n_horizon", "p_collision", "headway",
              "margin_q"):
        assert st[k] == ref[k], k
    assert np.array_equal(st["risk_count"], ref["risk_count"])
    assert abs(st["mean_dist"] - ref["mean_dist"]) <= 1e-12 * abs(ref["mean_dist"])


def test_small_arena_admits_by_footprint(B):
    scns = mixed_requests(16, seed=5)
    big = max(int(d["n_samples"]) for d in scns)
    fixed = B.Server.fixed_bytes(max_slots=16, n_streams=2, max_tick_samples=big,
                                 risk=RISK, margin_q=MQ, grid=GRID)
    with B.Server(fixed + (3 << 20), max_slots=16, n_streams=2, max_tick_samples=big,
                  risk=RISK, margin_q=MQ, grid=GRID) as srv:
        fps = [srv.footprint(int(d["n_samples"])) for d in scns]
        assert max(fps) <= 3 << 20 < sum(fps)   # not all fit at once
        tickets = [srv.submit(d) for d in scns]
        got = [srv.wait(t)[0] for t in tickets]
        info = srv.info()
    assert info["arena_peak"] <= info["arena_request_bytes"]
    assert info["completed"] == len(scns)
    for d, st in zip(scns, got):
        same(alone(B, d, "fp64"), st)


def test_concurrent_clients(B):
    scns = mixed_requests(32, seed=8, sizes=(2000, 5000, 9000))
    res = [None] * len(scns)
    with B.Server(128 << 20, max_slots=8, n_streams=2, tick_us=200,
                  max_tick_samples=1 << 16, risk=RISK, margin_q=MQ, grid=GRID) as srv:
        def client(k0):
            for k in range(k0, len(scns), 4):
                res[k] = srv.wait(srv.submit(scns[k]))[0]
        th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
        for t in th:
            t.start()
        for t in th:
            t.join()
    for d, st in zip(scns, res):
        same(alone(B, d, "fp64"), st)


def test_refusals(B):
    with B.Server(64 << 20, max_slots=4, n_streams=1, max_tick_samples=1 << 14) as srv:
        with pytest.raises(B.AebError) as e:
            # the closed-loop controller is not batched
            srv.submit(W.closed_loop(100))
        assert e.value.code == B.EINVAL
        with pytest.raises(B.AebError) as e:
            srv.submit(W.single(1 << 15))              # more than a launch holds
        assert e.value.code == B.ENOMEM
        with pytest.raises(B.AebError) as e:
            srv.poll(12345)
        assert e.value.code == B.ENOTFOUND
    with pytest.raises(B.AebError) as e:
        B.Server(1 << 20, max_tick_samples=1 << 20)     # arena too small
    assert e.value.code == B.ENOMEM


def test_rk4_requests_equal_alone(B):
    scns = [W.paper_preset(n, seed=40 + j, scenario_id=j) for j, n in
            enumerate((5000, 12000, 700, 20000))]
    with B.Server(128 << 20, max_slots=8, n_streams=2, tick_us=1000,
                  max_tick_samples=1 << 16, risk=RISK, margin_q=MQ, grid=GRID) as srv:
        tickets = [srv.submit(d) for d in scns]
        got = [srv.wait(t)[0] for t in tickets]
    for d, st in zip(scns, got):
        same(alone(B, d, "fp64"), st)
