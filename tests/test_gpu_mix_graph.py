"""Recorded graphs for changing mixes (aeb_graph_create_mix /
aeb_graph_launch_mix, and the server's per-bucket recordings): one recording
replays mixes of different scenario counts, sizes, steps and horizons, with
eager work and synchronisation between replays, and every replay's outputs
and statistics equal the eager batched launch (aeb_batch_rollout +
aeb_batch_reduce) of the same mix bit for bit."""
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


def to_np(out):
    import torch
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def same_out(a, b):
    for k in a:
        assert np.array_equal(a[k].view(np.uint8), b[k].view(np.uint8)), k


def same_stats(a, b):
    for k, v in a.items():
        w = b[k]
        if isinstance(v, np.ndarray):
            assert np.array_equal(v.view(np.uint8), w.view(np.uint8)), k
        elif isinstance(v, float):
            assert np.float64(v).tobytes() == np.float64(w).tobytes(), k
        else:
            assert v == w, k


def mixes(kind):
    """Mixes of 1 to 8 scenarios of the kind: uneven sizes, steps, horizons."""
    base = W.uneven_batch(40, max_samples=60_000)
    out = []
    for sel in ([3], [0, 1, 2, 5, 7], [8, 9, 10, 11, 12, 13, 14, 15], [20, 4]):
        mix = []
        for j in sel:
            d = dict(base[j])
            d.update({k: kind[k] for k in ("obstacle", "impact_exit", "nofma", "integrator")
                      if k in kind})
            if kind.get("obstacle") == "lead":
                d["lead_decel"] = kind["lead_decel"]
                d["gap"] = kind["gap"]
            mix.append(d)
        out.append(mix)
    return out


KINDS = {
    "stationary fp64": (dict(W.single(10)), "fp64"),
    "unfused fp64": (dict(W.single(10), nofma=True), "fp64"),
    "stationary fp32c": (dict(W.single(10)), "fp32c"),
    "lead fp64": (dict(W.sweep(n=10)[120]), "fp64"),
    "impact exit fp32c": (dict(W.single(10), impact_exit=True), "fp32c"),
}


@pytest.mark.parametrize("name", list(KINDS))
def test_mix_graph_replays_equal_eager(B, name):
    kind, prec = KINDS[name]
    g = B.MixGraph(kind, precision=prec, max_scn=8, max_samples=400_000, risk=RISK,
                   margin_q=MQ, grid=GRID)
    try:
        for rep in range(2):
            for mix in mixes(kind):
                outs = g.launch(mix)
                got = g.finish()
                want_outs = B.batch_rollout(mix, precision=prec)
                want = B.batch_reduce(want_outs, risk=RISK, margin_q=MQ, grid=GRID)
                for o, wo, st, ws in zip(outs, want_outs, got, want):
                    same_out(to_np(o), to_np(wo))
                    same_stats(st, ws)
    finally:
        g.close()


def test_mix_graph_perception_with_and_without(B):
    kind = W.perception(10)
    mix = [W.perception(20_000, seed=5), W.single(30_000, seed=6), W.perception(7_001, seed=7)]
    g = B.MixGraph(kind, max_scn=4, max_samples=100_000, risk=RISK, margin_q=MQ, grid=GRID)
    try:
        for _ in range(2):
            outs = g.launch(mix)
            got = g.finish()
            for d, o, st in zip(mix, outs, got):
                alone = B.rollout(d)
                same_out(to_np(o), to_np(alone))
                same_stats(st, B.reduce(alone, risk=RISK, margin_q=MQ, grid=GRID))
    finally:
        g.close()


def test_mix_graph_without_statistics(B):
    kind = W.single(10)
    mix = [W.single(5000, seed=3), W.single(777, seed=4)]
    g = B.MixGraph(kind, max_scn=2, max_samples=10_000, stats=False)
    try:
        outs = g.launch(mix)
        assert g.finish() is None
        for d, o in zip(mix, outs):
            same_out(to_np(o), to_np(B.rollout(d)))
    finally:
        g.close()


def test_mix_graph_rejects(B):
    kind = W.single(10)
    g = B.MixGraph(kind, max_scn=2, max_samples=10_000, risk=RISK)
    try:
        with pytest.raises(B.AebError):      # too many scenarios
            g.launch([W.single(100, seed=s) for s in range(3)])
        with pytest.raises(B.AebError):      # too many samples
            g.launch([W.single(6000, seed=1), W.single(6000, seed=2)])
        with pytest.raises(B.AebError):      # another kind
            g.launch([W.sweep(n=100)[3]])
        with pytest.raises(B.AebError):      # perception not recorded
            g.launch([W.perception(100)])
        g.launch([W.single(100, seed=1)])
        with pytest.raises(B.AebError):      # the previous replay not finished
            g.launch([W.single(100, seed=2)])
        g.finish()
    finally:
        g.close()
    with pytest.raises(B.AebError):                  # RK4 has no FP32C form
        B.MixGraph(W.paper_preset(10), precision="fp32c")
    with pytest.raises(B.AebError):                  # the controller runs scenario by scenario
        B.MixGraph(W.closed_loop(10))


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_server_recorded_equals_eager(B, prec):
    """The server's recorded ticks and its eager ticks give the same
    statistics, and both equal each request alone."""
    reqs = W.serving_stream(rate=1000.0, duration=10.0, seed=19, sizes=(3000, 12000, 40000),
                            probs=(0.5, 0.3, 0.2))
    scns = [d for _, d, _ in reqs[:30]]
    res = {}
    for eager in (False, True):
        with B.Server(256 << 20, precision=prec, max_slots=32, n_streams=3, tick_us=500,
                      max_tick_samples=1 << 18, risk=RISK, margin_q=MQ, grid=GRID,
                      eager=eager) as srv:
            tickets = [srv.submit(d) for d in scns]
            res[eager] = [srv.wait(t)[0] for t in tickets]
            assert srv.info()["failed"] == 0
    for d, a, b in zip(scns, res[False], res[True]):
        same_stats(a, b)
        alone = B.rollout(d, precision=prec)
        same_stats(a, B.reduce(alone, risk=RISK, margin_q=MQ, grid=GRID))
