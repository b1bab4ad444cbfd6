"""GPU tests of recorded launch sequences: every replay of a graph (with
eager work, synchronizations and overwritten outputs between replays) gives
the eager results bit for bit, and reads its parameter columns at replay
time."""
import numpy as np
import pytest

from paper_2604_27193_amd import workloads as W

pytestmark = pytest.mark.gpu

RISK = (0.05, 0.01)
MQ = (0.0, 0.5)
GRID = (30.0, 130.0, 32)


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2604_27193_amd import binding
    binding.lib()
    return binding


def host(out):
    return {k: v.cpu().numpy() for k, v in out.items() if hasattr(v, "cpu")}


def same_stats(a, b):
    for k in a:
        if isinstance(a[k], np.ndarray):
            assert np.array_equal(a[k], b[k]), k
        elif isinstance(a[k], float) and np.isnan(a[k]):
            assert np.isnan(b[k]), k
        else:
            assert a[k] == b[k], (k, a[k], b[k])


def same_out(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def eager_noise(B, torch):
    d = W.single(4000, seed=99, scenario_id=5)
    o = B.rollout(d)
    B.reduce(o, risk=RISK)
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["fp64", "fp32c", "rk4", "nofma", "fp32c_fixup"])
def test_graph_replays_equal_eager(B, prec):
    import torch
    d = W.single(30000, seed=12, scenario_id=3)
    if prec == "rk4":
        d, prec = W.paper_preset(30000, seed=12, scenario_id=3), "fp64"
    if prec == "nofma":
        d, prec = W.single(30000, seed=12, scenario_id=3, nofma=True), "fp64"
    ref_out = B.rollout(d, precision=prec)
    ref_st = B.reduce(ref_out, risk=RISK, margin_q=MQ, grid=GRID)
    ref = host(ref_out)
    g = B.Graph(d, precision=prec, risk=RISK, margin_q=MQ, grid=GRID)
    for rep in range(4):
        g.out["dist"].fill_(-1.0)
        g.out["status"].zero_()
        g.launch()
        st = g.finish()
        same_out(ref, host(g.out))
        same_stats(ref_st, st)
        eager_noise(B, torch)
    g.close()


def test_graph_reads_params_at_replay(B):
    import torch
    d1 = W.single(20000, seed=1, scenario_id=1)
    d2 = W.single(20000, seed=2, scenario_id=2)
    params = B.sample_params(d1)
    g = B.Graph(d1, params=params, risk=RISK)
    g.launch()
    st1 = g.finish()
    same_stats(B.reduce(B.rollout(d1, params=B.sample_params(d1)), risk=RISK), st1)
    # new parameter values in the same columns: the next replay uses them
    p2 = B.sample_params(d2)
    for c in B.COLUMNS:
        params[c].copy_(p2[c])
    torch.cuda.synchronize()
    g.launch()
    st2 = g.finish()
    same_stats(B.reduce(B.rollout(d2, params=p2), risk=RISK), st2)
    assert st1["mean_dist"] != st2["mean_dist"]
    g.close()


def test_batch_graph_replays_equal_eager(B):
    import torch
    scns = W.uneven_batch(6, max_samples=3000)
    ref_outs = B.batch_rollout(scns)
    ref_st = B.batch_reduce(ref_outs, risk=RISK, margin_q=MQ, grid=GRID)
    refs = [host(o) for o in ref_outs]
    g = B.Graph(scns, batch=True, risk=RISK, margin_q=MQ, grid=GRID)
    for rep in range(3):
        for o in g.out:
            o["dist"].fill_(-1.0)
        g.launch()
        sts = g.finish()
        for j in range(len(scns)):
            same_out(refs[j], host(g.out[j]))
            same_stats(ref_st[j], sts[j])
        eager_noise(B, torch)
    g.close()


def test_graph_rejects(B):
    with pytest.raises(B.AebError) as e:   # the controller in a batched graph is not recorded
        B.Graph([W.single(100), W.closed_loop(100)], batch=True)
    assert e.value.code == B.EINVAL
    with pytest.raises(B.AebError) as e:   # the fix-up is recorded for one scenario only
        B.Graph([W.single(100), W.single(200)], precision="fp32c_fixup", batch=True)
    assert e.value.code == B.EINVAL


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_two_graphs_pipelined_on_two_streams(B, prec):
    """Two graphs of one scenario (own outputs and scratch each) replayed on
    two streams with step k+1 launched before step k is collected, as the
    benchmark's throughput loop runs them: every step's outputs and
    statistics equal the eager call's."""
    import torch
    d = W.single(60000, seed=21, scenario_id=4)
    ref_out = B.rollout(d, precision=prec)
    ref_st = B.reduce(ref_out, risk=RISK, margin_q=MQ, grid=GRID)
    ref = host(ref_out)
    gs = [B.Graph(d, precision=prec, risk=RISK, margin_q=MQ, grid=GRID) for _ in range(2)]
    ss = [torch.cuda.Stream(), torch.cuda.Stream()]
    steps = 6
    gs[0].launch(ss[0])
    for k in range(1, steps + 1):
        if k < steps:
            gs[k % 2].launch(ss[k % 2])
        j = (k - 1) % 2
        same_stats(ref_st, gs[j].finish(ss[j]))
        same_out(ref, host(gs[j].out))
    for g in gs:
        g.close()
