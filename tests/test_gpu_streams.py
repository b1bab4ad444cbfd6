"""Calls in flight at once on different streams and threads.

The library's scratch pool hands each call blocks no other live call holds
and fences them with an event on the call's stream, so eager rollouts and
reductions of different scenarios on two streams -- or from two host threads,
while the pool grows under them -- each give the same bits as the same call
alone.
"""
import threading

import numpy as np
import pytest

from paper_2604_27193_amd import workloads as W
from test_gpu_parity import to_np

pytestmark = pytest.mark.gpu

RISK = (0.05, 0.01)
GRID = (30.0, 110.0, 41)


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2604_27193_amd import binding
    binding.lib()
    return binding


def alone(B, d, prec):
    out = B.rollout(d, precision=prec)
    st = B.reduce(out, risk=RISK, grid=GRID)
    return to_np(out), st


def same(B, got, ref):
    for k in ref:
        assert np.array_equal(got[k], ref[k]), k


def same_stats(a, b):
    for k, v in a.items():
        if isinstance(v, np.ndarray):
            assert np.array_equal(v, b[k]), k
        elif isinstance(v, float) and v != v:
            assert b[k] != b[k], k
        else:
            assert v == b[k], k


@pytest.mark.parametrize("prec", ["fp64", "fp32c_fixup"])
def test_two_streams_in_flight(B, prec):
    import torch
    da = W.single(600_000, seed=5)
    db = dict(W.sweep(n=400_000)[100])
    ra, sa = alone(B, da, prec)
    rb, sb = alone(B, db, prec)
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    oa, ob = B.alloc_outputs(600_000), B.alloc_outputs(400_000)
    torch.cuda.synchronize()
    for it in range(4):
        first, second = ((s1, da, oa), (s2, db, ob)) if it % 2 == 0 else ((s2, db, ob),
                                                                          (s1, da, oa))
        # both rollouts enqueued before either is collected
        B.rollout(first[1], precision=prec, out=first[2], stream=first[0])
        B.rollout(second[1], precision=prec, out=second[2], stream=second[0])
        ga = B.reduce(oa, risk=RISK, grid=GRID, stream=s1)
        gb = B.reduce(ob, risk=RISK, grid=GRID, stream=s2)
        torch.cuda.synchronize()
        same(B, to_np(oa), ra)
        same(B, to_np(ob), rb)
        same_stats(ga, sa)
        same_stats(gb, sb)


def test_two_threads_while_the_pool_grows(B):
    """Two host threads on their own streams, each cycling through scenarios of
    growing size (so the pool adds and replaces blocks while the other thread's
    work is in flight); every result equals its run alone."""
    import torch
    plans = {
        0: [W.single(n, seed=31 + k) for k, n in enumerate((20_000, 200_000, 900_000, 1_500_000))],
        1: [dict(W.sweep(n=n)[40 + k]) for k, n in enumerate((1_200_000, 30_000, 700_000))],
    }
    refs = {t: [alone(B, d, "fp64") for d in ds] for t, ds in plans.items()}
    torch.cuda.synchronize()
    errors = []

    def worker(t):
        try:
            st = torch.cuda.Stream()
            with torch.cuda.stream(st):
                for rep in range(3):
                    for d, (ref, sref) in zip(plans[t], refs[t]):
                        out = B.alloc_outputs(int(d["n_samples"]))
                        B.rollout(d, out=out, stream=st)
                        got = B.reduce(out, risk=RISK, grid=GRID, stream=st)
                        st.synchronize()
                        same(B, to_np(out), ref)
                        same_stats(got, sref)
        except Exception as e:  # reported by the main thread
            errors.append((t, repr(e)))

    th = [threading.Thread(target=worker, args=(t,)) for t in plans]
    for x in th:
        x.start()
    for x in th:
        x.join()
    torch.cuda.synchronize()
    assert not errors, errors


def test_capturing_stream_is_refused(B):
    """The pool's event fences cannot be recorded into a caller's graph: a
    rollout on a capturing stream is refused before anything is enqueued."""
    import torch
    d = W.single(1000)
    out = B.alloc_outputs(1000)
    torch.cuda.synchronize()
    st = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with pytest.raises(B.AebError, match="captured"):
        with torch.cuda.graph(g, stream=st):
            B.rollout(d, out=out)
    torch.cuda.synchronize()
