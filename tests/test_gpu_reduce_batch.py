"""The segmented reduction (aeb_batch_reduce: every kernel of the reduction
covers a group of output sets) against the single-set reduction and the
FP64 reference.

* the 1,000-scenario uneven batch (about 1.4e8 samples): every set's
  statistics equal aeb_reduce of that set alone, bit for bit;
* samples 0..999 of 32 of those scenarios, reduced as 32 sets of one call,
  against the reference's sort-based statistics of the same samples;
* sets with and without importance-sampling weights in one call;
* the radix-select fallback (a value bin with more than 8,192 equal values at
  a target rank): it runs, alone and inside a batch, and the statistics still
  equal the reference's.
"""
import numpy as np
import pytest

from paper_2604_27193_amd import workloads as W
from test_gpu_parity import MQ, RISK, GRID, compare_stats, to_np, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2604_27193_amd import binding
    binding.lib()
    return binding


def same_stats(a, b):
    for k, v in a.items():
        w = b[k]
        if isinstance(v, np.ndarray):
            assert np.array_equal(v.view(np.uint8), w.view(np.uint8)), k
        elif isinstance(v, float):
            assert np.float64(v).tobytes() == np.float64(w).tobytes(), k
        else:
            assert v == w, k


@pytest.fixture(scope="module")
def uneven(B):
    import torch
    scns = W.uneven_batch(1000)
    outs = B.batch_rollout(scns, precision="fp32c")
    torch.cuda.synchronize()
    yield scns, outs
    del outs
    torch.cuda.empty_cache()


def test_uneven_1000_batch_reduce_equals_alone(B, uneven):
    scns, outs = uneven
    got = B.batch_reduce(outs, risk=RISK, margin_q=MQ, grid=GRID)
    assert len(got) == 1000
    for o, st in zip(outs, got):
        same_stats(st, B.reduce(o, risk=RISK, margin_q=MQ, grid=GRID))


def test_uneven_subsets_batch_reduce_vs_reference(B, orc, uneven):
    """Samples 0..999 of 32 of the scenarios, rolled out from host-drawn
    parameters (the plain method: bit-identical to the reference's rollouts)
    and reduced as 32 sets of one call: the statistics equal the
    reference's sort-based ones of the same samples."""
    scns, _ = uneven
    pick = sorted(np.random.default_rng(34).choice(1000, 32, replace=False).tolist())
    sub = [dict(scns[j], n_samples=1000) for j in pick]
    outs = [B.rollout(d, params=upload(B.sample_params(d, device=False))) for d in sub]
    got = B.batch_reduce(outs, risk=RISK, margin_q=MQ, grid=GRID)
    for d, st in zip(sub, got):
        want = orc.reduce(orc.run(d, threads=min(8, orc.host_threads())), risk=RISK,
                          margin_q=MQ, grid=GRID)
        compare_stats(st, want)


def test_ragged_sets_and_views(B, orc):
    """Sets of 1, 2, 4,095, 4,096, 4,097 and 70,001 samples, some of them
    slices of one rollout's columns, in one call."""
    d = W.single(70_001, seed=21)
    host = B.sample_params(d, device=False)
    full = B.rollout(d, params=upload(host))
    ref = orc.run(d, threads=min(8, orc.host_threads()))
    cuts = [(0, 1), (5, 7), (100, 4195), (0, 4096), (9, 4106), (0, 70_001)]
    outs = [{k: v[a:b] for k, v in full.items()} for a, b in cuts]
    got = B.batch_reduce(outs, risk=RISK, margin_q=MQ, grid=GRID)
    for (a, b), st in zip(cuts, got):
        want = orc.reduce({k: v[a:b] for k, v in ref.items()}, risk=RISK, margin_q=MQ,
                          grid=GRID)
        compare_stats(st, want)


def test_weighted_and_plain_sets_together(B):
    dw = W.rare_event(20_000, integrator="euler")
    dp = W.single(30_000, seed=3)
    ow = B.rollout(dw)
    op = B.rollout(dp)
    got = B.batch_reduce([op, ow, op], risk=RISK, margin_q=MQ, grid=GRID)
    same_stats(got[0], B.reduce(op, risk=RISK, margin_q=MQ, grid=GRID))
    same_stats(got[1], B.reduce(ow, risk=RISK, margin_q=MQ, grid=GRID))
    same_stats(got[2], got[0])
    assert got[1]["weighted"] == 1 and got[0]["weighted"] == 0


def tied(n, n_tie, seed):
    """Synthetic outputs whose middle n_tie distances are one value (STOP),
    so the median's value bin holds n_tie > 8,192 samples."""
    rng = np.random.default_rng(seed)
    lo = (n - n_tie) // 2
    dist = np.concatenate([rng.uniform(30.0, 59.0, lo), np.full(n_tie, 60.0),
                           rng.uniform(61.0, 90.0, n - lo - n_tie)])
    rng.shuffle(dist)
    status = np.full(n, 1, np.uint8)
    status[dist > 62.0] |= 4
    return {"dist": dist, "status": status, "steps": np.full(n, 5000, np.int32),
            "margin": 62.0 - dist, "v_impact": np.zeros(n, np.float32)}


def test_radix_fallback_runs_and_matches(B, orc):
    syn = tied(50_000, 20_000, seed=9)
    want = orc.reduce(syn, risk=(0.5, 0.01), margin_q=(0.5,), grid=GRID)
    dev = upload(syn)
    before = B.reduce_fallbacks()
    got = B.reduce(dev, risk=(0.5, 0.01), margin_q=(0.5,), grid=GRID)
    assert B.reduce_fallbacks() == before + 1
    compare_stats(got, want)
    assert got["headway"][0] == 60.0
    # inside a batch: only the tied set takes the fallback
    other = upload(tied(9_000, 10, seed=10))
    before = B.reduce_fallbacks()
    got = B.batch_reduce([other, dev, other], risk=(0.5, 0.01), margin_q=(0.5,), grid=GRID)
    assert B.reduce_fallbacks() == before + 1
    compare_stats(got[1], want)
    same_stats(got[0], got[2])
    same_stats(got[0], B.reduce(other, risk=(0.5, 0.01), margin_q=(0.5,), grid=GRID))


@pytest.mark.parametrize("n", [1, 63, 4095, 4096, 4097, 25_000])
def test_small_set_paths_give_same_bits(B, orc, n):
    """A set of at most 4,096 samples (one element-pass block) is reduced by
    one workgroup (two kernels) when every set of the launch is that small,
    and by the eight element-pass and selection kernels when a larger set
    shares the launch: the same statistics bit for bit, and equal to the
    reference's."""
    d = W.single(n, seed=n, scenario_id=3)
    small = B.rollout(d)
    big = B.rollout(W.single(70_000, seed=5))
    alone = B.reduce(small, risk=RISK, margin_q=MQ, grid=GRID)         # one workgroup
    pair = B.batch_reduce([small, small], risk=RISK, margin_q=MQ, grid=GRID)
    mixed = B.batch_reduce([big, small], risk=RISK, margin_q=MQ, grid=GRID)  # eight kernels
    same_stats(alone, mixed[1])
    same_stats(alone, pair[0])
    same_stats(alone, pair[1])
    compare_stats(alone, orc.reduce(to_np(small), risk=RISK, margin_q=MQ, grid=GRID))
