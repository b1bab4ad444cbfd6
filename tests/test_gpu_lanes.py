"""Lane accounting of the integration kernels (aeb_timing_lanes): with timing
enabled, the wavefront sample-steps counted are at least the steps output and
the slots times the longest sample (a chunk runs as long as its longest
sample), and at most a top block per chunk beyond the longest sample."""
import numpy as np
import pytest

from paper_2604_27193_amd import workloads as W
from test_gpu_parity import to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2604_27193_amd import binding
    binding.lib()
    return binding


CASES = {
    "fp64 stationary": (W.single(100_000, seed=3), "fp64", None),
    "fp64 ragged": (W.single(4_097, seed=4), "fp64", None),
    "fp64 two per lane": (W.single(50_000, seed=5), "fp64", ("stationary", 64, 256, 0, 2)),
    "fp64 lead": (W.sweep(n=30_000)[77], "fp64", None),
    "fp64 controller": (W.closed_loop(30_000, seed=6), "fp64", None),
    "fp64 rk4": (W.paper_preset(20_000), "fp64", None),
    "fp32c stationary": (W.single(100_000, seed=7), "fp32c", None),
    "fp32c lead": (W.sweep(n=30_000)[77], "fp32c", None),
}


@pytest.mark.parametrize("name", list(CASES))
def test_lane_accounting(B, name):
    d, prec, shape = CASES[name]
    keep = None
    if shape:
        keep = B.tune_get(prec, shape[0])
        B.tune_set(prec, shape[0], *shape[1:])
    B.timing_enable(True)
    try:
        out = to_np(B.rollout(d, precision=prec))
        wave = B.timing_lanes()
    finally:
        B.timing_enable(False)
        if keep:
            B.tune_set(prec, shape[0], *keep)
    steps = out["steps"].astype(np.int64)
    lane = int(steps.sum())
    spw = 128 if shape and shape[4] == 2 else 64
    chunks = -(-len(steps) // spw)
    # every chunk runs at least as long as its longest sample, at most a top
    # block (128 steps, 50 with the controller) beyond the horizon
    assert lane <= wave <= chunks * spw * (int(steps.max()) + 128)
    assert wave >= spw * int(steps.max())
    print(name, "lane efficiency", lane / wave)


def test_batch_lane_accounting(B):
    scns = W.uneven_batch(6, max_samples=20_000)
    B.timing_enable(True)
    try:
        outs = [to_np(o) for o in B.batch_rollout(scns, precision="fp32c")]
        wave = B.timing_lanes()
    finally:
        B.timing_enable(False)
    lane = sum(int(o["steps"].astype(np.int64).sum()) for o in outs)
    assert lane <= wave <= 2 * lane


def test_no_timed_launch_is_reported(B):
    B.timing_enable(True)
    try:
        with pytest.raises(B.AebError) as e:
            B.timing_lanes()
        assert e.value.code == B.EAGAIN
    finally:
        B.timing_enable(False)
