"""aeb_rollout_noalloc (the rollout on the library's fixed per-device scratch
array, for callers that cannot allocate) against aeb_rollout on the same
inputs: every output of every sample identical, for two calls in a row on
one device, the second with fewer samples than the first (the array keeps
the first call's contents, which the second must not read).  Also: a
scenario whose scratch exceeds the array is refused before anything runs
(the largest accepted sizes are the ones the header states), and a call
captured into a HIP graph replays to the same results."""
import numpy as np
import pytest

from paper_2604_27193_amd import workloads as W

pytestmark = pytest.mark.gpu


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


def same(a, b):
    for k in a:
        assert np.array_equal(np.asarray(a[k]).view(np.uint8), np.asarray(b[k]).view(np.uint8)), k


def upload(cols):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to("cuda") for k, v in cols.items()}


CASES = [
    # (description, scenario builder of n, precision, host-drawn parameters)
    ("stationary fp64 plain", lambda n: W.single(n), "fp64", True),
    ("stationary fp32c in-kernel", lambda n: W.single(n, seed=5), "fp32c", False),
    ("stationary fp32c fix-up", lambda n: W.single(n, seed=6), "fp32c_fixup", False),
    ("lead sweep cell fp64", lambda n: dict(W.sweep(n=n)[200]), "fp64", False),
    ("lead sweep cell fp32c", lambda n: dict(W.sweep(n=n)[37]), "fp32c", False),
    ("perception fp64", lambda n: W.perception(n), "fp64", False),
    ("controller fp64", lambda n: W.closed_loop(n), "fp64", False),
    ("paper preset rk4", lambda n: W.paper_preset(n), "fp64", True),
]


@pytest.mark.parametrize("case", CASES, ids=[c[0] for c in CASES])
def test_noalloc_equals_rollout_two_calls(B, case):
    _, make, prec, plain = case
    for n in (300_000, 4_097):  # the second call smaller than the first
        d = make(n)
        params = upload(B.sample_params(d, device=False)) if plain else None
        want = to_np(B.rollout(d, params=params, precision=prec))
        got = to_np(B.rollout_noalloc(d, params=params, precision=prec))
        same(got, want)


def test_noalloc_refuses_beyond_its_array(B):
    import torch
    n = B.NOALLOC_SCRATCH_BYTES // 64  # 64-byte job records alone exceed it
    d = W.single(n)
    out = B.alloc_outputs(1)
    out_big = {k: torch.empty(n, dtype=v.dtype, device="cuda") for k, v in out.items()}
    with pytest.raises(RuntimeError, match="scratch"):
        B.rollout_noalloc(d, out=out_big)


@pytest.mark.parametrize("lead, limit", [(False, 418_604), (True, 380_544)],
                         ids=["stationary", "lead"])
def test_noalloc_limit_is_the_documented_one(B, lead, limit):
    """aeb.h states the largest scenario the array takes: that one runs (and
    equals aeb_rollout), one sample more is refused."""
    def make(n):
        return dict(W.sweep(n=n)[37]) if lead else W.single(n, seed=3)
    d = make(limit)
    want = to_np(B.rollout(d, precision="fp32c"))
    same(to_np(B.rollout_noalloc(d, precision="fp32c")), want)
    out = B.alloc_outputs(limit + 1)
    with pytest.raises(RuntimeError, match="scratch"):
        B.rollout_noalloc(make(limit + 1), out=out, precision="fp32c")


def test_noalloc_in_captured_graph(B):
    import torch
    d = W.single(50_000, seed=11)
    want = to_np(B.rollout(d))
    out = B.alloc_outputs(50_000)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        B.rollout_noalloc(d, out=out, stream=s)  # first call on the device: symbol lookup
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        B.rollout_noalloc(d, out=out, stream=s)
    for _ in range(3):
        for v in out.values():
            v.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        same(to_np(out), want)
