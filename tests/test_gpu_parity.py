"""GPU parity: every result of the HIP path against the FP64 reference on the
same seeded inputs.

Bars (the reference is exact FP64 of the same steps):
  * uniforms: bit-identical;
  * FP64 rollout: per-sample relative distance error <= 1e-12, status and step
    counts identical (the host-sampled plain method is expected bit-exact);
  * FP32 compensated rollout: relative distance error <= 1e-4, collision flags
    and end reasons identical except for samples the kernel flags as within
    the single-precision band of the boundary (none after the FP64 fix-up),
    v_impact within 0.05 m/s;
  * reduction: counts, order statistics and the risk curve identical, moments
    within 1e-12 relative.
"""
import numpy as np
import pytest

from paper_2604_27193_amd import workloads as W

pytestmark = pytest.mark.gpu

REL64 = 1e-12
REL32 = 1e-4


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


def upload(cols):
    import torch
    return {k: torch.from_numpy(np.ascontiguousarray(v)).to("cuda") for k, v in cols.items()}


def rel_err(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def check_fp64(got, ref, exact=False):
    assert np.array_equal(got["status"], ref["status"])
    assert np.array_equal(got["steps"], ref["steps"])
    assert rel_err(got["dist"], ref["dist"]).max() <= REL64
    m = np.abs(got["margin"] - ref["margin"])
    assert np.all(m <= REL64 * np.maximum(np.abs(ref["margin"]), np.abs(ref["dist"])) + 1e-12)
    assert np.all(np.abs(got["v_impact"] - ref["v_impact"]) <= 1e-6 * np.abs(ref["v_impact"]) + 1e-7)
    if exact:
        assert np.array_equal(got["dist"].view(np.uint64), ref["dist"].view(np.uint64))


def plain(B, d):
    host = B.sample_params(d, device=False)
    return B.rollout(d, params=upload(host))


# ---------------------------------------------------------------------------
# generator and sampler
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed,sid,slot,attempt,n", [(42, 0, 0, 0, 1_000_000),
                                                     (7, 2**33 + 9, 8, 3, 100_003)])
def test_device_uniforms_bitwise(B, orc, seed, sid, slot, attempt, n):
    got = B.uniforms(seed, sid, 5, n, slot, attempt, device=True).cpu().numpy()
    want = orc.uniforms(seed, sid, 5, n, slot, attempt)
    assert np.array_equal(got.view(np.uint64), want.view(np.uint64))


@pytest.mark.parametrize("row", range(3))
def test_device_uniforms_known_answers(B, row):
    # the kernel generator against the published Philox4x32-10 rows
    from test_oracle_rng import kat_as_uniform_call, kat_rows, kat_uniforms
    ctr, key, out = kat_rows()[row]
    seed, sid, i, slot, attempt = kat_as_uniform_call(ctr, key)
    got = B.uniforms(seed, sid, i, 1, slot, attempt, device=True).cpu().numpy().ravel()
    assert list(got) == kat_uniforms(out)


def test_device_sampler_matches_reference(B, orc):
    d = W.single(50_000)
    got = {k: v.cpu().numpy() for k, v in B.sample_params(d, device=True).items()}
    want = orc.sample(d)
    for c in ("mu", "crr", "tau"):                     # uniform draws: bit-identical
        assert np.array_equal(got[c], want[c]), c
    for c in ("v0", "mass", "grade", "sin_grade", "cos_grade", "cda", "gap"):
        assert rel_err(got[c], want[c] + (want[c] == 0)).max() <= 1e-14, c


# ---------------------------------------------------------------------------
# FP64 rollout
# ---------------------------------------------------------------------------
def test_plain_fp64_config0_exact(B, orc):
    d = W.single(10_000)
    got = to_np(plain(B, d))
    ref = orc.run(d)
    check_fp64(got, ref, exact=True)


@pytest.mark.parametrize("n,seed", [(1, 3), (63, 4), (64, 5), (257, 6), (4097, 7)])
def test_plain_fp64_ragged_sizes(B, orc, n, seed):
    d = W.single(n, seed=seed)
    check_fp64(to_np(plain(B, d)), orc.run(d), exact=True)


def test_device_rng_fp64(B, orc):
    d = W.single(20_000, seed=11, scenario_id=5)
    got = to_np(B.rollout(d, params=None))
    check_fp64(got, orc.run(d))


@pytest.mark.parametrize("variant", ["nofma", "impact_exit", "none", "rk4", "rk4_stationary",
                                     "paper_euler"])
def test_fp64_variants(B, orc, variant):
    if variant == "nofma":
        d = W.single(3000, nofma=True)
    elif variant == "impact_exit":
        d = W.single(3000, impact_exit=True)
    elif variant == "none":
        d = W.single(3000, obstacle="none")
    elif variant == "rk4":
        d = W.paper_preset(2000)
    elif variant == "rk4_stationary":
        d = W.single(2000, integrator="rk4")
    else:
        d = W.paper_preset(3000, integrator="euler")
    check_fp64(to_np(plain(B, d)), orc.run(d), exact=True)


@pytest.mark.parametrize("k", [0, 37, 100, 255])
def test_lead_vehicle_fp64(B, orc, k):
    d = W.sweep(n=1500)[k]
    check_fp64(to_np(plain(B, d)), orc.run(d), exact=True)
    check_fp64(to_np(B.rollout(d)), orc.run(d))


def test_uneven_scenarios_fp64(B, orc):
    for d in W.uneven_batch(6, max_samples=1500):
        check_fp64(to_np(B.rollout(d)), orc.run(d))


def test_full_size_sampled(B, orc):
    """Config-1 size, launch shape of the benchmark; 1,500 sampled indices."""
    d = W.single(1_048_576)
    got = to_np(plain(B, d))
    rng = np.random.default_rng(2024)
    idx = np.unique(np.concatenate([rng.integers(0, d["n_samples"], 1500),
                                    [0, 1, d["n_samples"] - 1]]))
    for i in idx:
        r = orc.run(d, first=int(i), count=1)
        assert got["status"][i] == r["status"][0] and got["steps"][i] == r["steps"][0]
        assert got["dist"][i] == r["dist"][0], i
    # properties that hold at any size
    st = got["status"]
    col = (st & B.COLLIDED) != 0
    host = B.sample_params(d, device=False)
    assert np.array_equal(col, got["dist"] > host["gap"])
    assert np.all(st & 3 == B.END_STOP)


def test_repeat_is_bitwise_deterministic(B):
    d = W.single(30_000)
    params = upload(B.sample_params(d, device=False))
    first = to_np(B.rollout(d, params=params))
    s0 = B.reduce(B.rollout(d, params=params), risk=(0.05,), grid=(40, 90, 51))
    for _ in range(5):
        again = to_np(B.rollout(d, params=params))
        for k in first:
            assert np.array_equal(first[k], again[k])
        s1 = B.reduce(B.rollout(d, params=params), risk=(0.05,), grid=(40, 90, 51))
        assert s1["mean_dist"] == s0["mean_dist"] and s1["sd_dist"] == s0["sd_dist"]


def test_invalid_arguments_raise(B):
    import torch
    with pytest.raises(B.AebError):
        B.rollout(dict(W.single(10), n_samples=0))
    d = W.single(100)
    out = B.alloc_outputs(99)
    with pytest.raises(B.AebError):
        B.rollout(d, out=out)
    with pytest.raises(B.AebError):
        B.rollout(dict(d, integrator="rk4", obstacle="lead"))
    torch.cuda.synchronize()


# ---------------------------------------------------------------------------
# FP32 compensated rollout
# ---------------------------------------------------------------------------
B_COLLIDED, B_BOUNDARY = 4, 8


def check_fp32c(got, ref, fixup=False, margin_abs=None):
    """Distance within 1e-4; flags and end reasons exact except samples flagged
    as within the boundary band (none of which remain after the FP64 fix-up);
    optionally the margin within margin_abs metres."""
    bnd = (got["status"] & B_BOUNDARY) != 0
    # a flagged sample lies at the boundary: its reference clearance (margin)
    # is within a step's travel of zero, and its own margin agrees with it
    assert np.all(np.abs(ref["margin"][bnd]) <= 0.1), ref["margin"][bnd]
    assert np.all(np.abs(got["margin"][bnd] - ref["margin"][bnd]) <= 0.1)
    if margin_abs is not None:
        ok_m = ~bnd
        assert np.all(np.abs(got["margin"] - ref["margin"])[ok_m] <= margin_abs)
    if fixup:
        assert not bnd.any()
    ok = ~bnd
    rel = rel_err(got["dist"], ref["dist"])[ok]
    assert rel.max() <= REL32, rel.max()
    assert np.array_equal(got["status"][ok] & B_COLLIDED, ref["status"][ok] & B_COLLIDED)
    assert np.array_equal(got["status"][ok] & 3, ref["status"][ok] & 3)
    col = ok & ((ref["status"] & B_COLLIDED) != 0)
    assert np.all(np.abs(got["v_impact"][col] - ref["v_impact"][col]) <= 0.05)
    assert np.all(np.abs(got["steps"][ok] - ref["steps"][ok]) <= 2)
    # a flag can only disagree within the band around the obstacle
    bad = (got["status"] & B_COLLIDED) != (ref["status"] & B_COLLIDED)
    assert np.all(bnd[bad])
    return rel, int(bnd.sum())


@pytest.mark.parametrize("mode", ["plain", "devrng"])
@pytest.mark.parametrize("prec", ["fp32c", "fp32c_fixup"])
def test_fp32c_config0(B, orc, mode, prec):
    d = W.single(20_000)
    params = upload(B.sample_params(d, device=False)) if mode == "plain" else None
    got = to_np(B.rollout(d, params=params, precision=prec))
    rel, nb = check_fp32c(got, orc.run(d), fixup=prec == "fp32c_fixup")
    print(f"{prec} config0 {mode}: max rel {rel.max():.2e} mean {rel.mean():.2e} boundary {nb}")


@pytest.mark.parametrize("k", [0, 40, 130, 255])
@pytest.mark.parametrize("prec", ["fp32c", "fp32c_fixup"])
def test_fp32c_lead(B, orc, k, prec):
    d = W.sweep(n=1000)[k]
    got = to_np(B.rollout(d, precision=prec))
    check_fp32c(got, orc.run(d), fixup=prec == "fp32c_fixup", margin_abs=2e-3)


@pytest.mark.parametrize("prec", ["fp32c", "fp32c_fixup"])
def test_fp32c_variants(B, orc, prec):
    for d in (W.single(2000, obstacle="none"), W.single(2000, impact_exit=True),
              W.single(1500, obstacle="none", dt=5e-4, horizon=15.0),
              W.single(2000, seed=17, nofma=True),  # the fix-up recomputes in the unfused form
              W.paper_preset(2000, integrator="euler"), W.single(1500, dt=5e-4, horizon=15.0),
              *W.uneven_batch(3, max_samples=1000)):
        check_fp32c(to_np(B.rollout(d, precision=prec)), orc.run(d), fixup=prec == "fp32c_fixup")


def test_fp32c_full_size_error_budget(B, orc):
    """1,048,576 samples: distance error against FP64 stays under 1e-4 everywhere
    and flags agree outside the band; sampled samples against the reference."""
    d = W.single(1_048_576)
    params = upload(B.sample_params(d, device=False))
    g64 = to_np(B.rollout(d, params=params))
    g32 = to_np(B.rollout(d, params=params, precision="fp32c"))
    rel = rel_err(g32["dist"], g64["dist"])
    assert rel.max() <= REL32
    bnd = (g32["status"] & B_BOUNDARY) != 0
    assert np.array_equal((g32["status"] & 7)[~bnd], (g64["status"] & 7)[~bnd])
    assert bnd.sum() < 1e-3 * d["n_samples"]
    print(f"fp32c 1M: max rel {rel.max():.2e} boundary {bnd.sum()}")


# ---------------------------------------------------------------------------
# block-structured path: edge cases of its guards
# ---------------------------------------------------------------------------
MU_AT_COMMAND = 6.0 / (9.81 - 6.0 * 0.55 / 2.7)   # friction limit equal to the command


@pytest.mark.parametrize("case", ["no_dead_time", "dead_2K", "dead_beyond_horizon",
                                  "horizon_cut", "horizon_short", "dt2ms", "mu_at_command",
                                  "wide_gap", "wide_gap_exit", "downhill"])
@pytest.mark.parametrize("prec", ["fp64", "fp32c", "rk4"])
def test_block_path_edges(B, orc, case, prec):
    d = W.single(3000, seed=77)
    if prec == "rk4":
        d["integrator"] = "rk4"
    d.update({
        "no_dead_time": dict(dead_time=0.0),
        "dead_2K": dict(dead_time=0.064),
        "dead_beyond_horizon": dict(dead_time=0.5, horizon=0.4),
        "horizon_cut": dict(horizon=4.2),
        "horizon_short": dict(horizon=0.033),
        "dt2ms": dict(dt=2e-3),
        "mu_at_command": dict(mu=("const", MU_AT_COMMAND)),
        "wide_gap": dict(gap=("normal", 55.0, 20.0)),
        "wide_gap_exit": dict(gap=("normal", 55.0, 20.0), impact_exit=True),
        "downhill": dict(grade=("normal", -0.25, 0.05), mu=("uniform", 0.3, 0.5)),
    }[case])
    ref = orc.run(d)
    got = to_np(B.rollout(d, precision="fp64" if prec == "rk4" else prec))
    if prec in ("fp64", "rk4"):
        check_fp64(got, ref)
    else:
        check_fp32c(got, ref)


def test_timing_hook(B):
    d = W.single(50_000)
    B.timing_enable(True)
    try:
        B.rollout(d)
        ms = B.timing_last()
        assert 0.0 < ms < 1000.0
    finally:
        B.timing_enable(False)


# ---------------------------------------------------------------------------
# reduction
# ---------------------------------------------------------------------------
RISK = (0.0, 0.5, 0.05, 0.01, 0.001)
MQ = (0.0, 0.01, 0.1, 0.5)
GRID = (30.0, 110.0, 161)


def compare_stats(got, want):
    for k in ("n", "n_collide", "n_stop", "n_impact", "n_horizon", "p_collision", "margin_min",
              "v_impact_max", "dist_min", "dist_max"):
        assert got[k] == want[k] or (np.isnan(got[k]) and np.isnan(want[k])), k
    assert got["headway"] == want["headway"]
    assert got["margin_q"] == want["margin_q"]
    assert np.array_equal(got["risk_count"], want["risk_count"])
    assert np.array_equal(got["risk_p"], want["risk_p"])
    for k in ("mean_dist", "sd_dist", "margin_mean"):
        if np.isnan(want[k]):
            assert np.isnan(got[k])
        else:
            assert abs(got[k] - want[k]) <= 1e-12 * max(abs(want[k]), 1.0), k


def test_reduce_on_rollout(B, orc):
    d = W.single(10_000)
    out = plain(B, d)
    got = B.reduce(out, risk=RISK, margin_q=MQ, grid=GRID)
    want = orc.reduce(orc.run(d), risk=RISK, margin_q=MQ, grid=GRID)
    compare_stats(got, want)


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (777, 2), (65_537, 3), (300_001, 4)])
def test_reduce_on_synthetic(B, orc, n, seed):
    from test_oracle_reduce import synthetic
    syn = synthetic(n, seed, ties=(seed % 2 == 0))
    got = B.reduce(upload(syn), risk=RISK, margin_q=MQ, grid=GRID)
    want = orc.reduce(syn, risk=RISK, margin_q=MQ, grid=GRID)
    compare_stats(got, want)


def test_horizon_beyond_block_path_limit(B, orc):
    """A horizon of 2,147,483,000 steps (within the 2^31 - 1 validation
    bound, beyond the block path's 2^31 - 4096): FP64 takes the checked
    kernel, which counts steps in 64 bits, and matches the reference (every
    sample stops long before the horizon); FP32C and a recorded graph say no."""
    d = W.single(1500, seed=8, horizon=2147483.0)
    check_fp64(to_np(plain(B, d)), orc.run(d), exact=True)
    with pytest.raises(B.AebError, match="2\\^31 - 4096"):
        B.rollout(d, precision="fp32c")
    with pytest.raises(B.AebError):
        B.Graph(d)


@pytest.mark.parametrize("k", [3, 70, 130, 255])
def test_lead_unfused_exact(B, orc, k):
    """The paper's rule of no fused operations with a decelerating lead vehicle
    (the block-structured kernel, lead state pinned per step): bit for bit."""
    d = dict(W.sweep(n=2500)[k], nofma=True)
    check_fp64(to_np(plain(B, d)), orc.run(d), exact=True)
