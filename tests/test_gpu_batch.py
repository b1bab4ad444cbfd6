"""GPU parity of the batched rollout: many scenarios of uneven sizes, steps,
horizons and obstacles in one launch, each scenario against the FP64
reference, and each equal to the same scenario rolled out alone."""
import numpy as np
import pytest

from paper_2604_27193_amd import workloads as W
from test_gpu_parity import check_fp32c, check_fp64, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2604_27193_amd import binding
    binding.lib()
    return binding


def test_batch_lead_sweep_fp64(B, orc):
    scns = W.sweep(n=800)[::21]
    outs = B.batch_rollout(scns)
    for d, o in zip(scns, outs):
        check_fp64(to_np(o), orc.run(d))


def test_batch_uneven_fp64(B, orc):
    scns = W.uneven_batch(24, max_samples=1200)
    assert len({d["dt"] for d in scns}) == 3
    outs = B.batch_rollout(scns)
    for d, o in zip(scns, outs):
        check_fp64(to_np(o), orc.run(d))


def test_batch_uneven_unfused(B, orc):
    """The paper's rule of no fused operations in one batched launch: every
    scenario equals the reference bit for bit and equals its launch alone."""
    scns = [dict(d, nofma=True) for d in W.uneven_batch(12, max_samples=1500)]
    outs = B.batch_rollout(scns)
    for d, o in zip(scns, outs):
        got = to_np(o)
        check_fp64(got, orc.run(d))
        alone = to_np(B.rollout(d))
        for c in got:
            assert np.array_equal(got[c], alone[c]), c


def test_batch_lead_sweep_unfused(B, orc):
    """Sixteen cells of the lead-vehicle sweep without fused operations in one
    batched launch: each equals the reference and its launch alone."""
    scns = [dict(d, nofma=True) for d in W.sweep(n=800)[::16]]
    outs = B.batch_rollout(scns)
    for d, o in zip(scns, outs):
        got = to_np(o)
        check_fp64(got, orc.run(d))
        alone = to_np(B.rollout(d))
        for c in got:
            assert np.array_equal(got[c], alone[c]), c


def test_batch_uneven_fp32c(B, orc):
    scns = W.uneven_batch(24, max_samples=1200)
    outs = B.batch_rollout(scns, precision="fp32c")
    for d, o in zip(scns, outs):
        check_fp32c(to_np(o), orc.run(d))


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_batch_equals_alone(B, prec):
    scns = W.uneven_batch(10, max_samples=3000) + [W.single(2000, seed=5, scenario_id=77)]
    outs = B.batch_rollout(scns, precision=prec)
    for d, o in zip(scns, outs):
        alone = to_np(B.rollout(d, precision=prec))
        got = to_np(o)
        for k in alone:
            assert np.array_equal(got[k], alone[k]), (prec, k)


def test_batch_tiny_and_ragged(B, orc):
    base = W.single(1)
    scns = [dict(base, n_samples=n, scenario_id=j) for j, n in enumerate([1, 2, 63, 65, 129, 1])]
    outs = B.batch_rollout(scns)
    for d, o in zip(scns, outs):
        check_fp64(to_np(o), orc.run(d))


def test_batch_reduce_matches_reference(B, orc):
    scns = W.uneven_batch(5, max_samples=2500)
    outs = B.batch_rollout(scns)
    risk, mq, grid = (0.5, 0.05, 0.01), (0.0, 0.5), (20.0, 120.0, 101)
    stats = B.batch_reduce(outs, risk=risk, margin_q=mq, grid=grid)
    for d, st in zip(scns, stats):
        ref = orc.reduce(orc.run(d), risk=risk, margin_q=mq, grid=grid)
        assert st["n_collide"] == ref["n_collide"] and st["p_collision"] == ref["p_collision"]
        assert st["headway"] == ref["headway"] and st["margin_q"] == ref["margin_q"]
        assert np.array_equal(st["risk_count"], ref["risk_count"])
        assert abs(st["mean_dist"] - ref["mean_dist"]) <= 1e-12 * ref["mean_dist"]


def test_batch_rk4_and_fp32_lead(B, orc):
    # RK4 (FP64) and FP32 with a lead vehicle in one batched launch each
    rk = [W.paper_preset(700, seed=s, scenario_id=s) for s in (1, 2, 3)]
    for d, o in zip(rk, B.batch_rollout(rk)):
        check_fp64(to_np(o), orc.run(d))
    lead = W.sweep(n=600)[40:43]
    for d, o in zip(lead, B.batch_rollout(lead, precision="fp32c")):
        check_fp32c(to_np(o), orc.run(d))


def test_batch_rejects_bad_batches(B):
    with pytest.raises(B.AebError):
        B.batch_rollout([W.single(10), W.single(10, obstacle="none")])
    with pytest.raises(B.AebError):
        B.batch_rollout([W.single(10)], precision="fp32c_fixup")
    with pytest.raises(B.AebError):
        B.batch_rollout([W.single(10), dict(W.single(10), dt=-1.0)])


@pytest.mark.parametrize("prec", ["fp64", "fp32c"])
def test_batch_lead_mixed_horizons(B, orc, prec):
    # lanes of near-equal predicted length but different horizons share
    # wavefronts: a lane ending at its horizon while its neighbours go on must
    # keep the margin it had when it ended
    base = W.sweep(n=3000)[160]
    scns = [dict(base, scenario_id=900 + j, horizon=h) for j, h in
            enumerate((0.8, 0.85, 0.9, 3.0))]
    outs = B.batch_rollout(scns, precision=prec)
    for d, o in zip(scns, outs):
        got, ref = to_np(o), orc.run(d)
        if prec == "fp64":
            check_fp64(got, ref)
        else:
            check_fp32c(got, ref, margin_abs=2e-3)
        assert ((ref["status"] & 3) == 3).any()        # some lanes end at the horizon


def _subset_stats(status, dist):
    col = (status & 4) != 0
    return col.mean(), np.percentile(dist, 99)


def test_sweep_full_size_subset(B, orc):
    """The 256-scenario lead-vehicle sweep at 100,000 samples each in one
    launch: on the first 1,000 samples of every scenario, FP64 equals the
    reference and FP32C's per-scenario P(collision) and p99 distance are
    within the stated tolerance of it."""
    import torch
    scns = W.sweep(n=100_000)
    got = {}
    for prec in ("fp64", "fp32c"):
        outs = B.batch_rollout(scns, precision=prec)
        torch.cuda.synchronize()
        got[prec] = [{k: v[:1000].cpu().numpy() for k, v in o.items()} for o in outs]
        del outs
        torch.cuda.empty_cache()
    worst_p, worst_q = 0.0, 0.0
    threads = orc.host_threads()
    for j, d in enumerate(scns):
        ref = orc.run(d, first=0, count=1000, threads=threads)
        check_fp64(got["fp64"][j], ref)
        g32 = got["fp32c"][j]
        check_fp32c(g32, ref, margin_abs=2e-3)
        p_ref, q_ref = _subset_stats(ref["status"], ref["dist"])
        p_32, q_32 = _subset_stats(g32["status"], g32["dist"])
        nb = int(((g32["status"] & 8) != 0).sum())
        assert abs(p_32 - p_ref) <= nb / 1000.0 + 1e-12, j
        # nb boundary samples may end differently (at the lead or not), which
        # moves an order statistic by at most nb ranks (unbounded past the ends)
        srt = np.sort(ref["dist"])
        lo = srt[989 - nb] * (1 - 1e-4) if 989 - nb >= 0 else -np.inf
        hi = srt[990 + nb] * (1 + 1e-4) if 990 + nb <= 999 else np.inf
        assert lo <= q_32 <= hi, (j, nb, q_32, q_ref)
        worst_p, worst_q = max(worst_p, abs(p_32 - p_ref)), max(worst_q, abs(q_32 - q_ref) / q_ref)
    print(f"sweep subset: max |dP| {worst_p:.2e}, max rel p99 error {worst_q:.2e}")


def test_uneven_full_size_sampled(B, orc):
    """The 1,000-scenario uneven batch at full size (about 1.4e8 samples) in
    one launch: the first and last sample of every scenario against the
    reference."""
    import torch
    scns = W.uneven_batch(1000)
    outs = B.batch_rollout(scns)
    torch.cuda.synchronize()
    for d, o in zip(scns, outs):
        n = int(d["n_samples"])
        for i in (0, n - 1):
            ref = orc.run(d, first=i, count=1)
            assert int(o["status"][i].item()) == int(ref["status"][0])
            assert int(o["steps"][i].item()) == int(ref["steps"][0])
            assert abs(float(o["dist"][i].item()) - ref["dist"][0]) <= 1e-12 * abs(ref["dist"][0])


def test_batch_unfused_runs_scenario_by_scenario(B, orc):
    scns = [W.single(900, seed=s, scenario_id=s, nofma=True) for s in (4, 5)]
    for d, o in zip(scns, B.batch_rollout(scns)):
        check_fp64(to_np(o), orc.run(d))
