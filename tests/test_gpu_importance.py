"""GPU parity of importance sampling (rare-event estimation, named in
Sec. VIII): proposal draws and likelihood-ratio weights against the FP64
reference, and the weighted collision-risk estimates of the reduction
(exact 128-bit fixed-point sums) against the reference's plain sums."""
import math

import numpy as np
import pytest
from scipy import stats as S

from paper_2604_27193_amd import workloads as W
from test_gpu_parity import check_fp64, rel_err, to_np, upload

pytestmark = pytest.mark.gpu

GRID = (90.0, 170.0, 81)


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2604_27193_amd import binding
    binding.lib()
    return binding


def weighted_ref(orc, d, ref_out=None, cols=None):
    out = ref_out if ref_out is not None else orc.run(d, threads=8)
    cols = cols if cols is not None else orc.sample(d)
    return out, orc.weighted_risk(out, np.exp(cols["log_weight"]), GRID)


def close(a, b, rel=1e-12, abs_=1e-300):
    a, b = np.asarray(a), np.asarray(b)
    assert np.all(np.abs(a - b) <= rel * np.abs(b) + abs_), np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300))


def test_device_log_weights(B, orc):
    d = W.rare_event(50_000)
    got = B.sample_params(d, device=True)["log_weight"].cpu().numpy()
    want = orc.sample(d)["log_weight"]
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("integrator", ["euler", "rk4"])
def test_plain_rollout_and_weights(B, orc, integrator):
    d = W.rare_event(20_000, integrator=integrator)
    host = B.sample_params(d, device=False)
    got = to_np(B.rollout(d, params=upload(host)))
    ref = orc.run(d, threads=8)
    check_fp64({k: v for k, v in got.items() if k != "weight"}, ref, exact=True)
    close(got["weight"], np.exp(orc.sample(d)["log_weight"]), rel=1e-15)


def test_weighted_estimates_match_reference(B, orc):
    d = W.rare_event(100_000, integrator="euler")
    out = B.rollout(d)                                  # weights drawn in-kernel
    st = B.reduce(out, grid=GRID)
    got = to_np(out)
    ref, wr = weighted_ref(orc, d)
    assert st["weighted"] == 1
    close(st["risk_pw"], wr["p"], rel=1e-11)
    close(st["risk_se"], wr["se"], rel=1e-8, abs_=1e-20)
    assert abs(st["weight_mean"] - np.exp(orc.sample(d)["log_weight"]).mean()) < 1e-12
    # the same estimator over the GPU's own outputs, in plain FP64 sums
    own = orc.weighted_risk(got, got["weight"], GRID)
    close(st["risk_pw"], own["p"], rel=1e-12)


def test_weighted_collision_probability(B, orc):
    d = dict(W.single(50_000), proposal={"gap": ("normal", 57.0, 2.0),
                                         "mass": ("normal", 1550.0, 75.0)})
    out = B.rollout(d)
    st = B.reduce(out, grid=(30.0, 110.0, 2))
    _, wr = weighted_ref(orc, d)
    assert abs(st["p_collision_w"] - wr["p_collision"]) <= 1e-12 * wr["p_collision"]
    assert abs(st["p_collision_se"] - wr["p_collision_se"]) <= 1e-8 * wr["p_collision_se"]


def test_unit_weights_give_the_counts(B):
    """Weights of 1 (no proposal, weights written): the weighted risk curve is
    the count-based one, bit for bit."""
    d = W.single(40_000)
    out = B.rollout(d, out=B.alloc_outputs(40_000, weight=True))
    assert bool((out["weight"] == 1.0).all())
    st = B.reduce(out, grid=(30.0, 110.0, 161))
    assert np.array_equal(st["risk_pw"], st["risk_p"])
    assert st["p_collision_w"] == st["p_collision"]


def test_deterministic_and_graph(B):
    d = W.rare_event(60_000)
    out = B.rollout(d)
    a = B.reduce(out, grid=GRID)
    for _ in range(3):
        b = B.reduce(B.rollout(d), grid=GRID)
        for k in ("risk_pw", "risk_se"):
            assert np.array_equal(a[k], b[k]), k
        assert a["p_collision_w"] == b["p_collision_w"] and a["weight_mean"] == b["weight_mean"]
    g = B.Graph(d, grid=GRID)
    for _ in range(3):
        g.launch()
        st = g.finish()
        assert np.array_equal(st["risk_pw"], a["risk_pw"])
    g.close()


def test_exact_rare_tail(B, orc):
    """Only v0 ~ N(30, 2) random (Euler, no obstacle): P(D > H0) is
    1 - Phi((v* - 30)/2) with D(v*) = H0; at P ~ 1e-6 the weighted estimate
    over 1,048,576 samples is within 4 standard errors of it."""
    def one(n, **over):
        d = W.paper_preset(n, integrator="euler")
        d.update({"mu": ("const", 0.8), "mass": ("const", 1500.0), "grade": ("const", 0.0),
                  "cda": ("const", 0.66)})
        d.update(over)
        return d
    target = 30.0 + 2.0 * 4.75
    H0 = orc.run(one(1, v0=("const", target)))["dist"][0]
    lo, hi = 30.0, 50.0
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if orc.run(one(1, v0=("const", mid)))["dist"][0] <= H0 else (lo, mid)
    exact = S.norm.sf((hi - 30.0) / 2.0)
    d = one(1_048_576, proposal={"v0": ("normal", target, 2.0)})
    st = B.reduce(B.rollout(d), grid=(H0 - 1.0, H0, 2))
    p, se = st["risk_pw"][1], st["risk_se"][1]
    assert se < 0.01 * p
    assert abs(p - exact) < 4 * se


def test_bad_weight_flagged(B):
    import torch
    d = W.rare_event(5000)
    out = B.rollout(d)
    out["weight"][17] = float("nan")
    torch.cuda.synchronize()
    st = B.reduce(out, grid=GRID)
    assert st["weighted"] == -1 and math.isnan(st["p_collision_w"])
    assert np.all(np.isnan(st["risk_pw"]))


def test_refusals(B):
    d = W.rare_event(1000)
    host = B.sample_params(d, device=False)
    missing = upload({k: v for k, v in host.items() if k != "log_weight"})
    with pytest.raises(B.AebError) as e:
        B.rollout(d, params=missing)
    assert e.value.code == B.EINVAL
    with B.Server(64 << 20, max_slots=2, n_streams=1, max_tick_samples=1 << 14) as srv:
        with pytest.raises(B.AebError) as e:
            srv.submit(d)
        assert e.value.code == B.EINVAL
