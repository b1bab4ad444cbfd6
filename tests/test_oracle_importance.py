"""Pins for the reference's importance sampling (rare-event estimation, named
in Section VIII): normal parameters drawn from normal proposals, each sample
weighted by its likelihood ratio p/q, and the weighted collision-risk
estimator with its standard error.

From outside the reference's code: the log weight against scipy's normal
log densities; E_q[w] = 1 and E_q[w x] = the nominal mean; a one-parameter
case with an exact answer (only v0 random, the stopping distance monotone
in v0, so P(D > H0) = P(v0 > v*) with D(v*) = H0 found by bisection) that the
weighted estimate matches at P ~ 1e-6 where plain sampling sees nothing; and
agreement with plain sampling at a moderate level on the full preset.
"""
import math

import numpy as np
import pytest
from scipy import stats as S

from paper_2604_27193_amd import workloads as W


def test_no_proposal_means_unit_weights(orc):
    d = W.paper_preset(2000)
    a = orc.sample(d)
    assert np.all(a["log_weight"] == 0.0)
    same = dict(d, proposal={"v0": d["v0"], "mu": d["mu"]})   # proposal = nominal
    b = orc.sample(same)
    for c in a:
        assert np.array_equal(a[c], b[c]), c


def test_log_weight_is_density_ratio(orc):
    d = W.rare_event(5000)
    cols = orc.sample(d)
    want = (S.norm.logpdf(cols["v0"], 30.0, 2.0) - S.norm.logpdf(cols["v0"], 36.0, 2.0)
            + S.norm.logpdf(cols["mu"], 0.8, 0.1) - S.norm.logpdf(cols["mu"], 0.55, 0.1))
    assert np.max(np.abs(cols["log_weight"] - want)) < 1e-10
    # the draws follow the proposals
    assert S.kstest(cols["v0"], S.norm(36.0, 2.0).cdf).pvalue > 1e-4
    assert S.kstest(cols["mu"], S.norm(0.55, 0.1).cdf).pvalue > 1e-4


def test_weight_moments(orc):
    n = 200_000
    d = dict(W.paper_preset(n), proposal={"v0": ("normal", 32.0, 2.5),
                                          "mu": ("normal", 0.7, 0.12)})
    cols = orc.sample(d)
    w = np.exp(cols["log_weight"])
    se = w.std() / math.sqrt(n)
    assert abs(w.mean() - 1.0) < 5 * se
    wx = w * cols["v0"]
    assert abs(wx.mean() - 30.0) < 5 * wx.std() / math.sqrt(n)


def one_param(n, **over):
    d = W.paper_preset(n, integrator="euler")
    d.update({"mu": ("const", 0.8), "mass": ("const", 1500.0), "grade": ("const", 0.0),
              "cda": ("const", 0.66)})
    d.update(over)
    return d


def stop_distance(orc, v0):
    return orc.run(one_param(1, v0=("const", float(v0))))["dist"][0]


def test_rare_tail_exact(orc):
    """Only v0 ~ N(30, 2) random: P(D > H0) = 1 - Phi((v* - 30) / 2)."""
    target = 30.0 + 2.0 * 4.75                         # P ~ 1e-6
    H0 = stop_distance(orc, target)
    lo, hi = 30.0, 50.0
    for _ in range(60):                                # D increases with v0
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if stop_distance(orc, mid) <= H0 else (lo, mid)
    exact = S.norm.sf((hi - 30.0) / 2.0)
    assert 5e-7 < exact < 2e-6
    n = 40_000
    d = one_param(n, proposal={"v0": ("normal", target, 2.0)})
    out = orc.run(d)
    w = np.exp(orc.sample(d)["log_weight"])
    est = orc.weighted_risk(out, w, (H0 - 1.0, H0, 2))
    p, se = est["p"][1], est["se"][1]
    assert se < 0.03 * p
    assert abs(p - exact) < 4 * se
    # plain sampling at the same N sees (almost surely) no such stop
    plain = orc.run(one_param(n))
    assert np.sum(plain["dist"] > H0) <= 1


def test_agrees_with_plain_sampling(orc):
    """Full Sec. IV-B preset at a level near 1e-2: the weighted estimate and
    plain sampling agree within their combined standard errors."""
    n = 60_000
    plain = orc.run(W.paper_preset(n, integrator="euler"), threads=8)
    H0 = float(np.quantile(plain["dist"], 0.99))
    p_plain = np.mean(plain["dist"] > H0)
    se_plain = math.sqrt(p_plain * (1 - p_plain) / n)
    d = W.rare_event(n, integrator="euler", v0_shift=3.0, mu_shift=-0.1)
    out = orc.run(d, threads=8)
    w = np.exp(orc.sample(d)["log_weight"])
    est = orc.weighted_risk(out, w, (H0 - 1.0, H0, 2))
    assert abs(est["p"][1] - p_plain) < 5 * math.hypot(est["se"][1], se_plain)
    assert est["se"][1] < se_plain          # the proposal concentrates on the tail


BAD = [{"proposal": {"tau": ("normal", 0.2, 0.01)}},
       {"proposal": {"v0": ("uniform", 20.0, 40.0)}},
       {"proposal": {"v0": ("normal", 36.0, 0.0)}},
       {"proposal": {"v0": ("normal", float("nan"), 2.0)}},
       {"v0": ("trunc_normal", 30.0, 2.0, 20.0, 40.0), "proposal": {"v0": ("normal", 36.0, 2.0)}},
       {"v0": ("normal", 30.0, 0.0), "proposal": {"v0": ("normal", 36.0, 2.0)}}]


@pytest.mark.parametrize("change", BAD)
def test_rejects_bad_proposals(orc, change):
    d = W.paper_preset(10)
    d.update(change)
    assert orc.validate(d) == orc.EINVAL


def test_accepts_rare_event_workload(orc):
    assert orc.validate(W.rare_event(10)) == orc.OK
