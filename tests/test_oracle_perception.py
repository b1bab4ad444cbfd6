"""Pins for the reference's perception model: a stochastic brake-trigger delay.

Perception effects (latency, dropout, occlusion) are the extension that
Section VIII names.  The reading built here: sensing runs in frames of period
P; the obstacle is hidden for the first floor(occlusion) frames; each later
frame detects it independently with probability 1 - p_dropout; braking is
requested at the end of the first run of ``confirm`` consecutive detections
plus a processing latency, and that request adds to the actuator dead time.
A trigger beyond the horizon means no braking at all.

Every check here comes from outside the reference's code: closed forms for
deterministic settings, the geometric law and an independently computed
Markov-chain law of the confirmation frame (chi-square), the exact coasting
shift of a drag-free run, and validation of every bad input.
"""
import math

import numpy as np
import pytest
from scipy import stats as S

from paper_2604_27193_amd import workloads as W


def flat(n=1, **over):
    """No drag, grade or rolling resistance: a coasting car keeps its speed."""
    d = W.single(n)
    d.update({"obstacle": "none", "dead_time": 0.0, "h_cog": 0.0, "v0": ("const", 25.3),
              "mu": ("const", 0.8), "tau": ("const", 0.15), "grade": ("const", 0.0),
              "crr": ("const", 0.0), "cda": ("const", 0.0), "mass": ("const", 1500.0),
              "gap": ("const", 1000.0), "horizon": 30.0})
    d.update(over)
    return d


def test_defaults_mean_no_perception(orc):
    d = W.single(3000)
    cols = orc.sample(d)
    assert np.all(cols["trigger"] == 0.0)
    explicit = dict(d, latency=("const", 0.0), occlusion=("const", 3.0), frame_period=0.0,
                    p_dropout=0.5, confirm=4)       # frames off: only latency counts
    a, b = orc.run(d), orc.run(explicit)
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_latency_only(orc):
    d = W.single(20000, latency=("uniform", 0.02, 0.18))
    t = orc.sample(d)["trigger"]
    assert t.min() >= 0.02 and t.max() <= 0.18
    assert abs(t.mean() - 0.10) < 5 * 0.16 / math.sqrt(12 * len(t))
    # a normal latency is clipped at zero: the clipped mass is Phi(-mean / sd)
    d = W.single(40000, latency=("normal", 0.01, 0.02))
    t = orc.sample(d)["trigger"]
    assert t.min() == 0.0
    p0 = S.norm.cdf(-0.5)
    assert abs(np.mean(t == 0.0) - p0) < 5 * math.sqrt(p0 * (1 - p0) / len(t))


@pytest.mark.parametrize("occ,confirm,want_frames", [(0.0, 1, 0), (2.7, 1, 2), (2.0, 3, 4),
                                                     (-1.5, 2, 1), (5.99, 5, 9)])
def test_no_dropout_closed_form(orc, occ, confirm, want_frames):
    """p_dropout = 0: detection at frame floor(occ) and confirmation confirm - 1
    frames later, so the trigger is (floor(occ)^+ + confirm - 1) P + latency."""
    P, lat = 0.04, 0.031
    d = W.single(64, latency=("const", lat), occlusion=("const", occ), frame_period=P,
                 p_dropout=0.0, confirm=confirm)
    t = orc.sample(d)["trigger"]
    assert np.all(np.abs(t - (want_frames * P + lat)) <= 1e-15)


def frames_of(t, P, lat):
    j = np.round((t - lat) / P)
    assert np.all(np.abs(j * P + lat - t) <= 1e-12)
    return j.astype(np.int64)


def confirmation_law(p, M, jmax):
    """P(J = j) for j < jmax, J the frame index that completes the first run of
    M detections, each frame detecting with probability 1 - p independently:
    forward recursion over the current run length."""
    q = 1.0 - p
    state = np.zeros(M)
    state[0] = 1.0
    law = np.zeros(jmax)
    for j in range(jmax):
        nxt = np.zeros(M)
        nxt[0] = p * state.sum()          # a miss resets the run
        law[j] = q * state[M - 1]         # a hit on a run of M-1 completes it
        nxt[1:] = q * state[:M - 1]
        state = nxt
    return law


def chi2_pvalue(counts, probs, n):
    exp = n * probs
    keep = exp >= 20
    obs, e = counts[keep], exp[keep]
    rest = n - e.sum()
    if rest > 1e-6 * n:                   # the pooled tail, when it has mass
        obs, e = np.append(obs, n - obs.sum()), np.append(e, rest)
    else:
        assert obs.sum() == n
    stat = ((obs - e) ** 2 / e).sum()
    return S.chi2.sf(stat, len(obs) - 1)


def test_confirmation_law_sanity():
    """The recursion against two closed forms: the geometric law for M = 1 and
    the mean (1 - q^M) / (p q^M) trials for M consecutive successes."""
    law = confirmation_law(0.3, 1, 60)
    assert np.allclose(law, 0.7 * 0.3 ** np.arange(60), atol=0, rtol=1e-13)
    p, M = 0.25, 3
    law = confirmation_law(p, M, 400)
    q = 1.0 - p
    assert abs(law.sum() - 1.0) < 1e-12
    assert abs((np.arange(400) + 1) @ law - (1 - q ** M) / (p * q ** M)) < 1e-9


@pytest.mark.parametrize("p,M,occ", [(0.3, 1, 0.0), (0.25, 3, 0.0), (0.5, 2, 3.0),
                                     (0.1, 5, 1.0)])
def test_confirmation_frame_law(orc, p, M, occ):
    P, lat, n = 0.05, 0.0, 120_000
    d = W.single(n, latency=("const", lat), occlusion=("const", occ), frame_period=P,
                 p_dropout=p, confirm=M, horizon=60.0)
    j = frames_of(orc.sample(d)["trigger"], P, lat) - int(occ)
    assert j.min() >= M - 1
    law = confirmation_law(p, M, 200)
    counts = np.bincount(j, minlength=200)[:200]
    assert chi2_pvalue(counts, law, n) > 1e-6
    # the first M frames after occlusion all detect with probability q^M
    assert abs(np.mean(j == M - 1) - (1 - p) ** M) < 5 * math.sqrt((1 - p) ** M / n)


def test_consecutive_frames_independent(orc):
    """Adjacent frames share one generator call: a pairing mistake would make
    them equal.  With M = 2, p = 1/2: P(J = 1) = 1/4, P(J = 2) = 1/8."""
    n = 80_000
    d = W.single(n, occlusion=("const", 0.0), frame_period=0.01, p_dropout=0.5, confirm=2)
    j = frames_of(orc.sample(d)["trigger"], 0.01, 0.0)
    for jj, want in ((1, 0.25), (2, 0.125), (3, 0.125)):
        assert abs(np.mean(j == jj) - want) < 5 * math.sqrt(want / n)


def test_occlusion_uniform_frames(orc):
    """Occlusion U(0, 4) hides floor(U) frames, uniform on {0, 1, 2, 3}."""
    n = 40_000
    d = W.single(n, occlusion=("uniform", 0.0, 4.0), frame_period=0.05, p_dropout=0.0,
                 confirm=1)
    j = frames_of(orc.sample(d)["trigger"], 0.05, 0.0)
    counts = np.bincount(j, minlength=4)
    assert len(counts) == 4
    assert chi2_pvalue(counts, np.full(4, 0.25), n) > 1e-6


def test_trigger_shifts_drag_free_stop(orc):
    """With no resistive force the car coasts at v0 until the command: a trigger
    that moves the command by k steps adds exactly k steps and k v0 dt metres."""
    base = flat(1)
    r0 = orc.run(base)
    n = 500
    d = flat(n, latency=("uniform", 0.0, 0.4), dead_time=0.05)
    t = orc.sample(d)["trigger"]
    r = orc.run(d)
    k = np.array([round((0.05 + ti) / 1e-3) for ti in t])
    assert np.array_equal(r["steps"], r0["steps"][0] + k)
    want = r0["dist"][0] + k * 1e-3 * 25.3
    assert np.all(np.abs(r["dist"] - want) <= 1e-9 * want)


def test_trigger_beyond_horizon_coasts(orc):
    """Never confirmed within the horizon: no braking, coasting to the horizon."""
    T = 2.0
    d = flat(8, horizon=T, occlusion=("const", 100.0), frame_period=0.05, confirm=1)
    assert np.all(np.isinf(orc.sample(d)["trigger"]))
    # an occlusion far beyond the frame count hides every frame as well
    huge = flat(4, horizon=T, occlusion=("const", 1e30), frame_period=0.05)
    assert np.all(np.isinf(orc.sample(huge)["trigger"]))
    r = orc.run(d)
    assert np.all(r["status"] & 3 == orc.END_HORIZON)
    assert np.all(r["steps"] == 2000)
    assert np.all(np.abs(r["dist"] - 25.3 * T) <= 1e-9 * 25.3 * T)
    # confirmed at the last frame inside the horizon, the command just fits
    d = flat(1, horizon=T, occlusion=("const", 39.0), frame_period=0.05, confirm=1)
    assert orc.sample(d)["trigger"][0] == pytest.approx(1.95, abs=1e-12)


def test_occlusion_between_last_frames(orc):
    """Only the first floor(occlusion) frames are hidden: an occlusion between
    the last frame index and the frame count leaves the last frame visible."""
    T, P = 10.0, 0.3                      # frames 0..33 (33 P = 9.9 s <= T)
    for occ, want in ((33.0, 33 * P), (33.5, 33 * P), (33.999, 33 * P), (34.0, np.inf),
                      (34.5, np.inf)):
        d = flat(2, horizon=T, occlusion=("const", occ), frame_period=P, confirm=1)
        t = orc.sample(d)["trigger"]
        assert np.all(t == want), (occ, t)
    # the command then starts inside the horizon: the rollout brakes at its end
    d = flat(1, horizon=T, occlusion=("const", 33.5), frame_period=P, confirm=1,
             dead_time=0.05)
    r = orc.run(d)
    assert r["steps"][0] == 10_000 and r["dist"][0] < 25.3 * T - 1e-6


def test_trigger_equals_extra_dead_time(orc):
    """In the full model (drag, grade, weight transfer, obstacle) a trigger T
    acts as dead time: same outputs as no perception with dead_time + T."""
    d = W.perception(200)
    cols = orc.sample(d)
    r = orc.run(d)
    for i in range(0, 200, 7):
        one = {k: v[i:i + 1] for k, v in cols.items()}
        e = dict(W.single(1), dead_time=d["dead_time"] + cols["trigger"][i])
        one_nop = dict(one, trigger=np.zeros(1))
        g = orc.rollout_given(e, one_nop)
        for k in r:
            assert r[k][i] == g[k][0], (i, k)


def test_perception_raises_collisions(orc):
    d0 = W.single(20000)
    d1 = W.perception(20000)
    r0, r1 = orc.run(d0), orc.run(d1)
    assert np.all(r1["dist"] >= r0["dist"])
    c0 = np.mean(r0["status"] & orc.COLLIDED > 0)
    c1 = np.mean(r1["status"] & orc.COLLIDED > 0)
    assert c1 > c0


BAD = [{"p_dropout": 1.0}, {"p_dropout": -0.1}, {"p_dropout": float("nan")},
       {"frame_period": -0.05}, {"frame_period": float("inf")}, {"confirm": 0},
       {"confirm": 65}, {"frame_period": 1e-6, "horizon": 10.0},
       {"latency": ("uniform", 0.2, 0.1)}, {"occlusion": ("normal", 1.0, -1.0)}]


@pytest.mark.parametrize("change", BAD)
def test_rejects_bad_perception(orc, change):
    d = W.perception(10)
    d.update(change)
    assert orc.validate(d) == orc.EINVAL


def test_accepts_perception_workload(orc):
    assert orc.validate(W.perception(10)) == orc.OK
