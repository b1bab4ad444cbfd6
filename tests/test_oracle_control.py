"""Pins for the reference's closed-loop controller (the controller assessment
named in Section VIII): a TTC-threshold controller ticking every ctl_period
on gap and closing speed measured with normal noise, raising a latched stage
(partial braking a_warn, then full braking a_cmd), each command after the
dead time.

Checks from outside the reference's code: thresholds that fire at the first
tick reproduce the open-loop rollout bit for bit; without noise, a constant
speed approach triggers at the tick a closed form predicts, and the run equals
the open-loop run with that much more dead time; two stages lie between the
runs that brake fully at either tick; the trigger probability at the first
tick matches the normal law of the measured TTC (gap noise, speed noise,
both: the two normals of a call are independent); an unchanged closing speed
never triggers; every bad input is rejected.
"""
import math

import numpy as np
import pytest
from scipy import stats as S

from paper_2604_27193_amd import workloads as W

DT = 1e-3


def flat(n=1, **over):
    """Constant speed until braking (no drag, grade or rolling resistance)."""
    d = W.single(n)
    d.update({"dead_time": 0.05, "h_cog": 0.0, "v0": ("const", 20.0),
              "mu": ("const", 0.8), "tau": ("const", 0.15), "grade": ("const", 0.0),
              "crr": ("const", 0.0), "cda": ("const", 0.0), "mass": ("const", 1500.0),
              "gap": ("const", 150.0), "horizon": 20.0})
    d.update(over)
    return d


def ctl(**over):
    c = {"ctl_period": 0.05, "ttc_warn": 0.0, "ttc_brake": 0.0, "a_warn": -3.0,
         "noise_gap": 0.0, "noise_v": 0.0}
    c.update(over)
    return c


def same(a, b):
    for k in a:
        assert np.array_equal(a[k], b[k]), k


@pytest.mark.parametrize("base", ["single", "rk4", "impact_exit"])
def test_fires_at_first_tick_equals_open_loop(orc, base):
    """(A lead starting at the ego's speed has no closing speed at the first
    tick, so it is left to the tests below.)"""
    d = {"single": W.single(2000), "rk4": W.single(1000, integrator="rk4"),
         "impact_exit": W.single(2000, impact_exit=True)}[base]
    closed = dict(d, **ctl(ttc_brake=math.inf, noise_gap=0.7, noise_v=0.4))
    same(orc.run(d), orc.run(closed))


@pytest.mark.parametrize("integrator", ["euler", "rk4"])
@pytest.mark.parametrize("tb,period", [(2.01, 0.05), (3.33, 0.02), (1.03, 0.1)])
def test_noise_free_trigger_tick(orc, integrator, tb, period):
    """v0 = 20 m/s toward a gap of 150 m: TTC at tick m is 7.5 - m P; the first
    tick below tb is m* = floor((7.5 - tb) / P) + 1, and braking then starts
    m* S + nd steps in: the open-loop run with that dead time."""
    d = flat(integrator=integrator)
    m_star = math.floor((7.5 - tb) / period) + 1
    assert abs((7.5 - tb) / period - round((7.5 - tb) / period)) > 0.05  # no tie at a tick
    per = round(period / DT)
    nd = round(0.05 / DT)
    closed = dict(d, **ctl(ctl_period=period, ttc_brake=tb))
    open_ = dict(d, dead_time=(m_star * per + nd) * DT)
    same(orc.run(open_), orc.run(closed))


def test_two_stages_between_single_stage_runs(orc):
    """Partial braking from the warning tick, full from the brake tick: the
    stopping distance lies between full braking from either tick."""
    d = flat(4)
    two = orc.run(dict(d, **ctl(ttc_warn=3.0, ttc_brake=2.0)))
    early = orc.run(dict(d, **ctl(ttc_brake=3.0)))
    late = orc.run(dict(d, **ctl(ttc_brake=2.0)))
    assert np.all(early["dist"] < two["dist"]) and np.all(two["dist"] < late["dist"])
    # a warning stage with a_warn = a_cmd is full braking from the warning tick
    same(early, orc.run(dict(d, **ctl(ttc_warn=3.0, ttc_brake=2.0, a_warn=d["a_cmd"]))))
    # a warning that brakes with zero deceleration changes nothing
    same(late, orc.run(dict(d, **ctl(ttc_warn=3.0, ttc_brake=2.0, a_warn=0.0))))


@pytest.mark.parametrize("sg,sv", [(2.0, 0.0), (0.0, 0.4), (1.5, 0.3)])
def test_first_tick_trigger_law(orc, sg, sv):
    """At tick 0 the measured TTC is (G + sg z1) / (v0 + sv z2); with tb chosen
    so that the measured gap and speed sit near the threshold the probability
    of braking at once is P(G + sg z1 < tb (v0 + sv z2)), a normal law."""
    n = 60_000
    G, v0, tb = 150.0, 20.0, 7.45
    d = flat(n, **ctl(ttc_brake=tb, noise_gap=sg, noise_v=sv))
    r = orc.run(d, threads=8)
    at_once = orc.run(flat(1, dead_time=0.05))            # braking from step nd
    fired = r["dist"] == at_once["dist"][0]
    p = S.norm.cdf((tb * v0 - G) / math.sqrt(sg ** 2 + (tb * sv) ** 2))
    assert 0.2 < p < 0.8
    assert abs(fired.mean() - p) < 5 * math.sqrt(p * (1 - p) / n)


def test_no_closing_speed_never_triggers(orc):
    """A lead at the ego's speed that never brakes: the closing speed starts at
    zero and only drag (on the ego) changes it, so TTC stays infinite or grows
    and no stage is ever raised: the open-loop run without a command."""
    d = W.sweep(n=200)[40]
    d.update({"lead_decel": ("const", 0.0), "horizon": 5.0})
    closed = dict(d, **ctl(ttc_warn=3.0, ttc_brake=2.0))
    same(orc.run(dict(d, dead_time=10.0)), orc.run(closed))


def test_closed_loop_workload(orc):
    d = W.closed_loop(4000)
    assert orc.validate(d) == orc.OK
    r = orc.run(d, threads=8)
    col = (r["status"] & orc.COLLIDED) != 0
    assert 0.1 < col.mean() < 0.9
    # braking later (lower thresholds) never helps
    r2 = orc.run(dict(d, ttc_warn=2.5, ttc_brake=1.5), threads=8)
    assert ((r2["status"] & orc.COLLIDED) != 0).mean() > col.mean()


BAD = [{"ctl_period": -0.05}, {"ctl_period": float("inf")}, {"ctl_period": 1e-5},
       {"obstacle": "none"}, {"latency": ("const", 0.1)}, {"ttc_warn": -1.0},
       {"ttc_brake": float("nan")}, {"a_warn": -7.0}, {"a_warn": 0.5},
       {"noise_gap": -0.1}, {"noise_v": float("inf")}, {"ctl_period": 1e-3, "horizon": 1e5}]


@pytest.mark.parametrize("change", BAD)
def test_rejects_bad_controller(orc, change):
    d = W.closed_loop(10)
    d.update(change)
    assert orc.validate(d) == orc.EINVAL
