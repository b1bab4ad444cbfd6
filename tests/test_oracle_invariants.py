"""Invariant pins for the reference: monotonicity of the stopping distance in
each physical parameter, the work-energy lower bound, equivalences between
readings that must agree bit for bit, and determinism of the sample stream."""
import numpy as np
import pytest

from paper_2604_27193_amd import workloads as W

N = 3000


@pytest.fixture(scope="module")
def base(orc):
    d = W.single(N)
    cols = orc.sample(d)
    out = orc.rollout_given(d, cols)
    return d, cols, out


def _perturbed(orc, d, cols, **changes):
    c2 = {k: v.copy() for k, v in cols.items()}
    for k, f in changes.items():
        c2[k] = f(c2[k])
    if "grade" in changes:
        c2["sin_grade"] = np.sin(c2["grade"])
        c2["cos_grade"] = np.cos(c2["grade"])
    return orc.rollout_given(d, c2)


@pytest.mark.parametrize("param,scale,direction", [
    ("mu", 1.05, -1), ("cda", 1.2, -1), ("crr", 1.3, -1), ("v0", 1.02, +1),
    ("tau", 1.1, +1), ("mass", 1.1, +1)])
def test_monotone_in_parameter(orc, base, param, scale, direction):
    d, cols, out = base
    new = _perturbed(orc, d, cols, **{param: lambda a: a * scale})
    diff = (new["dist"] - out["dist"]) * direction
    assert np.all(diff >= -1e-9), param
    assert np.mean(diff > 1e-6) > 0.5  # the parameter matters for most samples


def test_monotone_in_grade(orc, base):
    d, cols, out = base
    new = _perturbed(orc, d, cols, grade=lambda a: a + 0.01)
    assert np.all(new["dist"] <= out["dist"] + 1e-9)


def test_monotone_in_dead_time(orc, base):
    d, cols, out = base
    d2 = dict(d, dead_time=0.08)
    new = orc.rollout_given(d2, cols)
    assert np.all(new["dist"] >= out["dist"] - 1e-9)


def test_collision_monotone_in_gap(orc, base):
    d, cols, out = base
    col = out["status"] & orc.COLLIDED
    new = _perturbed(orc, d, cols, gap=lambda a: a + 3.0)
    col2 = new["status"] & orc.COLLIDED
    assert np.all(col2 <= col)
    assert np.array_equal(new["dist"], out["dist"])  # a stationary obstacle never changes D


def test_work_energy_lower_bound(orc, base):
    """With c >= 0 the speed never exceeds v0, so the deceleration is at most
    min(|a_cmd|, |alim|) + kd v0^2 + c and D >= v0^2 / (2 * that)."""
    d, cols, out = base
    g = d["g"]
    kd = 0.5 * d["rho"] * cols["cda"] / cols["mass"]
    c = g * cols["sin_grade"] + cols["crr"] * g * cols["cos_grade"]
    alim = cols["mu"] * g / (1.0 + cols["mu"] * d["h_cog"] / d["wheelbase"])
    dec = np.minimum(abs(d["a_cmd"]), alim) + kd * cols["v0"] ** 2 + c
    bound = cols["v0"] ** 2 / (2.0 * dec)
    sel = c >= 0
    assert sel.sum() > N // 4
    assert np.all(out["dist"][sel] >= bound[sel])


def test_state_clamp_equals_output_clamp(orc, base):
    """Saturating the realised brake or clamping the actuator state itself gives
    bit-identical Euler results for a step command with dt/tau <= 1."""
    d, cols, out = base
    alt = orc.rollout_given(d, cols, clamp_state=True)
    for k in out:
        assert np.array_equal(out[k], alt[k]), k


def test_stationary_flag_is_distance_beyond_gap(orc, base):
    d, cols, out = base
    col = (out["status"] & orc.COLLIDED) != 0
    assert np.array_equal(col, out["dist"] > cols["gap"])
    assert np.all(out["status"] & 3 == orc.END_STOP)
    assert np.array_equal(out["margin"], cols["gap"] - out["dist"])
    assert np.all(out["v_impact"][~col] == 0.0)
    assert np.all(out["v_impact"][col] > 0.0)
    assert 0.3 < col.mean() < 0.8


def test_impact_exit_agrees_with_run_to_stop(orc, base):
    d, cols, out = base
    ex = orc.rollout_given(dict(d, impact_exit=True), cols)
    col = (out["status"] & orc.COLLIDED) != 0
    assert np.array_equal((ex["status"] & orc.COLLIDED) != 0, col)
    assert np.array_equal(ex["v_impact"], out["v_impact"])
    for k in out:
        assert np.array_equal(ex[k][~col], out[k][~col]), k
    assert np.all(ex["status"][col] == orc.END_IMPACT | orc.COLLIDED)
    assert np.all(ex["steps"][col] <= out["steps"][col])
    assert np.all(ex["dist"][col] > cols["gap"][col])
    assert np.all(ex["margin"][col] < 0)


def test_fused_and_unfused_differ_only_by_rounding(orc, base):
    d, cols, out = base
    nf = orc.rollout_given(dict(d, nofma=True), cols)
    rel = np.abs(nf["dist"] - out["dist"]) / out["dist"]
    assert rel.max() < 1e-11
    assert np.mean(nf["dist"] != out["dist"]) > 0.5  # it is a different rounding


def test_euler_and_rk4_agree_to_first_order(orc):
    d = W.paper_preset(400)
    rk = orc.run(d)
    eu = orc.run(dict(d, integrator="euler"))
    diff = eu["dist"] - rk["dist"]
    assert np.all(np.abs(diff) <= d["dt"] * 40.0)
    assert np.all(diff > 0)  # explicit Euler's left sums overshoot


def test_euler_converges_first_order_in_dt(orc):
    d = W.single(200)
    fine = orc.run(dict(d, integrator="rk4", dt=2.5e-4))["dist"]
    e1 = orc.run(d)["dist"] - fine
    e2 = orc.run(dict(d, dt=5e-4))["dist"] - fine
    ratio = np.median(e1 / e2)
    assert abs(ratio - 2.0) < 0.1


def test_lead_mode_outputs_are_consistent(orc):
    d = W.sweep(n=400)[5 * 16 + 3]
    out = orc.run(d)
    end = out["status"] & 3
    col = (out["status"] & orc.COLLIDED) != 0
    assert np.array_equal(end == orc.END_IMPACT, col)  # a lead vehicle always ends the run
    assert np.all(out["margin"][col] < 0) and np.all(out["margin"][~col] >= 0)
    assert np.all(out["v_impact"][col] > 0)
    assert set(np.unique(end)) <= {orc.END_STOP, orc.END_IMPACT, orc.END_HORIZON}


def test_sub_ranges_and_threads_are_deterministic(orc):
    d = W.single(2000)
    a = orc.run(d)
    b = orc.run(d, threads=4)
    c = orc.run(d, first=777, count=300)
    for k in a:
        assert np.array_equal(a[k], b[k])
        assert np.array_equal(a[k][777:1077], c[k])
