"""Randomised parity on the GPU: scenarios drawn from a seeded generator over
the options the library supports together -- integrator, obstacle, impact
exit, the unfused form, step, horizon, dead time, command, distribution
means and spreads, the perception trigger, the closed-loop controller and
importance-sampling proposals -- a few hundred samples each.  FP64 with
host-drawn parameters equals the reference bit for bit; in-kernel draws agree
within 1e-12; the FP32 compensated form stays within its error budget where
it applies (explicit Euler without the controller)."""
import numpy as np
import pytest

from paper_2604_27193_amd import workloads as W
from test_gpu_parity import check_fp32c, check_fp64, plain, to_np

pytestmark = pytest.mark.gpu

N_SCENARIOS = 64


@pytest.fixture(scope="module")
def B():
    import torch
    assert torch.cuda.is_available()
    from paper_2604_27193_amd import binding
    binding.lib()
    return binding


def scenario(j):
    """Scenario j of the seeded family (numpy PCG64, seed 4242 + j)."""
    g = np.random.default_rng(4242 + j)
    d = W.single(int(g.integers(200, 500)), seed=int(g.integers(1, 10_000)), scenario_id=j)
    integ = "rk4" if g.random() < 0.25 else "euler"
    obstacle = str(g.choice(["none", "stationary", "lead"] if integ == "euler"
                            else ["none", "stationary"]))
    v0 = float(g.uniform(12.0, 35.0))
    mu_lo = float(g.uniform(0.2, 0.6))
    d.update({
        "integrator": integ, "obstacle": obstacle,
        "impact_exit": bool(g.random() < 0.3),
        "nofma": bool(integ == "euler" and g.random() < 0.15),
        "dt": float(g.choice([5e-4, 1e-3, 2e-3])),
        "horizon": float(g.uniform(3.0, 15.0)),
        "dead_time": float(g.uniform(0.0, 0.1)),
        "a_cmd": float(g.uniform(-8.0, -4.0)),
        "v0": ("trunc_normal", v0, float(g.uniform(0.5, 2.5)), v0 - 5.0, v0 + 5.0),
        "mu": ("uniform", mu_lo, mu_lo + float(g.uniform(0.1, 0.5))),
        "gap": ("normal", float(g.uniform(30.0, 90.0)), float(g.uniform(1.0, 5.0))),
    })
    if obstacle == "lead":
        d["lead_decel"] = ("normal", float(g.uniform(1.0, 5.0)), 0.5)
    extra = g.random()
    if extra < 0.2:
        # perception trigger
        d.update({"latency": ("trunc_normal", 0.08, 0.02, 0.03, 0.12),
                  "occlusion": ("uniform", 0.0, float(g.uniform(0.0, 6.0))),
                  "frame_period": float(g.choice([0.02, 0.05, 0.1])),
                  "p_dropout": float(g.uniform(0.0, 0.3)), "confirm": int(g.integers(1, 4))})
    elif extra < 0.4 and obstacle != "none":
        # closed-loop controller
        d.update({"ctl_period": float(g.choice([0.02, 0.03, 0.04, 0.05, 0.1])),
                  "ttc_warn": float(g.uniform(2.5, 4.0)), "ttc_brake": float(g.uniform(1.2, 2.4)),
                  "a_warn": float(g.uniform(-3.5, -1.0)), "noise_gap": float(g.uniform(0.0, 1.0)),
                  "noise_v": float(g.uniform(0.0, 0.5))})
        d["horizon"] = float(g.uniform(8.0, 15.0))
        d["gap"] = ("normal", float(g.uniform(60.0, 140.0)), 5.0)
    elif extra < 0.5:
        # importance sampling on the mass and the drag area (normal parameters)
        d["proposal"] = {"mass": ("normal", 1500.0 + float(g.uniform(-100, 100)), 90.0),
                         "cda": ("normal", 0.7 + float(g.uniform(-0.05, 0.05)), 0.06)}
    return d


def kinds(d):
    tags = [d["integrator"], d["obstacle"]]
    for key, tag in (("ctl_period", "controller"), ("frame_period", "perception"),
                     ("proposal", "importance")):
        if key in d:
            tags.append(tag)
    return "-".join(tags)


@pytest.mark.parametrize("j", range(N_SCENARIOS))
def test_random_scenario_fp64(B, orc, j):
    d = scenario(j)
    assert B.validate(d) == 0, kinds(d)
    ref = orc.run(d)
    check_fp64(to_np(plain(B, d)), ref, exact=True)
    check_fp64(to_np(B.rollout(d)), ref)


def fp32c_applies(d):
    """The FP32 compensated form covers explicit Euler without the controller."""
    return d["integrator"] == "euler" and "ctl_period" not in d


@pytest.mark.parametrize("j", [j for j in range(N_SCENARIOS) if fp32c_applies(scenario(j))])
def test_random_scenario_fp32c(B, orc, j):
    d = scenario(j)
    margin_abs = 2e-3 if d["obstacle"] == "lead" else None
    check_fp32c(to_np(B.rollout(d, precision="fp32c")), orc.run(d), margin_abs=margin_abs)


def test_family_covers_every_option():
    """The generator's scenarios include each integrator, obstacle and
    extension at least once (so the parity above spans them)."""
    seen = set()
    for j in range(N_SCENARIOS):
        d = scenario(j)
        seen.update(kinds(d).split("-"))
        if d["impact_exit"]:
            seen.add("impact_exit")
        if d["nofma"]:
            seen.add("nofma")
    for tag in ("euler", "rk4", "none", "stationary", "lead", "controller", "perception",
                "importance", "impact_exit", "nofma"):
        assert tag in seen, tag
