"""Scenario validation in the reference: every rejected input is rejected."""
import ctypes as C

import pytest

from paper_2604_27193_amd import workloads as W


BAD = [
    {"n_samples": 0}, {"n_samples": -5}, {"n_samples": 2**31},
    {"dt": 0.0}, {"dt": -1e-3}, {"horizon": 0.0}, {"dead_time": -0.01},
    {"horizon": 1e7, "dt": 1e-3},
    {"tau": ("uniform", 0.0005, 0.3)},          # dt/tau > 1 for explicit Euler
    {"tau": ("normal", 0.2, 0.05)},             # unbounded below
    {"integrator": "rk4", "obstacle": "lead"},
    {"mass": ("normal", 1500.0, -1.0)},
    {"v0": ("trunc_normal", 25.0, 1.0, 30.0, 20.0)},
    {"mu": ("uniform", 0.9, 0.4)},
    {"wheelbase": 0.0},
    {"a_cmd": float("nan")},
]


@pytest.mark.parametrize("change", BAD)
def test_rejects(orc, change):
    d = W.single(100)
    d.update(change)
    assert orc.validate(d) == orc.EINVAL


@pytest.mark.parametrize("d", [W.single(10_000), W.single(1_048_576), W.paper_preset(),
                               W.sweep(n=1000)[0], W.uneven_batch(20)[3],
                               dict(W.single(5), integrator="rk4", tau=("const", 0.15))])
def test_accepts_workloads(orc, d):
    assert orc.validate(d) == orc.OK


def test_rejects_unknown_enums(orc):
    s = orc.scenario(W.single(100))
    s.integrator = 7
    assert orc.lib().orc_validate(C.byref(s)) == orc.EINVAL
    s = orc.scenario(W.single(100))
    s.mu.kind = 9
    assert orc.lib().orc_validate(C.byref(s)) == orc.EINVAL


def test_run_refuses_invalid(orc):
    with pytest.raises(ValueError):
        orc.run(dict(W.single(10), dt=-1.0))
