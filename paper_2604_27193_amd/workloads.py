"""Seeded synthetic workloads: scenario descriptors and request streams.

This module only builds inputs.  It holds none of the model's arithmetic: a
scenario is a plain dict naming the integrator, the obstacle, the physical
constants and, for each uncertain parameter, its distribution as a tuple
``("const", x)``, ``("uniform", a, b)``, ``("normal", mean, sd)`` or
``("trunc_normal", mean, sd, lo, hi)``.  Per-sample values are never drawn
here; the counter-based generator on either side of a comparison does that
from (seed, scenario_id, sample index).  Scenario-level randomness (random
means of an uneven batch, arrival times of a request stream) comes from
numpy's PCG64 with the stated seed.

Workloads:
  * ``paper_preset`` -- Section IV-B: v0~N(30,2^2), mu~N(0.8,0.1^2),
    theta~N(0,0.05^2), m~N(1500,100^2), Cd~N(0.3,0.05^2) (frontal area 2.2 m^2),
    tau = 0.15 s, h = 0.5 m, L = 2.7 m, a_cmd = -6, RK4, dt = 1 ms, T = 10 s.
  * ``single`` -- one stationary-obstacle scenario with dead time, rolling
    resistance, truncated v0 and uniform mu/tau/Crr (10,000 or 1,048,576
    samples, explicit Euler, dt = 1 ms, T = 10 s).
  * ``sweep`` -- 16 v0 means x 16 mu means with a decelerating lead vehicle.
  * ``uneven_batch`` -- 1,000 scenarios with log-uniform sample counts, random
    horizons and steps, scenario means drawn from seed 7.
  * ``serving_stream`` -- Poisson arrivals of randomized single scenarios.
  * ``perception`` -- ``single`` with a stochastic brake trigger from frame
    sensing: occlusion, per-frame dropout, a confirmation run and latency.
  * ``closed_loop`` -- ``single`` with the obstacle farther ahead and a
    two-stage TTC-threshold controller on noisy measurements.
  * ``rare_event`` -- ``paper_preset`` with importance-sampling proposals for
    v0 and mu shifted toward long stopping distances.
"""
import numpy as np

G = 9.81
RHO = 1.225
FRONTAL_AREA = 2.2


def _base(seed, scenario_id, n):
    return {
        "seed": int(seed), "scenario_id": int(scenario_id), "n_samples": int(n),
        "integrator": "euler", "obstacle": "stationary", "impact_exit": False, "nofma": False,
        "dt": 1e-3, "horizon": 10.0, "dead_time": 0.05, "a_cmd": -6.0, "g": G, "rho": RHO,
        "h_cog": 0.55, "wheelbase": 2.7,
        "v0": ("trunc_normal", 25.0, 1.0, 20.0, 30.0),
        "mu": ("uniform", 0.4, 0.9),
        "mass": ("normal", 1500.0, 75.0),
        "grade": ("normal", 0.0, 0.02),
        "cda": ("normal", 0.7, 0.05),
        "crr": ("uniform", 0.01, 0.015),
        "tau": ("uniform", 0.1, 0.3),
        "gap": ("normal", 60.0, 2.0),
        "lead_decel": ("const", 0.0),
    }


def single(n=10_000, seed=42, scenario_id=0, **over):
    """Stationary obstacle, run to stop with the collision flag latched."""
    d = _base(seed, scenario_id, n)
    d.update(over)
    return d


def paper_preset(n=12_000, seed=2026, scenario_id=0, integrator="rk4", **over):
    """The uncertainty model and nominal parameters of Section IV-B."""
    d = _base(seed, scenario_id, n)
    d.update({
        "integrator": integrator, "obstacle": "none", "dead_time": 0.0, "h_cog": 0.5,
        "v0": ("normal", 30.0, 2.0),
        "mu": ("normal", 0.8, 0.1),
        "mass": ("normal", 1500.0, 100.0),
        "grade": ("normal", 0.0, 0.05),
        "cda": ("normal", 0.3 * FRONTAL_AREA, 0.05 * FRONTAL_AREA),
        "crr": ("const", 0.0),
        "tau": ("const", 0.15),
        "gap": ("const", 0.0),
    })
    d.update(over)
    return d


def sweep(n=100_000, seed=42, v0_means=None, mu_means=None):
    """16 x 16 grid of (v0 mean, mu mean) with a lead vehicle braking at N(3, 0.5)."""
    v0_means = np.linspace(10.0, 40.0, 16) if v0_means is None else v0_means
    mu_means = np.linspace(0.2, 1.0, 16) if mu_means is None else mu_means
    out = []
    for iv, vm in enumerate(v0_means):
        for im, mm in enumerate(mu_means):
            d = _base(seed, len(mu_means) * iv + im, n)
            d.update({
                "obstacle": "lead",
                "v0": ("trunc_normal", float(vm), 1.0, float(vm) - 5.0, float(vm) + 5.0),
                "mu": ("trunc_normal", float(mm), 0.05, 0.05, 1.5),
                "gap": ("normal", 40.0, 3.0),
                "lead_decel": ("normal", 3.0, 0.5),
            })
            out.append(d)
    return out


def _randomized(rng, seed, scenario_id, n):
    d = _base(seed, scenario_id, n)
    vm = float(rng.uniform(20.0, 30.0))
    mc = float(rng.uniform(0.5, 0.8))
    gm = float(rng.uniform(50.0, 70.0))
    d.update({
        "v0": ("trunc_normal", vm, 1.0, vm - 5.0, vm + 5.0),
        "mu": ("uniform", mc - 0.25, mc + 0.25),
        "gap": ("normal", gm, 2.0),
    })
    return d


def uneven_batch(n_scenarios=1000, seed=7, max_samples=None):
    """Scenario means, sizes, horizons and steps drawn from PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for k in range(n_scenarios):
        u = float(rng.uniform())
        n = int(np.floor(10.0 ** (3.0 + 3.0 * u)))
        if max_samples is not None:
            n = min(n, max_samples)
        d = _randomized(rng, seed, k, n)
        d["horizon"] = float(rng.uniform(3.0, 15.0))
        d["dt"] = float((0.5e-3, 1e-3, 2e-3)[int(rng.integers(0, 3))])
        out.append(d)
    return out


def serving_stream(rate, duration=60.0, seed=None, sizes=(25_000, 100_000, 1_000_000),
                   probs=(0.70, 0.25, 0.05), deadline=0.530):
    """Poisson arrivals at `rate` req/s; returns a list of (t_arrival, scenario, deadline)."""
    seed = 1000 + int(rate) if seed is None else seed
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    reqs = []
    k = 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration:
            break
        n = int(rng.choice(np.array(sizes), p=np.array(probs)))
        d = _randomized(rng, seed, k, n)
        reqs.append((t, d, deadline))
        k += 1
    return reqs


def perception(n=10_000, seed=42, scenario_id=0, **over):
    """The stationary-obstacle scenario with a stochastic brake trigger.

    Sensing runs at 20 Hz (frame period 50 ms); the obstacle is hidden for the
    first U(0, 4) frames, each later frame misses it with probability 0.1, and
    braking is requested after 3 consecutive detections plus a processing
    latency ~ N(80 ms, 20 ms) truncated to [30, 120] ms (120 ms being the
    perception allowance of the timing budget in Section VI-F;
    perception effects are the extension named in Section VIII).
    """
    d = single(n, seed, scenario_id)
    d.update({"latency": ("trunc_normal", 0.08, 0.02, 0.03, 0.12),
              "occlusion": ("uniform", 0.0, 4.0), "frame_period": 0.05,
              "p_dropout": 0.1, "confirm": 3})
    d.update(over)
    return d


def closed_loop(n=10_000, seed=42, scenario_id=0, **over):
    """The stationary-obstacle scenario under a TTC-threshold controller.

    The obstacle is far ahead (gap ~ N(120 m, 10 m)); at 20 Hz the controller
    measures gap and closing speed with noise (sd 0.5 m, 0.3 m/s), brakes
    partially at -3 m/s^2 once the measured TTC drops below 3.0 s and fully
    (a_cmd) below 2.0 s, each command after the 50 ms dead time; horizon 15 s.
    """
    d = single(n, seed, scenario_id)
    d.update({"gap": ("normal", 120.0, 10.0), "horizon": 15.0, "ctl_period": 0.05,
              "ttc_warn": 3.0, "ttc_brake": 2.0, "a_warn": -3.0, "noise_gap": 0.5,
              "noise_v": 0.3})
    d.update(over)
    return d


def rare_event(n=100_000, seed=2026, scenario_id=0, v0_shift=6.0, mu_shift=-0.25, **over):
    """The paper preset with importance sampling toward long stops: v0 drawn
    from N(30 + v0_shift, 2) and mu from N(0.8 + mu_shift, 0.1) (the nominal
    distributions of Sec. IV-B otherwise), each sample weighted by its
    likelihood ratio, for collision-risk levels far below 1/N."""
    d = paper_preset(n, seed, scenario_id)
    d["proposal"] = {"v0": ("normal", 30.0 + v0_shift, 2.0), "mu": ("normal", 0.8 + mu_shift, 0.1)}
    d.update(over)
    return d
