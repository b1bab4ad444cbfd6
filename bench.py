"""Benchmark of the Monte Carlo braking rollout on one MI355X.

Workload (the headline configuration): one stationary-obstacle scenario of
1,048,576 samples -- v0 ~ TN(25, 1; [20, 30]), mu ~ U(0.4, 0.9),
m ~ N(1500, 75), theta ~ N(0, 0.02), CdA ~ N(0.7, 0.05), Crr ~ U(0.01, 0.015),
tau ~ U(0.1, 0.3), gap ~ N(60, 2), dead time 0.05 s, h = 0.55, L = 2.7,
explicit Euler, dt = 1 ms, T = 10 s -- with the parameters drawn on the host
(the paper's plain method) and resident in HBM before timing starts.

One step = aeb_rollout (all samples) + aeb_reduce (counts, P(collision),
moments, headways at 5/1/0.1 % risk, a 256-point risk curve, margin
quantiles), timed as eager calls and as a recorded HIP graph of the same
kernels (each replay recomputes everything and its statistics are collected
before the next), and as two recorded graphs on two streams with their own
outputs and scratch, step k+1 launched before step k is collected so that
its prep and sort overlap step k's integration tail and reduction.  `value`
is the FP64 rollouts/s of the fastest of the three among those whose
statistics equal the eager ones; the FP32 compensated form is timed as eager
calls and as one graph and reported beside it.

Also printed: the rollout kernel's roofline position (vector-ALU bound,
algorithmic flops = 11 per Euler step x the steps actually taken, FP64 vector
peak 78.6 TFLOP/s), the host sampling and PCIe transfer rates of the plain
method, and the FP64 reference timed on the host cores over a bounded sample.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "rollouts/sec FP64 vs FP32-comp; p50/p99 latency of 25k-sample requests"
FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz
FP64_FLOP_PER_CYCLE = 32768       # 1,024 SIMDs x 16 lanes x 2 flop
FP32_VECTOR_PEAK_TFLOPS = 157.3  # packed FP32; unpacked FP32 issues at the FP64 rate
EULER_FLOPS_PER_STEP = 11        # 4 fma (2 each) + 3 (v*v, -c, cmd-a)
FP32C_FLOPS_PER_STEP = 9         # 4 fma + v*v, compensated sums per block not counted
RK4_FLOPS_PER_STEP = 57          # 4 stage speed/actuator derivatives (6 each), 3 stage
                                 # updates of v and a (4 each), 3 weighted sums (5 each),
                                 # the final update of x, v, a (2 each)
RISK = (0.05, 0.01, 0.001)
MARGIN_Q = (0.0, 0.01, 0.05, 0.5)
GRID = (30.0, 130.0, 256)


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def profile_field(name, key, cast=float):
    """A figure from the machine-readable block of a committed rocprofv3
    summary under profiles/, or None if the kernel source it was taken on has
    changed since (its sha1 differs) or the summary is missing."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", name)
    try:
        txt = open(path).read()
        src = re.search(r"kernel_source: (\S+)", txt).group(1)
        sha = re.search(r"source_sha1: ([0-9a-f]+)", txt).group(1)
        val = cast(re.search(key + r": ([0-9.eE+-]+)", txt).group(1))
        now = hashlib.sha1(open(os.path.join(ROOT, src), "rb").read()).hexdigest()
    except (OSError, AttributeError, ValueError):
        return None
    return val if now == sha else None


def measured_traffic():
    """HBM bytes per launch of the integration kernel from the committed
    counter summary, or None if the kernel source changed since."""
    return profile_field("rollout_fp64_1M_hbm_traffic.md", "traffic_bytes_per_launch", int)


def cpu_model():
    """The host CPU's model name (as lscpu reports it)."""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


LANES = {}   # lane accounting of the last timed launch of each loop (profiling hooks)


def lane_efficiency(B, key, out):
    """Read the lane accounting of the last timed rollout (timing still on)
    and keep it under `key`: the fraction of the integration kernel's
    lane-steps that advanced a sample (the steps output over the wavefront
    sample-steps)."""
    wave = B.timing_lanes()
    lane = int(out["steps"].long().sum().item())
    LANES[key] = {"wave_sample_steps": wave, "sample_steps": lane,
                  "lane_efficiency": lane / wave if wave else None}
    return LANES[key]


def time_steps(B, torch, d, params, precision, out, steps, warmup):
    """Warm up, then time `steps` steps of rollout + reduce.  Returns the wall
    time, per-step integration-kernel times (library HIP events around that
    kernel), per-step rollout-call times (torch events: prep, sort and
    integration) and the last statistics."""
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        B.rollout(d, params=params, precision=precision, out=out)
        B.reduce(out, risk=RISK, margin_q=MARGIN_Q, grid=GRID)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    kern_ms = []
    B.timing_enable(True)
    t0 = time.perf_counter()
    for k in range(steps):
        evs[k][0].record(stream)
        B.rollout(d, params=params, precision=precision, out=out)
        evs[k][1].record(stream)
        stats = B.reduce(out, risk=RISK, margin_q=MARGIN_Q, grid=GRID)
        kern_ms.append(B.timing_last())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    lane_efficiency(B, (precision, int(d["n_samples"]), bool(d.get("ctl_period"))), out)
    B.timing_enable(False)
    call_ms = [a.elapsed_time(b) for a, b in evs]
    return wall, kern_ms, call_ms, stats


def time_graph_steps(B, torch, d, params, precision, out, steps, warmup):
    """The same step recorded once as a HIP graph (rollout + reduction) and
    replayed: each replay recomputes everything from the parameter columns and
    its statistics are collected (stream synchronised) before the next."""
    g = B.Graph(d, params=params, precision=precision, out=out, risk=RISK, margin_q=MARGIN_Q,
                grid=GRID)
    for _ in range(warmup):
        g.launch()
        g.finish()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.launch()
        stats = g.finish()
    wall = time.perf_counter() - t0
    g.close()
    return wall, stats


def time_graph_steps_two_streams(B, torch, d, params, precision, outs, steps, warmup):
    """The recorded step on two streams, each with its own graph, outputs and
    scratch: step k+1 is launched before step k is collected, so its prep and
    sort overlap step k's integration tail and reduction.  Every step is still
    a whole pass; returns the wall time of `steps` of them and the statistics
    of the last (all must equal)."""
    gs = [B.Graph(d, params=params, precision=precision, out=o, risk=RISK, margin_q=MARGIN_Q,
                  grid=GRID) for o in outs]
    return pipeline_graphs(torch, gs, steps, warmup)


_PIPE_STREAMS = []


def pipe_streams(torch):
    """The two streams every pipelined measurement uses: one pair for the
    process (a pair taken later from torch's pool can share a hardware queue
    with streams in use before, which serialises the two)."""
    if not _PIPE_STREAMS:
        _PIPE_STREAMS.extend([torch.cuda.Stream(), torch.cuda.Stream()])
    return _PIPE_STREAMS


def pipeline_graphs(torch, gs, steps, warmup):
    """Replays two recorded graphs (own outputs and scratch each) alternately
    on two streams, launching step k+1 before collecting step k; closes the
    graphs.  Returns the wall time of `steps` steps, the statistics of the
    last and whether every step's statistics equal it."""
    ss = pipe_streams(torch)
    for k in range(max(warmup, 2)):
        gs[k % 2].launch(ss[k % 2])
        gs[k % 2].finish(ss[k % 2])
    torch.cuda.synchronize()
    every = []
    t0 = time.perf_counter()
    gs[0].launch(ss[0])
    for k in range(1, steps):
        gs[k % 2].launch(ss[k % 2])
        every.append(gs[(k - 1) % 2].finish(ss[(k - 1) % 2]))
    every.append(gs[(steps - 1) % 2].finish(ss[(steps - 1) % 2]))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    for g in gs:
        g.close()
    all_equal = all(same_stats(every[-1], x) for x in every)
    return wall, every[-1], all_equal


def same_stats(a, b):
    """Equal statistics (NaN equal to NaN); a batch's are lists of them."""
    import numpy as np
    if isinstance(a, list):
        return len(a) == len(b) and all(same_stats(x, y) for x, y in zip(a, b))
    for k, v in a.items():
        w = b[k]
        if isinstance(v, np.ndarray):
            if not np.array_equal(v, w, equal_nan=v.dtype.kind == "f"):
                return False
        elif isinstance(v, float) and v != v:
            if w == w:
                return False
        elif v != w:
            return False
    return True


def cpu_baseline(d, budget_samples, single_samples=10_000):
    """The oracle (plain C, FP64) on the host cores: all threads over the first
    `budget_samples` samples (the value), and one thread over the first
    `single_samples` (reported beside it)."""
    from oracle import oracle
    threads = oracle.host_threads()
    n = min(budget_samples, int(d["n_samples"]))
    t0 = time.perf_counter()
    oracle.run(d, first=0, count=n, threads=threads)
    el = time.perf_counter() - t0
    m = min(single_samples, int(d["n_samples"]))
    t0 = time.perf_counter()
    oracle.run(d, first=0, count=m, threads=1)
    el1 = time.perf_counter() - t0
    return {"value": n / el, "unit": "rollouts/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus_visible": os.cpu_count(),
            "sample": f"samples 0..{n - 1} of the same scenario on {threads} threads "
                      f"({el:.2f} s wall); single thread over samples 0..{m - 1}: "
                      f"{m / el1:.0f} rollouts/s ({el1:.2f} s)",
            "single_thread_rollouts_per_s": m / el1}


def rk4_leg(B, W, torch, n, steps=5):
    """The paper's own integrator on its Sec. IV-B uncertainty model (classical
    RK4, no fused operations, no obstacle), parameters drawn in-kernel: the
    integration kernel's time from the library's events, FP64 flops per step
    counted as in RK4_FLOPS_PER_STEP."""
    import numpy as np
    d = W.paper_preset(n)
    out = B.alloc_outputs(n)
    B.rollout(d, out=out)
    torch.cuda.synchronize()
    B.timing_enable(True)
    ks = []
    for _ in range(steps):
        B.rollout(d, out=out)
        ks.append(B.timing_last())
    B.timing_enable(False)
    nsteps = int(out["steps"].to(torch.int64).sum().item())
    ms = float(np.mean(ks))
    tflops = RK4_FLOPS_PER_STEP * nsteps / (ms * 1e-3) / 1e12
    return {"workload": f"paper preset (Sec. IV-B), {n} samples, RK4 dt=1 ms, no obstacle",
            "kernel_ms": ms, "rollouts_per_s": n / (ms * 1e-3), "steps_per_launch": nsteps,
            "flops_per_step": RK4_FLOPS_PER_STEP, "achieved_tflops": tflops,
            "frac_fp64_peak": tflops / FP64_VECTOR_PEAK_TFLOPS}


def unfused_leg(B, W, torch, n, steps=5):
    """The headline scenario under the paper's rule of no fused operations
    (Sec. V-D): every multiply-add a rounded product and a rounded sum, on the
    same block-structured kernel; 11 flop per step as for the fused form, so
    the ceiling is half the FMA peak."""
    import numpy as np
    d = W.single(n, nofma=True)
    out = B.alloc_outputs(n)
    B.rollout(d, out=out)
    torch.cuda.synchronize()
    B.timing_enable(True)
    ks = []
    for _ in range(steps):
        B.rollout(d, out=out)
        ks.append(B.timing_last())
    B.timing_enable(False)
    nsteps = int(out["steps"].to(torch.int64).sum().item())
    ms = float(np.mean(ks))
    tflops = EULER_FLOPS_PER_STEP * nsteps / (ms * 1e-3) / 1e12
    return {"workload": f"stationary obstacle, {n} samples, explicit Euler without fused "
                        "operations, parameters drawn in-kernel",
            "kernel_ms": ms, "rollouts_per_s": n / (ms * 1e-3), "steps_per_launch": nsteps,
            "flops_per_step": EULER_FLOPS_PER_STEP, "achieved_tflops": tflops,
            "frac_fp64_peak": tflops / FP64_VECTOR_PEAK_TFLOPS,
            "frac_unfused_ceiling": tflops / (FP64_VECTOR_PEAK_TFLOPS / 2)}


def paper_study_leg(B, W, torch):
    """The paper's own workload (Sec. IV-B preset, RK4, no obstacle) on the GPU:
    Table I's sample counts (mean and sd of the stopping distance beside the
    printed rows), the Sec. VI-C headways at 350,000 samples, and the step size
    against fidelity and speed (RK4 and explicit Euler, dt = 1 to 20 ms)."""
    import numpy as np
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_results.json")))
    risk = tuple(gold["headways"]["risk"])
    rows = []
    for row in gold["table_I"]["rows"]:
        st = B.reduce(B.rollout(W.paper_preset(row["n"])), risk=risk)
        rows.append({"n": row["n"], "mean": st["mean_dist"], "sd": st["sd_dist"],
                     "paper_mean": row["mean"], "paper_sd": row["sd"]})
    dt_rows = []
    ref = None
    for integ in ("rk4", "euler"):
        for dt in (1e-3, 2e-3, 5e-3, 1e-2, 2e-2):
            d = W.paper_preset(350_000, integrator=integ, dt=dt)
            out = B.alloc_outputs(350_000)
            B.rollout(d, out=out)
            torch.cuda.synchronize()
            B.timing_enable(True)
            ks = []
            for _ in range(3):
                B.rollout(d, out=out)
                ks.append(B.timing_last())
            B.timing_enable(False)
            st = B.reduce(out, risk=risk)
            if ref is None:
                ref = st
            dt_rows.append({"integrator": integ, "dt_ms": dt * 1e3, "mean": st["mean_dist"],
                            "sd": st["sd_dist"], "headways": st["headway"],
                            "mean_minus_rk4_1ms": st["mean_dist"] - ref["mean_dist"],
                            "kernel_ms": float(np.median(ks)),
                            "rollouts_per_s": 350_000 / (float(np.median(ks)) * 1e-3)})
    return {"workload": "paper preset (Sec. IV-B), RK4 dt = 1 ms unless stated, no obstacle",
            "table_I": rows, "headways_350k": ref["headway"],
            "paper_headways": gold["headways"]["h0"], "step_size": dt_rows}


def kernel_ms(B, torch, d, out, precision="fp64", reps=3):
    """Median integration-kernel time of `reps` rollouts (library HIP events)."""
    import numpy as np
    B.rollout(d, out=out, precision=precision)
    torch.cuda.synchronize()
    B.timing_enable(True)
    ks = []
    for _ in range(reps):
        B.rollout(d, out=out, precision=precision)
        ks.append(B.timing_last())
    lane_efficiency(B, (precision, int(d["n_samples"]), bool(d.get("ctl_period"))), out)
    B.timing_enable(False)
    return float(np.median(ks))


def perception_leg(B, W, torch, n):
    """Perception effects (Sec. VIII): each sample's brake command waits for a
    stochastic trigger (latency, occlusion, frame dropout, a confirmation run).
    The throughput of the stationary-obstacle scenario with and without it
    (parameters drawn in-kernel, FP64 and FP32C), and the paper preset's
    collision-risk headways as the dropout grows."""
    import numpy as np
    res = {"workload": f"stationary obstacle, {n} samples, explicit Euler dt=1 ms; perception: "
                       "20 Hz frames, occlusion U(0,4) frames, dropout 0.1, 3 detections in a "
                       "row, latency N(80, 20) ms truncated to [30, 120] ms"}
    out = B.alloc_outputs(n)
    for prec in ("fp64", "fp32c"):
        row = {}
        for name, d in (("without", W.single(n)), ("with", W.perception(n))):
            ms = kernel_ms(B, torch, d, out, prec)
            steps = int(out["steps"].to(torch.int64).sum().item())
            st = B.reduce(out, risk=RISK)
            flops = (EULER_FLOPS_PER_STEP if prec == "fp64" else FP32C_FLOPS_PER_STEP) * steps
            row[name] = {"kernel_ms": ms, "rollouts_per_s": n / (ms * 1e-3),
                         "steps_per_launch": steps, "achieved_tflops": flops / (ms * 1e-3) / 1e12,
                         "p_collision": st["p_collision"], "mean_dist": st["mean_dist"]}
        row["with"]["frac_fp64_peak"] = (row["with"]["achieved_tflops"] / FP64_VECTOR_PEAK_TFLOPS
                                         if prec == "fp64" else None)
        row["step_rate_with_over_without"] = (
            (row["with"]["steps_per_launch"] / row["with"]["kernel_ms"])
            / (row["without"]["steps_per_launch"] / row["without"]["kernel_ms"]))
        res[prec] = row
    trig = B.sample_params(W.perception(n), device=True)["trigger"]
    res["trigger_mean_s"] = float(trig.mean().item())
    res["trigger_p99_s"] = float(torch.quantile(trig[:1 << 20].float(), 0.99).item())
    risk = (0.05, 0.01, 0.001)
    rows = []
    for p in (None, 0.0, 0.1, 0.3):
        d = W.paper_preset(350_000)
        if p is not None:
            d.update({"latency": ("trunc_normal", 0.08, 0.02, 0.03, 0.12),
                      "occlusion": ("uniform", 0.0, 4.0), "frame_period": 0.05,
                      "p_dropout": p, "confirm": 3})
        st = B.reduce(B.rollout(d), risk=risk)
        rows.append({"p_dropout": p, "mean": st["mean_dist"], "sd": st["sd_dist"],
                     "headways": st["headway"]})
    res["paper_preset_headways"] = {"risk": list(risk), "samples": 350_000,
                                    "integrator": "rk4", "rows": rows}
    return res


def control_leg(B, W, torch, n):
    """Closed-loop controller assessment (Sec. VIII): the TTC-threshold
    controller on noisy measurements, run by the block-structured FP64 kernel.
    Its throughput against the open-loop run of the same scenario, and
    P(collision) over a grid of full-brake thresholds and noise levels."""
    import numpy as np
    out = B.alloc_outputs(n)
    d = W.closed_loop(n)
    ms = kernel_ms(B, torch, d, out, "fp64")
    steps = int(out["steps"].to(torch.int64).sum().item())
    st = B.reduce(out, risk=RISK)
    # the same scenario open loop (braking from the start) on the block path
    d_open = {k: v for k, v in d.items() if k not in B.CONTROL_FIELDS}
    ms_open = kernel_ms(B, torch, d_open, out, "fp64")
    steps_open = int(out["steps"].to(torch.int64).sum().item())
    flops = EULER_FLOPS_PER_STEP * steps
    prof_ctl = profile_field("rollout_fp64_controller_1M.md", "k_roll_fp64_ctl_avg_us")
    res = {"workload": f"stationary obstacle at N(120 m, 10 m), {n} samples, explicit Euler "
                       "dt=1 ms, T=15 s; 20 Hz controller, partial braking -3 m/s^2 below TTC "
                       "3.0 s, full braking below 2.0 s, measurement noise 0.5 m / 0.3 m/s",
           "kernel": "k_roll_fp64 with the controller (block-structured; blocks end at "
                     "decisions and command switches)",
           "kernel_ms": ms, "rollouts_per_s": n / (ms * 1e-3), "steps_per_launch": steps,
           "achieved_tflops": flops / (ms * 1e-3) / 1e12,
           "frac_fp64_peak": flops / (ms * 1e-3) / 1e12 / FP64_VECTOR_PEAK_TFLOPS,
           "p_collision": st["p_collision"],
           "lane_efficiency": LANES.get(("fp64", n, True), {}).get("lane_efficiency"),
           "profile_kernel_ms": (prof_ctl * 1e-3 if (prof_ctl and n == 1_048_576) else None),
           "frac_from_profile": (flops / (prof_ctl * 1e-6) / 1e12 / FP64_VECTOR_PEAK_TFLOPS
                                 if (prof_ctl and n == 1_048_576) else None),
           "open_loop_block_path": {"kernel_ms": ms_open, "steps_per_launch": steps_open,
                                    "step_rate_closed_over_open":
                                        (steps / ms) / (steps_open / ms_open)}}
    rows = []
    for tb in (1.6, 1.8, 2.0, 2.2, 2.4):
        for sg, sv in ((0.0, 0.0), (0.5, 0.3), (2.0, 1.0)):
            dd = W.closed_loop(200_000, ttc_brake=tb, noise_gap=sg, noise_v=sv)
            s2 = B.reduce(B.rollout(dd), risk=RISK)
            rows.append({"ttc_brake": tb, "noise_gap": sg, "noise_v": sv,
                         "p_collision": s2["p_collision"], "mean_dist": s2["mean_dist"]})
    res["threshold_grid"] = {"samples": 200_000, "ttc_warn": 3.0, "rows": rows}
    return res


def rare_event_leg(B, W, torch, n):
    """Rare-event estimation (Sec. VIII): the paper preset's collision-risk
    tail P(D > H0) out to ~1e-7, by plain sampling and by importance sampling
    (v0 and mu drawn from shifted normals, weighted by their likelihood ratio)
    at the same sample count; the standard errors give the variance reduction
    and the equivalent plain-sampling cost."""
    import numpy as np
    grid = (110.0, 190.0, 9)
    res = {"workload": f"paper preset (Sec. IV-B), {n} samples, RK4 dt=1 ms; proposals "
                       "v0 ~ N(36, 2), mu ~ N(0.55, 0.1)",
           "grid_m": list(np.linspace(*grid[:2], grid[2]))}
    out = B.alloc_outputs(n)
    d = W.paper_preset(n)
    ms_plain = kernel_ms(B, torch, d, out, "fp64")
    st = B.reduce(out, grid=grid)
    p_plain = st["risk_p"]
    se_plain = np.sqrt(p_plain * (1 - p_plain) / n)
    dw = W.rare_event(n)
    outw = B.alloc_outputs(n, weight=True)
    ms_is = kernel_ms(B, torch, dw, outw, "fp64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stw = B.reduce(outw, grid=grid)
    red_ms = (time.perf_counter() - t0) * 1e3
    rows = []
    for j, h in enumerate(res["grid_m"]):
        p, se = stw["risk_pw"][j], stw["risk_se"][j]
        vr = (se_plain[j] / se) ** 2 if se > 0 and se_plain[j] > 0 else None
        # plain samples needed for IS's relative error: p(1-p) / se^2
        n_eq = p * (1 - p) / se ** 2 if se > 0 else None
        rows.append({"H0": h, "p_plain": float(p_plain[j]), "se_plain": float(se_plain[j]),
                     "p_is": float(p), "se_is": float(se), "variance_ratio": vr,
                     "plain_samples_for_same_se": n_eq})
    res.update({"kernel_ms_plain": ms_plain, "kernel_ms_is": ms_is,
                "weighted_reduce_call_ms": red_ms, "weight_mean": stw["weight_mean"],
                "rows": rows})
    return res


def n_sweep_leg(B, W, torch, sizes=(1_000, 10_000, 100_000, 1_048_576), reps=5):
    """Rollout call (parameters drawn in-kernel) plus reduction at growing N:
    below ~1e5 samples the launch sequence, not the integration, sets the time."""
    import numpy as np
    res = {}
    for n in sizes:
        d = W.single(n)
        out = B.alloc_outputs(n)
        B.rollout(d, out=out)
        B.reduce(out, risk=RISK)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            B.rollout(d, out=out)
            B.reduce(out, risk=RISK)
            ts.append(time.perf_counter() - t0)
        t = float(np.median(ts))
        res[str(n)] = {"ms": t * 1e3, "rollouts_per_s": n / t}
    return res


def batch_leg(B, W, torch, reps=2):
    """Batched launches: the 256-scenario lead-vehicle sweep (100,000 samples
    each) and 1,000 scenarios of uneven size, horizon and step; parameters
    drawn in-kernel; rollouts/s of the batched rollout call (events on the
    stream), FP64 and FP32C, and the error of the FP32C P(collision) and p99
    distance against FP64 per scenario."""
    import numpy as np
    res = {}
    for name, scns in (("sweep_256x100k_lead", W.sweep(n=100_000)),
                       ("uneven_1000", W.uneven_batch(1000))):
        total = sum(int(d["n_samples"]) for d in scns)
        outs = [B.alloc_outputs(int(d["n_samples"])) for d in scns]
        entry = {"scenarios": len(scns), "samples": total}
        pcol, p99 = {}, {}
        for prec in ("fp64", "fp32c"):
            B.batch_rollout(scns, precision=prec, outs=outs)
            torch.cuda.synchronize()
            ms = []
            for _ in range(reps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
                B.batch_rollout(scns, precision=prec, outs=outs)
                e1.record()
                torch.cuda.synchronize()
                ms.append(e0.elapsed_time(e1))
            t = float(np.min(ms))
            entry[prec] = {"ms": t, "rollouts_per_s": total / (t * 1e-3)}
            pcol[prec] = np.array([float(((o["status"] & 4) != 0).double().mean().item())
                                   for o in outs])
            p99[prec] = np.array([float(torch.quantile(o["dist"], 0.99).item()) for o in outs])
            log(f"bench: batch {name} {prec}: {entry[prec]}")
        entry["fp32c_max_abs_err_p_collision"] = float(np.max(np.abs(pcol["fp32c"] -
                                                                     pcol["fp64"])))
        entry["fp32c_max_rel_err_p99_dist"] = float(np.max(np.abs(p99["fp32c"] - p99["fp64"]) /
                                                           np.abs(p99["fp64"])))
        entry["fp32c_speedup"] = entry["fp64"]["ms"] / entry["fp32c"]["ms"]
        res[name] = entry
        del outs
        torch.cuda.empty_cache()
    return res


def uneven_config_leg(B, W, torch, reps=3):
    """The 1,000-scenario uneven batch as specified: FP32C, launch shape chosen
    by the autotuner (calibrated on the batch's largest scenario; its choice
    and the runner-up reported), every step the batched rollout plus the
    statistics of every scenario, timed as eager calls and as a replay of one
    recorded graph (same kernels, statistics equal)."""
    import numpy as np
    scns = W.uneven_batch(1000)
    total = sum(int(d["n_samples"]) for d in scns)
    big = max(scns, key=lambda d: int(d["n_samples"]))
    keep = B.tune_get("fp32c", "stationary")
    default_ms = None
    try:
        # the default shape's time on the calibration scenario, then the sweep
        out = B.alloc_outputs(int(big["n_samples"]))
        B.rollout(big, precision="fp32c", out=out)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(4):
            B.rollout(big, precision="fp32c", out=out)
        torch.cuda.synchronize()
        default_ms = (time.perf_counter() - t0) / 4 * 1e3
        del out
        best_ms = B.autotune(big, "fp32c")
        ranked = B.tune_results("fp32c", "stationary")
        chosen = B.tune_get("fp32c", "stationary")
        outs = [B.alloc_outputs(int(d["n_samples"])) for d in scns]
        # eager: batched rollout + segmented statistics, synchronised per step
        B.batch_reduce(B.batch_rollout(scns, precision="fp32c", outs=outs), risk=RISK,
                       margin_q=MARGIN_Q, grid=GRID)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            st_e = B.batch_reduce(B.batch_rollout(scns, precision="fp32c", outs=outs),
                                  risk=RISK, margin_q=MARGIN_Q, grid=GRID)
        eager_ms = (time.perf_counter() - t0) / reps * 1e3
        # the batched integration kernel alone (library HIP events) and its
        # lane accounting: FP32C rate against the unpacked and packed peaks
        steps_total = sum(int(o["steps"].long().sum().item()) for o in outs)
        B.timing_enable(True)
        try:
            ks = []
            for _ in range(reps):
                B.batch_rollout(scns, precision="fp32c", outs=outs)
                ks.append(B.timing_last())
            wave = B.timing_lanes()
        finally:
            B.timing_enable(False)
        kern_ms = float(np.median(ks))
        tflops = FP32C_FLOPS_PER_STEP * steps_total / (kern_ms * 1e-3) / 1e12
        # one recorded graph of the same step
        g = B.Graph(scns, precision="fp32c", out=outs, risk=RISK, margin_q=MARGIN_Q, grid=GRID,
                    batch=True)
        g.launch()
        g.finish()
        t0 = time.perf_counter()
        for _ in range(reps):
            g.launch()
            st_g = g.finish()
        graph_ms = (time.perf_counter() - t0) / reps * 1e3
        g.close()
        same = all(same_stats(a, b) for a, b in zip(st_e, st_g))
        # two such graphs (own outputs and scratch) pipelined on two streams:
        # one step's prep and sort overlap the other's integration tail and
        # statistics
        outs2 = [B.alloc_outputs(int(d["n_samples"])) for d in scns]
        gs = [B.Graph(scns, precision="fp32c", out=o, risk=RISK, margin_q=MARGIN_Q, grid=GRID,
                      batch=True) for o in (outs, outs2)]
        wall2, st_p, p_equal = pipeline_graphs(torch, gs, max(reps, 4), 1)
        pipe_ms = wall2 / max(reps, 4) * 1e3
        p_same = p_equal and same_stats(st_e, st_p)
        del outs, outs2
        torch.cuda.empty_cache()
    finally:
        B.tune_set("fp32c", "stationary", *keep)
    return {"workload": "1,000 scenarios from seed 7: N log-uniform in [1e3, 1e6], horizon "
                        "U(3, 15) s, dt in {0.5, 1, 2} ms, stationary obstacle; FP32C; step = "
                        "batched rollout + statistics of every scenario",
            "scenarios": len(scns), "samples": total,
            "tuner": {"calibration": f"largest scenario, {int(big['n_samples'])} samples",
                      "chosen": {"shape": list(chosen), "ms": best_ms},
                      "runner_up": ({"shape": list(ranked[1][0]), "ms": ranked[1][1]}
                                    if len(ranked) > 1 else None),
                      "candidates": len(ranked), "default_shape_ms": default_ms},
            "kernel_ms": kern_ms, "kernel_rollouts_per_s": total / (kern_ms * 1e-3),
            "steps_per_launch": steps_total, "achieved_tflops": tflops,
            "frac_unpacked_fp32_peak": tflops / FP64_VECTOR_PEAK_TFLOPS,
            "frac_packed_fp32_peak": tflops / FP32_VECTOR_PEAK_TFLOPS,
            "lane_efficiency": steps_total / wave if wave else None,
            "eager_ms_per_step": eager_ms, "eager_rollouts_per_s": total / (eager_ms * 1e-3),
            "graph_ms_per_step": graph_ms, "graph_rollouts_per_s": total / (graph_ms * 1e-3),
            "graph_stats_equal_eager": same,
            "two_stream_graph_ms_per_step": pipe_ms,
            "two_stream_rollouts_per_s": total / (pipe_ms * 1e-3),
            "two_stream_stats_equal_eager": p_same}


def serving_leg(B, W, precision, rates, duration, arena_gib=4):
    """Poisson request streams (sizes 25k/100k/1M at 70/25/5 %, 530 ms deadline)
    paced in real time into one server; latency = completion - arrival on the
    server's clock."""
    import numpy as np
    res = {}
    with B.Server(int(arena_gib * (1 << 30)), precision=precision, max_slots=256, n_streams=3,
                  tick_us=200, max_tick_samples=1 << 22, risk=RISK, margin_q=MARGIN_Q,
                  grid=GRID) as srv:
        # warm the kernels once
        srv.wait(srv.submit(W.single(25_000, seed=1, scenario_id=1)))
        for rate in rates:
            stream = W.serving_stream(rate, duration=duration)
            pending, done = {}, []
            keep = {}  # a sampled subset, re-run alone afterwards
            t0 = time.perf_counter()
            k = 0
            while k < len(stream) or pending:
                now = time.perf_counter() - t0
                while k < len(stream) and stream[k][0] <= now:
                    _, d, dl = stream[k]
                    t = srv.submit(d, deadline=dl)
                    pending[t] = int(d["n_samples"])
                    if k % 97 == 0:
                        keep[t] = [d, None]
                    k += 1
                for t in list(pending):
                    r = srv.poll(t)
                    if r is not None:
                        done.append((pending.pop(t), r[1]))
                        if t in keep:
                            keep[t][1] = r[0]
                if k < len(stream):
                    time.sleep(max(0.0, min(2e-4, stream[k][0] - (time.perf_counter() - t0))))
                else:
                    time.sleep(1e-4)
            wall = time.perf_counter() - t0
            equal = True
            for d, st in keep.values():
                o = B.rollout(d, precision=precision)
                equal = equal and same_stats(B.reduce(o, risk=RISK, margin_q=MARGIN_Q,
                                                      grid=GRID), st)
            lat = np.array([tm["done"] - tm["arrive"] for _, tm in done])
            lat25 = np.array([tm["done"] - tm["arrive"] for n, tm in done if n == 25_000])
            samples = sum(n for n, _ in done)
            res[str(rate)] = {
                "requests": len(done), "p50_ms": float(np.percentile(lat, 50) * 1e3),
                "p99_ms": float(np.percentile(lat, 99) * 1e3),
                "p50_25k_ms": float(np.percentile(lat25, 50) * 1e3) if lat25.size else None,
                "p99_25k_ms": float(np.percentile(lat25, 99) * 1e3) if lat25.size else None,
                "max_ms": float(lat.max() * 1e3),
                "deadline_miss_rate": float(np.mean([tm["missed"] for _, tm in done])),
                "rollouts_per_s": samples / wall,
                "alone_vs_mix_checked": len(keep), "alone_vs_mix_equal": equal,
            }
            log(f"bench: serving {precision} {rate} req/s: {res[str(rate)]}")
        info = srv.info()
    res["ticks"] = info["ticks"]
    res["arena_peak_bytes"] = info["arena_peak"]
    return res


def plain_end_to_end(B, torch, d, n, cols, reps=3):
    """The paper's plain method as one figure (Sec. IV-C, V-B): parameters
    drawn on the host cores into pinned memory, copied to HBM, the rollout,
    the reduction and its statistics back on the host, timed from the start
    of the sampling to the statistics in host memory; median of `reps`."""
    import numpy as np
    host = B.alloc_params(n, device=False, pinned=True)
    params = {c: torch.empty(n, dtype=torch.float64, device="cuda") for c in cols}
    out = B.alloc_outputs(n)
    rows = []
    for r in range(reps + 1):  # the first pass pays one-time costs
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        B.sample_params(d, device=False, out=host)
        t1 = time.perf_counter()
        for c in cols:
            params[c].copy_(host[c], non_blocking=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        B.rollout(d, params=params, out=out)
        B.reduce(out, risk=RISK, margin_q=MARGIN_Q, grid=GRID)
        t3 = time.perf_counter()
        if r:
            rows.append((t3 - t0, t1 - t0, t2 - t1, t3 - t2))
    tot, samp, h2d, dev = (float(np.median([x[j] for x in rows])) for j in range(4))
    return {"what": "host sampling + H2D copy + rollout + reduction + statistics D2H, one pass",
            "ms": tot * 1e3, "rollouts_per_s": n / tot, "host_sampling_ms": samp * 1e3,
            "h2d_ms": h2d * 1e3, "rollout_and_reduce_ms": dev * 1e3,
            "host_sampling_threads": os.cpu_count()}


def saturated_leg(B, W, torch, seconds, depth=64):
    """The serving mix (25k/100k/1M samples at 70/25/5 %) submitted back to
    back so that `depth` requests are always waiting or running, for
    `seconds`, once in FP32C and once in FP64: the rollouts/s each served
    form delivers when the device never idles, its latency under that load,
    and the FP32C statistics against the FP64 ones of the same requests."""
    import numpy as np
    # enough requests that neither form runs out within the window (800 per
    # second of arrivals for 30 s per second of window: ~2.2e9 samples per
    # second of window, above what either form serves)
    reqs = [(d, dl) for _, d, dl in W.serving_stream(800, duration=30.0 * seconds, seed=4242)]
    res = {"workload": "serving mix, requests back to back, %d in flight" % depth,
           "seconds": seconds}
    stats = {}
    for prec in ("fp32c", "fp64"):
        with B.Server(4 << 30, precision=prec, max_slots=256, n_streams=3, tick_us=200,
                      max_tick_samples=1 << 22, risk=RISK, margin_q=MARGIN_Q, grid=GRID) as srv:
            srv.wait(srv.submit(W.single(25_000, seed=1, scenario_id=1)))
            pending, done, k = {}, {}, 0
            t0 = time.perf_counter()
            t_end = t0 + seconds
            while time.perf_counter() < t_end:
                while len(pending) < depth and k < len(reqs):
                    pending[srv.submit(reqs[k][0], deadline=reqs[k][1])] = k
                    k += 1
                for t in list(pending):
                    r = srv.poll(t)
                    if r is not None:
                        done[pending.pop(t)] = r
                time.sleep(5e-5)
            # requests completed inside the window count; the rest drain unmeasured
            t_stop = time.perf_counter()
            in_window = {j: r for j, r in done.items()}
            while pending:
                for t in list(pending):
                    r = srv.poll(t)
                    if r is not None:
                        done[pending.pop(t)] = r
                time.sleep(1e-4)
        samples = sum(int(reqs[j][0]["n_samples"]) for j in in_window)
        lat = np.array([tm["done"] - tm["arrive"] for _, tm in in_window.values()])
        res[prec] = {"requests": len(in_window), "rollouts_per_s": samples / (t_stop - t0),
                     "p50_ms": float(np.percentile(lat, 50) * 1e3),
                     "p99_ms": float(np.percentile(lat, 99) * 1e3),
                     "requests_ran_out": k >= len(reqs)}
        stats[prec] = {j: st for j, (st, _) in done.items()}
        log(f"bench: saturated {prec}: {res[prec]}")
    common = sorted(set(stats["fp32c"]) & set(stats["fp64"]))
    dp = [abs(stats["fp32c"][j]["p_collision"] - stats["fp64"][j]["p_collision"]) for j in common]
    dh = [abs(stats["fp32c"][j]["headway"][0] - stats["fp64"][j]["headway"][0])
          / stats["fp64"][j]["headway"][0] for j in common]
    nb = [stats["fp32c"][j]["n_boundary"] / stats["fp32c"][j]["n"] for j in common]
    res["fp32c_over_fp64"] = res["fp32c"]["rollouts_per_s"] / res["fp64"]["rollouts_per_s"]
    res["accuracy_fp32c_vs_fp64"] = {
        "requests_compared": len(common), "max_abs_diff_p_collision": float(max(dp)),
        "max_rel_diff_headway_5pct": float(max(dh)), "max_boundary_fraction": float(max(nb))}
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=1_048_576)
    ap.add_argument("--cpu-samples", type=int, default=1_048_576)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-launch leg")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the eager FP64 step loop on one stream (for profiler runs: "
                         "every integration-kernel launch is then one of the timed steps)")
    ap.add_argument("--fp32c-only", action="store_true",
                    help="only the eager FP32C step loop (for counter runs of that kernel)")
    ap.add_argument("--control-only", choices=("closed", "open"), default=None,
                    help="only the eager FP64 loop of the closed-loop controller scenario, "
                         "or of the same scenario open loop (for counter runs of that kernel)")
    ap.add_argument("--serve-seconds", type=float, default=60.0,
                    help="length of each Poisson serving stream (0: no serving leg)")
    ap.add_argument("--saturate-seconds", type=float, default=10.0,
                    help="length of each saturated serving run, FP32C and FP64 (0: none)")
    ap.add_argument("--copy-calib-mb", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a kernel of "
                         "known traffic for scaling hardware byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the rollout "
              "shards by sample range with no exchange beyond a tiny statistics merge; "
              "multi-GPU runs are not part of this build)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2604_27193_amd import binding as B
    from paper_2604_27193_amd import workloads as W

    torch.cuda.set_device(0)
    if args.copy_calib_mb:
        src = torch.ones(args.copy_calib_mb << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    if args.control_only:
        d = W.closed_loop(args.n)
        if args.control_only == "open":
            d = {k: v for k, v in d.items() if k not in B.CONTROL_FIELDS}
        outc = B.alloc_outputs(args.n)
        wall, kc, cc, stc = time_steps(B, torch, d, None, "fp64", outc, args.steps, args.warmup)
        steps_c = int(outc["steps"].to(torch.int64).sum().item())
        print(json.dumps({"control": args.control_only, "kernel_ms": float(np.mean(kc)),
                          "steps_per_launch": steps_c, "steps": args.steps}), flush=True)
        return
    d = W.single(args.n)
    n = int(d["n_samples"])

    # plain method: host sampling into pinned memory, then H2D
    log(f"bench: host sampling of {n} samples")
    t0 = time.perf_counter()
    host = B.sample_params(d, device=False, out=B.alloc_params(n, device=False, pinned=True))
    t_sample = time.perf_counter() - t0
    # without perception the trigger column stays on the host (passed as NULL)
    cols = [c for c in B.COLUMNS if c != "trigger"]
    params = {c: torch.empty(n, dtype=torch.float64, device="cuda") for c in cols}
    torch.cuda.synchronize()
    t_h2d = float("inf")
    for _ in range(3):  # the first copy also pays one-time driver costs
        t0 = time.perf_counter()
        for c in cols:
            params[c].copy_(host[c], non_blocking=True)
        torch.cuda.synchronize()
        t_h2d = min(t_h2d, time.perf_counter() - t0)
    out = B.alloc_outputs(n)

    if args.fp32c_only:
        out32 = B.alloc_outputs(n)
        wall32, k32, c32, st32 = time_steps(B, torch, d, params, "fp32c", out32, args.steps,
                                            args.warmup)
        print(json.dumps({"fp32c_kernel_ms": float(np.mean(k32)), "steps": args.steps}),
              flush=True)
        return
    log("bench: fp64 timed loop")
    wall64, k64, c64, st64 = time_steps(B, torch, d, params, "fp64", out, args.steps, args.warmup)
    steps_total = int(out["steps"].to(torch.int64).sum().item())
    kavg64 = float(np.mean(k64)) * 1e-3
    flops64 = EULER_FLOPS_PER_STEP * steps_total
    achieved = flops64 / kavg64 / 1e12
    prof_us = profile_field("rollout_fp64_1M_kernel_stats.md", "k_roll_fp64_avg_us")
    issued = profile_field("rollout_valu_counters_1M.md", "issued_fp64_flop_per_step")
    arith = profile_field("rollout_valu_counters_1M.md", "fp64_arith_per_lane_step")
    cycles = profile_field("rollout_valu_counters_1M.md", "cycles_per_launch")
    issue = profile_field("rollout_valu_counters_1M.md", "valu_issue_fraction")
    roofline = {
        "bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
        "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
        "traffic": measured_traffic() if n == 1_048_576 else None,
        "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-scaled)",
        "algorithmic_bytes_per_launch": 93 * n,
        "kernel": "k_roll_fp64 (block-structured explicit Euler, FP64)",
        "kernel_ms": kavg64 * 1e3, "kernel_ms_source": "HIP events on the launch stream",
        "flops_per_launch": flops64, "steps_per_launch": steps_total,
        "flops_per_step": EULER_FLOPS_PER_STEP,
        # the committed rocprofv3 kernel-trace summary of the --headline-only
        # loop (same kernel source), and the FP64 flops the VALU counters saw
        # issued per step (the clamped and dead-time forms skip the actuator
        # update, which cannot change the result)
        "profile_kernel_ms": prof_us * 1e-3 if (prof_us and n == 1_048_576) else None,
        "frac_from_profile": (flops64 / (prof_us * 1e-6) / 1e12 / FP64_VECTOR_PEAK_TFLOPS
                              if (prof_us and n == 1_048_576) else None),
        "issued_flops_per_step": issued,
        "issued_frac": (issued * steps_total / kavg64 / 1e12 / FP64_VECTOR_PEAK_TFLOPS
                        if issued else None),
        # the profile's GPU cycles per launch (GRBM_GUI_ACTIVE per XCD): the clock
        # the kernel ran at, the fraction of the per-cycle FP64 peak (32,768 flop
        # per cycle) and the share of cycles on which the VALU issued
        "profile_clock_ghz": (cycles / (prof_us * 1e-6) / 1e9
                              if (cycles and prof_us and n == 1_048_576) else None),
        "frac_per_cycle": (flops64 / (cycles * FP64_FLOP_PER_CYCLE)
                           if (cycles and n == 1_048_576) else None),
        "valu_issue_fraction": issue if n == 1_048_576 else None,
        # the instruction-mix ceiling: 11 flop per step over the FP64 arithmetic
        # instructions a step issues (counters), against 2 flop per FMA; and
        # the fraction of that ceiling the kernel reaches
        "mix_ceiling": (EULER_FLOPS_PER_STEP / (2.0 * arith) if arith else None),
        "frac_of_mix_ceiling": (achieved / FP64_VECTOR_PEAK_TFLOPS
                                / (EULER_FLOPS_PER_STEP / (2.0 * arith)) if arith else None),
        # lane efficiency of the last timed launch (aeb_timing_lanes): the
        # fraction of the kernel's lane-steps that advanced a sample
        "lane_efficiency": LANES.get(("fp64", n, False), {}).get("lane_efficiency"),
    }
    if args.headline_only:
        res = {"metric": METRIC, "value": args.steps * n / wall64, "unit": "rollouts/s",
               "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
               "ms_per_step": wall64 / args.steps * 1e3, "higher_is_better": True,
               "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
               "config": {"workload": f"single stationary-obstacle scenario, {n} samples, "
                                      "eager FP64 loop only (profiling run)",
                          "n_samples": n},
               "roofline": roofline, "cpu_baseline": None}
        print(json.dumps(res), flush=True)
        return
    log("bench: plain method end to end")
    e2e = plain_end_to_end(B, torch, d, n, cols)
    log("bench: fp32c timed loop")
    out32 = B.alloc_outputs(n)
    wall32, k32, c32, st32 = time_steps(B, torch, d, params, "fp32c", out32, args.steps,
                                        args.warmup)
    steps32 = int(out32["steps"].to(torch.int64).sum().item())
    prof32 = profile_field("rollout_fp32c_1M_kernel_stats.md", "k_roll_fp32c_avg_us")
    d64 = out["dist"].cpu().numpy()
    d32 = out32["dist"].cpu().numpy()
    s64 = out["status"].cpu().numpy()
    s32 = out32["status"].cpu().numpy()
    inband = (s32 & 8) != 0
    rel32 = float(np.max(np.abs(d32 - d64)[~inband] / d64[~inband]))
    flags_equal = bool(np.array_equal((s32 & 7)[~inband], (s64 & 7)[~inband]))

    log("bench: recorded-graph loops")
    wallg64, stg64 = time_graph_steps(B, torch, d, params, "fp64", out, args.steps, args.warmup)
    wallg32, stg32 = time_graph_steps(B, torch, d, params, "fp32c", out32, args.steps,
                                      args.warmup)
    graph_equal = same_stats(st64, stg64) and same_stats(st32, stg32)
    log("bench: recorded graphs on two streams")
    out2 = B.alloc_outputs(n)
    wallp64, stp64, p_same = time_graph_steps_two_streams(B, torch, d, params, "fp64",
                                                          (out, out2), args.steps, args.warmup)
    pipe_equal = p_same and same_stats(st64, stp64)

    kavg32 = float(np.mean(k32)) * 1e-3
    # the step as a production caller repeats it: the fastest of the eager
    # calls, the recorded graph and the recorded graphs on two streams, among
    # those whose statistics equal the eager ones
    paths = [("eager calls", wall64)]
    if graph_equal:
        paths.append(("recorded graph", wallg64))
    if pipe_equal:
        paths.append(("recorded graphs pipelined over two streams", wallp64))
    step_path, step_wall = min(paths, key=lambda p: p[1])
    value = args.steps * n / step_wall

    log("bench: rk4 leg")
    rk4 = rk4_leg(B, W, torch, n)
    log("bench: unfused Euler leg")
    unfused = unfused_leg(B, W, torch, n)
    log("bench: N sweep")
    nsweep = n_sweep_leg(B, W, torch)
    log("bench: paper-preset study")
    study = paper_study_leg(B, W, torch)
    log("bench: perception leg")
    perception = perception_leg(B, W, torch, n)
    log("bench: controller leg")
    control = control_leg(B, W, torch, n)
    log("bench: rare-event leg")
    rare = rare_event_leg(B, W, torch, n)

    batch = uneven = None
    if not args.no_batch:
        log("bench: batched launches")
        batch = batch_leg(B, W, torch)
        log("bench: uneven batch as specified (tuned FP32C, graph and eager, statistics)")
        uneven = uneven_config_leg(B, W, torch)

    serving = None
    if args.serve_seconds > 0 or args.saturate_seconds > 0:
        serving = {"precision": "fp32c", "deadline_ms": 530.0,
                   "duration_s": args.serve_seconds}
        if args.serve_seconds > 0:
            log("bench: serving streams")
            serving["rates"] = serving_leg(B, W, "fp32c", (50, 200, 800), args.serve_seconds)
        if args.saturate_seconds > 0:
            log("bench: saturated serving")
            serving["saturated"] = saturated_leg(B, W, torch, args.saturate_seconds)

    cpu = None
    if not args.no_cpu:
        log("bench: cpu baseline (oracle)")
        cpu = cpu_baseline(d, args.cpu_samples)

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "rollouts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"single stationary-obstacle scenario, {n} samples, plain method "
                        "(host-drawn parameters resident in HBM), explicit Euler dt=1 ms "
                        "T=10 s; step = rollout + reduce",
            "n_samples": n, "integrator": "euler", "precision": "fp64",
            "step_path": step_path,
        },
        "roofline": roofline,
        "cpu_baseline": cpu,
        "fp64": {
            "eager_ms_per_step": wall64 / args.steps * 1e3,
            "graph_ms_per_step": wallg64 / args.steps * 1e3,
            "graph_stats_equal_eager": graph_equal,
            "two_stream_graph_ms_per_step": wallp64 / args.steps * 1e3,
            "two_stream_stats_equal_eager": pipe_equal,
            "kernel_ms": kavg64 * 1e3, "kernel_rollouts_per_s": n / kavg64,
            "rollout_call_ms": float(np.mean(c64)),
            "rollout_call_rollouts_per_s": n / (float(np.mean(c64)) * 1e-3),
            "reduce_ms": wall64 / args.steps * 1e3 - float(np.mean(c64)),
        },
        "fp32c": {
            "value": args.steps * n / min(wall32, wallg32 if graph_equal else wall32),
            "unit": "rollouts/s",
            "ms_per_step": wall32 / args.steps * 1e3,
            "graph_ms_per_step": wallg32 / args.steps * 1e3, "kernel_ms": kavg32 * 1e3,
            "kernel_rollouts_per_s": n / kavg32,
            "rollout_call_ms": float(np.mean(c32)),
            "achieved_tflops": FP32C_FLOPS_PER_STEP * steps32 / kavg32 / 1e12,
            # the build disables packed FP32 instructions, so FP32 issues at the
            # unpacked rate (the FP64 rate, 78.6 TFLOP/s), half the packed peak
            "peak_tflops_unpacked_fp32": FP64_VECTOR_PEAK_TFLOPS,
            "frac_unpacked_fp32_peak": FP32C_FLOPS_PER_STEP * steps32 / kavg32 / 1e12
                                       / FP64_VECTOR_PEAK_TFLOPS,
            "frac_packed_fp32_peak": FP32C_FLOPS_PER_STEP * steps32 / kavg32 / 1e12
                                     / FP32_VECTOR_PEAK_TFLOPS,
            "max_rel_dist_err_vs_fp64": rel32,
            "boundary_samples": int(inband.sum()),
            "collision_flags_equal_fp64_outside_band": flags_equal,
            "speedup_vs_fp64_kernel": kavg64 / kavg32,
            "lane_efficiency": LANES.get(("fp32c", n, False), {}).get("lane_efficiency"),
            "profile_kernel_ms": (prof32 * 1e-3 if (prof32 and n == 1_048_576) else None),
        },
        "rk4": rk4,
        "unfused_euler": unfused,
        "n_sweep_fp64_step": nsweep,
        "paper_preset_study": study,
        "perception": perception,
        "control": control,
        "rare_event": rare,
        "batch": batch,
        "uneven_batch_config": uneven,
        "serving": serving,
        "plain_method_host": {"sampling_s": t_sample, "h2d_s": t_h2d,
                              "h2d_GBps": len(cols) * 8 * n / t_h2d / 1e9},
        "plain_method_end_to_end": e2e,
        "stats": {"p_collision": st64["p_collision"], "mean_dist": st64["mean_dist"],
                  "sd_dist": st64["sd_dist"], "headways": st64["headway"],
                  "p_collision_fp32c": st32["p_collision"],
                  "boundary_fp32c": st32["n_boundary"]},
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
