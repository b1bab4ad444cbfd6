"""ctypes binding of ``libaeb.so`` (declared in include/aeb.h).

Argument marshalling only: scenario dicts become ``aeb_scenario`` structs,
torch tensors become raw device pointers, the current torch stream becomes
the HIP stream.  Every computation runs in the library's HIP kernels (or, for
``sample_params(..., device=False)``, in the library's host sampler, which is
the paper's CPU sampling step).  If the library is not built, loading fails
with an error; there is no fallback.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaeb.so")
ABI_VERSION = 9     # the aeb_version() these structures match
NOALLOC_SCRATCH_BYTES = 32 << 20  # AEB_NOALLOC_SCRATCH_BYTES of aeb.h
SERVE_EAGER = 1                   # AEB_SERVE_EAGER of aeb.h

COLUMNS = ("v0", "mu", "mass", "grade", "sin_grade", "cos_grade", "cda", "crr", "tau", "gap",
           "lead_decel", "trigger", "log_weight")
DISTS = ("v0", "mu", "mass", "grade", "cda", "crr", "tau", "gap", "lead_decel")
# perception fields and their values when a scenario dict leaves them out
PERCEPTION_DEFAULTS = {"latency": ("const", 0.0), "occlusion": ("const", 0.0),
                       "frame_period": 0.0, "p_dropout": 0.0, "confirm": 1}
# closed-loop controller fields (absent: 0, the open-loop command)
CONTROL_FIELDS = ("ctl_period", "ttc_warn", "ttc_brake", "a_warn", "noise_gap", "noise_v")
INTEGRATORS = {"euler": 0, "rk4": 1}
OBSTACLES = {"none": 0, "stationary": 1, "lead": 2}
DIST_KINDS = {"const": 0, "uniform": 1, "normal": 2, "trunc_normal": 3}
PRECISIONS = {"fp64": 0, "fp32c": 1, "fp32c_fixup": 2}

OK, EINVAL, ENOMEM, EAGAIN, EDEVICE, ENOTFOUND = 0, -1, -2, -3, -4, -5
END_STOP, END_IMPACT, END_HORIZON, COLLIDED, BOUNDARY = 1, 2, 3, 4, 8

EXPORTS = ("aeb_last_error", "aeb_version", "aeb_validate", "aeb_uniforms", "aeb_sample_params",
           "aeb_rollout", "aeb_rollout_noalloc", "aeb_reduce", "aeb_batch_rollout",
           "aeb_batch_reduce",
           "aeb_timing_enable", "aeb_timing_last", "aeb_timing_lanes", "aeb_reduce_fallbacks", "aeb_ctl_approx_check", "aeb_ctl_math", "aeb_valu_probe",
           "aeb_server_fixed_bytes",
           "aeb_serve_footprint", "aeb_server_create", "aeb_server_destroy", "aeb_serve_submit",
           "aeb_serve_poll", "aeb_server_info_get", "aeb_graph_create", "aeb_graph_create_batch",
           "aeb_graph_launch", "aeb_graph_finish", "aeb_graph_destroy", "aeb_graph_create_mix",
           "aeb_graph_launch_mix", "aeb_tune_get",
           "aeb_tune_set", "aeb_tune_results", "aeb_tune_load", "aeb_autotune")


class AebError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"aeb error {code}: {msg}")
        self.code = code


class Dist(C.Structure):
    _fields_ = [("kind", C.c_int32), ("reserved", C.c_int32), ("p0", C.c_double),
                ("p1", C.c_double), ("lo", C.c_double), ("hi", C.c_double)]


class Scenario(C.Structure):
    _fields_ = ([("seed", C.c_uint64), ("scenario_id", C.c_uint64), ("n_samples", C.c_int64),
                 ("integrator", C.c_int32), ("obstacle", C.c_int32),
                 ("impact_exit", C.c_int32), ("nofma", C.c_int32)]
                + [(f, C.c_double) for f in ("dt", "horizon", "dead_time", "a_cmd", "g", "rho",
                                             "h_cog", "wheelbase")]
                + [(f, Dist) for f in DISTS]
                + [("latency", Dist), ("occlusion", Dist), ("frame_period", C.c_double),
                   ("p_dropout", C.c_double), ("confirm", C.c_int32), ("reserved2", C.c_int32)]
                + [(f, C.c_double) for f in CONTROL_FIELDS]
                + [("is_mask", C.c_int32), ("reserved3", C.c_int32), ("proposal", Dist * 9)])


class Params(C.Structure):
    _fields_ = [(f, C.c_void_p) for f in COLUMNS] + [("n", C.c_int64)]


class Outputs(C.Structure):
    _fields_ = [("dist", C.c_void_p), ("status", C.c_void_p), ("steps", C.c_void_p),
                ("margin", C.c_void_p), ("v_impact", C.c_void_p), ("weight", C.c_void_p),
                ("n", C.c_int64)]


class ReduceReq(C.Structure):
    _fields_ = [("n_risk", C.c_int32), ("n_margin_q", C.c_int32), ("n_grid", C.c_int32),
                ("reserved", C.c_int32), ("risk", C.c_double * 16),
                ("margin_q", C.c_double * 4), ("grid_lo", C.c_double), ("grid_hi", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_collide", C.c_int64), ("n_stop", C.c_int64),
                ("n_impact", C.c_int64), ("n_horizon", C.c_int64), ("n_boundary", C.c_int64),
                ("p_collision", C.c_double), ("mean_dist", C.c_double), ("sd_dist", C.c_double),
                ("dist_min", C.c_double), ("dist_max", C.c_double),
                ("headway", C.c_double * 16), ("margin_min", C.c_double),
                ("margin_mean", C.c_double), ("margin_q", C.c_double * 4),
                ("v_impact_max", C.c_float), ("reserved", C.c_int32),
                ("risk_count", C.c_int64 * 1024), ("risk_p", C.c_double * 1024),
                ("weighted", C.c_int32), ("reserved2", C.c_int32), ("p_collision_w", C.c_double),
                ("p_collision_se", C.c_double), ("weight_mean", C.c_double),
                ("risk_pw", C.c_double * 1024), ("risk_se", C.c_double * 1024)]


_lib = None


class TuneShape(C.Structure):
    _fields_ = [("k", C.c_int32), ("block", C.c_int32), ("waves_per_simd", C.c_int32),
                ("samples_per_thread", C.c_int32)]


class ServerCfg(C.Structure):
    _fields_ = [("arena", C.c_void_p), ("arena_bytes", C.c_uint64), ("max_slots", C.c_int32),
                ("precision", C.c_int32), ("n_streams", C.c_int32), ("tick_us", C.c_int32),
                ("max_queue", C.c_int32), ("flags", C.c_int32),
                ("max_tick_samples", C.c_int64), ("req", ReduceReq)]


class ReqTiming(C.Structure):
    _fields_ = [("arrive", C.c_double), ("admit", C.c_double), ("start", C.c_double),
                ("done", C.c_double), ("missed", C.c_int32), ("reserved", C.c_int32)]


class ServerInfo(C.Structure):
    _fields_ = [(f, C.c_uint64) for f in (
        "submitted", "completed", "failed", "missed", "ticks", "queued", "admitted", "running",
        "arena_in_use", "arena_peak", "arena_request_bytes", "fixed_bytes")]


def lib():
    """Load the built library (build it with __graft_entry__.build())."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() first")
        L = C.CDLL(LIB_PATH)
        if L.aeb_version() != ABI_VERSION:
            raise ImportError(f"{LIB_PATH} has ABI version {L.aeb_version()}, the binding "
                              f"needs {ABI_VERSION}; rebuild it with __graft_entry__.build()")
        P = C.POINTER
        L.aeb_last_error.restype = C.c_char_p
        L.aeb_validate.argtypes = [P(Scenario)]
        L.aeb_uniforms.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, C.c_int64, C.c_uint32,
                                   C.c_uint32, C.c_void_p, C.c_int, C.c_void_p]
        L.aeb_sample_params.argtypes = [P(Scenario), C.c_int64, C.c_int64, P(Params), C.c_int,
                                        C.c_void_p]
        L.aeb_rollout.argtypes = [P(Scenario), P(Params), C.c_int, P(Outputs), C.c_void_p]
        L.aeb_rollout_noalloc.argtypes = [P(Scenario), P(Params), C.c_int, P(Outputs),
                                          C.c_void_p]
        L.aeb_reduce.argtypes = [P(Outputs), P(ReduceReq), P(Stats), C.c_void_p]
        L.aeb_batch_rollout.argtypes = [P(Scenario), C.c_int, C.c_int, P(Outputs), C.c_void_p]
        L.aeb_batch_reduce.argtypes = [P(Outputs), C.c_int, P(ReduceReq), P(Stats), C.c_void_p]
        L.aeb_timing_enable.argtypes = [C.c_int]
        L.aeb_timing_last.argtypes = [P(C.c_float)]
        L.aeb_reduce_fallbacks.argtypes = [P(C.c_uint64)]
        L.aeb_timing_lanes.argtypes = [P(C.c_uint64)]
        L.aeb_ctl_approx_check.argtypes = [P(C.c_double), P(C.c_double), C.c_void_p]
        L.aeb_ctl_math.argtypes = [C.c_void_p, C.c_void_p, C.c_int64, C.c_void_p, C.c_void_p,
                                   C.c_void_p, C.c_int, C.c_void_p]
        L.aeb_valu_probe.argtypes = [C.c_int, C.c_int64, C.c_int, C.c_void_p, C.c_void_p]
        L.aeb_server_fixed_bytes.argtypes = [P(ServerCfg), P(C.c_uint64)]
        L.aeb_serve_footprint.argtypes = [P(ServerCfg), C.c_int64, P(C.c_uint64)]
        L.aeb_server_create.argtypes = [P(ServerCfg), P(C.c_void_p)]
        L.aeb_server_destroy.argtypes = [C.c_void_p]
        L.aeb_serve_submit.argtypes = [C.c_void_p, P(Scenario), C.c_double, P(C.c_uint64)]
        L.aeb_serve_poll.argtypes = [C.c_void_p, C.c_uint64, P(Stats), P(ReqTiming)]
        L.aeb_server_info_get.argtypes = [C.c_void_p, P(ServerInfo)]
        L.aeb_graph_create.argtypes = [P(Scenario), P(Params), C.c_int, P(Outputs),
                                       P(ReduceReq), C.c_void_p, P(C.c_void_p)]
        L.aeb_graph_create_batch.argtypes = [P(Scenario), C.c_int, C.c_int, P(Outputs),
                                             P(ReduceReq), C.c_void_p, P(C.c_void_p)]
        L.aeb_graph_launch.argtypes = [C.c_void_p, C.c_void_p]
        L.aeb_graph_create_mix.argtypes = [P(Scenario), C.c_int, C.c_int, C.c_int64,
                                           P(ReduceReq), P(C.c_void_p)]
        L.aeb_graph_launch_mix.argtypes = [C.c_void_p, P(Scenario), C.c_int, P(Outputs),
                                           C.c_void_p, C.c_void_p]
        L.aeb_graph_finish.argtypes = [C.c_void_p, C.c_void_p]
        L.aeb_graph_destroy.argtypes = [C.c_void_p]
        L.aeb_tune_get.argtypes = [C.c_int, C.c_int, P(TuneShape)]
        L.aeb_tune_set.argtypes = [C.c_int, C.c_int, P(TuneShape)]
        L.aeb_tune_results.argtypes = [C.c_int, C.c_int, P(TuneShape), P(C.c_float), C.c_int,
                                       P(C.c_int)]
        L.aeb_tune_load.argtypes = [C.c_char_p]
        L.aeb_autotune.argtypes = [P(Scenario), C.c_int, C.c_char_p, C.c_void_p, P(C.c_float)]
        _lib = L
    return _lib


def _check(rc):
    if rc != OK:
        raise AebError(rc, lib().aeb_last_error().decode())
    return rc


def _dist(spec):
    d = Dist()
    d.kind = DIST_KINDS[spec[0]]
    vals = [float(v) for v in spec[1:]] + [0.0] * (4 - len(spec[1:]))
    d.p0, d.p1, d.lo, d.hi = vals
    if spec[0] == "const":
        d.p1 = 0.0
    return d


def scenario(d):
    """Marshal a scenario dict (see workloads.py) into ``aeb_scenario``."""
    s = Scenario()
    s.seed = int(d["seed"]) & 0xFFFFFFFFFFFFFFFF
    s.scenario_id = int(d["scenario_id"]) & 0xFFFFFFFFFFFFFFFF
    s.n_samples = int(d["n_samples"])
    s.integrator = INTEGRATORS[d["integrator"]]
    s.obstacle = OBSTACLES[d["obstacle"]]
    s.impact_exit = int(bool(d.get("impact_exit", False)))
    s.nofma = int(bool(d.get("nofma", False)))
    for f in ("dt", "horizon", "dead_time", "a_cmd", "g", "rho", "h_cog", "wheelbase"):
        setattr(s, f, float(d[f]))
    for f in DISTS:
        setattr(s, f, _dist(d[f]))
    per = dict(PERCEPTION_DEFAULTS)
    per.update({k: d[k] for k in PERCEPTION_DEFAULTS if k in d})
    s.latency = _dist(per["latency"])
    s.occlusion = _dist(per["occlusion"])
    s.frame_period = float(per["frame_period"])
    s.p_dropout = float(per["p_dropout"])
    s.confirm = int(per["confirm"])
    for f in CONTROL_FIELDS:
        setattr(s, f, float(d.get(f, 0.0)))
    # importance sampling: {"param": distribution} drawn instead of the nominal
    mask = 0
    for name, spec in d.get("proposal", {}).items():
        j = DISTS.index(name)
        mask |= 1 << j
        s.proposal[j] = _dist(spec)
    s.is_mask = mask
    return s


def validate(d):
    return lib().aeb_validate(C.byref(scenario(d)))


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _torch():
    import torch
    return torch


def uniforms(seed, scenario_id, first, count, slot, attempt=0, device=True, stream=None):
    """(count, 2) float64 uniforms: a torch tensor on cuda:0 or a host numpy array."""
    if device:
        torch = _torch()
        out = torch.empty((count, 2), dtype=torch.float64, device="cuda")
        _check(lib().aeb_uniforms(seed, scenario_id, first, count, slot, attempt,
                                  C.c_void_p(out.data_ptr()), 1, _stream(stream)))
        return out
    out = np.empty((count, 2), dtype=np.float64)
    _check(lib().aeb_uniforms(seed, scenario_id, first, count, slot, attempt,
                              C.c_void_p(out.ctypes.data), 0, None))
    return out


def alloc_params(n, device=True, pinned=False):
    """Dict of the twelve float64 columns: cuda tensors, pinned host tensors or numpy arrays."""
    if device or pinned:
        torch = _torch()
        if device:
            return {c: torch.empty(n, dtype=torch.float64, device="cuda") for c in COLUMNS}
        return {c: torch.empty(n, dtype=torch.float64, pin_memory=True) for c in COLUMNS}
    return {c: np.empty(n, dtype=np.float64) for c in COLUMNS}


def _ptr(a):
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


def _params_struct(cols, n):
    """Columns by name; a missing trigger or log_weight column is passed as NULL
    (read as zeros)."""
    p = Params()
    for c in COLUMNS:
        setattr(p, c, _ptr(cols[c]) if c in cols or c not in ("trigger", "log_weight") else None)
    p.n = n
    return p


def sample_params(d, first=0, count=None, device=True, out=None, stream=None):
    """Draw parameter columns: on the GPU (device=True) or on the host cores."""
    if count is None:
        count = int(d["n_samples"]) - first
    if out is None:
        out = alloc_params(count, device=device)
    s = scenario(d)
    st = _stream(stream) if device else None
    _check(lib().aeb_sample_params(C.byref(s), first, count, C.byref(_params_struct(out, count)),
                                   1 if device else 0, st))
    return out


def alloc_outputs(n, weight=False):
    """Device output columns; weight=True adds the importance-sampling weights."""
    torch = _torch()
    out = {"dist": torch.empty(n, dtype=torch.float64, device="cuda"),
           "status": torch.empty(n, dtype=torch.uint8, device="cuda"),
           "steps": torch.empty(n, dtype=torch.int32, device="cuda"),
           "margin": torch.empty(n, dtype=torch.float64, device="cuda"),
           "v_impact": torch.empty(n, dtype=torch.float32, device="cuda")}
    if weight:
        out["weight"] = torch.empty(n, dtype=torch.float64, device="cuda")
    return out


def _outputs_struct(out):
    o = Outputs()
    for k in ("dist", "status", "steps", "margin", "v_impact"):
        setattr(o, k, out[k].data_ptr())
    o.weight = out["weight"].data_ptr() if "weight" in out else None
    o.n = out["dist"].numel()
    return o


def rollout(d, params=None, precision="fp64", out=None, stream=None):
    """Roll out every sample of scenario `d` on the GPU; params=None draws in-kernel."""
    n = int(d["n_samples"])
    if out is None:
        out = alloc_outputs(n, weight=bool(d.get("proposal")))
    s = scenario(d)
    pp = C.byref(_params_struct(params, n)) if params is not None else None
    _check(lib().aeb_rollout(C.byref(s), pp, PRECISIONS[precision],
                             C.byref(_outputs_struct(out)), _stream(stream)))
    return out


def rollout_noalloc(d, params=None, precision="fp64", out=None, stream=None):
    """rollout() through aeb_rollout_noalloc: the library's fixed per-device
    scratch array instead of its growable pool (`out` must be preallocated
    by callers that cannot allocate)."""
    n = int(d["n_samples"])
    if out is None:
        out = alloc_outputs(n, weight=bool(d.get("proposal")))
    s = scenario(d)
    pp = C.byref(_params_struct(params, n)) if params is not None else None
    _check(lib().aeb_rollout_noalloc(C.byref(s), pp, PRECISIONS[precision],
                                     C.byref(_outputs_struct(out)), _stream(stream)))
    return out


def reduce_request(risk=(), margin_q=(), grid=None):
    req = ReduceReq()
    req.n_risk = len(risk)
    for j, r in enumerate(risk):
        req.risk[j] = r
    req.n_margin_q = len(margin_q)
    for j, p in enumerate(margin_q):
        req.margin_q[j] = p
    if grid is not None:
        req.grid_lo, req.grid_hi, req.n_grid = float(grid[0]), float(grid[1]), int(grid[2])
    return req


def stats_dict(st, n_risk, n_mq, n_grid):
    return {
        "n": st.n, "n_collide": st.n_collide, "n_stop": st.n_stop, "n_impact": st.n_impact,
        "n_horizon": st.n_horizon, "n_boundary": st.n_boundary, "p_collision": st.p_collision,
        "mean_dist": st.mean_dist,
        "sd_dist": st.sd_dist, "dist_min": st.dist_min, "dist_max": st.dist_max,
        "headway": list(st.headway)[:n_risk], "margin_min": st.margin_min,
        "margin_mean": st.margin_mean, "margin_q": list(st.margin_q)[:n_mq],
        "v_impact_max": st.v_impact_max,
        "risk_count": np.array(st.risk_count[:n_grid], dtype=np.int64),
        "risk_p": np.array(st.risk_p[:n_grid], dtype=np.float64),
        "weighted": st.weighted, "p_collision_w": st.p_collision_w,
        "p_collision_se": st.p_collision_se, "weight_mean": st.weight_mean,
        "risk_pw": np.array(st.risk_pw[:n_grid], dtype=np.float64),
        "risk_se": np.array(st.risk_se[:n_grid], dtype=np.float64),
    }


def reduce(out, risk=(), margin_q=(), grid=None, stream=None):
    """Statistics of device outputs (blocks until they are on the host)."""
    req = reduce_request(risk, margin_q, grid)
    st = Stats()
    _check(lib().aeb_reduce(C.byref(_outputs_struct(out)), C.byref(req), C.byref(st),
                            _stream(stream)))
    return stats_dict(st, req.n_risk, req.n_margin_q, req.n_grid)


def reduce_fallbacks():
    """Reductions since load whose order statistics took the radix-select fallback."""
    c = C.c_uint64()
    _check(lib().aeb_reduce_fallbacks(C.byref(c)))
    return c.value


def ctl_approx_check(stream=None):
    """Largest errors of the controller screen's single-precision log2, sqrt,
    sin and cos over all their inputs, measured on the device, and the bounds
    the screen assumes: two 4-tuples (measured, bounds)."""
    m = (C.c_double * 4)()
    b = (C.c_double * 4)()
    _check(lib().aeb_ctl_approx_check(m, b, _stream(stream)))
    return tuple(m), tuple(b)


def ctl_math(a, x, device=False, stream=None):
    """The controller exact stage's (log a, sin x, cos x), evaluated by the
    library on the host (numpy float64 arrays in and out) or on the device
    (torch float64 CUDA tensors in and out)."""
    if device:
        torch = _torch()
        a = a.contiguous()
        x = x.contiguous()
        if a.dtype != torch.float64 or x.dtype != torch.float64 or a.numel() != x.numel():
            raise ValueError("ctl_math: two float64 tensors of one size")
        outs = [torch.empty_like(a) for _ in range(3)]
        _check(lib().aeb_ctl_math(a.data_ptr(), x.data_ptr(), a.numel(),
                                  *[o.data_ptr() for o in outs], 1, _stream(stream)))
        return tuple(outs)
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float64)
    x = np.ascontiguousarray(x, dtype=np.float64)
    if a.shape != x.shape:
        raise ValueError("ctl_math: two arrays of one size")
    outs = [np.empty_like(a) for _ in range(3)]
    _check(lib().aeb_ctl_math(a.ctypes.data, x.ctypes.data, a.size,
                              *[o.ctypes.data for o in outs], 0, None))
    return tuple(outs)


def valu_probe(fp32, threads, iters, stream=None):
    """Runs the counter-check kernel (aeb_valu_probe) and returns its output
    tensor (one sum per lane)."""
    torch = _torch()
    out = torch.empty(threads, dtype=torch.float32 if fp32 else torch.float64, device="cuda")
    _check(lib().aeb_valu_probe(1 if fp32 else 0, threads, iters, out.data_ptr(), _stream(stream)))
    return out


def timing_lanes():
    """Wavefront sample-steps of the last timed rollout on this thread: the
    launch's steps output summed over it is the lane efficiency."""
    w = C.c_uint64()
    _check(lib().aeb_timing_lanes(C.byref(w)))
    return w.value


def timing_enable(on=True):
    _check(lib().aeb_timing_enable(1 if on else 0))


def timing_last():
    """Duration (ms) of the last rollout's integration kernel on this thread."""
    ms = C.c_float()
    _check(lib().aeb_timing_last(C.byref(ms)))
    return ms.value


def batch_rollout(scns, precision="fp64", outs=None, stream=None):
    """Roll out every sample of several scenarios in one launch; returns a list of outputs."""
    k = len(scns)
    if outs is None:
        outs = [alloc_outputs(int(d["n_samples"]), weight=bool(d.get("proposal"))) for d in scns]
    sarr = (Scenario * k)(*[scenario(d) for d in scns])
    oarr = (Outputs * k)(*[_outputs_struct(o) for o in outs])
    _check(lib().aeb_batch_rollout(sarr, k, PRECISIONS[precision], oarr, _stream(stream)))
    return outs


def batch_reduce(outs, risk=(), margin_q=(), grid=None, stream=None):
    """Statistics of each output set of a batch (list of dicts)."""
    k = len(outs)
    req = reduce_request(risk, margin_q, grid)
    oarr = (Outputs * k)(*[_outputs_struct(o) for o in outs])
    st = (Stats * k)()
    _check(lib().aeb_batch_reduce(oarr, k, C.byref(req), st, _stream(stream)))
    return [stats_dict(st[j], req.n_risk, req.n_margin_q, req.n_grid) for j in range(k)]


class Server:
    """Continuous-batching evaluation server on the current device.  The arena
    is a torch uint8 tensor owned by this object (device memory handed to the
    library, which never frees it)."""

    def __init__(self, arena_bytes, precision="fp64", max_slots=256, n_streams=2, tick_us=200,
                 max_queue=4096, max_tick_samples=1 << 22, risk=(), margin_q=(), grid=None,
                 eager=False):
        torch = _torch()
        self.cfg = ServerCfg()
        self.cfg.flags = SERVE_EAGER if eager else 0
        self.cfg.max_slots = max_slots
        self.cfg.precision = PRECISIONS[precision]
        self.cfg.n_streams = n_streams
        self.cfg.tick_us = tick_us
        self.cfg.max_queue = max_queue
        self.cfg.max_tick_samples = max_tick_samples
        self.cfg.req = reduce_request(risk, margin_q, grid)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
        self.cfg.arena = self.arena.data_ptr()
        self.cfg.arena_bytes = int(arena_bytes)
        torch.cuda.synchronize()
        h = C.c_void_p()
        _check(lib().aeb_server_create(C.byref(self.cfg), C.byref(h)))
        self.h = h

    @staticmethod
    def fixed_bytes(precision="fp64", max_slots=256, n_streams=2, max_tick_samples=1 << 22,
                    risk=(), margin_q=(), grid=None):
        cfg = ServerCfg(max_slots=max_slots, precision=PRECISIONS[precision],
                        n_streams=n_streams, tick_us=0, max_queue=1,
                        max_tick_samples=max_tick_samples,
                        req=reduce_request(risk, margin_q, grid))
        b = C.c_uint64()
        _check(lib().aeb_server_fixed_bytes(C.byref(cfg), C.byref(b)))
        return b.value

    def footprint(self, n_samples):
        b = C.c_uint64()
        _check(lib().aeb_serve_footprint(C.byref(self.cfg), int(n_samples), C.byref(b)))
        return b.value

    def submit(self, d, deadline=0.530):
        """Queue one scenario; returns its ticket (raises AebError on refusal)."""
        t = C.c_uint64()
        _check(lib().aeb_serve_submit(self.h, C.byref(scenario(d)), float(deadline),
                                      C.byref(t)))
        return t.value

    def try_submit(self, d, deadline=0.530):
        """(return code, ticket) without raising."""
        t = C.c_uint64()
        rc = lib().aeb_serve_submit(self.h, C.byref(scenario(d)), float(deadline), C.byref(t))
        return rc, t.value

    def poll(self, ticket):
        """None while pending; else (stats dict, timing dict).  Raises on errors."""
        st, tm = Stats(), ReqTiming()
        rc = lib().aeb_serve_poll(self.h, int(ticket), C.byref(st), C.byref(tm))
        if rc == EAGAIN:
            return None
        _check(rc)
        req = self.cfg.req
        timing = {"arrive": tm.arrive, "admit": tm.admit, "start": tm.start, "done": tm.done,
                  "missed": bool(tm.missed)}
        return stats_dict(st, req.n_risk, req.n_margin_q, req.n_grid), timing

    def wait(self, ticket, timeout=60.0, sleep=1e-4):
        import time
        t_end = time.monotonic() + timeout
        while True:
            r = self.poll(ticket)
            if r is not None:
                return r
            if time.monotonic() > t_end:
                raise TimeoutError(f"ticket {ticket} still pending after {timeout} s")
            time.sleep(sleep)

    def info(self):
        inf = ServerInfo()
        _check(lib().aeb_server_info_get(self.h, C.byref(inf)))
        return {f: getattr(inf, f) for f, _ in ServerInfo._fields_}

    def close(self):
        if getattr(self, "h", None):
            _check(lib().aeb_server_destroy(self.h))
            self.h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """A recorded rollout (+ statistics) of one scenario, or of a fixed mix of
    scenarios in one batched launch, replayed with one launch.  Outputs are
    the device tensors given (or allocated here); statistics land in pinned
    host memory owned by this object."""

    def __init__(self, d, params=None, precision="fp64", out=None, risk=(), margin_q=(),
                 grid=None, stats=True, batch=False):
        torch = _torch()
        scns = list(d) if batch else [d]
        k = len(scns)
        if out is None:
            out = [alloc_outputs(int(x["n_samples"]), weight=bool(x.get("proposal")))
                   for x in scns] if batch else \
                alloc_outputs(int(scns[0]["n_samples"]), weight=bool(scns[0].get("proposal")))
        self.out = out
        outs = out if batch else [out]
        self.req = reduce_request(risk, margin_q, grid) if stats else None
        self._pin = torch.empty(C.sizeof(Stats) * k, dtype=torch.uint8, pin_memory=True)
        self._stats = (Stats * k).from_address(self._pin.data_ptr())
        h = C.c_void_p()
        req = C.byref(self.req) if stats else None
        if batch:
            sarr = (Scenario * k)(*[scenario(x) for x in scns])
            oarr = (Outputs * k)(*[_outputs_struct(o) for o in outs])
            _check(lib().aeb_graph_create_batch(sarr, k, PRECISIONS[precision], oarr, req,
                                                self._pin.data_ptr(), C.byref(h)))
        else:
            prm = C.byref(_params_struct(params, int(scns[0]["n_samples"]))) if params else None
            _check(lib().aeb_graph_create(C.byref(scenario(scns[0])), prm,
                                          PRECISIONS[precision],
                                          C.byref(_outputs_struct(outs[0])), req,
                                          self._pin.data_ptr(), C.byref(h)))
        self.k, self.batch, self.h = k, batch, h

    def launch(self, stream=None):
        _check(lib().aeb_graph_launch(self.h, _stream(stream)))

    def finish(self, stream=None):
        """Wait for the stream; returns the statistics (list for a batch)."""
        _check(lib().aeb_graph_finish(self.h, _stream(stream)))
        if self.req is None:
            return None
        r = self.req
        st = [stats_dict(self._stats[j], r.n_risk, r.n_margin_q, r.n_grid) for j in range(self.k)]
        return st if self.batch else st[0]

    def close(self):
        if getattr(self, "h", None):
            _check(lib().aeb_graph_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MixGraph:
    """One recording that replays any mix of up to max_scn scenarios of the
    kind of `kind` with at most max_samples samples in all (the batched
    rollout, plus the statistics of each scenario unless stats=False)."""

    def __init__(self, kind, precision="fp64", max_scn=16, max_samples=1 << 20, risk=(),
                 margin_q=(), grid=None, stats=True):
        self.req = reduce_request(risk, margin_q, grid) if stats else None
        h = C.c_void_p()
        _check(lib().aeb_graph_create_mix(C.byref(scenario(kind)), PRECISIONS[precision],
                                          int(max_scn), int(max_samples),
                                          C.byref(self.req) if stats else None, C.byref(h)))
        self.h = h
        self._st = None

    def launch(self, scns, outs=None, stream=None):
        """Replay for the scenarios `scns` (outputs allocated if not given);
        returns the outputs."""
        k = len(scns)
        if outs is None:
            outs = [alloc_outputs(int(d["n_samples"]), weight=bool(d.get("proposal")))
                    for d in scns]
        self._sarr = (Scenario * k)(*[scenario(d) for d in scns])
        self._oarr = (Outputs * k)(*[_outputs_struct(o) for o in outs])
        self._st = (Stats * k)() if self.req is not None else None
        _check(lib().aeb_graph_launch_mix(self.h, self._sarr, k, self._oarr,
                                          C.cast(self._st, C.c_void_p) if self._st else None,
                                          _stream(stream)))
        self.k = k
        return outs

    def finish(self, stream=None):
        """Wait for the replay; returns the statistics (list) or None."""
        _check(lib().aeb_graph_finish(self.h, _stream(stream)))
        if self.req is None:
            return None
        r = self.req
        return [stats_dict(self._st[j], r.n_risk, r.n_margin_q, r.n_grid) for j in range(self.k)]

    def close(self):
        if getattr(self, "h", None):
            _check(lib().aeb_graph_destroy(self.h))
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def tune_get(precision="fp64", obstacle="stationary"):
    """(k, block, waves_per_simd, samples_per_thread) of the integration kernel's launch."""
    t = TuneShape()
    _check(lib().aeb_tune_get(PRECISIONS[precision], OBSTACLES[obstacle], C.byref(t)))
    return t.k, t.block, t.waves_per_simd, t.samples_per_thread


def tune_set(precision, obstacle, k, block, waves_per_simd, samples_per_thread=1):
    t = TuneShape(k, block, waves_per_simd, samples_per_thread)
    _check(lib().aeb_tune_set(PRECISIONS[precision], OBSTACLES[obstacle], C.byref(t)))


def tune_results(precision="fp64", obstacle="stationary", max_n=256):
    """The last autotune's candidates, fastest first: [((k, block, waves, spt), ms), ...]."""
    shapes = (TuneShape * max_n)()
    ms = (C.c_float * max_n)()
    cnt = C.c_int()
    _check(lib().aeb_tune_results(PRECISIONS[precision], OBSTACLES[obstacle], shapes, ms, max_n,
                                  C.byref(cnt)))
    return [((t.k, t.block, t.waves_per_simd, t.samples_per_thread), ms[j])
            for j, t in enumerate(shapes[:min(cnt.value, max_n)])]


def tune_load(path):
    _check(lib().aeb_tune_load(os.fsencode(path)))


def autotune(d, precision="fp64", cache_path=None, stream=None):
    """Time every launch shape on scenario d; keeps the fastest; returns its ms."""
    ms = C.c_float()
    _check(lib().aeb_autotune(C.byref(scenario(d)), PRECISIONS[precision],
                              os.fsencode(cache_path) if cache_path else None, _stream(stream),
                              C.byref(ms)))
    return ms.value
