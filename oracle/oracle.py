"""ctypes front end of the FP64 reference (test infrastructure only).

Scenarios are plain dicts (see ``SCENARIO_KEYS``); distributions are tuples
``("const", x)``, ``("uniform", a, b)``, ``("normal", mean, sd)`` or
``("trunc_normal", mean, sd, lo, hi)``.  Every function here marshals
arguments and calls the C reference in ``aeb_oracle.c``; the arithmetic of the
model lives only there.
"""
import ctypes as C
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from . import build as _build

COLUMNS = ("v0", "mu", "mass", "grade", "sin_grade", "cos_grade", "cda", "crr", "tau",
           "gap", "lead_decel", "trigger", "log_weight")
DISTS = ("v0", "mu", "mass", "grade", "cda", "crr", "tau", "gap", "lead_decel")
SLOTS = {name: k for k, name in enumerate(DISTS)}
SLOTS.update({"latency": 9, "occlusion": 10, "detect": 11, "control": 12})
# perception (absent from a scenario dict: no perception)
PERCEPTION_DEFAULTS = {"latency": ("const", 0.0), "occlusion": ("const", 0.0),
                       "frame_period": 0.0, "p_dropout": 0.0, "confirm": 1}
# closed-loop controller (absent: open loop)
CONTROL_FIELDS = ("ctl_period", "ttc_warn", "ttc_brake", "a_warn", "noise_gap", "noise_v")
INTEGRATORS = {"euler": 0, "rk4": 1}
OBSTACLES = {"none": 0, "stationary": 1, "lead": 2}
DIST_KINDS = {"const": 0, "uniform": 1, "normal": 2, "trunc_normal": 3}

END_STOP, END_IMPACT, END_HORIZON, COLLIDED = 1, 2, 3, 4
OK, EINVAL = 0, -1


class Dist(C.Structure):
    _fields_ = [("kind", C.c_int32), ("pad", C.c_int32), ("p0", C.c_double),
                ("p1", C.c_double), ("lo", C.c_double), ("hi", C.c_double)]


class Scenario(C.Structure):
    _fields_ = ([("seed", C.c_uint64), ("scenario_id", C.c_uint64), ("n_samples", C.c_int64),
                 ("integrator", C.c_int32), ("obstacle", C.c_int32),
                 ("impact_exit", C.c_int32), ("nofma", C.c_int32)]
                + [(f, C.c_double) for f in ("dt", "horizon", "dead_time", "a_cmd", "g", "rho",
                                             "h_cog", "wheelbase")]
                + [(f, Dist) for f in DISTS]
                + [("latency", Dist), ("occlusion", Dist), ("frame_period", C.c_double),
                   ("p_dropout", C.c_double), ("confirm", C.c_int32), ("pad2", C.c_int32)]
                + [(f, C.c_double) for f in CONTROL_FIELDS]
                + [("is_mask", C.c_int32), ("pad3", C.c_int32), ("proposal", Dist * 9)])


class ReduceReq(C.Structure):
    _fields_ = [("n_risk", C.c_int32), ("n_margin_q", C.c_int32), ("n_grid", C.c_int32),
                ("pad", C.c_int32), ("risk", C.c_double * 16), ("margin_q", C.c_double * 4),
                ("grid_lo", C.c_double), ("grid_hi", C.c_double)]


class Stats(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_collide", C.c_int64), ("n_stop", C.c_int64),
                ("n_impact", C.c_int64), ("n_horizon", C.c_int64),
                ("p_collision", C.c_double), ("mean_dist", C.c_double), ("sd_dist", C.c_double),
                ("dist_min", C.c_double), ("dist_max", C.c_double),
                ("headway", C.c_double * 16), ("margin_min", C.c_double),
                ("margin_mean", C.c_double), ("margin_q", C.c_double * 4),
                ("v_impact_max", C.c_float), ("pad", C.c_int32),
                ("risk_count", C.c_int64 * 1024), ("risk_p", C.c_double * 1024)]


_lib = None


def lib():
    """Load the reference library, compiling it first if it is missing or stale."""
    global _lib
    if _lib is None:
        path = _build.build(force=False)
        L = C.CDLL(path)
        P = C.POINTER
        L.orc_validate.argtypes = [P(Scenario)]
        L.orc_philox4x32_10.argtypes = [P(C.c_uint32), P(C.c_uint32), P(C.c_uint32)]
        L.orc_uniforms.argtypes = [C.c_uint64, C.c_uint64, C.c_int64, C.c_int64, C.c_uint32,
                                   C.c_uint32, P(C.c_double)]
        L.orc_sample_range.argtypes = [P(Scenario), C.c_int64, C.c_int64, P(P(C.c_double))]
        L.orc_run_range.argtypes = [P(Scenario), C.c_int64, C.c_int64, P(C.c_double),
                                    P(C.c_uint8), P(C.c_int32), P(C.c_double), P(C.c_float)]
        L.orc_rollout_given.argtypes = [P(Scenario), P(P(C.c_double)), C.c_int64, C.c_int,
                                        P(C.c_double), P(C.c_uint8), P(C.c_int32),
                                        P(C.c_double), P(C.c_float)]
        L.orc_weighted_risk.argtypes = [P(C.c_double), P(C.c_uint8), P(C.c_double), C.c_int64,
                                         C.c_double, C.c_double, C.c_int32, P(C.c_double),
                                         P(C.c_double), P(C.c_double), P(C.c_double)]
        L.orc_reduce.argtypes = [P(C.c_double), P(C.c_uint8), P(C.c_double), P(C.c_float),
                                 C.c_int64, P(ReduceReq), P(Stats)]
        _lib = L
    return _lib


def _dist(spec):
    d = Dist()
    kind = spec[0]
    d.kind = DIST_KINDS[kind]
    vals = list(spec[1:]) + [0.0] * (4 - len(spec[1:]))
    d.p0, d.p1, d.lo, d.hi = (float(v) for v in vals)
    if kind == "const":
        d.p1 = 0.0
    return d


def scenario(d):
    """Marshal a scenario dict into the reference's struct."""
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
        j = SLOTS[name]
        mask |= 1 << j
        s.proposal[j] = _dist(spec)
    s.is_mask = mask
    return s


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def validate(d):
    return lib().orc_validate(C.byref(scenario(d)))


def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(v) & 0xFFFFFFFF for v in ctr])
    k = (C.c_uint32 * 2)(*[int(v) & 0xFFFFFFFF for v in key])
    o = (C.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return [int(v) for v in o]


def uniforms(seed, scenario_id, first, count, slot, attempt=0):
    """(count, 2) array of the two uniforms of each generator call."""
    out = np.empty(2 * count, dtype=np.float64)
    rc = lib().orc_uniforms(seed, scenario_id, first, count, slot, attempt, _dptr(out))
    if rc != OK:
        raise ValueError("orc_uniforms rejected its arguments")
    return out.reshape(count, 2)


def sample(d, first=0, count=None):
    """Dict of the twelve parameter columns for samples [first, first+count)."""
    if count is None:
        count = int(d["n_samples"]) - first
    cols = [np.empty(count, dtype=np.float64) for _ in COLUMNS]
    arr = (C.POINTER(C.c_double) * 13)(*[_dptr(c) for c in cols])
    rc = lib().orc_sample_range(C.byref(scenario(d)), first, count, arr)
    if rc != OK:
        raise ValueError("orc_sample_range rejected its arguments")
    return dict(zip(COLUMNS, cols))


def _alloc_out(n):
    return {"dist": np.empty(n, np.float64), "status": np.empty(n, np.uint8),
            "steps": np.empty(n, np.int32), "margin": np.empty(n, np.float64),
            "v_impact": np.empty(n, np.float32)}


def _out_ptrs(o, lo, hi):
    P = C.POINTER
    return (o["dist"][lo:hi].ctypes.data_as(P(C.c_double)),
            o["status"][lo:hi].ctypes.data_as(P(C.c_uint8)),
            o["steps"][lo:hi].ctypes.data_as(P(C.c_int32)),
            o["margin"][lo:hi].ctypes.data_as(P(C.c_double)),
            o["v_impact"][lo:hi].ctypes.data_as(P(C.c_float)))


def run(d, first=0, count=None, threads=1):
    """Sample and roll out [first, first+count); optional static split over threads."""
    if count is None:
        count = int(d["n_samples"]) - first
    s = scenario(d)
    if lib().orc_validate(C.byref(s)) != OK:
        raise ValueError("scenario rejected by the reference validator")
    o = _alloc_out(count)
    threads = max(1, min(int(threads), count if count > 0 else 1))
    bounds = [count * t // threads for t in range(threads + 1)]

    def work(t):
        lo, hi = bounds[t], bounds[t + 1]
        rc = lib().orc_run_range(C.byref(s), first + lo, hi - lo, *_out_ptrs(o, lo, hi))
        if rc != OK:
            raise ValueError("orc_run_range failed")

    if threads == 1:
        work(0)
    else:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, range(threads)))
    return o


def rollout_given(d, cols, clamp_state=False):
    """Roll out caller-given parameter columns (dict keyed by COLUMNS)."""
    n = len(cols["v0"])
    arrs = [np.ascontiguousarray(cols[c] if c in cols else np.zeros(n), dtype=np.float64)
            for c in COLUMNS]
    arr = (C.POINTER(C.c_double) * 13)(*[_dptr(a) for a in arrs])
    o = _alloc_out(n)
    rc = lib().orc_rollout_given(C.byref(scenario(d)), arr, n, int(bool(clamp_state)),
                                 *_out_ptrs(o, 0, n))
    if rc != OK:
        raise ValueError("orc_rollout_given failed")
    return o


def weighted_risk(out, weight, grid):
    """Importance-sampling estimates: P(D > H0_j) and its standard error on the
    grid (lo, hi, n), and P(collision) with its standard error."""
    n = len(out["dist"])
    lo, hi, ng = float(grid[0]), float(grid[1]), int(grid[2])
    p = np.empty(ng, np.float64)
    se = np.empty(ng, np.float64)
    pc, pcs = C.c_double(), C.c_double()
    dist = np.ascontiguousarray(out["dist"], np.float64)
    status = np.ascontiguousarray(out["status"], np.uint8)
    w = np.ascontiguousarray(weight, np.float64)
    rc = lib().orc_weighted_risk(_dptr(dist), status.ctypes.data_as(C.POINTER(C.c_uint8)),
                                 _dptr(w), n, lo, hi, ng, _dptr(p), _dptr(se), C.byref(pc),
                                 C.byref(pcs))
    if rc != OK:
        raise ValueError("orc_weighted_risk rejected its arguments")
    return {"p": p, "se": se, "p_collision": pc.value, "p_collision_se": pcs.value}


def reduce(out, risk=(), margin_q=(), grid=None):
    """Sort-based statistics of one rollout batch; grid = (lo, hi, n_points)."""
    n = len(out["dist"])
    req = ReduceReq()
    req.n_risk = len(risk)
    for j, r in enumerate(risk):
        req.risk[j] = r
    req.n_margin_q = len(margin_q)
    for j, p in enumerate(margin_q):
        req.margin_q[j] = p
    if grid is not None:
        req.grid_lo, req.grid_hi, req.n_grid = float(grid[0]), float(grid[1]), int(grid[2])
    st = Stats()
    P = C.POINTER
    dist = np.ascontiguousarray(out["dist"], np.float64)
    status = np.ascontiguousarray(out["status"], np.uint8)
    margin = np.ascontiguousarray(out["margin"], np.float64)
    vimp = np.ascontiguousarray(out["v_impact"], np.float32)
    rc = lib().orc_reduce(_dptr(dist), status.ctypes.data_as(P(C.c_uint8)), _dptr(margin),
                          vimp.ctypes.data_as(P(C.c_float)), n, C.byref(req), C.byref(st))
    if rc != OK:
        raise ValueError("orc_reduce rejected its arguments")
    ng = req.n_grid
    return {
        "n": st.n, "n_collide": st.n_collide, "n_stop": st.n_stop, "n_impact": st.n_impact,
        "n_horizon": st.n_horizon, "p_collision": st.p_collision, "mean_dist": st.mean_dist,
        "sd_dist": st.sd_dist, "dist_min": st.dist_min, "dist_max": st.dist_max,
        "headway": list(st.headway)[:len(risk)], "margin_min": st.margin_min,
        "margin_mean": st.margin_mean, "margin_q": list(st.margin_q)[:len(margin_q)],
        "v_impact_max": st.v_impact_max,
        "risk_count": np.array(st.risk_count[:ng], dtype=np.int64),
        "risk_p": np.array(st.risk_p[:ng], dtype=np.float64),
    }


def host_threads():
    """Threads the reference may use on this host."""
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1
