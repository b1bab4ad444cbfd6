// abi.cpp -- the C ABI of include/aeb.h: argument checking, scenario
// validation, the host-side sampler of the plain method (Sec. IV-C) and
// dispatch to the kernel launchers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include <sched.h>

#include "aeb.h"
#include "aeb_common.h"
#include "ctl_math.h"
#include "aeb_runtime.h"

namespace aeb {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// ---------------------------------------------------------------------------
// scratch pool
//
// Device blocks per device, each with an event recorded on the stream of the
// call that last used it.  A call takes blocks inside a ScratchScope: a block
// no other call holds, preferring one last used on the same stream (stream
// order protects it) or one whose event has completed; otherwise a new block,
// or, once the pool holds POOL_SOFT blocks, a fitting block whose event the
// call's stream waits for on the device.  A block is freed (to grow it) only
// when no call holds it and after its event has completed, so no queued work
// can touch freed memory.
// ---------------------------------------------------------------------------
namespace {
struct Block {
  void* ptr = nullptr;
  size_t bytes = 0;
  hipEvent_t ev = nullptr;     // recorded on `last` when the last holder released it
  hipStream_t last = nullptr;
  bool busy = false;           // held by a live scope
  bool fenced = false;         // ev has been recorded
};
constexpr int MAX_DEV = 64;
constexpr size_t POOL_SOFT = 8;
std::mutex g_pool_mu;
std::vector<Block*> g_pool[MAX_DEV];

struct Timing {
  bool on = false;
  bool recorded = false;
  int dev = -1;
  hipEvent_t start = nullptr, stop = nullptr;
  unsigned long long* lanes = nullptr;  // lane accounting of the timed launch (device)
  bool lanes_armed = false;  // the next timed launch counts lanes
  bool lanes_valid = false;  // the last timed launch counted lanes
};
thread_local Timing g_timing;
thread_local ScratchScope* g_scope = nullptr;

bool block_idle(const Block* b, hipStream_t st) {
  if (!b->fenced || b->last == st) return true;
  return hipEventQuery(b->ev) == hipSuccess;
}

// Called with g_pool_mu held.  Returns a block of at least `bytes` for work on
// `st`, marked busy, or nullptr with the error set.
Block* acquire(int dev, size_t bytes, hipStream_t st) {
  std::vector<Block*>& pool = g_pool[dev];
  Block* pick = nullptr;
  for (Block* b : pool)  // a fitting block that is idle for this stream, smallest first
    if (!b->busy && b->bytes >= bytes && block_idle(b, st) && (!pick || b->bytes < pick->bytes))
      pick = b;
  bool wait = false;
  if (!pick && pool.size() >= POOL_SOFT) {
    for (Block* b : pool)  // a fitting block still in flight on another stream
      if (!b->busy && b->bytes >= bytes && (!pick || b->bytes < pick->bytes)) pick = b;
    wait = pick != nullptr;
  }
  if (!pick) {
    // grow: replace the smallest block nobody holds -- below POOL_SOFT blocks
    // only one idle for this stream, beyond it any (after its last work) --
    // or add one
    Block* old = nullptr;
    const bool full = pool.size() >= POOL_SOFT;
    for (Block* b : pool)
      if (!b->busy && (full || block_idle(b, st)) && (!old || b->bytes < old->bytes)) old = b;
    size_t want = bytes < (size_t(1) << 20) ? (size_t(1) << 20) : bytes;
    want = (want + 4095) & ~size_t(4095);
    if (old) {
      if ((old->fenced && hipEventSynchronize(old->ev) != hipSuccess) || hipFree(old->ptr) != hipSuccess) {
        set_error("scratch: could not release a pool block");
        return nullptr;
      }
      old->ptr = nullptr;
      old->bytes = 0;
      old->fenced = false;
      pick = old;
    } else {
      pick = new (std::nothrow) Block;
      if (!pick) {
        set_error("scratch: host allocation failed");
        return nullptr;
      }
      if (hipEventCreateWithFlags(&pick->ev, hipEventDisableTiming) != hipSuccess) {
        delete pick;
        set_error("scratch: hipEventCreate failed");
        return nullptr;
      }
      pool.push_back(pick);
    }
    if (hipMalloc(&pick->ptr, want) != hipSuccess) {
      pick->ptr = nullptr;
      set_error("scratch: hipMalloc of " + std::to_string(want) + " bytes failed");
      return nullptr;
    }
    pick->bytes = want;
  }
  if (wait && hipStreamWaitEvent(st, pick->ev, 0) != hipSuccess) {
    set_error("scratch: hipStreamWaitEvent failed");
    return nullptr;
  }
  pick->busy = true;
  return pick;
}

// Called with g_pool_mu held: fence the block's work on `st` and hand it back.
void release(Block* b, hipStream_t st) {
  if (hipEventRecord(b->ev, st) == hipSuccess) {
    b->fenced = true;
    b->last = st;
  } else {
    // no fence: make sure its work is done before anyone else takes it
    (void)hipStreamSynchronize(st);
    b->fenced = false;
  }
  b->busy = false;
}
}  // namespace

ScratchScope::ScratchScope(hipStream_t st) : st_(st), outer_(g_scope) {
  if (hipGetDevice(&dev_) != hipSuccess || dev_ < 0 || dev_ >= MAX_DEV) dev_ = -1;
  g_scope = this;
}

ScratchScope::~ScratchScope() {
  {
    std::lock_guard<std::mutex> lock(g_pool_mu);
    for (void* h : held_)
      if (h) release(static_cast<Block*>(h), st_);
  }
  g_scope = outer_;
}

void* scratch_slot(int slot, size_t bytes, hipStream_t stream) {
  ScratchScope* sc = g_scope;
  if (!sc || sc->st_ != stream || sc->dev_ < 0 || slot < 0 || slot >= ScratchScope::SLOTS) {
    set_error("scratch: no scratch scope for this call (internal error)");
    return nullptr;
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cap) == hipSuccess && cap != hipStreamCaptureStatusNone) {
    set_error("scratch: the pool's blocks are fenced by events and cannot be captured; record "
              "graphs with aeb_graph_create");
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_pool_mu);
  Block* have = static_cast<Block*>(sc->held_[slot]);
  if (have && have->bytes >= bytes) return have->ptr;
  if (have) {
    release(have, stream);
    sc->held_[slot] = nullptr;
  }
  Block* b = acquire(sc->dev_, bytes, stream);
  if (!b) return nullptr;
  sc->held_[slot] = b;
  return b->ptr;
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
static bool dist_ok(const aeb_dist& d) {
  switch (d.kind) {
    case AEB_DIST_CONST:
      return std::isfinite(d.p0);
    case AEB_DIST_UNIFORM:
      return std::isfinite(d.p0) && std::isfinite(d.p1) && d.p0 <= d.p1;
    case AEB_DIST_NORMAL:
      return std::isfinite(d.p0) && std::isfinite(d.p1) && d.p1 >= 0.0;
    case AEB_DIST_TRUNC_NORMAL:
      return std::isfinite(d.p0) && std::isfinite(d.p1) && d.p1 >= 0.0 && std::isfinite(d.lo) &&
             std::isfinite(d.hi) && d.lo < d.hi;
    default:
      return false;
  }
}

// lowest value a distribution can produce
static double support_min(const aeb_dist& d) {
  switch (d.kind) {
    case AEB_DIST_CONST:
    case AEB_DIST_UNIFORM:
      return d.p0;
    case AEB_DIST_TRUNC_NORMAL:
      return d.lo;
    default:
      return d.p1 == 0.0 ? d.p0 : -INFINITY;
  }
}

int validate(const aeb_scenario& s) {
  if (s.n_samples < 1 || s.n_samples > 0x7fffffffLL) return fail(AEB_EINVAL, "n_samples out of [1, 2^31-1]");
  if (s.integrator != AEB_EULER && s.integrator != AEB_RK4) return fail(AEB_EINVAL, "unknown integrator");
  if (s.obstacle < AEB_OBS_NONE || s.obstacle > AEB_OBS_LEAD) return fail(AEB_EINVAL, "unknown obstacle");
  if (s.integrator == AEB_RK4 && s.obstacle == AEB_OBS_LEAD)
    return fail(AEB_EINVAL, "the lead-vehicle model needs the Euler integrator");
  if (s.impact_exit != 0 && s.impact_exit != 1) return fail(AEB_EINVAL, "impact_exit must be 0 or 1");
  if (s.nofma != 0 && s.nofma != 1) return fail(AEB_EINVAL, "nofma must be 0 or 1");
  if (!(s.dt > 0.0) || !std::isfinite(s.dt)) return fail(AEB_EINVAL, "dt must be positive");
  if (!(s.horizon > 0.0) || !std::isfinite(s.horizon)) return fail(AEB_EINVAL, "horizon must be positive");
  if (!(s.dead_time >= 0.0) || !std::isfinite(s.dead_time)) return fail(AEB_EINVAL, "dead_time must be >= 0");
  double steps = s.horizon / s.dt;
  if (!(steps >= 1.0) || steps > 2147483647.0) return fail(AEB_EINVAL, "horizon/dt out of [1, 2^31-1]");
  if (!std::isfinite(s.a_cmd) || !std::isfinite(s.g) || !std::isfinite(s.rho) || !std::isfinite(s.h_cog))
    return fail(AEB_EINVAL, "non-finite physical constant");
  if (!(s.wheelbase > 0.0) || !std::isfinite(s.wheelbase)) return fail(AEB_EINVAL, "wheelbase must be positive");
  const aeb_dist* all[9] = {&s.v0, &s.mu, &s.mass, &s.grade, &s.cda, &s.crr, &s.tau, &s.gap, &s.lead_decel};
  static const char* names[9] = {"v0", "mu", "mass", "grade", "cda", "crr", "tau", "gap", "lead_decel"};
  for (int k = 0; k < 9; ++k)
    if (!dist_ok(*all[k])) return fail(AEB_EINVAL, std::string("invalid distribution for ") + names[k]);
  if (!dist_ok(s.latency)) return fail(AEB_EINVAL, "invalid distribution for latency");
  if (!dist_ok(s.occlusion)) return fail(AEB_EINVAL, "invalid distribution for occlusion");
  if (!(s.frame_period >= 0.0) || !std::isfinite(s.frame_period))
    return fail(AEB_EINVAL, "frame_period must be >= 0 and finite");
  if (s.frame_period > 0.0 && !(s.horizon / s.frame_period <= 1.0e6))
    return fail(AEB_EINVAL, "more than 1e6 sensing frames over the horizon");
  if (!(s.p_dropout >= 0.0 && s.p_dropout < 1.0)) return fail(AEB_EINVAL, "p_dropout out of [0, 1)");
  if (s.confirm < 1 || s.confirm > 64) return fail(AEB_EINVAL, "confirm out of [1, 64]");
  if (!(s.ctl_period >= 0.0) || !std::isfinite(s.ctl_period))
    return fail(AEB_EINVAL, "ctl_period must be >= 0 and finite");
  if (s.ctl_period > 0.0) {
    const long long per = std::llround(s.ctl_period / s.dt);
    if (per < 1) return fail(AEB_EINVAL, "ctl_period shorter than half a step");
    if (!(s.horizon / s.dt / static_cast<double>(per) < 16777216.0))
      return fail(AEB_EINVAL, "2^24 or more controller decisions over the horizon");
    if (s.obstacle == AEB_OBS_NONE) return fail(AEB_EINVAL, "the controller needs an obstacle");
    if (perception_on(s)) return fail(AEB_EINVAL, "the controller and perception exclude each other");
    if (!(s.ttc_warn >= 0.0) || !(s.ttc_brake >= 0.0))
      return fail(AEB_EINVAL, "TTC thresholds must be >= 0");
    if (!std::isfinite(s.a_warn) || !(s.a_cmd <= s.a_warn && s.a_warn <= 0.0))
      return fail(AEB_EINVAL, "a_warn must lie in [a_cmd, 0]");
    if (!(s.noise_gap >= 0.0) || !std::isfinite(s.noise_gap) || !(s.noise_v >= 0.0) ||
        !std::isfinite(s.noise_v))
      return fail(AEB_EINVAL, "measurement noise sds must be >= 0 and finite");
  }
  if (s.is_mask & ~0x1BF)
    return fail(AEB_EINVAL, "importance sampling covers normal parameters other than tau");
  for (int j = 0; j < 9; ++j) {
    if (!((s.is_mask >> j) & 1)) continue;
    const aeb_dist& q = s.proposal[j];
    if (all[j]->kind != AEB_DIST_NORMAL || q.kind != AEB_DIST_NORMAL || !(all[j]->p1 > 0.0) ||
        !(q.p1 > 0.0) || !dist_ok(q))
      return fail(AEB_EINVAL, std::string("importance sampling of ") + names[j] +
                                  " needs normal distribution and proposal with sd > 0");
  }
  double tmin = support_min(s.tau);
  if (!(tmin > 0.0)) return fail(AEB_EINVAL, "tau distribution can reach 0");
  if (s.integrator == AEB_EULER && tmin < s.dt)
    return fail(AEB_EINVAL, "explicit Euler needs tau >= dt for every sample");
  return AEB_OK;
}

bool timing_suspend(bool off) {
  const bool was = g_timing.on;
  if (off) g_timing.on = false;
  return was;
}

void timing_resume(bool was) { g_timing.on = was; }

// the events and the lane counters of the current device (made on first use)
static bool timing_ready() {
  Timing& t = g_timing;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  if (t.dev != dev) {
    if (t.start) (void)hipEventDestroy(t.start);
    if (t.stop) (void)hipEventDestroy(t.stop);
    if (t.lanes) (void)hipFree(t.lanes);
    t.start = t.stop = nullptr;
    t.lanes = nullptr;
    t.dev = -1;
    if (hipEventCreate(&t.start) != hipSuccess || hipEventCreate(&t.stop) != hipSuccess ||
        hipMalloc(&t.lanes, sizeof(unsigned long long)) != hipSuccess)
      return false;
    t.dev = dev;
  }
  return true;
}

unsigned long long* timing_lanes() {
  if (!g_timing.on || !timing_ready()) return nullptr;
  g_timing.lanes_armed = true;
  return g_timing.lanes;
}

void timing_begin(hipStream_t stream) {
  Timing& t = g_timing;
  if (!t.on || !timing_ready()) return;
  // a launch that did not arm the counters (the checked kernels) has none
  t.lanes_valid = t.lanes_armed;
  t.lanes_armed = false;
  (void)hipEventRecord(t.start, stream);
}

void timing_end(hipStream_t stream) {
  Timing& t = g_timing;
  if (!t.on || !t.stop) return;
  if (hipEventRecord(t.stop, stream) == hipSuccess) t.recorded = true;
}

int64_t horizon_steps(const aeb_scenario& s) { return std::llround(s.horizon / s.dt); }
int64_t dead_steps(const aeb_scenario& s) { return std::llround(s.dead_time / s.dt); }

static int host_threads() {
  cpu_set_t set;
  if (sched_getaffinity(0, sizeof(set), &set) == 0) {
    int c = CPU_COUNT(&set);
    if (c > 0) return c;
  }
  unsigned h = std::thread::hardware_concurrency();
  return h ? static_cast<int>(h) : 1;
}

static bool params_complete(const aeb_params* p) {
  return p && p->v0 && p->mu && p->mass && p->grade && p->sin_grade && p->cos_grade && p->cda &&
         p->crr && p->tau && p->gap && p->lead_decel;
}

static bool outputs_complete(const aeb_outputs* o) {
  return o && o->dist && o->status && o->steps && o->margin && o->v_impact;
}

}  // namespace aeb

using namespace aeb;

namespace aeb {

int rollout_args(const aeb_scenario* scn, const aeb_params* params, int precision,
                 const aeb_outputs* out, ParamSrc* src) {
  if (!scn || !outputs_complete(out)) return fail(AEB_EINVAL, "aeb_rollout: null argument");
  int rc = validate(*scn);
  if (rc != AEB_OK) return rc;
  if (precision != AEB_FP64 && precision != AEB_FP32C && precision != AEB_FP32C_FIXUP)
    return fail(AEB_EINVAL, "unknown precision");
  if (out->n != scn->n_samples) return fail(AEB_EINVAL, "outputs length differs from n_samples");
  *src = ParamSrc{};
  if (params) {
    if (!params_complete(params)) return fail(AEB_EINVAL, "aeb_rollout: incomplete parameter columns");
    if (params->n != scn->n_samples) return fail(AEB_EINVAL, "parameter length differs from n_samples");
    if (perception_on(*scn) && !params->trigger)
      return fail(AEB_EINVAL, "aeb_rollout: a scenario with perception needs the trigger column");
    if (scn->is_mask && !params->log_weight)
      return fail(AEB_EINVAL, "aeb_rollout: importance sampling needs the log_weight column");
    *src = ParamSrc{params->v0, params->mu,  params->mass, params->sin_grade, params->cos_grade,
                    params->cda, params->crr, params->tau, params->gap, params->lead_decel,
                    params->trigger, params->log_weight};
  }
  return AEB_OK;
}

int check_reduce_req(const aeb_reduce_req& req) {
  if (req.n_risk < 0 || req.n_risk > AEB_MAX_RISK || req.n_margin_q < 0 ||
      req.n_margin_q > AEB_MAX_MARGIN_Q || req.n_grid < 0 || req.n_grid > AEB_MAX_GRID ||
      req.n_grid == 1)
    return fail(AEB_EINVAL, "aeb_reduce: request sizes out of range");
  for (int j = 0; j < req.n_risk; ++j)
    if (!(req.risk[j] >= 0.0 && req.risk[j] < 1.0)) return fail(AEB_EINVAL, "risk level outside [0,1)");
  for (int j = 0; j < req.n_margin_q; ++j)
    if (!(req.margin_q[j] >= 0.0 && req.margin_q[j] < 1.0))
      return fail(AEB_EINVAL, "margin quantile outside [0,1)");
  if (req.n_grid >= 2 && !(req.grid_lo < req.grid_hi && std::isfinite(req.grid_lo) &&
                            std::isfinite(req.grid_hi)))
    return fail(AEB_EINVAL, "headway grid needs finite grid_lo < grid_hi");
  return AEB_OK;
}

}  // namespace aeb

extern "C" {

const char* aeb_last_error(void) { return g_err.c_str(); }

int aeb_version(void) { return 9; }

int aeb_timing_enable(int on) {
  g_timing.on = on != 0;
  g_timing.recorded = false;
  g_timing.lanes_valid = g_timing.lanes_armed = false;
  return AEB_OK;
}

int aeb_reduce_fallbacks(uint64_t* count) {
  if (!count) return fail(AEB_EINVAL, "aeb_reduce_fallbacks: null argument");
  *count = reduce_fallback_count();
  return AEB_OK;
}

int aeb_ctl_approx_check(double* measured, double* bounds, void* stream) {
  if (!measured || !bounds) return fail(AEB_EINVAL, "aeb_ctl_approx_check: null argument");
  return launch_approx_check(measured, bounds, static_cast<hipStream_t>(stream));
}

int aeb_ctl_math(const double* a, const double* x, int64_t n, double* log_a, double* sin_x,
                 double* cos_x, int on_device, void* stream) {
  if (n < 0 || (n > 0 && (!a || !x || !log_a || !sin_x || !cos_x)))
    return fail(AEB_EINVAL, "aeb_ctl_math: bad argument");
  if (on_device)
    return launch_ctl_math(a, x, n, log_a, sin_x, cos_x, static_cast<hipStream_t>(stream));
  for (int64_t i = 0; i < n; ++i) {
    log_a[i] = ctl_log(a[i]);
    ctl_sincos(x[i], &sin_x[i], &cos_x[i]);
  }
  return AEB_OK;
}

int aeb_valu_probe(int fp32, int64_t threads, int iters, void* out, void* stream) {
  if (!out || threads <= 0 || threads % 256 != 0 || threads / 256 > 0x7fffffff || iters < 0)
    return fail(AEB_EINVAL, "aeb_valu_probe: bad argument");
  return launch_valu_probe(fp32, threads, iters, out, static_cast<hipStream_t>(stream));
}

int aeb_timing_lanes(uint64_t* wave_sample_steps) {
  if (!wave_sample_steps) return fail(AEB_EINVAL, "aeb_timing_lanes: null argument");
  Timing& t = g_timing;
  if (!t.recorded || !t.lanes) return fail(AEB_EAGAIN, "no timed rollout on this thread");
  if (!t.lanes_valid)
    return fail(AEB_EAGAIN, "the last timed rollout ran a checked kernel (no lane accounting)");
  AEB_HIP(hipEventSynchronize(t.stop));
  unsigned long long h = 0;
  AEB_HIP(hipMemcpy(&h, t.lanes, sizeof(h), hipMemcpyDeviceToHost));
  *wave_sample_steps = h;
  return AEB_OK;
}

int aeb_timing_last(float* ms) {
  if (!ms) return fail(AEB_EINVAL, "aeb_timing_last: null argument");
  Timing& t = g_timing;
  if (!t.recorded) return fail(AEB_EAGAIN, "no timed rollout on this thread");
  AEB_HIP(hipEventSynchronize(t.stop));
  AEB_HIP(hipEventElapsedTime(ms, t.start, t.stop));
  return AEB_OK;
}

int aeb_validate(const aeb_scenario* scn) {
  if (!scn) return fail(AEB_EINVAL, "null scenario");
  int rc = validate(*scn);
  if (rc == AEB_OK) g_err.clear();
  return rc;
}

int aeb_uniforms(uint64_t seed, uint64_t scenario_id, int64_t first, int64_t count, uint32_t slot,
                 uint32_t attempt, double* out, int on_device, void* stream) {
  if (!out || first < 0 || count < 0 || first + count > (int64_t(1) << 32) || slot > 255 ||
      attempt > 0xFFFFFF)
    return fail(AEB_EINVAL, "aeb_uniforms: bad arguments");
  if (count == 0) return AEB_OK;
  if (on_device)
    return launch_uniforms(seed, scenario_id, first, count, slot, attempt, out,
                           static_cast<hipStream_t>(stream));
  for (int64_t k = 0; k < count; ++k) {
    U2 u = uniform2(seed, scenario_id, static_cast<uint64_t>(first + k), slot, attempt);
    out[2 * k] = u.a;
    out[2 * k + 1] = u.b;
  }
  return AEB_OK;
}

int aeb_sample_params(const aeb_scenario* scn, int64_t first, int64_t count, const aeb_params* out,
                      int on_device, void* stream) {
  if (!scn || !params_complete(out)) return fail(AEB_EINVAL, "aeb_sample_params: null argument");
  int rc = validate(*scn);
  if (rc != AEB_OK) return rc;
  if (first < 0 || count < 0 || first + count > (int64_t(1) << 32))
    return fail(AEB_EINVAL, "aeb_sample_params: sample range out of [0, 2^32)");
  if (perception_on(*scn) && !out->trigger)
    return fail(AEB_EINVAL, "aeb_sample_params: a scenario with perception needs the trigger column");
  if (scn->is_mask && !out->log_weight)
    return fail(AEB_EINVAL,
                "aeb_sample_params: importance sampling needs the log_weight column");
  if (count == 0) return AEB_OK;
  if (on_device) return launch_sample(*scn, first, count, *out, static_cast<hipStream_t>(stream));
  // the paper's plain method: draw on the host with host libm, all cores
  const aeb_scenario s = *scn;
  const aeb_params p = *out;
  auto work = [&](int64_t lo, int64_t hi) {
    for (int64_t k = lo; k < hi; ++k) {
      Sample q = draw_sample(s, static_cast<uint64_t>(first + k));
      p.v0[k] = q.v0;
      p.mu[k] = q.mu;
      p.mass[k] = q.mass;
      p.grade[k] = q.grade;
      p.sin_grade[k] = q.sin_grade;
      p.cos_grade[k] = q.cos_grade;
      p.cda[k] = q.cda;
      p.crr[k] = q.crr;
      p.tau[k] = q.tau;
      p.gap[k] = q.gap;
      p.lead_decel[k] = q.lead_decel;
      if (p.trigger) p.trigger[k] = q.trigger;
      if (p.log_weight) p.log_weight[k] = q.log_w;
    }
  };
  int nt = host_threads();
  if (count < 4096) nt = 1;
  if (nt > 256) nt = 256;
  if (nt == 1) {
    work(0, count);
  } else {
    std::vector<std::thread> th;
    th.reserve(nt);
    for (int t = 0; t < nt; ++t) th.emplace_back(work, count * t / nt, count * (t + 1) / nt);
    for (auto& t : th) t.join();
  }
  return AEB_OK;
}

int aeb_rollout(const aeb_scenario* scn, const aeb_params* params, int precision,
                const aeb_outputs* out, void* stream) {
  ParamSrc src{};
  const int rc = rollout_args(scn, params, precision, out, &src);
  if (rc != AEB_OK) return rc;
  OutCols oc{out->dist, out->status, out->steps, out->margin, out->v_impact, out->weight};
  ScratchScope scope(static_cast<hipStream_t>(stream));
  return launch_rollout(*scn, params ? &src : nullptr, precision, oc, scn->n_samples,
                        static_cast<hipStream_t>(stream));
}

int aeb_batch_rollout(const aeb_scenario* scns, int n_scn, int precision, const aeb_outputs* outs,
                      void* stream) {
  if (!scns || !outs || n_scn < 1) return fail(AEB_EINVAL, "aeb_batch_rollout: empty batch");
  if (precision != AEB_FP64 && precision != AEB_FP32C)
    return fail(AEB_EINVAL, "aeb_batch_rollout: precision must be AEB_FP64 or AEB_FP32C");
  int64_t total = 0;
  std::vector<OutCols> oc(n_scn);
  for (int j = 0; j < n_scn; ++j) {
    int rc = validate(scns[j]);
    if (rc != AEB_OK) return fail(rc, "scenario " + std::to_string(j) + ": " + g_err);
    if (!outputs_complete(&outs[j]) || outs[j].n != scns[j].n_samples)
      return fail(AEB_EINVAL, "outputs of scenario " + std::to_string(j) + " do not match it");
    if (scns[j].integrator != scns[0].integrator || scns[j].obstacle != scns[0].obstacle ||
        scns[j].impact_exit != scns[0].impact_exit || scns[j].nofma != scns[0].nofma)
      return fail(AEB_EINVAL, "batched scenarios must share integrator, obstacle, impact_exit, nofma");
    total += scns[j].n_samples;
    oc[j] = OutCols{outs[j].dist, outs[j].status, outs[j].steps, outs[j].margin, outs[j].v_impact,
                    outs[j].weight};
  }
  if (total > 0xffffffffLL) return fail(AEB_EINVAL, "a batch holds at most 2^32 - 1 samples");
  ScratchScope scope(static_cast<hipStream_t>(stream));
  return launch_batch(scns, n_scn, precision, oc.data(), static_cast<hipStream_t>(stream));
}

int aeb_batch_reduce(const aeb_outputs* outs, int n_scn, const aeb_reduce_req* req, aeb_stats* stats,
                     void* stream) {
  if (!outs || !stats || !req || n_scn < 1) return fail(AEB_EINVAL, "aeb_batch_reduce: empty batch");
  const int rc = check_reduce_req(*req);
  if (rc != AEB_OK) return rc;
  std::vector<OutCols> oc(n_scn);
  std::vector<int64_t> ns(n_scn);
  for (int j = 0; j < n_scn; ++j) {
    if (!outputs_complete(&outs[j])) return fail(AEB_EINVAL, "aeb_batch_reduce: null argument");
    if (outs[j].n < 1 || outs[j].n > 0x7fffffffLL)
      return fail(AEB_EINVAL, "aeb_batch_reduce: n out of [1, 2^31-1]");
    oc[j] = OutCols{outs[j].dist, outs[j].status, outs[j].steps, outs[j].margin, outs[j].v_impact,
                    outs[j].weight};
    ns[j] = outs[j].n;
  }
  ScratchScope scope(static_cast<hipStream_t>(stream));
  return launch_batch_reduce(oc.data(), ns.data(), n_scn, *req, stats,
                             static_cast<hipStream_t>(stream));
}

int aeb_reduce(const aeb_outputs* out, const aeb_reduce_req* req, aeb_stats* host_out, void* stream) {
  if (!outputs_complete(out) || !req || !host_out) return fail(AEB_EINVAL, "aeb_reduce: null argument");
  if (out->n < 1 || out->n > 0x7fffffffLL) return fail(AEB_EINVAL, "aeb_reduce: n out of [1, 2^31-1]");
  const int rc = check_reduce_req(*req);
  if (rc != AEB_OK) return rc;
  OutCols oc{out->dist, out->status, out->steps, out->margin, out->v_impact, out->weight};
  ScratchScope scope(static_cast<hipStream_t>(stream));
  return launch_reduce(oc, out->n, *req, host_out, static_cast<hipStream_t>(stream));
}

}  // extern "C"
