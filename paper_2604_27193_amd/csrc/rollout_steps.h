// rollout_steps.h -- per-sample integrators of the braking model
// (eq. (7)-(9)), one sample per lane, with the termination tests of Sec. V-C:
// after every step, impact (strict x > gap + x_lead), then stop (v <= 0),
// then horizon.
//
// FP64 forms: explicit Euler with four fused multiply-adds (or none when
// NOFMA), RK4 without fused operations.  These checked per-step forms serve
// RK4, the unfused Euler form, the closed-loop controller and the FP64
// recomputation of FP32 boundary samples; the explicit-Euler throughput path
// is kernels_fast.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "aeb_common.h"
#include "ctl_math.h"

namespace aeb {

struct Result {
  double dist;
  double margin;
  int32_t steps;
  uint8_t status;
  float vimp;
};

struct Lane {
  double v0, gap, lead;  // initial speed, initial gap, lead deceleration
  Consts k;
  double tau;
  double trig;           // perception delay (s)
  uint64_t index;        // the sample's index (keys the controller's noise)
  double log_w;          // importance-sampling log likelihood ratio
};

// ---------------------------------------------------------------------------
// Closed-loop controller (Sec. VIII's controller assessment).  Every `period`
// steps it measures gap and closing speed with additive normal noise (the
// cosine and sine Box-Muller normals of one generator call per decision),
// forms TTC and raises its latched stage; a stage's command starts nd steps
// after the decision.
// ---------------------------------------------------------------------------
struct CtlArgs {
  int64_t period;
  double ttc_warn, ttc_brake, a_warn, noise_gap, noise_v;
  uint64_t seed, sid;
};

inline CtlArgs ctl_args(const aeb_scenario& s) {
  CtlArgs a{};
  if (control_on(s)) a.period = std::llround(s.ctl_period / s.dt);
  a.ttc_warn = s.ttc_warn;
  a.ttc_brake = s.ttc_brake;
  a.a_warn = s.a_warn;
  a.noise_gap = s.noise_gap;
  a.noise_v = s.noise_v;
  a.seed = s.seed;
  a.sid = s.scenario_id;
  return a;
}

struct Ctl {
  int64_t next_tick, on1, on2;  // next decision step; first steps of the two commands
  uint32_t tick;                // decisions taken
  int stage;
};

__device__ inline Ctl ctl_start() {
  Ctl c;
  c.next_tick = 0;
  c.on1 = c.on2 = INT64_MAX;
  c.tick = 0;
  c.stage = 0;
  return c;
}

// The stage decision asks for from the measurement noise's uniforms u (the
// cosine and sine Box-Muller normals of one generator call) and the true gap
// and closing speed: measured TTC below ttc_brake asks for full braking,
// below ttc_warn for partial braking.
// The logarithm, sine and cosine are ctl_math.h's, written for these
// arguments (a few registers where a general library routine costs the
// integration kernel a wavefront per SIMD), accurate to about an ulp like any
// libm: the outcome equals another FP64 evaluation's unless the measured TTC
// lies within about 1e-15 (relative) of a threshold.
__device__ inline int ctl_exact(const CtlArgs& A, U2 u, double gap_true, double closing) {
  const double r = sqrt(-2.0 * ctl_log(u.a));
  const double ang = 6.283185307179586 * u.b;
  double sn, cs;
  ctl_sincos(ang, &sn, &cs);
  const double g = gap_true + A.noise_gap * (r * cs);
  const double cl = closing + A.noise_v * (r * sn);
  const double ttc = cl > 0.0 ? g / cl : INFINITY;
  return ttc < A.ttc_brake ? 2 : (ttc < A.ttc_warn ? 1 : 0);
}

// the stage decision `tick` asks for, from the true gap and closing speed
__device__ inline int ctl_want(const CtlArgs& A, uint64_t index, uint32_t tick, double gap_true,
                               double closing) {
  return ctl_exact(A, uniform2(A.seed, A.sid, index, AEB_SLOT_CONTROL, tick), gap_true, closing);
}

// The decision's outcome when every measured gap in [g_lo, g_hi] and closing
// speed in [c_lo, c_hi] gives it, else -1.  The outcome is the new stage when
// the decision raises it (then it equals ctl_exact's value), and a value at
// most `stage` when it does not.  Margins of 1e-9 (relative, plus 1e-9
// absolute) cover the rounding of the exact evaluation.  Thresholds are >= 0.
__device__ inline int ctl_box(const CtlArgs& A, int stage, double g_lo, double g_hi, double c_lo,
                              double c_hi) {
  // every measured TTC at or above t (an infinite TTC included)
  auto above = [&](double t) {
    if (c_hi <= 0.0) return true;
    const double b = t * c_hi;
    return g_lo > 0.0 && g_lo >= b + 1e-9 * (fabs(b) + 1.0);
  };
  // every measured TTC below t
  auto below = [&](double t) {
    const double b = t * c_lo;
    return c_lo > 0.0 && g_hi <= b - 1e-9 * (fabs(b) + 1.0);
  };
  if (below(A.ttc_brake)) return 2;
  if (stage >= 1) return above(A.ttc_brake) ? stage : -1;
  if (above(fmax(A.ttc_warn, A.ttc_brake))) return 0;
  if (above(A.ttc_brake) && below(A.ttc_warn)) return 1;
  return -1;
}

// Before any draw: the Box-Muller radius is below 8.572 (the smallest
// uniform is 2^-53), so the measured gap and closing speed lie within
// R = 8.6 noise standard deviations of the true ones.
__device__ inline int ctl_screen(const CtlArgs& A, int stage, double gap_true, double closing) {
  constexpr double R = 8.6;
  const double eg = A.noise_gap * R, ev = A.noise_v * R;
  return ctl_box(A, stage, gap_true - eg, gap_true + eg, closing - ev, closing + ev);
}

// Bounds on the single-precision hardware approximations the estimate below
// uses, over every input that reaches them (the device measures the actual
// maxima exhaustively: aeb_ctl_approx_check):
//   CTL_EL  |v_log_f32(a) - log2(a)| / max(1, |log2(a)|), a in [2^-53, 1]
//   CTL_ES  |v_sqrt_f32(x) - sqrt(x)| / sqrt(x), x in [2^-24, 80]
//   CTL_ET  |v_sin_f32(b) - sin(2 pi b)| and the cosine's, b in [2^-53, 1]
//           (the instruction's argument is in revolutions)
constexpr double CTL_EL = 1e-6;
constexpr double CTL_ES = 1e-6;
constexpr double CTL_ET = 1e-5;

// After the draw: the noise estimated in single precision with an error box
// around it, then ctl_box on the box; -1 when the box straddles a threshold
// (the exact evaluation decides).  Error terms, for the radius r = sqrt(s),
// s = -2 ln(u.a), and its estimate r' = v_sqrt_f32(s'):
//   a = float(u.a) moves log2 by at most 2^-24 / ln 2 (< 8.6e-8), so
//   |s' - s| <= D = 2 ln 2 (CTL_EL + 8.6e-8) + (CTL_EL + 2^-21) s' (the
//   log's error relative to |log2 a| > 1, and the float constant and
//   product roundings, 2^-23 s' with room);
//   |sqrt(s') - r| <= D / max(r', sqrt(D0)) with D0 the absolute part of D,
//   and |r' - sqrt(s')| <= 2 CTL_ES r';
//   b = float(u.b) moves the angle by at most 2 pi 2^-24 < 3.8e-7.
// Then |noise_gap (r cos - r' cos')| <= noise_gap (er + r' et), likewise for
// the closing speed with the sine.
__device__ inline int ctl_fast(const CtlArgs& A, int stage, double gap_true, double closing,
                               U2 u) {
  const float a = static_cast<float>(u.a), b = static_cast<float>(u.b);
  const float s2 = fmaxf(-1.3862943611198906f * __builtin_amdgcn_logf(a), 0.0f);
  const float rf = __builtin_amdgcn_sqrtf(s2);
  const double r = rf, cs = __builtin_amdgcn_cosf(b), sn = __builtin_amdgcn_sinf(b);
  constexpr double D0 = 2.0 * 0.6931471805599453 * (CTL_EL + 8.6e-8);
  const double d = D0 + (CTL_EL + 0x1p-21) * static_cast<double>(s2);
  const double er = d / fmax(r, 5e-4) + 2.0 * CTL_ES * r;  // 5e-4 < sqrt(D0) = 1.18e-3
  const double et = CTL_ET + 3.8e-7;
  const double eg = A.noise_gap * (er + r * et) * 1.0001;
  const double ev = A.noise_v * (er + r * et) * 1.0001;
  const double g = gap_true + A.noise_gap * (r * cs);
  const double c = closing + A.noise_v * (r * sn);
  return ctl_box(A, stage, g - eg, g + eg, c - ev, c + ev);
}

__device__ inline void ctl_decide(const CtlArgs& A, Ctl& c, uint64_t index, int64_t step,
                                  int64_t nd, double gap_true, double closing) {
  const int want = ctl_want(A, index, c.tick, gap_true, closing);
  if (want > c.stage) {
    if (want == 2)
      c.on2 = step + nd;
    else
      c.on1 = step + nd;
    c.stage = want;
  }
  c.tick += 1;
  c.next_tick += A.period;
}

__device__ inline double ctl_command(const Ctl& c, int64_t step, double a_cmd, double a_warn) {
  if (step >= c.on2) return a_cmd;
  if (step >= c.on1) return a_warn;
  return 0.0;
}

// ---------------------------------------------------------------------------
// Explicit Euler, FP64.  Per step k (cmd = a_cmd once k >= nd, else 0):
//   abe = max(a, alim); acc = fma(-kd, v*v, abe) - c
//   x' = fma(dt, v, x); v' = fma(dt, acc, v); a' = fma(dt/tau, cmd - a, a)
//   lead: xl' = fma(dt, vl, xl); vl' = max(fma(-dt, al, vl), 0)
// ---------------------------------------------------------------------------
template <int OBS, bool NOFMA, bool CTL = false>
__device__ inline Result euler_fp64(const Lane& L, double dt, double a_cmd, int64_t nd,
                                    int64_t nmax, int impact_exit, const CtlArgs* ca = nullptr) {
  const double kt = dt / L.tau;
  const double nkd = -L.k.kd, c = L.k.c, alim = L.k.alim;
  double x = 0.0, v = L.v0, a = 0.0;
  double xl = 0.0, vl = (OBS == AEB_OBS_LEAD) ? L.v0 : 0.0;
  const double gap0 = L.gap;
  double margin = (gap0 + xl) - x;
  bool collided = false;
  float vimp = 0.0f;
  int end = 0;
  int64_t step = 0;
  Ctl cs = ctl_start();
  for (;;) {
    double cmd;
    if (CTL) {
      if (step == cs.next_tick) ctl_decide(*ca, cs, L.index, step, nd, (gap0 + xl) - x, v - vl);
      cmd = ctl_command(cs, step, a_cmd, ca->a_warn);
    } else {
      cmd = step >= nd ? a_cmd : 0.0;
    }
    const double abe = fmax(a, alim);
    const double v2 = v * v;
    double acc, xn, vn, an;
    if (NOFMA) {
      acc = (abe - L.k.kd * v2) - c;
      xn = dt * v + x;
      vn = dt * acc + v;
      an = kt * (cmd - a) + a;
    } else {
      acc = fma(nkd, v2, abe) - c;
      xn = fma(dt, v, x);
      vn = fma(dt, acc, v);
      an = fma(kt, cmd - a, a);
    }
    if (OBS == AEB_OBS_LEAD) {
      const double xln = NOFMA ? dt * vl + xl : fma(dt, vl, xl);
      const double t = NOFMA ? vl - dt * L.lead : fma(-dt, L.lead, vl);
      xl = xln;
      vl = t > 0.0 ? t : 0.0;
    }
    x = xn;
    v = vn;
    a = an;
    ++step;
    const double gap_now = gap0 + xl;
    const double m = gap_now - x;
    margin = m < margin ? m : margin;
    if (OBS != AEB_OBS_NONE && x > gap_now) {
      if (!collided) {
        collided = true;
        vimp = static_cast<float>(v - vl);
      }
      if (OBS == AEB_OBS_LEAD || impact_exit) {
        end = AEB_END_IMPACT;
        break;
      }
    }
    if (v <= 0.0) {
      end = AEB_END_STOP;
      break;
    }
    if (step == nmax) {
      end = AEB_END_HORIZON;
      break;
    }
  }
  Result r;
  r.dist = x;
  r.margin = margin;
  r.steps = static_cast<int32_t>(step);
  r.status = static_cast<uint8_t>(end | (collided ? AEB_COLLIDED : 0));
  r.vimp = vimp;
  return r;
}

// ---------------------------------------------------------------------------
// Classical RK4, FP64, no fused operations.  f(x, v, a) =
//   (v, (max(a, alim) - kd (v v)) - c, (cmd - a) / tau)
// with the command held over the step at its start-of-step value.
// ---------------------------------------------------------------------------
struct S3 {
  double x, v, a;
};

__device__ inline S3 rk_rhs(const Consts& k, double rt, double cmd, S3 y) {
  S3 d;
  d.x = y.v;
  d.v = (fmax(y.a, k.alim) - k.kd * (y.v * y.v)) - k.c;
  d.a = (cmd - y.a) * rt;
  return d;
}

__device__ inline S3 rk_axpy(S3 y, double h, S3 d) {
  S3 o;
  o.x = y.x + h * d.x;
  o.v = y.v + h * d.v;
  o.a = y.a + h * d.a;
  return o;
}

template <int OBS, bool CTL = false>
__device__ inline Result rk4_fp64(const Lane& L, double dt, double a_cmd, int64_t nd,
                                  int64_t nmax, int impact_exit, const CtlArgs* ca = nullptr) {
  const double h2 = 0.5 * dt, h6 = dt / 6.0, rt = 1.0 / L.tau;
  const double gap0 = L.gap;
  S3 y{0.0, L.v0, 0.0};
  double margin = gap0 - y.x;
  bool collided = false;
  float vimp = 0.0f;
  int end = 0;
  int64_t step = 0;
  Ctl cs = ctl_start();
  for (;;) {
    double cmd;
    if (CTL) {
      if (step == cs.next_tick) ctl_decide(*ca, cs, L.index, step, nd, gap0 - y.x, y.v);
      cmd = ctl_command(cs, step, a_cmd, ca->a_warn);
    } else {
      cmd = step >= nd ? a_cmd : 0.0;
    }
    S3 k1 = rk_rhs(L.k, rt, cmd, y);
    S3 k2 = rk_rhs(L.k, rt, cmd, rk_axpy(y, h2, k1));
    S3 k3 = rk_rhs(L.k, rt, cmd, rk_axpy(y, h2, k2));
    S3 k4 = rk_rhs(L.k, rt, cmd, rk_axpy(y, dt, k3));
    S3 sum;
    sum.x = ((k1.x + 2.0 * k2.x) + 2.0 * k3.x) + k4.x;
    sum.v = ((k1.v + 2.0 * k2.v) + 2.0 * k3.v) + k4.v;
    sum.a = ((k1.a + 2.0 * k2.a) + 2.0 * k3.a) + k4.a;
    y = rk_axpy(y, h6, sum);
    ++step;
    const double m = gap0 - y.x;
    margin = m < margin ? m : margin;
    if (OBS == AEB_OBS_STATIONARY && y.x > gap0) {
      if (!collided) {
        collided = true;
        vimp = static_cast<float>(y.v);
      }
      if (impact_exit) {
        end = AEB_END_IMPACT;
        break;
      }
    }
    if (y.v <= 0.0) {
      end = AEB_END_STOP;
      break;
    }
    if (step == nmax) {
      end = AEB_END_HORIZON;
      break;
    }
  }
  Result r;
  r.dist = y.x;
  r.margin = margin;
  r.steps = static_cast<int32_t>(step);
  r.status = static_cast<uint8_t>(end | (collided ? AEB_COLLIDED : 0));
  r.vimp = vimp;
  return r;
}

// Kahan-compensated FP32 sum (the FP32 compensated form of kernels_fast.hip
// keeps its distance and lead clearance in these).
struct Kahan32 {
  float hi = 0.0f, lo = 0.0f;
  __device__ inline void add(float y_in) {
    float y = y_in - lo;
    float t = hi + y;
    lo = (t - hi) - y;
    hi = t;
  }
  __device__ inline double value(float partial) const {
    return (static_cast<double>(hi) - static_cast<double>(lo)) + static_cast<double>(partial);
  }
};

}  // namespace aeb
