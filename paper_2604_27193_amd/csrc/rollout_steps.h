// rollout_steps.h -- per-sample integrators of the braking model
// (eq. (7)-(9)), one sample per lane, with the termination tests of Sec. V-C:
// after every step, impact (strict x > gap + x_lead), then stop (v <= 0),
// then horizon.
//
// FP64 forms are the library's exact path: explicit Euler with four fused
// multiply-adds (or none when NOFMA), RK4 without fused operations.  The FP32
// form is the compensated served variant.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "aeb_common.h"

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
};

// ---------------------------------------------------------------------------
// Explicit Euler, FP64.  Per step k (cmd = a_cmd once k >= nd, else 0):
//   abe = max(a, alim); acc = fma(-kd, v*v, abe) - c
//   x' = fma(dt, v, x); v' = fma(dt, acc, v); a' = fma(dt/tau, cmd - a, a)
//   lead: xl' = fma(dt, vl, xl); vl' = max(fma(-dt, al, vl), 0)
// ---------------------------------------------------------------------------
template <int OBS, bool NOFMA>
__device__ inline Result euler_fp64(const Lane& L, double dt, double a_cmd, int64_t nd,
                                    int64_t nmax, int impact_exit) {
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
  for (;;) {
    const double cmd = step >= nd ? a_cmd : 0.0;
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

template <int OBS>
__device__ inline Result rk4_fp64(const Lane& L, double dt, double a_cmd, int64_t nd,
                                  int64_t nmax, int impact_exit) {
  const double h2 = 0.5 * dt, h6 = dt / 6.0, rt = 1.0 / L.tau;
  const double gap0 = L.gap;
  S3 y{0.0, L.v0, 0.0};
  double margin = gap0 - y.x;
  bool collided = false;
  float vimp = 0.0f;
  int end = 0;
  int64_t step = 0;
  for (;;) {
    const double cmd = step >= nd ? a_cmd : 0.0;
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

// ---------------------------------------------------------------------------
// FP32 compensated Euler.  The same model rewritten for single precision:
//   * the actuator is carried as its deviation from the command, e = a - cmd,
//     which decays as e' = fma(-dt/tau, e, e) (the rate keeps the precision of
//     dt/tau; a product with 1 - dt/tau would not);
//   * the brake term with grade and rolling folded in is
//     max(e + (cmd - c), alim - c), so acc = fma(-kd, v v, that);
//   * each speed is a float base plus a small in-block increment; the base
//     absorbs the increment every KB steps with an exact two-sum, so rounding
//     never accumulates at the scale of the speed itself;
//   * positions are summed in blocks of KB increments dt*v, each block sum
//     added to a Kahan pair; the clearance to a lead vehicle likewise.
// Distances, the collision decision and the margin are finished in FP64.
// `boundary` reports an outcome that single precision cannot decide; the
// caller recomputes such samples in FP64.
// ---------------------------------------------------------------------------
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

// base + increment with an exact carry (|base| >= |increment| assumed)
struct Split32 {
  float base, inc;
  __device__ inline void carry() {
    float t = base + inc;
    inc = inc - (t - base);
    base = t;
  }
};

__device__ inline Split32 split_of(double v) {
  Split32 s;
  s.base = static_cast<float>(v);
  s.inc = static_cast<float>(v - static_cast<double>(s.base));
  return s;
}

template <int OBS>
__device__ inline Result euler_fp32c(const Lane& L, double dt, double a_cmd, int64_t nd,
                                     int64_t nmax, int impact_exit, double band, bool& boundary) {
  constexpr int KB = 32;
  const double kt = dt / L.tau;
  const float dtf = static_cast<float>(dt);
  const float nkd = static_cast<float>(-L.k.kd);
  const float nkt = static_cast<float>(-kt);
  const float alc = static_cast<float>(L.k.alim - L.k.c);
  const float t_dead = static_cast<float>(0.0 - L.k.c);    // cmd - c before the command
  const float t_brake = static_cast<float>(a_cmd - L.k.c);  // cmd - c after it
  const float e_jump = static_cast<float>(-a_cmd);          // e = a - cmd jumps when cmd does
  const float gapf = static_cast<float>(L.gap);
  const float al = static_cast<float>(L.lead);
  const float bandf = static_cast<float>(band);
  Split32 V = split_of(L.v0), VL = split_of(L.v0);
  float vc = V.base + V.inc, vlc = vc;
  float e = 0.0f;
  float p = 0.0f, pg = 0.0f;
  Kahan32 X, G;
  G.hi = gapf;
  G.lo = static_cast<float>(static_cast<double>(gapf) - L.gap);
  float gmin = gapf, gprev = gapf;
  bool collided = false;
  float vimp = 0.0f;
  int end = 0;
  int64_t step = 0;
  boundary = false;
  for (;;) {
    if (step == nd) e += e_jump;
    const float tc = step >= nd ? t_brake : t_dead;
    const float q = vc * vc;
    const float m = fmaxf(e + tc, alc);
    const float acc = fmaf(nkd, q, m);
    const float vb = vc;
    p = fmaf(dtf, vc, p);
    if (OBS == AEB_OBS_LEAD) {
      pg = fmaf(dtf, vlc - vc, pg);
      VL.inc = fmaf(-dtf, al, VL.inc);
    }
    V.inc = fmaf(dtf, acc, V.inc);
    e = fmaf(nkt, e, e);
    ++step;
    if ((step & (KB - 1)) == 0) {
      X.add(p);
      p = 0.0f;
      V.carry();
      if (OBS == AEB_OBS_LEAD) {
        G.add(pg);
        pg = 0.0f;
        VL.carry();
      }
    }
    vc = V.base + V.inc;
    if (OBS == AEB_OBS_LEAD) {
      vlc = fmaxf(VL.base + VL.inc, 0.0f);
      const float g = (G.hi - G.lo) + pg;
      gmin = fminf(gmin, g);
      if (g < 0.0f) {
        collided = true;
        vimp = vc - vlc;
        end = AEB_END_IMPACT;
        boundary = fabsf(gprev) < bandf || fabsf(g) < bandf;
        break;
      }
      gprev = g;
    } else if (OBS == AEB_OBS_STATIONARY && !collided) {
      if ((X.hi - X.lo) + p > gapf) {
        collided = true;
        vimp = vc;
        if (impact_exit) {
          end = AEB_END_IMPACT;
          // the crossing step is in doubt if either side of it is within the band
          const double xe = X.value(p);
          boundary = fabs(xe - L.gap) < band || fabs(L.gap - (xe - static_cast<double>(dtf * vb))) < band;
          break;
        }
      }
    }
    if (vc <= 0.0f) {
      end = AEB_END_STOP;
      break;
    }
    if (step == nmax) {
      end = AEB_END_HORIZON;
      break;
    }
  }
  Result res;
  res.dist = X.value(p);
  res.steps = static_cast<int32_t>(step);
  if (OBS == AEB_OBS_LEAD) {
    res.margin = static_cast<double>(gmin);
    if (!collided) boundary = boundary || (gmin < bandf);
  } else {
    const double mg = L.gap - res.dist;
    res.margin = mg < L.gap ? mg : L.gap;
    if (OBS == AEB_OBS_STATIONARY) {
      // the flag is decided in FP64 on the compensated distance
      const double clear = L.gap - res.dist;
      if (impact_exit) {
        if (!collided) boundary = clear < band;
      } else {
        collided = res.dist > L.gap;
        boundary = fabs(clear) < band;
        if (!collided) vimp = 0.0f;
      }
    }
  }
  res.status = static_cast<uint8_t>(end | (collided ? AEB_COLLIDED : 0));
  res.vimp = collided ? vimp : 0.0f;
  return res;
}

}  // namespace aeb
