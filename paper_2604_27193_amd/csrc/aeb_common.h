// aeb_common.h -- arithmetic shared by the host sampler and the kernels of
// the library: the counter-based generator, the parameter distributions and
// the per-sample constants of the force balance.
//
// Everything here is __host__ __device__ and compiled with -ffp-contract=off,
// so host and device evaluate the same expression trees; only libm
// (log, cos, sin, sqrt) differs between host and device.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "aeb.h"

namespace aeb {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).  Ten rounds of: two
// 32x32->64 products of counter words 0 and 2 with fixed multipliers; the new
// counter takes the low halves in place and xors the high halves into the
// other words together with the round key; the key then advances by the Weyl
// constants.
// ---------------------------------------------------------------------------
struct Ctr {
  uint32_t w[4];
};

__host__ __device__ inline void mulhilo(uint32_t a, uint32_t b, uint32_t& hi, uint32_t& lo) {
  uint64_t p = static_cast<uint64_t>(a) * static_cast<uint64_t>(b);
  hi = static_cast<uint32_t>(p >> 32);
  lo = static_cast<uint32_t>(p);
}

__host__ __device__ inline Ctr philox4x32_10(Ctr c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t hi_a, lo_a, hi_b, lo_b;
    mulhilo(0xD2511F53u, c.w[0], hi_a, lo_a);
    mulhilo(0xCD9E8D57u, c.w[2], hi_b, lo_b);
    Ctr n;
    n.w[0] = hi_b ^ c.w[1] ^ k0;
    n.w[1] = lo_b;
    n.w[2] = hi_a ^ c.w[3] ^ k1;
    n.w[3] = lo_a;
    c = n;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return c;
}

// Two uniforms in (0,1) from one call: 52 top bits of each 64-bit half plus 1/2.
struct U2 {
  double a, b;
};

__host__ __device__ inline double unit52(uint64_t w) {
  return (static_cast<double>(w >> 12) + 0.5) * 0x1p-52;
}

__host__ __device__ inline U2 uniform2(uint64_t seed, uint64_t sid, uint64_t i, uint32_t slot,
                                       uint32_t attempt) {
  Ctr c;
  c.w[0] = static_cast<uint32_t>(i);
  c.w[1] = slot | (attempt << 8);
  c.w[2] = static_cast<uint32_t>(sid);
  c.w[3] = static_cast<uint32_t>(sid >> 32);
  Ctr o = philox4x32_10(c, static_cast<uint32_t>(seed), static_cast<uint32_t>(seed >> 32));
  U2 u;
  u.a = unit52((static_cast<uint64_t>(o.w[1]) << 32) | o.w[0]);
  u.b = unit52((static_cast<uint64_t>(o.w[3]) << 32) | o.w[2]);
  return u;
}

// Box-Muller, cosine branch.
__host__ __device__ inline double box_muller(U2 u) {
  const double two_pi = 6.283185307179586;
  double l = log(u.a);
  double rad = sqrt(-2.0 * l);
  double th = two_pi * u.b;
  return rad * cos(th);
}

__host__ __device__ inline double draw(const aeb_dist& d, uint64_t seed, uint64_t sid, uint64_t i,
                                       uint32_t slot) {
  if (d.kind == AEB_DIST_CONST) return d.p0;
  if (d.kind == AEB_DIST_UNIFORM) {
    U2 u = uniform2(seed, sid, i, slot, 0);
    return d.p0 + (d.p1 - d.p0) * u.a;
  }
  if (d.kind == AEB_DIST_NORMAL) {
    U2 u = uniform2(seed, sid, i, slot, 0);
    return d.p0 + d.p1 * box_muller(u);
  }
  // truncated normal: up to 16 counter-indexed attempts, then clamp
  double val = d.p0;
  for (uint32_t j = 0; j < 16; ++j) {
    U2 u = uniform2(seed, sid, i, slot, j);
    val = d.p0 + d.p1 * box_muller(u);
    if (val >= d.lo && val <= d.hi) return val;
  }
  return val < d.lo ? d.lo : d.hi;
}

// ---------------------------------------------------------------------------
// Perception (sensing latency, dropout and occlusion; Sec. VIII): the delay
// from the start of the rollout to the brake request.  Frames come every
// frame_period seconds; the first floor(occlusion) cannot see the object; a
// later frame j detects it when its uniform (word j mod 2 of the call with
// attempt j / 2 on the DETECT slot) is at least p_dropout; the request
// follows the frame that completes `confirm` detections in a row, plus the
// processing latency.  No such frame up to the horizon: +inf.
// ---------------------------------------------------------------------------
__host__ __device__ inline bool perception_on(const aeb_scenario& s) {
  return !(s.latency.kind == AEB_DIST_CONST && s.latency.p0 == 0.0 && s.frame_period == 0.0);
}

__host__ __device__ inline double trigger_delay(const aeb_scenario& s, uint64_t i) {
  double lat = draw(s.latency, s.seed, s.scenario_id, i, AEB_SLOT_LATENCY);
  if (!(lat > 0.0)) lat = 0.0;
  if (s.frame_period == 0.0) return lat;
  const double occ = draw(s.occlusion, s.seed, s.scenario_id, i, AEB_SLOT_OCCLUSION);
  // frames j = 0 .. last with j * frame_period <= horizon (at most 1e6 + 1)
  const int64_t last = static_cast<int64_t>(floor(s.horizon / s.frame_period));
  int64_t j = 0;
  // the first floor(occ) frames are hidden; beyond the frame count, all of them
  if (occ > 0.0)
    j = occ < static_cast<double>(last + 1) ? static_cast<int64_t>(floor(occ)) : last + 1;
  const int64_t first = j;
  int run = 0;
  U2 u{0.0, 0.0};
  for (; j <= last; ++j) {
    if ((j & 1) == 0 || j == first)
      u = uniform2(s.seed, s.scenario_id, i, AEB_SLOT_DETECT, static_cast<uint32_t>(j >> 1));
    const double uj = (j & 1) ? u.b : u.a;
    run = uj >= s.p_dropout ? run + 1 : 0;
    if (run == s.confirm) return static_cast<double>(j) * s.frame_period + lat;
  }
  return INFINITY;
}

// The closed-loop controller replaces the open-loop command when on.
__host__ __device__ inline bool control_on(const aeb_scenario& s) { return s.ctl_period > 0.0; }

// First step with the brake command for a sample with trigger delay `trig`:
// llround((dead_time + trig) / dt), capped at nmax (a command at or beyond the
// last step is never applied, so every value from nmax up acts the same).
__host__ __device__ inline int64_t command_step(const aeb_scenario& s, double trig, int64_t nmax) {
  const double q = round((s.dead_time + trig) / s.dt);
  return q < static_cast<double>(nmax) ? static_cast<int64_t>(q) : nmax;
}

// One realised parameter vector.
struct Sample {
  double v0, mu, mass, grade, sin_grade, cos_grade, cda, crr, tau, gap, lead_decel;
  double trigger;  // perception delay (s), 0 without perception
  double log_w;    // importance-sampling log likelihood ratio, 0 without
};

// Parameter `slot`: from its proposal when importance sampling covers it
// (adding log p(x) - log q(x) to lw), else from its own distribution.
__host__ __device__ inline double draw_param(const aeb_scenario& s, const aeb_dist& d, uint64_t i,
                                             uint32_t slot, double& lw) {
  if (!((s.is_mask >> slot) & 1)) return draw(d, s.seed, s.scenario_id, i, slot);
  const aeb_dist& q = s.proposal[slot];
  const double x = draw(q, s.seed, s.scenario_id, i, slot);
  const double zp = (x - d.p0) / d.p1;
  const double zq = (x - q.p0) / q.p1;
  lw += log(q.p1 / d.p1) + (0.5 * (zq * zq) - 0.5 * (zp * zp));
  return x;
}

__host__ __device__ inline Sample draw_sample(const aeb_scenario& s, uint64_t i) {
  Sample p;
  double lw = 0.0;
  p.v0 = draw_param(s, s.v0, i, AEB_SLOT_V0, lw);
  p.mu = draw_param(s, s.mu, i, AEB_SLOT_MU, lw);
  p.mass = draw_param(s, s.mass, i, AEB_SLOT_MASS, lw);
  p.grade = draw_param(s, s.grade, i, AEB_SLOT_GRADE, lw);
  p.sin_grade = sin(p.grade);
  p.cos_grade = cos(p.grade);
  p.cda = draw_param(s, s.cda, i, AEB_SLOT_CDA, lw);
  p.crr = draw_param(s, s.crr, i, AEB_SLOT_CRR, lw);
  p.tau = draw_param(s, s.tau, i, AEB_SLOT_TAU, lw);
  p.gap = draw_param(s, s.gap, i, AEB_SLOT_GAP, lw);
  p.lead_decel = draw_param(s, s.lead_decel, i, AEB_SLOT_LEAD, lw);
  p.trigger = perception_on(s) ? trigger_delay(s, i) : 0.0;
  p.log_w = lw;
  return p;
}

// ---------------------------------------------------------------------------
// Per-sample constants of eq. (4)-(6).
//   kd   = ((rho/2) CdA) / m              drag deceleration per v^2
//   c    = g sin(th) + (Crr g) cos(th)    grade plus rolling resistance
//   alim = -(mu g / (1 + (mu h) / L))     eq. (5) solved with signed a < 0
// ---------------------------------------------------------------------------
struct Consts {
  double kd, c, alim;
};

__host__ __device__ inline Consts derive(const aeb_scenario& s, double mu, double mass,
                                         double sin_g, double cos_g, double cda, double crr) {
  Consts k;
  double half_rho = 0.5 * s.rho;
  double drag_num = half_rho * cda;
  k.kd = drag_num / mass;
  double grade_term = s.g * sin_g;
  double roll_coef = crr * s.g;
  double roll_term = roll_coef * cos_g;
  k.c = grade_term + roll_term;
  double mu_g = mu * s.g;
  double mu_h = mu * s.h_cog;
  double transfer = mu_h / s.wheelbase;
  double denom = 1.0 + transfer;
  k.alim = -(mu_g / denom);
  return k;
}

}  // namespace aeb
