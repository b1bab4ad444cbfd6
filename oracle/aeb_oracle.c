/*
 * aeb_oracle.c -- the FP64 reference for the stochastic braking rollout.
 *
 * TEST INFRASTRUCTURE ONLY (see aeb_oracle.h).  Plain sequential C: one sample
 * at a time, every operation written out in the order the model states it.
 *
 * Paper map:
 *   state (x, v, a_brake,actual), command a_brake,cmd ......... eq. (1)-(2)
 *   force balance dv/dt = a - rho Cd Af v^2 / (2m) - g sin(theta)  eq. (4)
 *   friction limit under weight transfer ...................... eq. (5)
 *   first-order actuator lag .................................. eq. (6)
 *   complete system ........................................... eq. (7)-(9)
 *   fixed-step integration, dt = 1 ms, T_max = 10 s ........... Sec. IV-B, IV-D
 *   termination at v <= 0, D_stop = x(t_stop) ................. eq. (3), Sec. V-D
 *   P(collision | H0) = P(D_stop > H0), minimum safe headway .. eq. (20), Sec. VI-C
 *   random inputs drawn from a fixed seed ..................... Sec. IV-B, IV-C
 */
#include "aeb_oracle.h"

#include <limits.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Counter-based generator: Philox4x32-10 as defined by Salmon, Moraes, Dror  */
/* and Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11).  Each     */
/* round multiplies counter words 0 and 2 by two fixed odd constants, keeps   */
/* the 64-bit products, and recombines the high halves with the other two     */
/* counter words and the round key; the key advances by two Weyl increments.  */
/* ------------------------------------------------------------------------ */

static const uint32_t PHILOX_M0 = 0xD2511F53u;
static const uint32_t PHILOX_M1 = 0xCD9E8D57u;
static const uint32_t PHILOX_W0 = 0x9E3779B9u;
static const uint32_t PHILOX_W1 = 0xBB67AE85u;

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += PHILOX_W0;
      k1 += PHILOX_W1;
    }
    uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
    uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    uint32_t n0 = hi1 ^ c1 ^ k0;
    uint32_t n1 = lo1;
    uint32_t n2 = hi0 ^ c3 ^ k1;
    uint32_t n3 = lo0;
    c0 = n0;
    c1 = n1;
    c2 = n2;
    c3 = n3;
  }
  out[0] = c0;
  out[1] = c1;
  out[2] = c2;
  out[3] = c3;
}

/* 52-bit uniform strictly inside (0,1): the top 52 bits of a 64-bit word plus
 * one half, scaled by 2^-52.  Every value is exact in binary64. */
static double word_to_uniform(uint64_t w) {
  double m = (double)(w >> 12);
  return (m + 0.5) * 0x1p-52;
}

void orc_uniform_pair(uint64_t seed, uint64_t scenario_id, uint64_t i, uint32_t slot,
                      uint32_t attempt, double u[2]) {
  uint32_t ctr[4], key[2], o[4];
  ctr[0] = (uint32_t)i;
  ctr[1] = slot | (attempt << 8);
  ctr[2] = (uint32_t)scenario_id;
  ctr[3] = (uint32_t)(scenario_id >> 32);
  key[0] = (uint32_t)seed;
  key[1] = (uint32_t)(seed >> 32);
  orc_philox4x32_10(ctr, key, o);
  uint64_t w0 = ((uint64_t)o[1] << 32) | (uint64_t)o[0];
  uint64_t w1 = ((uint64_t)o[3] << 32) | (uint64_t)o[2];
  u[0] = word_to_uniform(w0);
  u[1] = word_to_uniform(w1);
}

int orc_uniforms(uint64_t seed, uint64_t scenario_id, int64_t first, int64_t count,
                 uint32_t slot, uint32_t attempt, double* out) {
  if (count < 0 || first < 0) return ORC_EINVAL;
  for (int64_t k = 0; k < count; ++k) {
    double u[2];
    orc_uniform_pair(seed, scenario_id, (uint64_t)(first + k), slot, attempt, u);
    out[2 * k] = u[0];
    out[2 * k + 1] = u[1];
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Distributions of the uncertain parameters (eq. (11)-(15) and the uniform   */
/* and truncated forms of the configured workloads).  A normal variate is the */
/* cosine branch of the Box-Muller transform on the two uniforms of one call. */
/* ------------------------------------------------------------------------ */

static const double TWO_PI = 6.283185307179586;  /* binary64 nearest 2*pi */
#define TRUNC_ATTEMPTS 16

static double std_normal(const double u[2]) {
  double lg = log(u[0]);
  double r = sqrt(-2.0 * lg);
  double ang = TWO_PI * u[1];
  return r * cos(ang);
}

double orc_draw(const orc_dist* d, uint64_t seed, uint64_t scenario_id, uint64_t i,
                uint32_t slot) {
  double u[2];
  switch (d->kind) {
    case ORC_D_CONST:
      return d->p0;
    case ORC_D_UNIFORM:
      orc_uniform_pair(seed, scenario_id, i, slot, 0, u);
      return d->p0 + (d->p1 - d->p0) * u[0];
    case ORC_D_NORMAL:
      orc_uniform_pair(seed, scenario_id, i, slot, 0, u);
      return d->p0 + d->p1 * std_normal(u);
    case ORC_D_TRUNC_NORMAL: {
      /* rejection: attempt j uses its own counter; after the last attempt the
       * final candidate is clamped into the support */
      double val = d->p0;
      for (uint32_t j = 0; j < TRUNC_ATTEMPTS; ++j) {
        orc_uniform_pair(seed, scenario_id, i, slot, j, u);
        val = d->p0 + d->p1 * std_normal(u);
        if (val >= d->lo && val <= d->hi) return val;
      }
      if (val < d->lo) return d->lo;
      return d->hi;
    }
    default:
      return NAN;
  }
}

/* ------------------------------------------------------------------------ */
/* Perception trigger delay (see orc_scenario).  Frame j (captured at time    */
/* j * frame_period) sees the object if j >= the occluded frame count and its */
/* own uniform (slot DETECT, word j of the generator calls) is at least       */
/* p_dropout.  The object is confirmed at the frame that completes `confirm`  */
/* consecutive detections; frames are searched until the horizon.             */
/* ------------------------------------------------------------------------ */

static int perception_on(const orc_scenario* s) {
  return !(s->latency.kind == ORC_D_CONST && s->latency.p0 == 0.0 && s->frame_period == 0.0);
}

double orc_trigger_delay(const orc_scenario* s, uint64_t i) {
  const uint64_t seed = s->seed, sid = s->scenario_id;
  double lat = orc_draw(&s->latency, seed, sid, i, ORC_SLOT_LATENCY);
  if (!(lat > 0.0)) lat = 0.0;
  if (s->frame_period == 0.0) return lat;
  double occ = orc_draw(&s->occlusion, seed, sid, i, ORC_SLOT_OCCLUSION);
  const long long frames = (long long)floor(s->horizon / s->frame_period) + 1;
  long long hidden = 0;  /* occluded frames; more than all of them hides every frame */
  if (occ > 0.0) hidden = occ < (double)frames ? (long long)floor(occ) : frames;
  int run = 0;
  for (long long j = 0; j < frames; ++j) {
    int seen = 0;
    if (j >= hidden) {
      double u[2];
      orc_uniform_pair(seed, sid, i, ORC_SLOT_DETECT, (uint32_t)(j / 2), u);
      seen = u[j % 2] >= s->p_dropout;
    }
    run = seen ? run + 1 : 0;
    if (run == s->confirm) return (double)j * s->frame_period + lat;
  }
  return INFINITY;
}

/* ------------------------------------------------------------------------ */
/* Closed-loop controller (see orc_scenario).  A decision at tick m reads the */
/* state after m * period steps: the measured gap and closing speed carry    */
/* the cosine and sine Box-Muller normals of generator call                  */
/* (index, CONTROL slot, attempt m) times their noise sds.                   */
/* ------------------------------------------------------------------------ */

typedef struct {
  long long period;     /* steps between decisions */
  long long next_tick;  /* step of the next decision */
  long long on1, on2;   /* steps from which the warning / full command applies */
  uint32_t tick;        /* decisions taken */
  int stage;
} ctl_state;

static int control_on(const orc_scenario* s) { return s->ctl_period > 0.0; }

static void ctl_init(const orc_scenario* s, ctl_state* c) {
  c->period = llround(s->ctl_period / s->dt);
  c->next_tick = 0;
  c->on1 = c->on2 = LLONG_MAX;
  c->tick = 0;
  c->stage = 0;
}

static void ctl_decide(const orc_scenario* s, const orc_sample* p, ctl_state* c, long long step,
                       long long nd, double gap_true, double closing) {
  double u[2];
  orc_uniform_pair(s->seed, s->scenario_id, p->index, ORC_SLOT_CONTROL, c->tick, u);
  const double r = sqrt(-2.0 * log(u[0]));
  const double ang = TWO_PI * u[1];
  const double g = gap_true + s->noise_gap * (r * cos(ang));
  const double cl = closing + s->noise_v * (r * sin(ang));
  const double ttc = cl > 0.0 ? g / cl : INFINITY;
  const int want = ttc < s->ttc_brake ? 2 : (ttc < s->ttc_warn ? 1 : 0);
  if (want > c->stage) {
    if (want == 2)
      c->on2 = step + nd;
    else
      c->on1 = step + nd;
    c->stage = want;
  }
  c->tick += 1;
  c->next_tick += c->period;
}

static double ctl_command(const orc_scenario* s, const ctl_state* c, long long step) {
  if (step >= c->on2) return s->a_cmd;
  if (step >= c->on1) return s->a_warn;
  return 0.0;
}

/* first step with the brake command: the dead time plus the trigger delay */
static long long command_step(const orc_scenario* s, const orc_sample* p) {
  const double q = (s->dead_time + p->trigger) / s->dt;
  if (!(q < 4.0e18)) return LLONG_MAX;
  return llround(q);
}

/* Parameter `slot`: drawn from its proposal when importance sampling covers
 * it (then its log likelihood ratio log p(x) - log q(x) is added to *log_w),
 * else from its own distribution. */
static double draw_param(const orc_scenario* s, const orc_dist* d, uint64_t i, uint32_t slot,
                         double* log_w) {
  if (!((s->is_mask >> slot) & 1)) return orc_draw(d, s->seed, s->scenario_id, i, slot);
  const orc_dist* q = &s->proposal[slot];
  const double x = orc_draw(q, s->seed, s->scenario_id, i, slot);
  const double zp = (x - d->p0) / d->p1;
  const double zq = (x - q->p0) / q->p1;
  *log_w += log(q->p1 / d->p1) + (0.5 * (zq * zq) - 0.5 * (zp * zp));
  return x;
}

void orc_sample_one(const orc_scenario* s, uint64_t i, orc_sample* p) {
  double lw = 0.0;
  p->v0 = draw_param(s, &s->v0, i, ORC_SLOT_V0, &lw);
  p->mu = draw_param(s, &s->mu, i, ORC_SLOT_MU, &lw);
  p->mass = draw_param(s, &s->mass, i, ORC_SLOT_MASS, &lw);
  p->grade = draw_param(s, &s->grade, i, ORC_SLOT_GRADE, &lw);
  p->sin_grade = sin(p->grade);
  p->cos_grade = cos(p->grade);
  p->cda = draw_param(s, &s->cda, i, ORC_SLOT_CDA, &lw);
  p->crr = draw_param(s, &s->crr, i, ORC_SLOT_CRR, &lw);
  p->tau = draw_param(s, &s->tau, i, ORC_SLOT_TAU, &lw);
  p->gap = draw_param(s, &s->gap, i, ORC_SLOT_GAP, &lw);
  p->lead_decel = draw_param(s, &s->lead_decel, i, ORC_SLOT_LEAD, &lw);
  p->trigger = perception_on(s) ? orc_trigger_delay(s, i) : 0.0;
  p->index = i;
  p->log_w = lw;
}

int orc_sample_range(const orc_scenario* s, int64_t first, int64_t count, double* const cols[13]) {
  if (first < 0 || count < 0) return ORC_EINVAL;
  for (int64_t k = 0; k < count; ++k) {
    orc_sample p;
    orc_sample_one(s, (uint64_t)(first + k), &p);
    cols[0][k] = p.v0;
    cols[1][k] = p.mu;
    cols[2][k] = p.mass;
    cols[3][k] = p.grade;
    cols[4][k] = p.sin_grade;
    cols[5][k] = p.cos_grade;
    cols[6][k] = p.cda;
    cols[7][k] = p.crr;
    cols[8][k] = p.tau;
    cols[9][k] = p.gap;
    cols[10][k] = p.lead_decel;
    cols[11][k] = p.trigger;
    cols[12][k] = p.log_w;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Scenario validation.                                                       */
/* ------------------------------------------------------------------------ */

static int dist_ok(const orc_dist* d) {
  switch (d->kind) {
    case ORC_D_CONST:
      return isfinite(d->p0);
    case ORC_D_UNIFORM:
      return isfinite(d->p0) && isfinite(d->p1) && d->p0 <= d->p1;
    case ORC_D_NORMAL:
      return isfinite(d->p0) && isfinite(d->p1) && d->p1 >= 0.0;
    case ORC_D_TRUNC_NORMAL:
      return isfinite(d->p0) && isfinite(d->p1) && d->p1 >= 0.0 && isfinite(d->lo) &&
             isfinite(d->hi) && d->lo < d->hi;
    default:
      return 0;
  }
}

/* smallest value the distribution can produce (-inf for an untruncated normal) */
static double dist_min(const orc_dist* d) {
  switch (d->kind) {
    case ORC_D_CONST:
      return d->p0;
    case ORC_D_UNIFORM:
      return d->p0;
    case ORC_D_TRUNC_NORMAL:
      return d->lo;
    default:
      return d->p1 == 0.0 ? d->p0 : -INFINITY;
  }
}

int orc_validate(const orc_scenario* s) {
  if (s->n_samples <= 0 || s->n_samples > 0x7fffffffLL) return ORC_EINVAL;
  if (s->integrator != ORC_EULER && s->integrator != ORC_RK4) return ORC_EINVAL;
  if (s->obstacle < ORC_OBS_NONE || s->obstacle > ORC_OBS_LEAD) return ORC_EINVAL;
  if (s->integrator == ORC_RK4 && s->obstacle == ORC_OBS_LEAD) return ORC_EINVAL;
  if (s->impact_exit != 0 && s->impact_exit != 1) return ORC_EINVAL;
  if (s->nofma != 0 && s->nofma != 1) return ORC_EINVAL;
  if (!(s->dt > 0.0) || !isfinite(s->dt)) return ORC_EINVAL;
  if (!(s->horizon > 0.0) || !isfinite(s->horizon)) return ORC_EINVAL;
  if (!(s->dead_time >= 0.0) || !isfinite(s->dead_time)) return ORC_EINVAL;
  double steps = s->horizon / s->dt;
  if (!(steps >= 1.0) || steps > 2147483647.0) return ORC_EINVAL;
  if (!isfinite(s->a_cmd) || !isfinite(s->g) || !isfinite(s->rho) || !isfinite(s->h_cog))
    return ORC_EINVAL;
  if (!(s->wheelbase > 0.0) || !isfinite(s->wheelbase)) return ORC_EINVAL;
  const orc_dist* all[9] = {&s->v0, &s->mu, &s->mass, &s->grade, &s->cda,
                            &s->crr, &s->tau, &s->gap, &s->lead_decel};
  for (int k = 0; k < 9; ++k)
    if (!dist_ok(all[k])) return ORC_EINVAL;
  /* perception: finite distributions, a dropout probability in [0, 1), at
   * most 1e6 frames over the horizon, 1 to 64 confirming detections */
  if (!dist_ok(&s->latency) || !dist_ok(&s->occlusion)) return ORC_EINVAL;
  if (!(s->frame_period >= 0.0) || !isfinite(s->frame_period)) return ORC_EINVAL;
  if (s->frame_period > 0.0 && !(s->horizon / s->frame_period <= 1.0e6)) return ORC_EINVAL;
  if (!(s->p_dropout >= 0.0 && s->p_dropout < 1.0)) return ORC_EINVAL;
  if (s->confirm < 1 || s->confirm > 64) return ORC_EINVAL;
  /* controller: a whole positive number of steps per tick, fewer than 2^24
   * ticks over the horizon, an obstacle to measure, no perception trigger,
   * thresholds >= 0 (+inf allowed), a_cmd <= a_warn <= 0, noise sds >= 0 */
  if (!(s->ctl_period >= 0.0) || !isfinite(s->ctl_period)) return ORC_EINVAL;
  if (s->ctl_period > 0.0) {
    const long long per = llround(s->ctl_period / s->dt);
    if (per < 1) return ORC_EINVAL;
    if (!(s->horizon / s->dt / (double)per < 16777216.0)) return ORC_EINVAL;
    if (s->obstacle == ORC_OBS_NONE || perception_on(s)) return ORC_EINVAL;
    if (!(s->ttc_warn >= 0.0) || !(s->ttc_brake >= 0.0)) return ORC_EINVAL;
    if (!isfinite(s->a_warn) || !(s->a_cmd <= s->a_warn && s->a_warn <= 0.0)) return ORC_EINVAL;
    if (!(s->noise_gap >= 0.0) || !isfinite(s->noise_gap)) return ORC_EINVAL;
    if (!(s->noise_v >= 0.0) || !isfinite(s->noise_v)) return ORC_EINVAL;
  }
  /* importance sampling: normal parameters with normal proposals (not tau,
   * which must stay positive), sds > 0 */
  if (s->is_mask & ~0x1BF) return ORC_EINVAL;
  {
    const orc_dist* nom[9] = {&s->v0, &s->mu, &s->mass, &s->grade, &s->cda,
                              &s->crr, &s->tau, &s->gap, &s->lead_decel};
    for (int j = 0; j < 9; ++j) {
      if (!((s->is_mask >> j) & 1)) continue;
      const orc_dist* q = &s->proposal[j];
      if (nom[j]->kind != ORC_D_NORMAL || q->kind != ORC_D_NORMAL) return ORC_EINVAL;
      if (!(nom[j]->p1 > 0.0) || !(q->p1 > 0.0) || !dist_ok(q)) return ORC_EINVAL;
    }
  }
  /* the explicit actuator update needs dt/tau <= 1 for every sample */
  if (!(dist_min(&s->tau) > 0.0)) return ORC_EINVAL;
  if (s->integrator == ORC_EULER && dist_min(&s->tau) < s->dt) return ORC_EINVAL;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Per-sample constants of the force balance (eq. (4)-(6)).                   */
/* ------------------------------------------------------------------------ */

typedef struct {
  double kd;    /* rho * CdA / (2 m): drag deceleration per v^2 */
  double c;     /* grade plus rolling resistance: g sin(th) + Crr g cos(th) */
  double alim;  /* friction limit solved from eq. (5) with signed a < 0 */
} orc_consts;

static void derive(const orc_scenario* s, const orc_sample* p, orc_consts* k) {
  double half_rho = 0.5 * s->rho;
  double drag_num = half_rho * p->cda;
  k->kd = drag_num / p->mass;
  double grade_term = s->g * p->sin_grade;
  double roll_coef = p->crr * s->g;
  double roll_term = roll_coef * p->cos_grade;
  k->c = grade_term + roll_term;
  /* a >= -mu g (1 + (h/L)(a/g)) holds with equality at a = -mu g / (1 + mu h / L) */
  double mu_g = p->mu * s->g;
  double mu_h = p->mu * s->h_cog;
  double transfer = mu_h / s->wheelbase;
  double denom = 1.0 + transfer;
  k->alim = -(mu_g / denom);
}

static double max2(double a, double b) { return a > b ? a : b; }

/* ------------------------------------------------------------------------ */
/* Explicit Euler, one step per dt, with the termination tests after every    */
/* step: impact (strict x > gap), then stop (v <= 0), then horizon.           */
/* ------------------------------------------------------------------------ */

static void rollout_euler(const orc_scenario* s, const orc_sample* p, int clamp_state,
                          orc_result* r) {
  orc_consts k;
  derive(s, p, &k);
  const double dt = s->dt;
  const double kt = dt / p->tau;
  const long long nd = command_step(s, p);
  const long long nmax = llround(s->horizon / dt);
  const int lead = s->obstacle == ORC_OBS_LEAD;
  const int nofma = s->nofma;

  double x = 0.0, v = p->v0, a = 0.0;
  double xl = 0.0, vl = lead ? p->v0 : 0.0;
  const double al = p->lead_decel;
  const double gap0 = p->gap;
  double margin = (gap0 + xl) - x;
  int collided = 0, end = 0;
  float vimp = 0.0f;
  long long step = 0;
  const int ctl = control_on(s);
  ctl_state cs;
  ctl_init(s, &cs);

  for (;;) {
    double cmd;
    if (ctl) {
      if (step == cs.next_tick) ctl_decide(s, p, &cs, step, nd, (gap0 + xl) - x, v - vl);
      cmd = ctl_command(s, &cs, step);
    } else {
      cmd = step >= nd ? s->a_cmd : 0.0;
    }
    /* realised brake deceleration cannot exceed the friction limit */
    double abe = clamp_state ? a : max2(a, k.alim);
    double v2 = v * v;
    double acc, xn, vn, an;
    if (nofma) {
      acc = (abe - k.kd * v2) - k.c;
      xn = dt * v + x;
      vn = dt * acc + v;
      an = kt * (cmd - a) + a;
    } else {
      acc = fma(-k.kd, v2, abe) - k.c;
      xn = fma(dt, v, x);
      vn = fma(dt, acc, v);
      an = fma(kt, cmd - a, a);
    }
    if (clamp_state) an = max2(an, k.alim);
    double xln = xl, vln = vl;
    if (lead) {
      xln = nofma ? dt * vl + xl : fma(dt, vl, xl);
      double t = nofma ? vl - dt * al : fma(-dt, al, vl);
      vln = t > 0.0 ? t : 0.0;
    }
    x = xn;
    v = vn;
    a = an;
    xl = xln;
    vl = vln;
    ++step;

    double gap_now = gap0 + xl;
    double m = gap_now - x;
    if (m < margin) margin = m;
    if (s->obstacle != ORC_OBS_NONE && x > gap_now) {
      if (!collided) {
        collided = 1;
        vimp = (float)(v - vl);
      }
      if (s->impact_exit || lead) {
        end = ORC_END_IMPACT;
        break;
      }
    }
    if (v <= 0.0) {
      end = ORC_END_STOP;
      break;
    }
    if (step == nmax) {
      end = ORC_END_HORIZON;
      break;
    }
  }
  r->dist = x;
  r->margin = margin;
  r->steps = (int32_t)step;
  r->status = (uint8_t)(end | (collided ? ORC_COLLIDED : 0));
  r->v_impact = vimp;
}

/* ------------------------------------------------------------------------ */
/* Classical fourth-order Runge-Kutta (the paper's integrator, Sec. IV-D),    */
/* written without fused operations.  The brake command is held constant over */
/* each step at its start-of-step value (zero-order hold on the step grid):   */
/* the dead time is a whole number of steps, so the command switches exactly  */
/* on a step boundary and every stage of one step sees the same command.      */
/* ------------------------------------------------------------------------ */

typedef struct {
  double x, v, a;
} orc_state;

static orc_state rhs(const orc_consts* k, double rt, double cmd, orc_state y) {
  orc_state d;
  d.x = y.v;
  d.v = (max2(y.a, k->alim) - k->kd * (y.v * y.v)) - k->c;
  d.a = (cmd - y.a) * rt;
  return d;
}

static orc_state axpy(orc_state y, double h, orc_state d) {
  orc_state o;
  o.x = y.x + h * d.x;
  o.v = y.v + h * d.v;
  o.a = y.a + h * d.a;
  return o;
}

static void rollout_rk4(const orc_scenario* s, const orc_sample* p, orc_result* r) {
  orc_consts k;
  derive(s, p, &k);
  const double dt = s->dt;
  const double h2 = 0.5 * dt;
  const double h6 = dt / 6.0;
  const double rt = 1.0 / p->tau;
  const long long nd = command_step(s, p);
  const long long nmax = llround(s->horizon / dt);
  const double gap0 = p->gap;

  orc_state y = {0.0, p->v0, 0.0};
  double margin = gap0 - y.x;
  int collided = 0, end = 0;
  float vimp = 0.0f;
  long long step = 0;
  const int ctl = control_on(s);
  ctl_state cs;
  ctl_init(s, &cs);

  for (;;) {
    double cmd;
    if (ctl) {
      if (step == cs.next_tick) ctl_decide(s, p, &cs, step, nd, gap0 - y.x, y.v);
      cmd = ctl_command(s, &cs, step);
    } else {
      cmd = step >= nd ? s->a_cmd : 0.0;
    }
    orc_state k1 = rhs(&k, rt, cmd, y);
    orc_state k2 = rhs(&k, rt, cmd, axpy(y, h2, k1));
    orc_state k3 = rhs(&k, rt, cmd, axpy(y, h2, k2));
    orc_state k4 = rhs(&k, rt, cmd, axpy(y, dt, k3));
    orc_state sum;
    sum.x = ((k1.x + 2.0 * k2.x) + 2.0 * k3.x) + k4.x;
    sum.v = ((k1.v + 2.0 * k2.v) + 2.0 * k3.v) + k4.v;
    sum.a = ((k1.a + 2.0 * k2.a) + 2.0 * k3.a) + k4.a;
    y = axpy(y, h6, sum);
    ++step;

    double m = gap0 - y.x;
    if (m < margin) margin = m;
    if (s->obstacle == ORC_OBS_STATIONARY && y.x > gap0) {
      if (!collided) {
        collided = 1;
        vimp = (float)y.v;
      }
      if (s->impact_exit) {
        end = ORC_END_IMPACT;
        break;
      }
    }
    if (y.v <= 0.0) {
      end = ORC_END_STOP;
      break;
    }
    if (step == nmax) {
      end = ORC_END_HORIZON;
      break;
    }
  }
  r->dist = y.x;
  r->margin = margin;
  r->steps = (int32_t)step;
  r->status = (uint8_t)(end | (collided ? ORC_COLLIDED : 0));
  r->v_impact = vimp;
}

void orc_rollout_one(const orc_scenario* s, const orc_sample* p, int clamp_state, orc_result* r) {
  if (s->integrator == ORC_RK4)
    rollout_rk4(s, p, r);
  else
    rollout_euler(s, p, clamp_state, r);
}

int orc_run_range(const orc_scenario* s, int64_t first, int64_t count, double* dist,
                  uint8_t* status, int32_t* steps, double* margin, float* v_impact) {
  if (orc_validate(s) != ORC_OK || first < 0 || count < 0) return ORC_EINVAL;
  for (int64_t k = 0; k < count; ++k) {
    orc_sample p;
    orc_result r;
    orc_sample_one(s, (uint64_t)(first + k), &p);
    orc_rollout_one(s, &p, 0, &r);
    dist[k] = r.dist;
    status[k] = r.status;
    steps[k] = r.steps;
    margin[k] = r.margin;
    v_impact[k] = r.v_impact;
  }
  return ORC_OK;
}

int orc_rollout_given(const orc_scenario* s, const double* const cols[13], int64_t n,
                      int clamp_state, double* dist, uint8_t* status, int32_t* steps,
                      double* margin, float* v_impact) {
  if (n < 0) return ORC_EINVAL;
  for (int64_t k = 0; k < n; ++k) {
    orc_sample p;
    orc_result r;
    p.v0 = cols[0][k];
    p.mu = cols[1][k];
    p.mass = cols[2][k];
    p.grade = cols[3][k];
    p.sin_grade = cols[4][k];
    p.cos_grade = cols[5][k];
    p.cda = cols[6][k];
    p.crr = cols[7][k];
    p.tau = cols[8][k];
    p.gap = cols[9][k];
    p.lead_decel = cols[10][k];
    p.trigger = cols[11][k];
    p.index = (uint64_t)k;
    p.log_w = cols[12][k];
    orc_rollout_one(s, &p, clamp_state, &r);
    dist[k] = r.dist;
    status[k] = r.status;
    steps[k] = r.steps;
    margin[k] = r.margin;
    v_impact[k] = r.v_impact;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Reduction by sorting (eq. (20) and the minimum-safe-headway rule of        */
/* Sec. VI-C).  A sample that did not end in a stop has no stopping distance  */
/* inside the horizon and counts as +infinity (censored).                     */
/* ------------------------------------------------------------------------ */

static int cmp_double(const void* pa, const void* pb) {
  double a = *(const double*)pa, b = *(const double*)pb;
  return (a > b) - (a < b);
}

int orc_weighted_risk(const double* dist, const uint8_t* status, const double* weight, int64_t n,
                      double grid_lo, double grid_hi, int32_t n_grid, double* p, double* se,
                      double* p_collision, double* p_collision_se) {
  if (n < 2 || n_grid < 0 || n_grid == 1 || n_grid > ORC_MAX_GRID) return ORC_EINVAL;
  const double nd = (double)n;
  for (int32_t j = 0; j < n_grid; ++j) {
    const double h = grid_lo + (double)j * ((grid_hi - grid_lo) / (double)(n_grid - 1));
    double s1 = 0.0, s2 = 0.0;
    for (int64_t i = 0; i < n; ++i) {
      const double d = (status[i] & 3) == ORC_END_STOP ? dist[i] : INFINITY;
      if (d > h) {
        s1 += weight[i];
        s2 += weight[i] * weight[i];
      }
    }
    p[j] = s1 / nd;
    se[j] = sqrt(fmax(s2 / nd - p[j] * p[j], 0.0) / (nd - 1.0));
  }
  double c1 = 0.0, c2 = 0.0;
  for (int64_t i = 0; i < n; ++i)
    if (status[i] & ORC_COLLIDED) {
      c1 += weight[i];
      c2 += weight[i] * weight[i];
    }
  *p_collision = c1 / nd;
  *p_collision_se = sqrt(fmax(c2 / nd - (*p_collision) * (*p_collision), 0.0) / (nd - 1.0));
  return ORC_OK;
}

int orc_reduce(const double* dist, const uint8_t* status, const double* margin,
               const float* v_impact, int64_t n, const orc_reduce_req* req, orc_stats* out) {
  if (n <= 0 || req->n_risk < 0 || req->n_risk > ORC_MAX_RISK || req->n_margin_q < 0 ||
      req->n_margin_q > ORC_MAX_MQ || req->n_grid < 0 || req->n_grid > ORC_MAX_GRID ||
      req->n_grid == 1)
    return ORC_EINVAL;
  for (int j = 0; j < req->n_risk; ++j)
    if (!(req->risk[j] >= 0.0 && req->risk[j] < 1.0)) return ORC_EINVAL;
  for (int j = 0; j < req->n_margin_q; ++j)
    if (!(req->margin_q[j] >= 0.0 && req->margin_q[j] < 1.0)) return ORC_EINVAL;
  if (req->n_grid >= 2 && !(req->grid_lo < req->grid_hi)) return ORC_EINVAL;

  memset(out, 0, sizeof(*out));
  out->n = n;
  double sum = 0.0, msum = 0.0;
  double dmin = INFINITY, dmax = -INFINITY, mmin = INFINITY;
  float vmax = 0.0f;
  for (int64_t i = 0; i < n; ++i) {
    int end = status[i] & 3;
    if (status[i] & ORC_COLLIDED) {
      out->n_collide++;
      if (v_impact[i] > vmax) vmax = v_impact[i];
    }
    if (end == ORC_END_STOP) {
      out->n_stop++;
      sum += dist[i];
      if (dist[i] < dmin) dmin = dist[i];
      if (dist[i] > dmax) dmax = dist[i];
    } else if (end == ORC_END_IMPACT) {
      out->n_impact++;
    } else if (end == ORC_END_HORIZON) {
      out->n_horizon++;
    }
    msum += margin[i];
    if (margin[i] < mmin) mmin = margin[i];
  }
  out->p_collision = (double)out->n_collide / (double)n;
  out->v_impact_max = vmax;
  out->margin_min = mmin;
  out->margin_mean = msum / (double)n;
  if (out->n_stop > 0) {
    double mean = sum / (double)out->n_stop;
    out->mean_dist = mean;
    out->dist_min = dmin;
    out->dist_max = dmax;
    if (out->n_stop > 1) {
      double ss = 0.0;
      for (int64_t i = 0; i < n; ++i)
        if ((status[i] & 3) == ORC_END_STOP) {
          double d = dist[i] - mean;
          ss += d * d;
        }
      out->sd_dist = sqrt(ss / (double)(out->n_stop - 1));
    } else {
      out->sd_dist = NAN;
    }
  } else {
    out->mean_dist = NAN;
    out->sd_dist = NAN;
    out->dist_min = NAN;
    out->dist_max = NAN;
  }

  /* censored stopping distances, ascending */
  double* srt = (double*)malloc((size_t)n * sizeof(double));
  if (!srt) return ORC_EINVAL;
  for (int64_t i = 0; i < n; ++i)
    srt[i] = ((status[i] & 3) == ORC_END_STOP) ? dist[i] : INFINITY;
  qsort(srt, (size_t)n, sizeof(double), cmp_double);
  /* H(r): the smallest value with at most floor(r N) samples above it */
  for (int j = 0; j < req->n_risk; ++j) {
    int64_t m = (int64_t)floor(req->risk[j] * (double)n);
    out->headway[j] = srt[n - m - 1];
  }
  /* collision-risk curve: #{D > H0_j} on an even headway grid */
  if (req->n_grid >= 2) {
    double step = (req->grid_hi - req->grid_lo) / (double)(req->n_grid - 1);
    for (int j = 0; j < req->n_grid; ++j) {
      double h0 = req->grid_lo + (double)j * step;
      /* first position whose value is > h0 (binary search on exact compares) */
      int64_t lo = 0, hi = n;
      while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (srt[mid] > h0)
          hi = mid;
        else
          lo = mid + 1;
      }
      out->risk_count[j] = n - lo;
      out->risk_p[j] = (double)(n - lo) / (double)n;
    }
  }
  /* lower quantiles of the clearance margin */
  for (int64_t i = 0; i < n; ++i) srt[i] = margin[i];
  qsort(srt, (size_t)n, sizeof(double), cmp_double);
  for (int j = 0; j < req->n_margin_q; ++j) {
    int64_t m = (int64_t)floor(req->margin_q[j] * (double)n);
    out->margin_q[j] = srt[m];
  }
  free(srt);
  return ORC_OK;
}
