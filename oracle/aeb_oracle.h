/*
 * aeb_oracle.h -- plain, slow, sequential FP64 reference for the Monte Carlo
 * braking rollout of "Real-Time GPU-Accelerated Monte Carlo Evaluation of
 * Safety-Critical AEB Systems Under Uncertainty" (Karjol, Alawneh).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no source with the HIP library: it
 * has its own counter-based generator, its own distributions, its own derived
 * constants and its own integrators, all written from the paper's Sections
 * III-IV and the readings listed in the design notes.
 *
 * Every routine is scalar and handles one sample at a time.  Build with
 *   gcc -O2 -ffp-contract=off -fno-fast-math
 * so that no multiply-add is fused except where fma() is written out.
 */
#ifndef AEB_ORACLE_H
#define AEB_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_EULER = 0, ORC_RK4 = 1 };
enum { ORC_OBS_NONE = 0, ORC_OBS_STATIONARY = 1, ORC_OBS_LEAD = 2 };
enum { ORC_D_CONST = 0, ORC_D_UNIFORM = 1, ORC_D_NORMAL = 2, ORC_D_TRUNC_NORMAL = 3 };
/* status byte: low two bits = why the rollout ended, bit 2 = collision latched */
enum { ORC_END_STOP = 1, ORC_END_IMPACT = 2, ORC_END_HORIZON = 3, ORC_COLLIDED = 4 };
enum { ORC_OK = 0, ORC_EINVAL = -1 };

/* Random-parameter slots: the counter word that separates the draws of one
 * sample (Section IV-B lists the random parameters; the lead-vehicle slot is
 * the future-work extension of Section VIII). */
enum {
  ORC_SLOT_V0 = 0, ORC_SLOT_MU = 1, ORC_SLOT_MASS = 2, ORC_SLOT_GRADE = 3,
  ORC_SLOT_CDA = 4, ORC_SLOT_CRR = 5, ORC_SLOT_TAU = 6, ORC_SLOT_GAP = 7,
  ORC_SLOT_LEAD = 8, ORC_SLOT_LATENCY = 9, ORC_SLOT_OCCLUSION = 10, ORC_SLOT_DETECT = 11,
  ORC_SLOT_CONTROL = 12
};

typedef struct {
  int32_t kind;   /* ORC_D_* */
  int32_t pad;
  double p0, p1;  /* CONST: value p0; UNIFORM: [p0,p1]; NORMAL: mean p0, sd p1 */
  double lo, hi;  /* TRUNC_NORMAL support */
} orc_dist;

typedef struct {
  uint64_t seed;
  uint64_t scenario_id;
  int64_t n_samples;
  int32_t integrator;   /* ORC_EULER | ORC_RK4 */
  int32_t obstacle;     /* ORC_OBS_* */
  int32_t impact_exit;  /* stationary obstacle: end the rollout at impact */
  int32_t nofma;        /* 1: Euler uses separate multiply and add (paper's literal rule) */
  double dt, horizon, dead_time, a_cmd, g, rho, h_cog, wheelbase;
  orc_dist v0, mu, mass, grade, cda, crr, tau, gap, lead_decel;
  /* Perception (the sensing effects Section VIII lists as future work): the
   * brake command starts after the dead time plus a per-sample trigger delay,
   * the sensing latency plus the time until the object is confirmed.  Frames
   * arrive every frame_period seconds; the first `occlusion` frames cannot
   * see the object; a visible frame misses it with probability p_dropout;
   * `confirm` consecutive detections confirm it.  frame_period = 0 leaves the
   * latency alone.  latency = CONST 0 and frame_period = 0: no perception. */
  orc_dist latency;    /* seconds, clamped at 0 */
  orc_dist occlusion;  /* frames, rounded down, clamped at 0 */
  double frame_period, p_dropout;
  int32_t confirm;
  int32_t pad2;
  /* Closed-loop controller (the controller assessment Section VIII names):
   * every ctl_period seconds (a whole number of steps, llround(ctl_period /
   * dt)) it measures the gap and the closing speed with additive normal
   * noise (sd noise_gap, noise_v), forms TTC = gap / closing speed (+inf if
   * the measured closing speed is not positive) and raises its stage, which
   * never falls: TTC < ttc_warn -> stage 1 (command a_warn), TTC < ttc_brake
   * -> stage 2 (command a_cmd); a new stage's command starts dead_time
   * later.  ctl_period = 0: the open-loop command of dead_time. */
  double ctl_period, ttc_warn, ttc_brake, a_warn, noise_gap, noise_v;
  /* Importance sampling (rare-event estimation, Section VIII): parameter j
   * (slot order v0 .. lead_decel) with bit j of is_mask set is drawn from
   * proposal[j] instead of its distribution; both must be NORMAL.  The
   * sample's likelihood ratio p(xi) / q(xi) is the product over those
   * parameters of (sd_q / sd_p) exp(z_q^2 / 2 - z_p^2 / 2), z the
   * standardised value under each. */
  int32_t is_mask;
  int32_t pad3;
  orc_dist proposal[9];
} orc_scenario;

/* One sample's realised parameter vector (xi^(i) of Section IV-A). */
typedef struct {
  double v0, mu, mass, grade, sin_grade, cos_grade, cda, crr, tau, gap, lead_decel;
  double trigger;  /* perception trigger delay (s); +inf: the object is never confirmed */
  uint64_t index;  /* the sample's index (keys the controller's measurement noise) */
  double log_w;    /* log likelihood ratio of importance sampling (0 without) */
} orc_sample;

typedef struct {
  double dist;      /* x at exit (D_stop of eq. (3)/(10) when the exit is a stop) */
  double margin;    /* min over steps of (gap0 + x_lead) - x */
  int32_t steps;    /* number of integration steps taken */
  uint8_t status;   /* ORC_END_* | ORC_COLLIDED */
  float v_impact;   /* ego minus lead speed at the first crossing, else 0 */
} orc_result;

#define ORC_MAX_RISK 16
#define ORC_MAX_MQ 4
#define ORC_MAX_GRID 1024

typedef struct {
  int32_t n_risk, n_margin_q, n_grid, pad;
  double risk[ORC_MAX_RISK];        /* risk levels r in [0,1) for headways H(r) */
  double margin_q[ORC_MAX_MQ];      /* lower quantile levels p in [0,1) of the margin */
  double grid_lo, grid_hi;          /* headway grid for the collision-risk curve */
} orc_reduce_req;

typedef struct {
  int64_t n, n_collide, n_stop, n_impact, n_horizon;
  double p_collision, mean_dist, sd_dist, dist_min, dist_max;
  double headway[ORC_MAX_RISK];
  double margin_min, margin_mean;
  double margin_q[ORC_MAX_MQ];
  float v_impact_max;
  int32_t pad;
  int64_t risk_count[ORC_MAX_GRID];
  double risk_p[ORC_MAX_GRID];
} orc_stats;

int orc_validate(const orc_scenario* s);

/* Philox4x32 with 10 rounds (Salmon et al., SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* The two uniforms of one generator call: counter (i, slot | attempt<<8,
 * scenario id), key = seed.  Each is ((w >> 12) + 1/2) * 2^-52. */
void orc_uniform_pair(uint64_t seed, uint64_t scenario_id, uint64_t i, uint32_t slot,
                      uint32_t attempt, double u[2]);
int orc_uniforms(uint64_t seed, uint64_t scenario_id, int64_t first, int64_t count,
                 uint32_t slot, uint32_t attempt, double* out /* 2*count */);

double orc_draw(const orc_dist* d, uint64_t seed, uint64_t scenario_id, uint64_t i,
                uint32_t slot);
void orc_sample_one(const orc_scenario* s, uint64_t i, orc_sample* out);

/* Perception trigger delay of sample i (seconds, +inf if never confirmed). */
double orc_trigger_delay(const orc_scenario* s, uint64_t i);

/* SoA parameter columns, in this order: v0 mu mass grade sin_grade cos_grade
 * cda crr tau gap lead_decel trigger log_weight.  cols[c] points at `count`
 * doubles. */
int orc_sample_range(const orc_scenario* s, int64_t first, int64_t count, double* const cols[13]);

void orc_rollout_one(const orc_scenario* s, const orc_sample* p, int clamp_state, orc_result* r);

/* Draw and roll out samples [first, first+count). */
int orc_run_range(const orc_scenario* s, int64_t first, int64_t count, double* dist,
                  uint8_t* status, int32_t* steps, double* margin, float* v_impact);

/* Roll out caller-given parameter columns (same order as orc_sample_range). */
int orc_rollout_given(const orc_scenario* s, const double* const cols[13], int64_t n,
                      int clamp_state, double* dist, uint8_t* status, int32_t* steps,
                      double* margin, float* v_impact);

/* Importance-sampling estimates over the samples' weights w (likelihood
 * ratios): for each headway H0_j of the grid, P(D > H0_j) = sum w 1[D > H0_j]
 * / n with D censored to +inf unless the sample stopped, and its standard
 * error sqrt((sum w^2 1[.] / n - P^2) / (n - 1)); the same for the collision
 * flag.  Plain sums in index order. */
int orc_weighted_risk(const double* dist, const uint8_t* status, const double* weight, int64_t n,
                      double grid_lo, double grid_hi, int32_t n_grid, double* p, double* se,
                      double* p_collision, double* p_collision_se);

int orc_reduce(const double* dist, const uint8_t* status, const double* margin,
               const float* v_impact, int64_t n, const orc_reduce_req* req, orc_stats* out);

#ifdef __cplusplus
}
#endif
#endif
