/*
 * aeb.h -- C ABI of the MI355X Monte Carlo library for emergency-braking (AEB)
 * evaluation under uncertainty.
 *
 * The operations follow "Real-Time GPU-Accelerated Monte Carlo Evaluation of
 * Safety-Critical AEB Systems Under Uncertainty" (Karjol, Alawneh):
 *   - per-sample parameter vectors xi^(i) drawn from a fixed seed (Sec. IV-A..C);
 *   - a rollout of the longitudinal model of eq. (1)-(9) per sample until the
 *     vehicle stops (eq. (3), (10)), integrated with a fixed step (Sec. IV-D);
 *   - the statistics of Sec. VI: P(collision | H0) = P(D_stop > H0) (eq. (20)),
 *     the collision-risk curve and minimum safe headways (Sec. VI-C), moments of
 *     the stopping distance (Sec. VI-B, Table I).
 * Extensions beyond the paper, all named in its future-work section (Sec. VIII):
 *   brake dead time, rolling resistance, a decelerating lead vehicle, and an
 *   FP32 form with compensated summation (mixed precision).
 *
 * Conventions
 *   - Every function returns AEB_OK (0) or a negative AEB_E* code; no C++
 *     exception crosses this boundary.  aeb_last_error() gives a message for the
 *     last failure on the calling thread.
 *   - Pointers documented as "device" must point at memory of the current HIP
 *     device (hipMalloc'd, e.g. by torch); "host" pointers at ordinary memory.
 *     The caller owns every pointer it passes; the library never frees them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the legacy default
 *     stream).  Device work is enqueued on it; functions documented as
 *     "asynchronous" return before the work completes.
 *   - All functions act on the HIP device that is current on the calling thread.
 *   - The library keeps a per-device pool of scratch blocks for sorting and
 *     reduction partials; it grows on demand (hipMalloc) and lives until
 *     process exit.  A call that needs scratch (aeb_rollout, aeb_reduce,
 *     aeb_batch_rollout, aeb_batch_reduce, aeb_autotune) holds its blocks
 *     while it enqueues work and then fences them with an event on its
 *     stream; another call reuses a block only once that work is done (or
 *     after its stream waits for the event on the device), and a block is
 *     freed to grow it only after its event has completed.  Calls on
 *     different streams and threads may therefore be in flight at once.
 *     These calls cannot be captured into a caller's graph (AEB_EINVAL on a
 *     capturing stream): record graphs with aeb_graph_create*.
 */
#ifndef AEB_H
#define AEB_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ---- */
#define AEB_OK 0
#define AEB_EINVAL (-1)    /* an argument or scenario failed validation */
#define AEB_ENOMEM (-2)    /* a device or host allocation failed, or a request exceeds capacity */
#define AEB_EAGAIN (-3)    /* not ready yet (serving: request pending, queue full) */
#define AEB_EDEVICE (-4)   /* a HIP runtime call failed */
#define AEB_ENOTFOUND (-5) /* unknown ticket */

/* ---- enumerations ---- */
enum { AEB_EULER = 0, AEB_RK4 = 1 };                 /* integrator (Sec. IV-D) */
enum { AEB_OBS_NONE = 0, AEB_OBS_STATIONARY = 1, AEB_OBS_LEAD = 2 };
enum { AEB_DIST_CONST = 0, AEB_DIST_UNIFORM = 1, AEB_DIST_NORMAL = 2, AEB_DIST_TRUNC_NORMAL = 3 };
/* arithmetic of the rollout: FP64; FP32 compensated with samples whose outcome
 * lies within the single-precision band of the collision boundary flagged; the
 * same with the flagged samples recomputed in FP64 */
enum { AEB_FP64 = 0, AEB_FP32C = 1, AEB_FP32C_FIXUP = 2 };
/* status byte of one sample: low two bits = why it ended, bit 2 = collision
 * latched, bit 3 = FP32 outcome within the band of the collision boundary */
enum { AEB_END_STOP = 1, AEB_END_IMPACT = 2, AEB_END_HORIZON = 3, AEB_COLLIDED = 4,
       AEB_BOUNDARY = 8 };
/* counter slots of the random parameters, one generator stream each */
enum {
  AEB_SLOT_V0 = 0, AEB_SLOT_MU = 1, AEB_SLOT_MASS = 2, AEB_SLOT_GRADE = 3, AEB_SLOT_CDA = 4,
  AEB_SLOT_CRR = 5, AEB_SLOT_TAU = 6, AEB_SLOT_GAP = 7, AEB_SLOT_LEAD = 8,
  AEB_SLOT_LATENCY = 9, AEB_SLOT_OCCLUSION = 10, AEB_SLOT_DETECT = 11, AEB_SLOT_CONTROL = 12
};

/* Distribution of one uncertain parameter (eq. (11)-(15) use NORMAL).
 * CONST: value p0.  UNIFORM: p0 + (p1 - p0) u.  NORMAL: p0 + p1 z with z the
 * cosine branch of Box-Muller.  TRUNC_NORMAL: NORMAL redrawn (attempt j uses
 * its own counter, j < 16) until it falls in [lo, hi], then clamped. */
typedef struct {
  int32_t kind;
  int32_t reserved;
  double p0, p1, lo, hi;
} aeb_dist;

/* One braking scenario (Sec. III-IV).  Units SI; angles in radians.
 *   seed, scenario_id: key and counter words of the generator; sample i of a
 *     scenario is a pure function of (seed, scenario_id, i).
 *   n_samples: N, 1 <= N <= 2^31 - 1.
 *   integrator: AEB_EULER (explicit Euler, four fused multiply-adds per step
 *     unless nofma) or AEB_RK4 (classical RK4, no fused operations).
 *   nofma: 1 for the paper's rule of no fused operations in AEB_FP64 explicit
 *     Euler (each multiply-add a rounded product and a rounded sum); the FP32
 *     compensated forms have their own arithmetic and ignore it (the fix-up
 *     mode recomputes its flagged samples in the FP64 form it names).
 *   obstacle: NONE (only the stopping distance), STATIONARY (obstacle at the
 *     sampled gap; the rollout runs to a stop with the collision flag latched,
 *     or ends at impact if impact_exit), LEAD (lead vehicle starting at the
 *     sampled gap with the ego's initial speed and braking at the sampled
 *     lead_decel until it stands still; the rollout ends at impact).  LEAD needs
 *     AEB_EULER.
 *   dt, horizon: step and T_max; the rollout takes at most llround(horizon/dt)
 *     steps.  dead_time: the brake command is zero for the first
 *     llround((dead_time + trigger)/dt) steps and a_cmd afterwards, trigger
 *     being the sample's perception delay (0 without perception).
 *   g, rho, h_cog, wheelbase: eq. (4)-(5) constants.
 *   v0 .. lead_decel: distributions; cda is the product C_d A_f (m^2), grade is
 *     theta, tau the actuator time constant of eq. (6).
 *   Perception (sensing latency, dropout and occlusion, the perception effects
 *   of Sec. VIII), giving each sample a brake-trigger delay:
 *     latency: processing delay (s), values below 0 taken as 0.
 *     frame_period: sensing period P (s); 0 = no frames, trigger = latency.
 *     occlusion: frames during which the object is hidden: the first
 *       floor(occlusion) frames (values below 0 taken as 0) cannot detect it.
 *     p_dropout: probability in [0, 1) that a later frame misses the object;
 *       frame j's decision uses the uniform of word j mod 2 of the generator
 *       call (i, AEB_SLOT_DETECT | (j / 2) << 8, ...), detected if u >= p.
 *     confirm: detections in a row (1..64) that confirm the object.
 *     trigger = J P + latency with J the first frame that completes `confirm`
 *     consecutive detections, searched over frames j with j P <= horizon;
 *     +inf (no braking) if there is none.  latency CONST 0 and frame_period 0
 *     switch perception off (trigger = 0) and draw nothing.
 *   Closed-loop controller (the controller assessment of Sec. VIII), on when
 *   ctl_period > 0; replaces the open-loop command, needs an obstacle and no
 *   perception:
 *     ctl_period: decision period, rounded to S = llround(ctl_period/dt) >= 1
 *       steps; decision m reads the state after m S steps.
 *     noise_gap, noise_v: sds of additive normal noise on the measured gap
 *       (gap + x_lead - x) and closing speed (v - v_lead): the cosine and sine
 *       Box-Muller normals of the call (i, AEB_SLOT_CONTROL | m << 8, ...).
 *     TTC = measured gap / measured closing speed (+inf if the latter <= 0);
 *     the controller's stage only rises: TTC < ttc_warn -> 1 (command a_warn,
 *     a_cmd <= a_warn <= 0), TTC < ttc_brake -> 2 (command a_cmd).  The
 *     command of a stage raised at decision step k applies from step
 *     k + llround(dead_time/dt).
 *   Importance sampling (rare-event estimation, Sec. VIII): parameter j in
 *   slot order (v0, mu, mass, grade, cda, crr, tau, gap, lead_decel) with bit
 *   j of is_mask set is drawn from proposal[j] instead of its distribution
 *   (both NORMAL with sd > 0; not tau).  The sample's log likelihood ratio
 *   log p(xi) - log q(xi) is the sum over those parameters of
 *   log(sd_q / sd_p) + (z_q^2 / 2 - z_p^2 / 2), z the standardised value
 *   under each; its exponential is the sample's weight. */
typedef struct {
  uint64_t seed;
  uint64_t scenario_id;
  int64_t n_samples;
  int32_t integrator;
  int32_t obstacle;
  int32_t impact_exit;
  int32_t nofma;
  double dt, horizon, dead_time, a_cmd, g, rho, h_cog, wheelbase;
  aeb_dist v0, mu, mass, grade, cda, crr, tau, gap, lead_decel;
  aeb_dist latency, occlusion;
  double frame_period, p_dropout;
  int32_t confirm;
  int32_t reserved2;
  double ctl_period, ttc_warn, ttc_brake, a_warn, noise_gap, noise_v;
  int32_t is_mask;
  int32_t reserved3;
  aeb_dist proposal[9];
} aeb_scenario;

/* Structure-of-arrays parameter columns, each `n` doubles (host or device,
 * as the called function states).  sin_grade/cos_grade hold sin/cos of grade;
 * trigger the perception delay in seconds (+inf: never confirmed).  A NULL
 * trigger column reads as zeros; a scenario with perception needs it.
 * log_weight: the importance-sampling log likelihood ratio; NULL reads as
 * zeros; a scenario with importance sampling needs it. */
typedef struct {
  double *v0, *mu, *mass, *grade, *sin_grade, *cos_grade, *cda, *crr, *tau, *gap, *lead_decel;
  double* trigger;
  double* log_weight;
  int64_t n;
} aeb_params;

/* Per-sample outputs (device), each `n` elements:
 *   dist: position x at exit (the stopping distance D_stop when status is STOP);
 *   status: AEB_END_* | AEB_COLLIDED;  steps: integration steps taken;
 *   margin: min over steps of (gap + x_lead) - x;
 *   v_impact: ego minus lead speed at the first step with x > gap + x_lead, else 0;
 *   weight: optional (NULL: not written); the sample's importance-sampling
 *     weight exp(log likelihood ratio), 1 without importance sampling.  A
 *     reduction over outputs with weights adds the weighted estimates. */
typedef struct {
  double* dist;
  uint8_t* status;
  int32_t* steps;
  double* margin;
  float* v_impact;
  double* weight;
  int64_t n;
} aeb_outputs;

#define AEB_MAX_RISK 16
#define AEB_MAX_MARGIN_Q 4
#define AEB_MAX_GRID 1024

/* What aeb_reduce computes beyond the counts and moments:
 *   risk[j] (0 <= r < 1): minimum safe headway H(r) = the smallest sample value v
 *     with #{D_i > v} <= floor(r N), D censored to +inf unless status is STOP;
 *   margin_q[j] (0 <= p < 1): lower quantile = the (floor(p N)+1)-th smallest margin;
 *   grid: n_grid (0 or 2..1024) headways H0_j = grid_lo + j (grid_hi - grid_lo)/(n_grid-1)
 *     for the collision-risk curve P(D > H0_j). */
typedef struct {
  int32_t n_risk, n_margin_q, n_grid, reserved;
  double risk[AEB_MAX_RISK];
  double margin_q[AEB_MAX_MARGIN_Q];
  double grid_lo, grid_hi;
} aeb_reduce_req;

/* Statistics of one batch of outputs.  Counts are exact (n_boundary counts
 * AEB_BOUNDARY samples); p_collision and
 * risk_p are count/N with one correctly rounded division; mean/sd are over
 * STOP samples (sd with N_stop - 1; NaN when undefined); headway/margin_q are
 * exact order statistics of the outputs. */
typedef struct {
  int64_t n, n_collide, n_stop, n_impact, n_horizon, n_boundary;
  double p_collision, mean_dist, sd_dist, dist_min, dist_max;
  double headway[AEB_MAX_RISK];
  double margin_min, margin_mean;
  double margin_q[AEB_MAX_MARGIN_Q];
  float v_impact_max;
  int32_t reserved;
  int64_t risk_count[AEB_MAX_GRID];
  double risk_p[AEB_MAX_GRID];
  /* with weights (importance sampling): weighted = 1 and, with w the
   * weights, P(collision) = sum w [collided] / N and on the grid
   * P(D > H0_j) = sum w [D > H0_j] / N, each with its standard error
   * sqrt((sum w^2 [.] / N - P^2) / (N - 1)); the sums are exact (128-bit
   * fixed point scaled to the largest weight), so repeated calls give the
   * same bits.  weighted = 0 without weights; -1 if a weight was not finite
   * and >= 0 (the weighted fields are then NaN). */
  int32_t weighted;
  int32_t reserved2;
  double p_collision_w, p_collision_se, weight_mean;
  double risk_pw[AEB_MAX_GRID];
  double risk_se[AEB_MAX_GRID];
} aeb_stats;

/* Message of the last failure on this thread ("" if none).  Library
 * plumbing; no passage of the paper defines it. */
const char* aeb_last_error(void);

/* Library ABI version (increments on incompatible changes).  Library
 * plumbing; no passage of the paper defines it. */
int aeb_version(void);

/* Validate a scenario: AEB_OK or AEB_EINVAL (with aeb_last_error() set).
 * The physical constraints come from the model of Sec. III: a positive
 * actuator time constant (eq. (6)), a positive wheelbase (eq. (5)), a step
 * that the explicit update of eq. (7)-(9) keeps stable (dt <= tau); the
 * others bound what the kernels' integer step counters can hold.
 * Rejects N outside [1, 2^31-1]; dt, horizon not positive and finite;
 * horizon/dt outside [1, 2^31-1]; negative dead_time; wheelbase <= 0; unknown
 * enums; non-finite distribution parameters, sd < 0, uniform p0 > p1,
 * truncation lo >= hi; a tau distribution that can reach 0 (or, for Euler,
 * values below dt); RK4 combined with a lead vehicle; for perception:
 * frame_period negative or not finite, more than 1e6 frames over the horizon,
 * p_dropout outside [0, 1), confirm outside [1, 64]; for the controller:
 * ctl_period negative, not finite or below half a step, 2^24 or more
 * decisions over the horizon, no obstacle, perception on, a TTC threshold
 * below 0 or NaN, a_warn outside [a_cmd, 0], noise sds negative or not
 * finite. */
int aeb_validate(const aeb_scenario* scn);

/* Raw generator output (Sec. IV-B "fixed seed"; Philox4x32-10 of Salmon et
 * al., SC'11): for sample i in [first, first+count) the call with counter
 * (i, slot | attempt << 8, lo32(scenario_id), hi32(scenario_id)) and key
 * (lo32(seed), hi32(seed)) yields words o0..o3; out[2k] and out[2k+1] are
 * ((w >> 12) + 0.5) * 2^-52 for w = o1:o0 and o3:o2.  `out` is host memory
 * (on_device = 0, computed on the host) or device memory (on_device = 1,
 * computed by a kernel, asynchronous on `stream`).  The two sides give
 * bit-identical values.  i must stay below 2^32. */
int aeb_uniforms(uint64_t seed, uint64_t scenario_id, int64_t first, int64_t count, uint32_t slot,
                 uint32_t attempt, double* out, int on_device, void* stream);

/* Draw parameter vectors xi^(i) for samples [first, first+count) into `out`
 * (columns of at least `count` doubles; out->n is ignored).  on_device = 0:
 * the paper's plain method (Sec. IV-C) -- drawn on the host (all host cores,
 * host libm), `out` host memory, synchronous.  on_device = 1: drawn by a
 * kernel into device columns, asynchronous on `stream`; uniforms are
 * bit-identical to the host's, transcendentals may differ by a few ulp. */
int aeb_sample_params(const aeb_scenario* scn, int64_t first, int64_t count, const aeb_params* out,
                      int on_device, void* stream);

/* Roll out all scn->n_samples samples (Sec. IV-D, V): per sample, integrate
 * eq. (7)-(9) from x = 0, v = v0, a = 0 until v <= 0 (STOP), the obstacle is
 * passed (IMPACT, if the rollout ends there) or the horizon is reached
 * (HORIZON), and write one entry of each output column.
 *   params: device parameter columns with params->n == n_samples (the plain
 *     method), or NULL to draw each sample's parameters inside the kernel from
 *     the counter generator (no per-sample input traffic).
 *   precision: AEB_FP64 (results equal to a sequential FP64 evaluation of the
 *     same steps), AEB_FP32C (FP32 state with compensated distance and, for
 *     long rollouts, compensated speed; FP64 derived constants, final
 *     distance and collision decision; samples whose distance or clearance is
 *     within 1 mm + 1e-4 gap of the obstacle -- the form's relative distance
 *     tolerance at the obstacle -- get AEB_BOUNDARY in their status)
 *     or AEB_FP32C_FIXUP (as AEB_FP32C, then the flagged samples are
 *     recomputed in FP64, so every collision flag is exact).  A scenario with
 *     the closed-loop controller takes AEB_FP64 only (AEB_EINVAL otherwise):
 *     the block-structured path with blocks that end at every decision (both
 *     Euler forms and RK4).  The
 *     block-structured path counts steps in 32 bits: a horizon plus dead time
 *     beyond 2^31 - 4096 steps takes the checked FP64 kernel (AEB_FP32C:
 *     AEB_EINVAL).
 *   out: device output columns with out->n == n_samples.
 * Asynchronous on `stream`.  May grow the scratch arena on first use. */
int aeb_rollout(const aeb_scenario* scn, const aeb_params* params, int precision,
                const aeb_outputs* out, void* stream);

/* For callers that cannot allocate device memory while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * aeb_rollout with the same arguments, results and errors, whose scratch is a
 * fixed library-owned device array of AEB_NOALLOC_SCRATCH_BYTES per device
 * instead of the growable pool.  The array holds the sorted path's per-sample
 * job records, sort keys and permutation, command steps and FP32 fix-up list
 * (80 bytes per sample, 88 with a lead vehicle, plus 66 KB): 32 MiB covers
 * 380,544 samples with a lead vehicle and 418,604 without.  A scenario
 * that needs more returns AEB_ENOMEM (use aeb_rollout); nothing is enqueued
 * then.  The call makes no hipMalloc/hipFree or other allocation and no
 * synchronisation, so it can be captured into a caller's graph.  Each device
 * holds its array from the library's first use of it until the process ends;
 * every call on one device uses that device's array and overwrites it, so
 * calls whose work overlaps on one device (two streams, two threads, or a
 * call made before an earlier one's kernels have run) race and give wrong
 * results: order them on one stream or synchronise between them.  The array
 * keeps the last call's contents; the kernels clear what must start at zero.
 * The timing hooks (aeb_timing_enable) are off inside this call.
 * Asynchronous on `stream`. */
#define AEB_NOALLOC_SCRATCH_BYTES (32LL << 20)
int aeb_rollout_noalloc(const aeb_scenario* scn, const aeb_params* params, int precision,
                        const aeb_outputs* out, void* stream);

/* Batched rollout (an extension: the paper evaluates one scenario per launch,
 * Sec. V-A; many small launches sit in its kernel-overhead regime, Sec. VI-E,
 * and one launch over many scenarios leaves it).  Each sample is the rollout
 * of aeb_rollout (Sec. IV-D, V).
 * All samples of n_scn scenarios in one sorted launch of the
 * persistent kernel (one lane per sample, wavefronts claiming chunks of the
 * length-sorted permutation), each sample's parameters drawn in-kernel from
 * (seed, scenario_id, index) of its scenario.  Scenarios may differ in every
 * distribution, N, dt, horizon, dead time and a_cmd, but must share
 * integrator, obstacle, impact_exit and nofma; sum of n_samples <= 2^32 - 1.
 *   scns: host array of n_scn scenarios (n_scn >= 1).
 *   outs: host array of n_scn output descriptors (device columns,
 *     outs[j].n == scns[j].n_samples); results equal those of aeb_rollout
 *     with params == NULL on each scenario alone.
 *   precision: AEB_FP64 or AEB_FP32C (AEB_FP32C_FIXUP is not accepted).
 * Returns after the launch has been enqueued and its (host) scenario tables
 * consumed; the outputs are ready after a sync of `stream`. */
int aeb_batch_rollout(const aeb_scenario* scns, int n_scn, int precision, const aeb_outputs* outs,
                      void* stream);

/* The statistics of Sec. VI (eq. (20), Sec. VI-B, VI-C) per scenario of a
 * batch: stats[j] (host array of n_scn) receives exactly what aeb_reduce(outs[j],
 * req) gives, bit for bit.  The sets are reduced together: every kernel of the
 * reduction covers a group of consecutive sets (each with its own scratch,
 * up to 256 MiB of scratch per group), so a batch of many small scenarios
 * costs a few launch sequences rather than one per scenario.  Sets with and
 * without importance-sampling weights may be mixed.  Uses the scratch pool;
 * waits for completion. */
int aeb_batch_reduce(const aeb_outputs* outs, int n_scn, const aeb_reduce_req* req,
                     aeb_stats* stats, void* stream);

/* Profiling aid for the GPU execution time the paper measures (Sec. VI-E,
 * eq. (17)).  While enabled on the calling thread, aeb_rollout brackets
 * its integration kernel with two HIP events on its stream; aeb_timing_last
 * waits for the second and returns the kernel's duration in milliseconds for
 * the last aeb_rollout call of this thread (AEB_EAGAIN if there was none). */
int aeb_timing_enable(int on);
int aeb_timing_last(float* ms);

/* Lane accounting of the last timed aeb_rollout (or aeb_batch_rollout) on
 * this thread, the measure of the sample-per-lane mapping that the paper's
 * discussion of divergence from early termination (Sec. V-C) calls for:
 * *wave_sample_steps = the sum over the integration kernel's wavefront
 * chunks of the steps the wavefront ran times its sample slots (64, or 128
 * with two samples per lane).  The sum of the launch's steps output over it
 * is the lane efficiency, the fraction of lane-steps that advanced a sample.
 * Waits for that kernel.  AEB_EAGAIN if there was no timed launch, or if it
 * ran the checked one-sample-per-lane kernel (horizons beyond the block
 * path), which keeps no such count. */
int aeb_timing_lanes(uint64_t* wave_sample_steps);

/* Self-check of the closed-loop controller's decision screen (Sec. VIII's
 * controller: measured TTC from noisy gap and closing speed).  Where the
 * noise can change a decision, the rollout kernels first estimate it with
 * the GPU's single-precision log2, sqrt, sin and cos instructions inside an
 * error box and take the exact double-precision evaluation only where the
 * box straddles a threshold, so decisions equal the exact ones provided the
 * instructions stay within the box's bounds.  This call measures their
 * largest errors on the device over every input that can reach them (about
 * 2.5e9 evaluations, a few milliseconds) and writes measured[0..3] (log2
 * relative to max(1, |log2 a|), sqrt relative, sin and cos of 2 pi b
 * absolute) and the bounds the screen assumes, bounds[0..3].  Every
 * measured value must not exceed its bound.  Allocates 32 bytes of device
 * memory; synchronises `stream`. */
int aeb_ctl_approx_check(double* measured, double* bounds, void* stream);

/* The natural logarithm, sine and cosine that the controller's exact-stage
 * decision uses (the measurement noise's Box-Muller radius and angle, Sec.
 * VIII's controller), written for the arguments that reach them (a in
 * [2^-53, 1], x in [0, 2 pi)) and accurate to within an ulp there.  For i <
 * n: log_a[i] = log(a[i]), sin_x[i] = sin(x[i]), cos_x[i] = cos(x[i]).  With
 * on_device the five arrays are device memory and the call is asynchronous on
 * `stream`; otherwise they are host memory and the host evaluates the same
 * arithmetic (the results are meant to be the same bits).  n = 0 does
 * nothing; n < 0 or a null array with n > 0 returns AEB_EINVAL. */
int aeb_ctl_math(const double* a, const double* x, int64_t n, double* log_a, double* sin_x,
                 double* cos_x, int on_device, void* stream);

/* Diagnostic for the measurement (not the method): a kernel of known
 * instruction counts, against which the VALU counters of a profiler are
 * checked before they are read on the rollout kernels.  `threads` lanes (a
 * multiple of 256) each run `iters` rounds of 8 independent fused
 * multiply-adds in double precision (fp32 = 0) or single precision (fp32 !=
 * 0), then add their 8 values up (7 adds, no multiplies); each lane writes
 * its sum to out[lane] (device memory of `threads` doubles or floats).
 * Asynchronous on `stream`; AEB_EINVAL for a bad size. */
int aeb_valu_probe(int fp32, int64_t threads, int iters, void* out, void* stream);

/* Metric of the exact order statistics (Sec. VI-C headways, margin
 * quantiles): the number of reductions (aeb_reduce, aeb_batch_reduce per set,
 * graphs, serving) since the library was loaded whose selection fell back
 * from the in-LDS sort of one value bin (a bin with more than 8,192 samples,
 * e.g. many equal values) to the radix select over the whole array. */
int aeb_reduce_fallbacks(uint64_t* count);

/* The statistics of Sec. VI: P(collision) = P(D_stop > H0) (eq. (20)), the
 * risk curve and minimum safe headways (Sec. VI-C), moments of D_stop
 * (Sec. VI-B, Table I), margins.
 * Statistics of `out` (device columns, out->n >= 1) as described for
 * aeb_stats/aeb_reduce_req.  Kernels run on `stream`; the function waits for
 * them and fills *host_out before returning. */
int aeb_reduce(const aeb_outputs* out, const aeb_reduce_req* req, aeb_stats* host_out,
               void* stream);

/* ---- launch shapes and the autotuner ----
 *
 * The block-structured integration kernel (Sec. V's one-thread-per-sample
 * mapping, reorganised as described for aeb_rollout) has four launch
 * parameters per precision (AEB_FP64, AEB_FP32C) and obstacle kind: k, the
 * steps per unchecked block (16, 32 or 64; AEB_FP64 also 128), the workgroup
 * size (64, 128, 256), waves_per_simd (0: one workgroup per `block` (or
 * 2 x `block`) samples in one pass; 1..32: a persistent grid of that many
 * wavefronts per SIMD claiming chunks of 64 (or 128) samples), and
 * samples_per_thread (1; or 2 for AEB_FP64 explicit Euler in the fused form
 * without a lead vehicle or controller: each lane integrates two sorted
 * samples, interleaving their steps; other scenarios of such an entry run
 * one sample per lane).  Results do not depend on them.  The table starts
 * from built-in defaults; if the environment variable AEB_TUNE_CACHE names a
 * cache file it is loaded at first use. */
typedef struct {
  int32_t k, block, waves_per_simd, samples_per_thread;
} aeb_tune_shape;
int aeb_tune_get(int precision, int obstacle, aeb_tune_shape* shape);
int aeb_tune_set(int precision, int obstacle, const aeb_tune_shape* shape);

/* The candidates the last aeb_autotune on this (precision, obstacle) timed,
 * fastest first: *count of them; the first min(max, *count) shapes and their
 * median times (ms, whole rollout call) are written to shapes and ms. */
int aeb_tune_results(int precision, int obstacle, aeb_tune_shape* shapes, float* ms, int max,
                     int* count);

/* (The launch configuration of Sec. V-A: block size and threads per sample.)
 * Load a cache written by aeb_autotune (AEB_EINVAL for a missing or malformed
 * file; entries are validated before any is used). */
int aeb_tune_load(const char* path);

/* (Sec. V-A fixes one launch configuration, 256 threads per block, one
 * thread per sample; this chooses it by measurement on this GPU.)
 * Time every candidate shape on `calib` (parameters drawn in-kernel; a few
 * launches each, synchronous on `stream`), keep the fastest for (precision,
 * calib->obstacle), return its time for the whole rollout call in *best_ms
 * (may be NULL) and, if cache_path is not NULL, write the table as JSON. */
int aeb_autotune(const aeb_scenario* calib, int precision, const char* cache_path, void* stream,
                 float* best_ms);

/* ---- recorded launch sequences (HIP graphs) ----
 *
 * The steady-state evaluation of one scenario (or of a fixed mix of
 * scenarios) on fixed buffers -- the rollout of Sec. IV-D/V plus, if `req` is
 * given, the statistics of Sec. VI per output set -- recorded once and then
 * replayed with a single launch, which removes the per-kernel launch cost of
 * repeated evaluations.  Each replay recomputes everything from the inputs
 * (parameter columns as they are at replay time, or the in-kernel generator)
 * and gives the same results as the eager calls.  The graph owns its device
 * scratch (allocated at creation) and, for batches, pinned copies of the
 * scenario tables.  Only the sorted block-structured path is recorded: FP64
 * explicit Euler (fused or unfused form) or RK4, FP32C explicit Euler (for
 * one scenario also with the FP64 fix-up of its flagged samples);
 * AEB_EINVAL for the fix-up mode in batched graphs, the closed-loop
 * controller in FP32C or in batched graphs (in any of their scenarios), and
 * a horizon plus dead time beyond 2^31 - 4096 steps. */
typedef struct aeb_graph aeb_graph;

/* (Removes the per-launch overhead the paper identifies at small N,
 * Sec. VI-E; the recorded work is that of aeb_rollout and aeb_reduce.)
 * One scenario: params (device columns, or NULL for the in-kernel generator),
 * out (device outputs, n_samples long), req (NULL: rollout only) and
 * host_stats: pinned host memory (hipHostMalloc) that each replay's
 * statistics are copied into; valid after aeb_graph_finish. */
int aeb_graph_create(const aeb_scenario* scn, const aeb_params* params, int precision,
                     const aeb_outputs* out, const aeb_reduce_req* req, aeb_stats* host_stats,
                     aeb_graph** graph);

/* (As aeb_graph_create, for the batched launch.)
 * A fixed mix of n_scn scenarios as one batched launch (as aeb_batch_rollout)
 * followed by the statistics of every scenario (the segmented reduction of
 * aeb_batch_reduce, all sets in one launch sequence) into host_stats[j]
 * (pinned, n_scn). */
int aeb_graph_create_batch(const aeb_scenario* scns, int n_scn, int precision,
                           const aeb_outputs* outs, const aeb_reduce_req* req,
                           aeb_stats* host_stats, aeb_graph** graph);

/* (A batched launch of changing mixes -- the serving path's steady-state
 * ticks, Sec. VI-F -- without the per-kernel launch cost, Sec. VI-E.)
 * A recording that replays ANY mix of up to max_scn scenarios with at most
 * max_samples samples in all, each of the kind of `kind` (the same
 * integrator, obstacle, impact_exit and nofma; perception allowed in the mix
 * only if `kind` has it; importance sampling only if `kind` has it): the
 * batched rollout of aeb_batch_rollout and, if req is not NULL, the
 * statistics of every scenario (aeb_batch_reduce).  Every grid covers the
 * capacity and the kernels read the mix's sizes from device tables, which
 * the graph's first nodes copy from pinned memory the graph owns, so a
 * replay only rewrites those tables.  The graph owns its device memory
 * (tables, rollout and reduction scratch for the capacity).  precision:
 * AEB_FP64 or AEB_FP32C.  AEB_EINVAL for a kind the batched path cannot run
 * (the closed-loop controller, RK4 in FP32C). */
int aeb_graph_create_mix(const aeb_scenario* kind, int precision, int max_scn,
                         int64_t max_samples, const aeb_reduce_req* req, aeb_graph** graph);

/* Replay a mix graph for n_scn scenarios (host array, each fitting the
 * graph's kind and capacity) with outputs outs[j] (device columns,
 * outs[j].n == scns[j].n_samples).  Asynchronous on `stream`; results equal
 * aeb_batch_rollout (and aeb_batch_reduce) of the same mix bit for bit.
 * host_stats (host array of n_scn, may be pageable; NULL if the graph has no
 * statistics) is filled by aeb_graph_finish, which must follow every replay
 * before the next (the replay reads the graph's pinned tables). */
int aeb_graph_launch_mix(aeb_graph* graph, const aeb_scenario* scns, int n_scn,
                         const aeb_outputs* outs, aeb_stats* host_stats, void* stream);

/* Enqueue one replay on `stream` (asynchronous).  (Graph plumbing; no
 * passage of the paper.) */
int aeb_graph_launch(aeb_graph* graph, void* stream);

/* Wait for `stream`; where a replay's order statistics needed the radix
 * fallback (rare), compute it; afterwards host_stats holds the statistics. */
int aeb_graph_finish(aeb_graph* graph, void* stream);

/* Release the graph, its scratch and pinned tables (graph plumbing). */
int aeb_graph_destroy(aeb_graph* graph);

/* ---- serving: continuous batching of evaluation requests ----
 *
 * Sec. VI bounds one Monte Carlo evaluation by 530 ms (700 ms of braking
 * budget minus perception and decision time).  A server takes requests (one
 * scenario each, parameters drawn in-kernel from its seed and id) as they
 * arrive, admits them in arrival order while their device footprint fits the
 * free part of a caller-provided arena and a slot is free, packs admitted
 * requests of one kind (integrator, obstacle, impact_exit, nofma) into one
 * sorted multi-scenario launch followed by one segmented reduction over its
 * requests (as aeb_batch_reduce), and
 * rotates launches over its streams so that work overlaps on the device.  A
 * request's statistics equal those of aeb_rollout (params == NULL) plus
 * aeb_reduce on the same scenario alone, bit for bit.  A worker thread of
 * the server drives admission, launches and completion; all entry points
 * are thread-safe. */
typedef struct aeb_server aeb_server;

/* Server configuration.
 *   arena, arena_bytes: device memory of the current device, owned by the
 *     caller (e.g. a torch tensor) and untouched by anyone else until
 *     aeb_server_destroy returns; the server carves its per-stream launch
 *     scratch (aeb_server_fixed_bytes) from the front and request
 *     footprints from the rest.
 *   max_slots: requests admitted or running at once (1..1024).
 *   precision: AEB_FP64 or AEB_FP32C.
 *   n_streams: launch streams (1..8), created by the server at the default
 *     priority; one launch in flight per stream.
 *   tick_us: while a launch is in flight, admitted requests wait up to this
 *     long (0..1e6 us) for others to share their launch.
 *   max_queue: waiting requests beyond which submit returns AEB_EAGAIN.
 *   flags: 0, or AEB_SERVE_EAGER to issue every launch's copies and kernels
 *     one by one instead of replaying a recorded graph (for comparison).
 *     By default a launch replays a HIP graph recorded once per stream and
 *     bucket -- kind, perception on or off, scenario count rounded up to a
 *     power of two, samples rounded up to a power of two (at least 2^15,
 *     at most max_tick_samples) -- whose first nodes copy the launch's
 *     scenario and set tables from pinned memory, so every mix that falls
 *     in a bucket replays the same recording.
 *   max_tick_samples: samples per launch (1..2^31-1); also the largest
 *     request.
 *   req: the statistics computed for every request (as for aeb_reduce). */
#define AEB_SERVE_EAGER 1
typedef struct {
  void* arena;
  uint64_t arena_bytes;
  int32_t max_slots;
  int32_t precision;
  int32_t n_streams;
  int32_t tick_us;
  int32_t max_queue;
  int32_t flags;
  int64_t max_tick_samples;
  aeb_reduce_req req;
} aeb_server_cfg;

/* Timestamps of one request, in seconds on the server's steady clock since
 * its creation: arrival (submit), admission, launch, and completion as seen
 * by the worker; missed = done - arrive exceeded the request's deadline. */
typedef struct {
  double arrive, admit, start, done;
  int32_t missed, reserved;
} aeb_req_timing;

/* Counters of a server: requests submitted, completed (including failed),
 * failed, past their deadline; launches; requests now queued, admitted,
 * running; arena bytes held by requests now and at most. */
typedef struct {
  uint64_t submitted, completed, failed, missed, ticks;
  uint64_t queued, admitted, running;
  uint64_t arena_in_use, arena_peak, arena_request_bytes, fixed_bytes;
} aeb_server_info;

/* (Admission by device footprint, for the Sec. VI-F request stream.)
 * Arena bytes a server with this configuration keeps for its streams (the
 * rest holds request footprints), and the footprint of one request of
 * n_samples samples. */
int aeb_server_fixed_bytes(const aeb_server_cfg* cfg, uint64_t* bytes);
int aeb_serve_footprint(const aeb_server_cfg* cfg, int64_t n_samples, uint64_t* bytes);

/* (The Sec. VI-F real-time evaluation as a service.)
 * Create a server on the current device (AEB_EINVAL for a bad
 * configuration, AEB_ENOMEM if the arena cannot hold the fixed part plus one
 * request of max_tick_samples samples). */
int aeb_server_create(const aeb_server_cfg* cfg, aeb_server** out);

/* (Server plumbing; no passage of the paper.)
 * Finish all accepted requests, stop the worker, release the streams and
 * pinned staging; results not polled yet are dropped.  NULL is accepted. */
int aeb_server_destroy(aeb_server* srv);

/* One Monte Carlo evaluation of Sec. IV-VI under the 530 ms budget of
 * Sec. VI-F (deadline_s).
 * Queue one evaluation (non-blocking).  AEB_EINVAL: invalid scenario or one
 * the batched path cannot run (RK4 in FP32C, the closed-loop controller);
 * AEB_ENOMEM: its footprint exceeds the request part of the arena or its
 * sample count max_tick_samples; AEB_EAGAIN: the queue is full.  deadline_s:
 * latency budget used for miss accounting (e.g. 0.530). */
int aeb_serve_submit(aeb_server* srv, const aeb_scenario* scn, double deadline_s,
                     uint64_t* ticket);

/* The statistics of Sec. VI for one request, and its latency against the
 * Sec. VI-F budget.
 * Collect a request: AEB_OK with *out (and *timing, if not NULL) filled once
 * it is done, after which the ticket is forgotten; AEB_EAGAIN while pending;
 * AEB_ENOTFOUND for an unknown or already collected ticket; the request's
 * own error if its execution failed. */
int aeb_serve_poll(aeb_server* srv, uint64_t ticket, aeb_stats* out, aeb_req_timing* timing);

/* Counters of the server (server plumbing; deadline misses against the
 * Sec. VI-F budget). */
int aeb_server_info_get(aeb_server* srv, aeb_server_info* out);

#ifdef __cplusplus
}
#endif
#endif /* AEB_H */
