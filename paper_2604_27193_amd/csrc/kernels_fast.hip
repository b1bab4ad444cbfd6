// kernels_fast.hip -- the throughput path of the explicit-Euler rollout (the
// configurations of Sec. IV with dead time and rolling resistance, and the
// lead-vehicle extension of Sec. VIII), FP64 and FP32-compensated, for one
// scenario or a batch of scenarios in one launch.
//
// Three stages:
//  1. prep: per sample, load (or draw) the parameters, derive the constants
//     of eq. (4)-(6), predict the number of steps to the stop from a
//     closed-form approximation of the braking phases, and classify the
//     sample (friction-limited or not).  Writes a 64-byte job record and a
//     sort key; counts keys in an LDS histogram.
//  2. counting sort of the keys: samples with the same predicted length land
//     in the same wavefront, longest first, so a wavefront's lanes finish
//     together and long wavefronts start early.
//  3. rollout: each lane integrates one sample.  Steps run in unchecked
//     blocks of K steps whenever no lane can stop, reach the horizon or pass
//     its command switch inside the block (guaranteed by per-lane bounds; the
//     switch is the dead time, plus the sample's own perception delay when
//     the scenario has one, and then the sort groups equal switch steps);
//     otherwise single steps with every test.  Inside a block the step takes
//     the cheapest form that gives bit-identical results in the current
//     phase: dead time (a = 0), generic, never-limited (max(a, alim) = a) or
//     friction-limited (max(a, alim) = alim for good, actuator update dead).
//     A crossing of the obstacle inside a block is found afterwards by
//     replaying that block from its saved start state.  The grid is
//     persistent: each wavefront claims the next 64 sorted samples through an
//     atomic counter until none are left (longest first, dynamically balanced).
#include <hip/hip_runtime.h>

#include <vector>

#include "aeb_common.h"
#include "aeb_runtime.h"
#include "fast_path.h"
#include "rollout_steps.h"
#include "tune.h"

namespace aeb {

namespace {

// The step and block helpers of the FP64 integration are always inlined: an
// out-of-line call takes the lane state by reference, which puts it in
// scratch memory (the compiler declined to inline the largest forms).
#define HOT __device__ __attribute__((always_inline)) inline

// sort keys: 64 coarse length bins x 2 classes x 64 fine levels; with the
// controller 64 decision ticks x 2 classes x 128 length levels (the sort's
// kernels take the key count as a template argument: their per-bin loops
// cost latency on small launches)
constexpr int NBINS = 8192;
constexpr int NBINS_CTL = 16384;
// The sort's kernels (prep, scan, scatter) run in workgroups of one wavefront
// per SIMD: beside a running integration kernel (four wavefronts per SIMD)
// each CU has room for one such workgroup, so the next launch's preparation
// overlaps the current integration when launches are pipelined on two streams.
constexpr int PREP_BLOCK = 256;
constexpr int PREP_SAMPLES = 4096;                     // samples per scatter block
constexpr int PREP_PER = PREP_SAMPLES / PREP_BLOCK;    // samples per scatter thread
// The drawing prep kernel takes one sample per thread, and its key histogram
// is a kernel of its own.  (A loop over several samples per thread, to share
// a block histogram's flush, let the compiler hoist the constants of the
// draws' log, sqrt, sine and cosine out of the loop and hold them in
// registers: 231 VGPRs, two wavefronts per SIMD, against 113 without it; and
// a block histogram per 256 samples costs more than the draws save.)  The
// plain method's prep, which draws nothing, keeps PREP_PER samples per thread
// with the histogram fused in (k_prep_cols).
inline unsigned prep_grid(int64_t n) {
  return static_cast<unsigned>((n + PREP_BLOCK - 1) / PREP_BLOCK);
}
template <bool DEVRNG>
constexpr int prep_threads() { return PREP_BLOCK; }

// Closed-form estimate of the stopping time (s): dead time at zero brake,
// first-order ramp of the brake to the friction limit (or to the command),
// then constant deceleration; drag taken at a third of the squared speed.
__device__ inline float predict_stop_time(float v0, float kd, float c, float alim, float tau,
                                          float acmd, float td) {
  const float amag = -acmd;  // command magnitude
  if (!(amag > 0.0f)) return INFINITY;
  float v1 = v0 - (c + kd * v0 * v0) * td;
  if (v1 <= 0.0f) return td;
  if (alim > acmd) {  // limited: the ramp stops at alim
    const float lim = -alim;
    const float ratio = alim / acmd;  // in (0, 1)
    const float ss = -tau * log1pf(-ratio);
    const float dv = amag * ss - tau * lim + (c + kd * v1 * v1 * 0.5f) * ss;
    const float v2 = v1 - dv;
    if (v2 <= 0.0f) return td + ss * (v1 / fmaxf(v1 - v2, 1e-6f));
    const float den = lim + c + kd * v2 * v2 * (1.0f / 3.0f);
    if (!(den > 0.0f)) return INFINITY;
    return td + ss + v2 / den;
  }
  const float den = amag + c + kd * v1 * v1 * (1.0f / 3.0f);
  if (!(den > 0.0f)) return INFINITY;
  return td + (v1 + amag * tau) / den;
}

// Predicted stop time under the closed-loop controller with a stationary
// obstacle, for the sort only (noise left out): constant speed until the
// first decision with TTC below ttc_warn, then the partial command (after
// the dead time and, roughly, the actuator lag) until the first decision with
// TTC below ttc_brake, then the full command as in predict_stop_time.
// Decisions fall on the controller's tick grid (period per); *t_full gets
// the predicted time of the full-braking decision.
__device__ inline float predict_ctl_stop_time(float v0, float gap, float tw, float tb, float aw,
                                              float per, float dead, float kd, float c,
                                              float alim, float tau, float acmd,
                                              float* t_full) {
  *t_full = 0.0f;
  if (!(v0 > 0.0f)) return dead;
  auto tick = [&](float t) { return ceilf(fmaxf(t, 0.0f) / per) * per; };
  float t_b, v_b;
  if (!(tw > tb)) {
    // no partial stage: full braking from the first decision below ttc_brake
    t_b = tick(gap / v0 - tb);
    v_b = v0;
  } else {
    const float t_w = tick(gap / v0 - tw);
    const float delay = dead + tau;
    const float g0 = gap - v0 * (t_w + delay);  // gap when the partial braking bites
    if (g0 <= tb * v0) {
      t_b = tick(gap / v0 - tb);
      v_b = v0;
    } else {
      // gap g0 - v0 s + aw s^2 / 2 reaches tb (v0 - aw s): smallest root
      float sroot;
      if (aw < 1e-6f) {
        sroot = (g0 - tb * v0) / v0;
      } else {
        const float bq = v0 - tb * aw;
        const float disc = bq * bq - 2.0f * aw * (g0 - tb * v0);
        // the partial braking alone stops the vehicle first
        *t_full = t_w + delay + v0 / aw;
        if (!(disc >= 0.0f) || bq <= 0.0f) return *t_full;
        sroot = (bq - sqrtf(disc)) / aw;
        if (sroot * aw >= v0) return *t_full;
      }
      t_b = tick(t_w + delay + sroot);
      v_b = fmaxf(v0 - aw * (t_b - t_w - delay), 0.0f);
    }
  }
  *t_full = t_b;
  return t_b + predict_stop_time(v_b, kd, c, alim, tau, acmd, dead);
}

// Inputs of the prep stage: one scenario (uniform) or a batch table.
struct PrepArgs {
  aeb_scenario s;          // single scenario
  ParamSrc src;            // its parameter columns (plain method)
  int64_t n;               // samples in the launch
  int nd, nmax;            // single scenario's step counts
  float cap;               // step count that maps to the last sort bin
  const aeb_scenario* scns;  // batch: scenarios
  const ScnDev* tab;         // batch: per-scenario constants and offsets
  int n_scn;
  int32_t* nds;              // per-sample command step (launches with perception), else null
  int ctl;                   // closed-loop controller (single scenario)
  double* weight;            // single scenario: importance-sampling weights out (or null)
  const BatchHdr* hdr;       // batch on device tables: n, cap and n_scn from here (else null)
};

// One sample: its parameters (drawn, or loaded from the plain method's
// columns), its job record and its sort key.
// (i: global index; j, local: its scenario and its index there)
template <bool DEVRNG, bool BATCH>
HOT uint32_t prep_sample(const PrepArgs& a, int64_t i, uint32_t j, int64_t local, float capf,
                         Job* jobs, LeadJob* leads) {
  const aeb_scenario& s = BATCH ? a.scns[j] : a.s;
  const int nd = BATCH ? a.tab[j].nd : a.nd;
  const int nmax = BATCH ? a.tab[j].nmax : a.nmax;
  double v0, mu, mass, sg, cg, cda, crr, tau, gap, lead, trig, lw;
  if (DEVRNG) {
    Sample q = draw_sample(s, static_cast<uint64_t>(local));
    v0 = q.v0; mu = q.mu; mass = q.mass; sg = q.sin_grade; cg = q.cos_grade;
    cda = q.cda; crr = q.crr; tau = q.tau; gap = q.gap; lead = q.lead_decel;
    trig = q.trigger;
    lw = q.log_w;
  } else {
    v0 = a.src.v0[i]; mu = a.src.mu[i]; mass = a.src.mass[i]; sg = a.src.sin_g[i];
    cg = a.src.cos_g[i]; cda = a.src.cda[i]; crr = a.src.crr[i]; tau = a.src.tau[i];
    gap = a.src.gap[i]; lead = a.src.lead[i];
    trig = a.src.trig ? a.src.trig[i] : 0.0;
    lw = a.src.logw ? a.src.logw[i] : 0.0;
  }
  // the importance-sampling weight goes straight to the sample's output
  double* wout = BATCH ? a.tab[j].out.weight : a.weight;
  if (wout) wout[local] = exp(lw);
  // with perception every sample has its own command step
  int ndl = nd;
  if (a.nds) {
    ndl = static_cast<int>(command_step(s, trig, nmax));
    a.nds[i] = ndl;
  }
  const Consts k = derive(s, mu, mass, sg, cg, cda, crr);
  Job J;
  J.v0 = v0;
  J.nkd = -k.kd;
  J.c = k.c;
  J.alim = k.alim;
  J.kt = s.integrator == AEB_RK4 ? 1.0 / tau : s.dt / tau;  // Euler: dt/tau; RK4: 1/tau
  J.gap = gap;
  // |acc| <= min(|a_cmd|, |alim|) + kd vmax^2 + |c|, with vmax the largest
  // speed the sample can reach (only a downhill pull can raise it)
  const double creach = k.c < 0.0 ? -k.c : 0.0;
  const double vmax = fabs(v0) + s.horizon * creach;
  const double brake = fmin(fabs(s.a_cmd), fabs(k.alim));
  J.dmax = (brake + fabs(k.kd) * vmax * vmax + fabs(k.c)) * 1.0001 + 1e-9;
  // classify and predict
  const bool limited = !(k.alim < s.a_cmd - 1e-6);
  float td = static_cast<float>(ndl) * static_cast<float>(s.dt);
  if (a.ctl && s.obstacle == AEB_OBS_LEAD) {
    // approach until the full-brake threshold, for the sort only: a lead
    // braking at `lead` from the ego's speed (closing speed lead t, gap
    // closed by lead t^2 / 2)
    const float T = static_cast<float>(s.ttc_brake), G = static_cast<float>(gap);
    const float A = static_cast<float>(lead);
    td += A > 0.0f ? sqrtf(T * T + 2.0f * G / A) - T : static_cast<float>(s.horizon);
  }
  float t, t_full = -1.0f;
  if (a.ctl && s.obstacle != AEB_OBS_LEAD)
    t = predict_ctl_stop_time(static_cast<float>(v0), static_cast<float>(gap),
                              static_cast<float>(s.ttc_warn), static_cast<float>(s.ttc_brake),
                              -static_cast<float>(s.a_warn), static_cast<float>(s.ctl_period),
                              static_cast<float>(ndl) * static_cast<float>(s.dt),
                              static_cast<float>(k.kd), static_cast<float>(k.c),
                              static_cast<float>(k.alim), static_cast<float>(tau),
                              static_cast<float>(s.a_cmd), &t_full);
  else
    t = predict_stop_time(static_cast<float>(v0), static_cast<float>(k.kd),
                          static_cast<float>(k.c), static_cast<float>(k.alim),
                          static_cast<float>(tau), static_cast<float>(s.a_cmd), td);
  float steps = t / static_cast<float>(s.dt);
  if (!(steps < static_cast<float>(nmax))) steps = static_cast<float>(nmax);
  if (!(steps > 0.0f)) steps = 0.0f;
  J.pred = steps;
  J.scn = j;
  jobs[i] = J;
  if (leads) leads[i].decel = lead;
  const uint32_t u = static_cast<uint32_t>(fminf(steps, capf) * (4096.0f / (capf + 1.0f)));
  const uint32_t ud = 4095u - (u > 4095u ? 4095u : u);  // longest first
  // within a coarse length bin: finer length; with perception 8 finer length
  // levels, then the command step in 16-step bins, so a wavefront's lanes
  // end close together and switch the command within a few steps of each
  // other (each distinct switch step cuts the wavefront's blocks)
  const uint32_t fine =
      a.nds ? (((ud >> 3) & 7u) << 3) | ((static_cast<uint32_t>(ndl) >> 4) & 7u) : ud & 63u;
  uint32_t key = ((ud >> 6) << 7) | (limited ? 0u : 64u) | fine;
  // with the controller: first the tick of the predicted full-braking
  // decision (modulo 64, latest first), so a wavefront's lanes reach the
  // thresholds, where the noise can decide and the whole wavefront draws
  // it, at the same ticks; then the class and the length in 128 levels, so
  // that they also stop close together (each lane's stop takes the
  // wavefront down the block ladder)
  if (t_full >= 0.0f) {
    const uint32_t tk =
        static_cast<uint32_t>(t_full / static_cast<float>(s.ctl_period) + 0.5f) & 63u;
    key = ((63u - tk) << 8) | (limited ? 0u : 128u) | (ud >> 5);
  }
  return key;
}

template <bool DEVRNG, bool BATCH>
__global__ __launch_bounds__(prep_threads<DEVRNG>()) void k_prep(PrepArgs a, Job* jobs,
                                                                 LeadJob* leads, uint32_t* keys) {
  constexpr int NT = prep_threads<DEVRNG>();
  // a recorded mix reads its sizes from the device header
  const int64_t n_all = a.hdr ? a.hdr->total : a.n;
  const float capf = a.hdr ? a.hdr->cap : a.cap;
  const int n_scn = a.hdr ? a.hdr->n_scn : a.n_scn;
  if (!BATCH) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * NT + threadIdx.x;
    if (i < n_all) keys[i] = prep_sample<DEVRNG, false>(a, i, 0u, i, capf, jobs, leads);
    return;
  }
  // A batch: the launch covers an index space where every scenario starts on
  // a multiple of 64, so each wavefront holds samples of one scenario, found
  // from the wavefront's first index: its table entry and scenario are then
  // uniform (scalar loads, no per-lane copies of the scenario in registers).
  const int64_t pw = static_cast<int64_t>(blockIdx.x) * NT +
                     __builtin_amdgcn_readfirstlane(threadIdx.x & ~63u);
  int lo = 0, hi = n_scn - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.tab[mid].poff <= pw)
      lo = mid;
    else
      hi = mid - 1;
  }
  const uint32_t j = static_cast<uint32_t>(lo);
  const int64_t off = a.tab[j].off;
  const int64_t n_j = (lo + 1 < n_scn ? a.tab[lo + 1].off : n_all) - off;
  const int64_t local = pw - a.tab[j].poff + (threadIdx.x & 63);
  if (local < n_j) keys[off + local] = prep_sample<DEVRNG, true>(a, off + local, j, local, capf,
                                                                  jobs, leads);
}

// The plain method's prep (parameters from the columns: no draws, so nothing
// for the compiler to hoist): PREP_PER samples per thread with the key
// histogram in LDS, flushed with one atomic per key the block holds, so no
// separate histogram pass.
template <int NB>
__global__ __launch_bounds__(PREP_BLOCK) void k_prep_cols(PrepArgs a, Job* jobs, LeadJob* leads,
                                                          uint32_t* keys, uint32_t* ghist) {
  __shared__ uint32_t hist[NB];
  for (int j = threadIdx.x; j < NB; j += PREP_BLOCK) hist[j] = 0;
  __syncthreads();
  const int64_t base_i = static_cast<int64_t>(blockIdx.x) * PREP_SAMPLES;
  for (int r = 0; r < PREP_PER; ++r) {
    const int64_t i = base_i + r * PREP_BLOCK + threadIdx.x;
    if (i >= a.n) break;
    const uint32_t key = prep_sample<false, false>(a, i, 0u, i, a.cap, jobs, leads);
    keys[i] = key;
    atomicAdd(&hist[key], 1u);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < NB; j += PREP_BLOCK)
    if (hist[j]) atomicAdd(&ghist[j], hist[j]);
}

// Key histogram: per block of PREP_SAMPLES keys in LDS, then one global
// atomic per key the block holds.
template <int NB>
__global__ __launch_bounds__(PREP_BLOCK) void k_hist(const uint32_t* keys, int64_t n,
                                                     uint32_t* ghist, const BatchHdr* hdr) {
  if (hdr) n = hdr->total;
  __shared__ uint32_t hist[NB];
  for (int j = threadIdx.x; j < NB; j += PREP_BLOCK) hist[j] = 0;
  __syncthreads();
  uint32_t key[PREP_PER];
  const int64_t base_i = static_cast<int64_t>(blockIdx.x) * (PREP_BLOCK * PREP_PER);
#pragma unroll
  for (int r = 0; r < PREP_PER; ++r) {
    const int64_t i = base_i + r * PREP_BLOCK + threadIdx.x;
    key[r] = i < n ? keys[i] : NB;
  }
#pragma unroll
  for (int r = 0; r < PREP_PER; ++r)
    if (key[r] < NB) atomicAdd(&hist[key[r]], 1u);
  __syncthreads();
  for (int j = threadIdx.x; j < NB; j += PREP_BLOCK)
    if (hist[j]) atomicAdd(&ghist[j], hist[j]);
}

// exclusive scan of the key histogram into bucket offsets (one block); also
// clears the integration kernel's chunk counter
template <int NB>
__global__ __launch_bounds__(PREP_BLOCK) void k_scan(uint32_t* hist, unsigned long long* counter) {
  if (threadIdx.x == 0) *counter = 0ull;
  __shared__ uint32_t part[PREP_BLOCK];
  constexpr int PER = NB / PREP_BLOCK;
  uint32_t loc[PER];
  uint32_t sum = 0;
  for (int j = 0; j < PER; ++j) {
    loc[j] = hist[threadIdx.x * PER + j];
    sum += loc[j];
  }
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < PREP_BLOCK; off <<= 1) {
    uint32_t v = threadIdx.x >= static_cast<unsigned>(off) ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t base = part[threadIdx.x] - sum;
  for (int j = 0; j < PER; ++j) {
    hist[threadIdx.x * PER + j] = base;
    base += loc[j];
  }
}

// Placement: each block ranks its samples per key in LDS, reserves one range
// per key with a single global atomic, then writes the permutation.
template <int NB>
__global__ __launch_bounds__(PREP_BLOCK) void k_scatter(const uint32_t* keys, int64_t n,
                                                        uint32_t* offs, uint32_t* perm,
                                                        const BatchHdr* hdr) {
  if (hdr) n = hdr->total;
  __shared__ uint32_t cnt[NB];
  for (int j = threadIdx.x; j < NB; j += PREP_BLOCK) cnt[j] = 0;
  __syncthreads();
  uint32_t key[PREP_PER], rank[PREP_PER];
  const int64_t base_i = static_cast<int64_t>(blockIdx.x) * (PREP_BLOCK * PREP_PER);
  // every key load in flight before the first LDS rank
#pragma unroll
  for (int r = 0; r < PREP_PER; ++r) {
    const int64_t i = base_i + r * PREP_BLOCK + threadIdx.x;
    key[r] = i < n ? keys[i] : 0u;
  }
#pragma unroll
  for (int r = 0; r < PREP_PER; ++r) {
    const int64_t i = base_i + r * PREP_BLOCK + threadIdx.x;
    rank[r] = i < n ? atomicAdd(&cnt[key[r]], 1u) : 0u;
  }
  __syncthreads();
  // the range reservations, 16 keys of the thread at a time: every atomic of
  // a group is in flight before the first result is read (one after another
  // they set the kernel's time on small launches)
  constexpr int G = 16;
  static_assert(NB % (G * PREP_BLOCK) == 0, "key count");
  for (int j0 = threadIdx.x; j0 < NB; j0 += G * PREP_BLOCK) {
    uint32_t c[G], o[G];
#pragma unroll
    for (int q = 0; q < G; ++q) c[q] = cnt[j0 + q * PREP_BLOCK];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      o[q] = 0u;
      if (c[q]) o[q] = atomicAdd(&offs[j0 + q * PREP_BLOCK], c[q]);
    }
#pragma unroll
    for (int q = 0; q < G; ++q) cnt[j0 + q * PREP_BLOCK] = o[q];
  }
  __syncthreads();
  for (int r = 0; r < PREP_PER; ++r) {
    const int64_t i = base_i + r * PREP_BLOCK + threadIdx.x;
    if (i < n) perm[cnt[key[r]] + rank[r]] = static_cast<uint32_t>(i);
  }
}

__global__ void k_zero(uint32_t* p, int64_t n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

// ---------------------------------------------------------------------------
// FP64 block forms.  All four give the canonical step's x and v bit for bit:
//   G: abe = max(a, alim); acc = fma(-kd, v v, abe) - c; x, v, a fma updates
//   F: never limited (alim < a_cmd): max(a, alim) = a
//   C: limited for good (a <= alim < a_cmd): abe = alim, a no longer read
//   D: dead time (cmd = 0, a = 0): abe = 0 exactly, a stays 0
// ---------------------------------------------------------------------------
struct St64 {
  double x, v, a;
};

// lead vehicle and the running minimum of the clearance (gap + x_lead) - x
struct Ld64 {
  double xl, vl, gmin;
};

// ---------------------------------------------------------------------------
// Classical RK4 (Sec. IV-D) in the same forms, no fused operations, the
// command held over the step.  Stage derivative of the speed:
//   (max(a, alim) - kd v v) - c, written (m + (-kd) (v v)) - c (the same bits);
// the position's stages are the stage speeds.  Job.kt holds 1/tau here.
// ---------------------------------------------------------------------------
template <int FORM>
__device__ inline double rk_dv(const Job& J, double v, double a) {
  double m;
  if (FORM == FORM_G)
    m = fmax(a, J.alim);
  else if (FORM == FORM_F)
    m = a;
  else if (FORM == FORM_C)
    m = J.alim;
  else
    m = 0.0;  // dead time: a = 0 exactly and max(0, alim) = 0
  return (m + J.nkd * (v * v)) - J.c;
}

template <int FORM>
__device__ inline void rk4_step(St64& s, const Job& J, double dt, double h2, double h6,
                                double cmd) {
  constexpr bool ACT = FORM == FORM_G || FORM == FORM_F;  // the actuator is read
  const double v1 = s.v, a1 = s.a;
  const double k1v = rk_dv<FORM>(J, v1, a1);
  const double k1a = ACT ? (cmd - a1) * J.kt : 0.0;
  const double v2 = v1 + h2 * k1v, a2 = ACT ? a1 + h2 * k1a : a1;
  const double k2v = rk_dv<FORM>(J, v2, a2);
  const double k2a = ACT ? (cmd - a2) * J.kt : 0.0;
  const double v3 = v1 + h2 * k2v, a3 = ACT ? a1 + h2 * k2a : a1;
  const double k3v = rk_dv<FORM>(J, v3, a3);
  const double k3a = ACT ? (cmd - a3) * J.kt : 0.0;
  const double v4 = v1 + dt * k3v, a4 = ACT ? a1 + dt * k3a : a1;
  const double k4v = rk_dv<FORM>(J, v4, a4);
  s.x = s.x + h6 * (((v1 + 2.0 * v2) + 2.0 * v3) + v4);
  s.v = v1 + h6 * (((k1v + 2.0 * k2v) + 2.0 * k3v) + k4v);
  if (ACT) {
    const double k4a = (cmd - a4) * J.kt;
    s.a = a1 + h6 * (((k1a + 2.0 * k2a) + 2.0 * k3a) + k4a);
  }
}

// Kernel tag of explicit Euler in the unfused form (the paper's rule of no
// fused operations): every a*b + c below a rounded product, then a rounded sum.
constexpr int EULER_NOFMA = 2;

// a*b + c: one fused multiply-add, or (unfused) a rounded product and a
// rounded sum (the build contracts nothing implicitly).  The canonical step's
// (abe - kd v v) and vl - dt al equal abe + (-kd)(v v) and vl + (-dt) al bit
// for bit (negation is exact), so one form serves both.
template <bool NF>
__device__ inline double mad(double a, double b, double c) {
  return NF ? a * b + c : fma(a, b, c);
}

template <int FORM, int K, bool LEAD, int INTEG = AEB_EULER>
HOT void block64(St64& s, Ld64& l, const Job& J, double al, double dt, double cmd) {
  constexpr bool NF = INTEG == EULER_NOFMA;
  if (INTEG == AEB_RK4) {
    const double h2 = 0.5 * dt, h6 = dt / 6.0;
#pragma unroll
    for (int j = 0; j < K; ++j) rk4_step<FORM>(s, J, dt, h2, h6, cmd);
    return;
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const double q = s.v * s.v;
    double acc;
    if (FORM == FORM_G) {
      acc = mad<NF>(J.nkd, q, fmax(s.a, J.alim)) - J.c;
      s.a = mad<NF>(J.kt, cmd - s.a, s.a);
    } else if (FORM == FORM_F) {
      acc = mad<NF>(J.nkd, q, s.a) - J.c;
      s.a = mad<NF>(J.kt, cmd - s.a, s.a);
    } else if (FORM == FORM_C) {
      acc = mad<NF>(J.nkd, q, J.alim) - J.c;
    } else {  // FORM_D
      acc = mad<NF>(J.nkd, q, 0.0) - J.c;
    }
    s.x = mad<NF>(dt, s.v, s.x);
    s.v = mad<NF>(dt, acc, s.v);
    if (LEAD) {
      l.xl = mad<NF>(dt, l.vl, l.xl);
      l.vl = fmax(mad<NF>(-dt, al, l.vl), 0.0);
      l.gmin = fmin(l.gmin, (J.gap + l.xl) - s.x);
    }
    // unfused: each step's position sum happens at its step (else the
    // compiler defers the sums and holds every step's product in a register)
    if (NF) asm volatile("" : "+v"(s.x));
    if (NF && LEAD) {  // likewise the lead vehicle's state, and no step interleaved with the next
      asm volatile("" : "+v"(l.xl), "+v"(l.vl), "+v"(l.gmin), "+v"(s.v));
      __builtin_amdgcn_sched_barrier(0);
    }
  }
}

template <bool LEAD, int INTEG = AEB_EULER>
HOT void step64(St64& s, Ld64& l, const Job& J, double al, double dt, double cmd) {
  constexpr bool NF = INTEG == EULER_NOFMA;
  if (INTEG == AEB_RK4) {
    rk4_step<FORM_G>(s, J, dt, 0.5 * dt, dt / 6.0, cmd);
    return;
  }
  const double q = s.v * s.v;
  const double acc = mad<NF>(J.nkd, q, fmax(s.a, J.alim)) - J.c;
  s.a = mad<NF>(J.kt, cmd - s.a, s.a);
  s.x = mad<NF>(dt, s.v, s.x);
  s.v = mad<NF>(dt, acc, s.v);
  if (LEAD) {
    l.xl = mad<NF>(dt, l.vl, l.xl);
    l.vl = fmax(mad<NF>(-dt, al, l.vl), 0.0);
  }
}

// Scenario constants a lane works with: uniform kernel arguments for one
// scenario, the scenario table in a batch.
struct Ctx {
  double dt, a_cmd;
  int nd, nmax, impact_exit;
  OutCols out;
  const ScnDev* tab;
  const int32_t* nds;  // per-sample command steps (perception), else null
  CtlArgs ca;          // the closed-loop controller (kernels instantiated for it)
  const BatchHdr* hdr; // a recorded mix: the launch's sample count (else null)
  // profiling (timing enabled): the sum over chunks of the steps the
  // wavefront ran times its sample slots (the steps output sums the useful
  // ones: lane efficiency is their ratio), else null
  unsigned long long* lanes;
};

// Lane accounting of one chunk: the wavefront ran k steps for spw sample
// slots (one atomic per chunk, from its first lane).
__device__ inline void count_lanes(unsigned long long* lanes, int k, int spw) {
  if ((threadIdx.x & 63) == 0)
    atomicAdd(lanes, static_cast<unsigned long long>(k) * static_cast<unsigned long long>(spw));
}

struct LaneScn {
  double dt, a_cmd;
  int nd, nmax;
};

template <bool BATCH>
__device__ inline LaneScn lane_scn(const Ctx& c, const Job& J, bool valid, uint32_t g) {
  LaneScn r;
  if (BATCH) {
    const ScnDev& t = c.tab[J.scn];
    r.dt = t.dt;
    r.a_cmd = t.a_cmd;
    r.nd = t.nd;
    r.nmax = t.nmax;
  } else {
    r.dt = c.dt;
    r.a_cmd = c.a_cmd;
    r.nd = c.nd;
    r.nmax = c.nmax;
  }
  if (c.nds && valid) r.nd = c.nds[g];
  return r;
}

// A uniform value passed through an identity DPP move (quad_perm [0,1,2,3]):
// the same bits, which the compiler then keeps in a vector register as a lane
// value.  Measured on the compensated FP32 kernel with a stationary obstacle:
// its scenario constants and limits as lane values (as in a batch) take 79
// VGPRs instead of 85, six wavefronts per SIMD instead of five, and the
// single-scenario launch runs 5-6 % faster.
__device__ inline int lane_value(int x) {
  return __builtin_amdgcn_update_dpp(0, x, 0xe4, 0xf, 0xf, false);
}

__device__ inline double lane_value(double x) {
  const long long b = __double_as_longlong(x);
  const int lo = lane_value(static_cast<int>(b)), hi = lane_value(static_cast<int>(b >> 32));
  return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
}

__device__ inline LaneScn lane_values(LaneScn r) {
  r.dt = lane_value(r.dt);
  r.a_cmd = lane_value(r.a_cmd);
  r.nd = lane_value(r.nd);
  r.nmax = lane_value(r.nmax);
  return r;
}

// Output columns and the sample's index in them (read only at the store, so
// that the pointers are not held through the integration).
template <bool BATCH>
__device__ inline OutCols lane_out(const Ctx& c, const Job& J, uint32_t g, int64_t& local) {
  if (BATCH) {
    const ScnDev& t = c.tab[J.scn];
    local = static_cast<int64_t>(g) - t.off;
    return t.out;
  }
  local = g;
  return c.out;
}

// Largest step index a block may end on without a per-step test: a block
// never straddles the command switch nd and ends before the last step
// nmax - 1 (the horizon test fires after that step).  The launch-wide
// limit of a wavefront is the minimum over its active lanes; it only grows
// as k passes a lane's nd or lanes finish, so it is refreshed once k reaches it.
__device__ inline int lane_lim(int k, int nd, int nmax) {
  return k < nd ? min(nd, nmax - 1) : nmax - 1;
}

// Minimum over the wavefront (every lane active), left in every lane: DPP row
// shifts of 1, 2, 4, 8 lanes give each row's minimum in its lane 15, the row
// broadcasts of lanes 15 and 31 carry it to lane 63.  Register moves, no LDS.
template <int CTRL, int ROW_MASK>
__device__ inline int dpp_min(int x) {
  return min(x, __builtin_amdgcn_update_dpp(INT_MAX, x, CTRL, ROW_MASK, 0xf, false));
}

__device__ inline int wave_min(int x) {
  x = dpp_min<0x111, 0xf>(x);  // row_shr:1
  x = dpp_min<0x112, 0xf>(x);  // row_shr:2
  x = dpp_min<0x114, 0xf>(x);  // row_shr:4
  x = dpp_min<0x118, 0xf>(x);  // row_shr:8
  x = dpp_min<0x142, 0xa>(x);  // row_bcast:15 into rows 1 and 3
  x = dpp_min<0x143, 0xc>(x);  // row_bcast:31 into rows 2 and 3
  return __builtin_amdgcn_readlane(x, 63);
}

// varnd: nd or nmax differ between lanes (a batch, or per-sample command steps)
__device__ inline int wave_lim(bool varnd, bool active, int k, int nd, int nmax) {
  // nd, nmax are uniform: say so, so that the tests on the limit are scalar
  if (!varnd) return __builtin_amdgcn_readfirstlane(lane_lim(k, nd, nmax));
  return wave_min(active ? lane_lim(k, nd, nmax) : INT_MAX);
}

// claim the next 64 sorted positions for this wavefront
__device__ inline int64_t claim(unsigned long long* counter) {
  unsigned long long base = 0;
  if ((threadIdx.x & 63) == 0) base = atomicAdd(counter, 64ull);
  const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(base));
  const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(base >> 32));
  return static_cast<int64_t>((static_cast<unsigned long long>(hi) << 32) | lo);
}

// The next 64 sorted positions of a wavefront.  First pass: the wavefront's
// own slice of its workgroup's range.  Later passes of a persistent launch:
// chunks claimed from the counter beyond the range the whole grid covered in
// its first pass (so the launch does not start with every wavefront
// contending for one atomic); a one-pass launch stops after the first.
__device__ inline int64_t next_chunk(unsigned long long* counter, int persistent, int pass,
                                     int64_t n) {
  if (pass == 0)
    return static_cast<int64_t>(blockIdx.x) * blockDim.x +
           __builtin_amdgcn_readfirstlane(threadIdx.x & ~63u);
  if (!persistent) return n;
  return claim(counter) + static_cast<int64_t>(gridDim.x) * blockDim.x;
}

// Lane state and per-lane flags of the FP64 integration.
struct Lane64 {
  St64 s, sv;  // state, and start state of the block where the obstacle was passed
  Ld64 l, lv;  // lead vehicle, and its state at that block start
  int sk, se;  // step index at that block start, and at its end
  int on1, on2, stage;  // controller: first steps of its two commands (INT_MAX: none), stage
  bool active, collided, pend, clamped, free_lane, limited;
};

// The lane's brake command at step kk (constant inside every block: blocks
// end at every command switch), and the first step with any command.
template <bool CTL>
__device__ inline double lane_cmd(const Lane64& L, const LaneScn& c, double a_warn, int kk) {
  if (!CTL) return kk >= c.nd ? c.a_cmd : 0.0;
  return kk >= L.on2 ? c.a_cmd : (kk >= L.on1 ? a_warn : 0.0);
}

template <bool CTL>
__device__ inline int first_cmd(const Lane64& L, const LaneScn& c) {
  return CTL ? min(L.on1, L.on2) : c.nd;
}

// Controller block limit of a lane: its next command switch, and the last step.
__device__ inline int ctl_lim(const Lane64& L, int k, int nmax) {
  // the earlier of the switches still ahead (either may be unset, INT_MAX)
  int sw = INT_MAX;
  if (L.on1 > k) sw = L.on1;
  if (L.on2 > k) sw = min(sw, L.on2);
  return min(sw, nmax - 1);
}

// wnd: the smallest nd of the wavefront's lanes (the whole block is dead time
// for every lane when k + B <= wnd)
template <int OBS, int B, int INTEG, bool CTL>
HOT void run_block64(Lane64& L, const Job& J, double al, const LaneScn& c, int k, int wnd,
                     int impact_exit, double a_warn) {
  constexpr bool LEAD = OBS == AEB_OBS_LEAD;
  const double cmd = lane_cmd<CTL>(L, c, a_warn, k);
  const int fcmd = first_cmd<CTL>(L, c);
  if (OBS != AEB_OBS_NONE && !L.collided) {
    L.sv = L.s;
    if (LEAD) L.lv = L.l;
    L.sk = k;
    L.se = k + B;
  }
  if (k + B <= wnd) {
    block64<FORM_D, B, LEAD, INTEG>(L.s, L.l, J, al, c.dt, cmd);
  } else if (__all(!L.active || L.clamped)) {
    block64<FORM_C, B, LEAD, INTEG>(L.s, L.l, J, al, c.dt, cmd);
  } else if (__all(!L.active || L.free_lane)) {
    block64<FORM_F, B, LEAD, INTEG>(L.s, L.l, J, al, c.dt, cmd);
  } else {
    block64<FORM_G, B, LEAD, INTEG>(L.s, L.l, J, al, c.dt, cmd);
    L.clamped = L.clamped || (L.limited && k + B > fcmd && L.s.a <= J.alim);
  }
  if (OBS == AEB_OBS_STATIONARY && L.active && !L.collided && L.s.x > J.gap) {
    L.collided = true;
    L.pend = true;
    if (impact_exit) L.active = false;
  }
  if (LEAD && L.active && L.l.gmin < 0.0) {  // the lead was reached inside the block
    L.collided = true;
    L.pend = true;
    L.active = false;
  }
}

// Consecutive K-step blocks in one steady form (every active lane friction-
// limited for good, or every one never limited), for as long as no lane can
// stop or reach the block limit wl inside the next block.  A lane's block
// start state is kept only through its block; where the obstacle is passed
// inside a block, that state becomes the lane's replay start.  Returns the
// step index after the last block.
template <int OBS, int K, int FORM, int INTEG>
HOT int run_steady(Lane64& L, const Job& J, double al, double dt, double cmd, int k, int wl,
                   double thr, int impact_exit, double& xmax) {
  constexpr bool LEAD = OBS == AEB_OBS_LEAD;
  do {
    const St64 b = L.s;
    const Ld64 bl = L.l;
    // in 16-step pieces whose position is pinned in a register at the end of
    // each: with no obstacle nothing inside the run reads the position, and
    // the compiler would otherwise hold every step's speed for a position
    // update sunk to the end of the run (hundreds of registers)
#pragma unroll
    for (int q = 0; q < K / 16; ++q) {
      block64<FORM, 16, LEAD, INTEG>(L.s, L.l, J, al, dt, cmd);
      asm volatile("" : "+v"(L.s.x));
    }
    if (K % 16 != 0) block64<FORM, K % 16, LEAD, INTEG>(L.s, L.l, J, al, dt, cmd);
    if (INTEG == AEB_RK4 && L.active) xmax = fmax(xmax, L.s.x);
    bool hit = false;
    if (OBS == AEB_OBS_STATIONARY) hit = L.active && !L.collided && L.s.x > J.gap;
    if (LEAD) hit = L.active && L.l.gmin < 0.0;  // the lead was reached inside the block
    if (hit) {
      L.sv = b;
      if (LEAD) L.lv = bl;
      L.sk = k;
      L.se = k + K;
      L.collided = true;
      L.pend = true;
      if (LEAD || impact_exit) L.active = false;
    }
    k += K;
  } while (k + K <= wl && __any(L.active) && !__any(L.active && L.s.v <= thr));
  return k;
}

template <int OBS, int K, bool BATCH, int INTEG = AEB_EULER, bool CTL = false>
__global__ __launch_bounds__(256) void k_roll_fp64(const Job* __restrict__ jobs,
                                                   const LeadJob* __restrict__ leads,
                                                   const uint32_t* __restrict__ perm, int64_t n,
                                                   Ctx ctx, unsigned long long* counter,
                                                   int persistent) {
  if (ctx.hdr) n = ctx.hdr->total;  // a recorded mix: its size from the device header
  // block ladder as a lane approaches its stop: K steps, then KM, then KS,
  // then single checked steps (a level runs while no lane can stop inside it)
  constexpr int KS = 4;
  constexpr int KM = K > 16 ? 16 : KS;
  // with the controller, decisions every few tens of steps leave short
  // remainders: a 2-step level before the single steps
  constexpr int K2 = CTL ? 2 : KS;
  constexpr bool LEAD = OBS == AEB_OBS_LEAD;
  for (int pass = 0;; ++pass) {
    const int64_t base = next_chunk(counter, persistent, pass, n);
    if (base >= n) break;
    const int64_t pos = base + (threadIdx.x & 63);
    const bool valid = pos < n;
    const uint32_t g = valid ? perm[pos] : 0u;
    Job J;
    if (valid) {
      J = jobs[g];
    } else {
      J = Job{1.0, 0.0, 0.0, -1.0, 0.5, 1e30, 1.0, 0.0f, 0u};
    }
    const double al = (LEAD && valid) ? leads[g].decel : 0.0;
    const LaneScn c = lane_scn<BATCH>(ctx, J, valid, g);
    const bool varnd = BATCH || ctx.nds;
    // every lane is in its dead time for blocks ending at or before wnd (with
    // the controller: until its first command, known once decided)
    int wnd = CTL ? INT_MAX
                  : __builtin_amdgcn_readfirstlane(varnd ? wave_min(valid ? c.nd : INT_MAX) : c.nd);
    // v above these cannot reach 0 within a block (|dv/dt| <= dmax)
    const double thr_k = static_cast<double>(K) * c.dt * J.dmax;
    const double thr_m = static_cast<double>(KM) * c.dt * J.dmax;
    const double thr_s = static_cast<double>(KS) * c.dt * J.dmax;
    const double thr_2 = static_cast<double>(K2) * c.dt * J.dmax;
    // the smallest block level and its stopping bound
    constexpr int KMIN = K2 < KS ? K2 : KS;
    const double thr_min = K2 < KS ? thr_2 : thr_s;
    Lane64 L;
    L.on1 = L.on2 = INT_MAX;
    L.stage = 0;
    L.s = St64{0.0, J.v0, 0.0};
    L.l = Ld64{0.0, LEAD ? J.v0 : 0.0, J.gap};
    L.sv = L.s;
    L.lv = L.l;
    L.sk = L.se = 0;
    L.active = valid;
    L.collided = L.pend = L.clamped = false;
    // never limited: a >= a_cmd - (rounding) > alim, so max(a, alim) = a
    L.free_lane = J.alim < c.a_cmd - 1e-6;
    // limited for good once a <= alim: a never climbs above max(a, a_cmd) < alim
    L.limited = J.alim > c.a_cmd + 1e-9;
    int end = 0, steps = 0;
    // margin: with a lead vehicle the running minimum of the clearance, taken
    // when the lane ends (later blocks keep integrating an ended lane's state)
    double dist = 0.0, margin = J.gap;
    // RK4's last step may move the position back (stage speeds below zero as
    // the vehicle stops): the margin then comes from the largest position,
    // tracked over the checked steps (blocks run only while every stage
    // speed is positive, so inside them the position rises)
    double xmax = 0.0;
    float vimp = 0.0f;
    int k = 0, wl = -1;
    // controller: the next decision step and the decisions taken (uniform)
    int ktick = 0;
    uint32_t tick = 0;
    // every lane has ended by its step nmax (the horizon test fires at k + 1 == nmax)
    for (;;) {
      // the step index is the same in every lane: keep it (and the branches on it) scalar
      k = __builtin_amdgcn_readfirstlane(k);
      if (!__any(L.active)) break;
      if (CTL) {
        if (k == ktick) {
          // decision on the state after k steps; a raised stage's command
          // starts nd steps later.  Once every active lane is at the full
          // stage no decision can change anything: decisions stop, and so do
          // the block limits at decision steps.
          if (!__any(L.active && L.stage < 2)) {
            ktick = INT_MAX;
          } else {
            if (L.active && L.stage < 2) {
              const double gt = LEAD ? (J.gap + L.l.xl) - L.s.x : (J.gap + 0.0) - L.s.x;
              const double cl = LEAD ? L.s.v - L.l.vl : L.s.v - 0.0;
              // the noise is drawn only where it can change the decision,
              // estimated in single precision with an error box, and
              // evaluated exactly only where the box straddles a threshold
              int want = ctl_screen(ctx.ca, L.stage, gt, cl);
              if (want < 0) {
                const U2 u = uniform2(ctx.ca.seed, ctx.ca.sid, g, AEB_SLOT_CONTROL, tick);
                want = ctl_fast(ctx.ca, L.stage, gt, cl, u);
                if (want < 0) want = ctl_exact(ctx.ca, u, gt, cl);
              }
              if (want > L.stage) {
                if (want == 2)
                  L.on2 = k + c.nd;
                else
                  L.on1 = k + c.nd;
                L.stage = want;
              }
            }
            ++tick;
            // past the last step no decision can act
            const int64_t nk = static_cast<int64_t>(ktick) + ctx.ca.period;
            ktick = nk < c.nmax ? static_cast<int>(nk) : INT_MAX;
          }
          wnd = wave_min(valid ? min(L.on1, L.on2) : INT_MAX);
          wl = -1;
        }
        if (k >= wl) wl = min(ktick, wave_min(L.active ? ctl_lim(L, k, c.nmax) : INT_MAX));
      } else if (!varnd || k >= wl) {
        wl = wave_lim(varnd, L.active, k, c.nd, c.nmax);
      }
      if (k + K <= wl && !__any(L.active && L.s.v <= thr_k)) {
        // past every lane's dead time, in a form no later block changes:
        // a run of blocks without the per-block bookkeeping
        const bool past = k + K > wnd;
        if (past && __all(!L.active || L.clamped)) {
          k = run_steady<OBS, K, FORM_C, INTEG>(L, J, al, c.dt, 0.0, k, wl, thr_k,
                                                ctx.impact_exit, xmax);
        } else if (past && __all(!L.active || L.free_lane)) {
          const double cmd = lane_cmd<CTL>(L, c, ctx.ca.a_warn, k);
          k = run_steady<OBS, K, FORM_F, INTEG>(L, J, al, c.dt, cmd, k, wl, thr_k,
                                                ctx.impact_exit, xmax);
        } else {
          run_block64<OBS, K, INTEG, CTL>(L, J, al, c, k, wnd, ctx.impact_exit, ctx.ca.a_warn);
          if (INTEG == AEB_RK4 && L.active) xmax = fmax(xmax, L.s.x);
          k += K;
        }
      } else if (KM > KS && k + KM <= wl && !__any(L.active && L.s.v <= thr_m)) {
        run_block64<OBS, KM, INTEG, CTL>(L, J, al, c, k, wnd, ctx.impact_exit, ctx.ca.a_warn);
        if (INTEG == AEB_RK4 && L.active) xmax = fmax(xmax, L.s.x);
        k += KM;
      } else if (k + KS <= wl && !__any(L.active && L.s.v <= thr_s)) {
        run_block64<OBS, KS, INTEG, CTL>(L, J, al, c, k, wnd, ctx.impact_exit, ctx.ca.a_warn);
        if (INTEG == AEB_RK4 && L.active) xmax = fmax(xmax, L.s.x);
        k += KS;
      } else if (K2 < KS && k + K2 <= wl && !__any(L.active && L.s.v <= thr_2)) {
        run_block64<OBS, K2, INTEG, CTL>(L, J, al, c, k, wnd, ctx.impact_exit, ctx.ca.a_warn);
        if (INTEG == AEB_RK4 && L.active) xmax = fmax(xmax, L.s.x);
        k += K2;
      } else {
        // checked single steps, in a loop of their own for as long as no
        // block level fits (a lane within the smallest level's stopping
        // bound, or the block limit closer than that level) and no decision
        // step or block limit is reached
        do {
          const double cmd = lane_cmd<CTL>(L, c, ctx.ca.a_warn, k);
          if (L.active) {
            step64<LEAD, INTEG>(L.s, L.l, J, al, c.dt, cmd);
            if (INTEG == AEB_RK4) xmax = fmax(xmax, L.s.x);
            if (k >= first_cmd<CTL>(L, c))
              L.clamped = L.clamped || (L.limited && L.s.a <= J.alim);
            bool impact = false;
            if (LEAD) {
              const double gk = (J.gap + L.l.xl) - L.s.x;
              L.l.gmin = fmin(L.l.gmin, gk);
              impact = gk < 0.0;
            } else if (OBS == AEB_OBS_STATIONARY) {
              impact = L.s.x > J.gap;
            }
            if (impact && !L.collided) {
              L.collided = true;
              vimp = static_cast<float>(LEAD ? L.s.v - L.l.vl : L.s.v);
            }
            if (impact && (LEAD || ctx.impact_exit)) {
              L.active = false;
              end = AEB_END_IMPACT;
              steps = k + 1;
              dist = L.s.x;
            }
            if (L.active) {
              if (L.s.v <= 0.0) {
                L.active = false;
                end = AEB_END_STOP;
                steps = k + 1;
                dist = L.s.x;
              } else if (k + 1 == c.nmax) {
                L.active = false;
                end = AEB_END_HORIZON;
                steps = k + 1;
                dist = L.s.x;
              }
            }
            if (LEAD && !L.active) margin = L.l.gmin;
          }
          k += 1;
        } while (k < wl && !(CTL && k == ktick) && __any(L.active) &&
                 (k + KMIN > wl || __any(L.active && L.s.v <= thr_min)));
      }
    }
    // replay the block in which each pending lane passed the obstacle.  Inside
    // that block every speed stays positive, so the position rises (and with
    // a lead vehicle the running minimum of the clearance can only fall): a
    // chunk of RB steps that ends inside the block holds the crossing exactly
    // when its end state shows it.  Chunks without the crossing are skipped
    // whole; the one holding it then runs step by step.  The generic form is
    // the canonical step, so both reproduce the block's states bit for bit.
    if (OBS != AEB_OBS_NONE && __any(L.pend)) {
      St64 r = L.sv;
      Ld64 rl = L.lv;
      int kr = L.sk;
      constexpr int RB = 8;
      if (K > RB) {
        // the command is constant over a block
        const double cmd = lane_cmd<CTL>(L, c, ctx.ca.a_warn, kr);
        bool skip = L.pend;
        for (int it = 0; it < K / RB; ++it) {
          skip = skip && kr + RB <= L.se;
          if (!__any(skip)) break;
          if (skip) {
            St64 t = r;
            Ld64 tl = rl;
            block64<FORM_G, RB, LEAD, INTEG>(t, tl, J, al, c.dt, cmd);
            if (LEAD ? tl.gmin < 0.0 : t.x > J.gap) {
              skip = false;
            } else {
              r = t;
              rl = tl;
              kr += RB;
            }
          }
        }
      }
      // the replay is bit-identical to the block, so the crossing recurs within it
      for (int it = 0; it <= K; ++it) {
        if (!__any(L.pend)) break;
        if (L.pend) {
          const double cmd = lane_cmd<CTL>(L, c, ctx.ca.a_warn, kr);
          step64<LEAD, INTEG>(r, rl, J, al, c.dt, cmd);
          ++kr;
          bool impact;
          if (LEAD) {
            const double gk = (J.gap + rl.xl) - r.x;
            rl.gmin = fmin(rl.gmin, gk);
            impact = gk < 0.0;
          } else {
            impact = r.x > J.gap;
          }
          if (impact) {
            L.pend = false;
            vimp = static_cast<float>(LEAD ? r.v - rl.vl : r.v);
            if (LEAD || ctx.impact_exit) {
              end = AEB_END_IMPACT;
              steps = kr;
              dist = r.x;
              xmax = r.x;
              margin = rl.gmin;
            }
          }
        }
      }
    }
    if (L.pend) vimp = __builtin_nanf("");  // unreachable; makes a broken replay visible
    if (ctx.lanes) count_lanes(ctx.lanes, k, 64);
    if (valid) {
      if (!LEAD) {
        const double mg = J.gap - (INTEG == AEB_RK4 ? xmax : dist);
        margin = mg < J.gap ? mg : J.gap;
      }
      int64_t i;
      const OutCols o = lane_out<BATCH>(ctx, J, g, i);
      o.dist[i] = dist;
      o.margin[i] = margin;
      o.steps[i] = steps;
      o.status[i] = static_cast<uint8_t>(end | (L.collided ? AEB_COLLIDED : 0));
      o.vimp[i] = L.collided ? vimp : 0.0f;
    }
  }
}

// ---------------------------------------------------------------------------
// Two samples per lane (explicit Euler, fused form, no obstacle or a
// stationary one, no controller): lane l of a wavefront integrates the
// sorted positions base + l and base + 64 + l of a 128-sample chunk, so a
// wavefront's block bookkeeping, ladder and replay serve twice the samples
// and every block interleaves two independent dependency chains.  The forms,
// ladder, block limits and crossing replay are those of k_roll_fp64, taken
// over both samples of every lane; each sample's steps are the canonical
// step's, bit for bit.
// ---------------------------------------------------------------------------
template <int FORM, int K>
HOT void block64x2(St64 (&s)[2], const Job (&J)[2], double dt0, double dt1, double cmd0,
                   double cmd1) {
  Ld64 l{};
#pragma unroll
  for (int j = 0; j < K; ++j) {
    block64<FORM, 1, false, AEB_EULER>(s[0], l, J[0], 0.0, dt0, cmd0);
    block64<FORM, 1, false, AEB_EULER>(s[1], l, J[1], 0.0, dt1, cmd1);
    // each step's position sums happen at their step (else the compiler
    // defers them and holds the speeds of many steps in registers)
    asm volatile("" : "+v"(s[0].x), "+v"(s[1].x));
  }
}

template <int OBS, int B>
HOT void run_block64x2(Lane64 (&L)[2], const Job (&J)[2], const LaneScn (&c)[2], int k, int wnd,
                       int impact_exit) {
  double cmd[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    cmd[q] = k >= c[q].nd ? c[q].a_cmd : 0.0;
    if (OBS != AEB_OBS_NONE && !L[q].collided) {
      L[q].sv = L[q].s;
      L[q].sk = k;
      L[q].se = k + B;
    }
  }
  St64 s[2] = {L[0].s, L[1].s};
  if (k + B <= wnd) {
    block64x2<FORM_D, B>(s, J, c[0].dt, c[1].dt, cmd[0], cmd[1]);
  } else if (__all((!L[0].active || L[0].clamped) && (!L[1].active || L[1].clamped))) {
    block64x2<FORM_C, B>(s, J, c[0].dt, c[1].dt, cmd[0], cmd[1]);
  } else if (__all((!L[0].active || L[0].free_lane) && (!L[1].active || L[1].free_lane))) {
    block64x2<FORM_F, B>(s, J, c[0].dt, c[1].dt, cmd[0], cmd[1]);
  } else {
    block64x2<FORM_G, B>(s, J, c[0].dt, c[1].dt, cmd[0], cmd[1]);
#pragma unroll
    for (int q = 0; q < 2; ++q)
      L[q].clamped = L[q].clamped || (L[q].limited && k + B > c[q].nd && s[q].a <= J[q].alim);
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    L[q].s = s[q];
    if (OBS == AEB_OBS_STATIONARY && L[q].active && !L[q].collided && L[q].s.x > J[q].gap) {
      L[q].collided = true;
      L[q].pend = true;
      if (impact_exit) L[q].active = false;
    }
  }
}

// runs of steady blocks for both samples of every lane (see run_steady)
template <int OBS, int K, int FORM>
HOT int run_steady_x2(Lane64 (&L)[2], const Job (&J)[2], const LaneScn (&c)[2], double cmd0,
                      double cmd1, int k, int wl, const double (&thr)[2], int impact_exit) {
  St64 s[2] = {L[0].s, L[1].s};
  do {
    const St64 b0 = s[0], b1 = s[1];
#pragma unroll
    for (int q = 0; q < K / 16; ++q) {
      block64x2<FORM, 16>(s, J, c[0].dt, c[1].dt, cmd0, cmd1);
      asm volatile("" : "+v"(s[0].x), "+v"(s[1].x));
    }
    if (K % 16 != 0) block64x2<FORM, K % 16>(s, J, c[0].dt, c[1].dt, cmd0, cmd1);
    if (OBS == AEB_OBS_STATIONARY) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (L[q].active && !L[q].collided && s[q].x > J[q].gap) {
          L[q].sv = q == 0 ? b0 : b1;
          L[q].sk = k;
          L[q].se = k + K;
          L[q].collided = true;
          L[q].pend = true;
          if (impact_exit) L[q].active = false;
        }
      }
    }
    k += K;
  } while (k + K <= wl && __any(L[0].active || L[1].active) &&
           !__any((L[0].active && s[0].v <= thr[0]) || (L[1].active && s[1].v <= thr[1])));
  L[0].s = s[0];
  L[1].s = s[1];
  return k;
}

// the next 128 sorted positions of a wavefront (see next_chunk)
__device__ inline int64_t next_chunk2(unsigned long long* counter, int persistent, int pass,
                                      int64_t n) {
  if (pass == 0)
    return 2 * (static_cast<int64_t>(blockIdx.x) * blockDim.x +
                __builtin_amdgcn_readfirstlane(threadIdx.x & ~63u));
  if (!persistent) return n;
  unsigned long long b = 0;
  if ((threadIdx.x & 63) == 0) b = atomicAdd(counter, 128ull);
  const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(b));
  const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(b >> 32));
  return static_cast<int64_t>((static_cast<unsigned long long>(hi) << 32) | lo) +
         2 * static_cast<int64_t>(gridDim.x) * blockDim.x;
}

template <int OBS, int K, bool BATCH>
__global__ __launch_bounds__(256) void k_roll_fp64x2(const Job* __restrict__ jobs,
                                                     const uint32_t* __restrict__ perm,
                                                     int64_t n, Ctx ctx,
                                                     unsigned long long* counter,
                                                     int persistent) {
  if (ctx.hdr) n = ctx.hdr->total;  // a recorded mix: its size from the device header
  constexpr int KS = 4;
  constexpr int KM = K > 16 ? 16 : KS;
  for (int pass = 0;; ++pass) {
    const int64_t base = next_chunk2(counter, persistent, pass, n);
    if (base >= n) break;
    bool valid[2];
    uint32_t g[2];
    Job J[2];
    LaneScn c[2];
    Lane64 L[2];
    double thr_k[2], thr_m[2], thr_s[2], dist[2], margin[2];
    float vimp[2];
    int end[2], steps[2];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int64_t pos = base + 64 * q + (threadIdx.x & 63);
      valid[q] = pos < n;
      g[q] = valid[q] ? perm[pos] : 0u;
      J[q] = valid[q] ? jobs[g[q]] : Job{1.0, 0.0, 0.0, -1.0, 0.5, 1e30, 1.0, 0.0f, 0u};
      c[q] = lane_scn<BATCH>(ctx, J[q], valid[q], g[q]);
      thr_k[q] = static_cast<double>(K) * c[q].dt * J[q].dmax;
      thr_m[q] = static_cast<double>(KM) * c[q].dt * J[q].dmax;
      thr_s[q] = static_cast<double>(KS) * c[q].dt * J[q].dmax;
      L[q].on1 = L[q].on2 = INT_MAX;
      L[q].stage = 0;
      L[q].s = St64{0.0, J[q].v0, 0.0};
      L[q].l = Ld64{0.0, 0.0, J[q].gap};
      L[q].sv = L[q].s;
      L[q].lv = L[q].l;
      L[q].sk = L[q].se = 0;
      L[q].active = valid[q];
      L[q].collided = L[q].pend = L[q].clamped = false;
      L[q].free_lane = J[q].alim < c[q].a_cmd - 1e-6;
      L[q].limited = J[q].alim > c[q].a_cmd + 1e-9;
      dist[q] = 0.0;
      margin[q] = J[q].gap;
      vimp[q] = 0.0f;
      end[q] = steps[q] = 0;
    }
    const bool varnd = BATCH || ctx.nds;
    int wnd = __builtin_amdgcn_readfirstlane(
        varnd ? wave_min(min(valid[0] ? c[0].nd : INT_MAX, valid[1] ? c[1].nd : INT_MAX))
              : c[0].nd);
    int k = 0, wl = -1;
    for (;;) {
      k = __builtin_amdgcn_readfirstlane(k);
      if (!__any(L[0].active || L[1].active)) break;
      if (!varnd) {
        wl = __builtin_amdgcn_readfirstlane(lane_lim(k, c[0].nd, c[0].nmax));
      } else if (k >= wl) {
        const int l0 = L[0].active ? lane_lim(k, c[0].nd, c[0].nmax) : INT_MAX;
        const int l1 = L[1].active ? lane_lim(k, c[1].nd, c[1].nmax) : INT_MAX;
        wl = wave_min(min(l0, l1));
      }
      if (k + K <= wl && !__any((L[0].active && L[0].s.v <= thr_k[0]) ||
                                (L[1].active && L[1].s.v <= thr_k[1]))) {
        const bool past = k + K > wnd;
        if (past && __all((!L[0].active || L[0].clamped) && (!L[1].active || L[1].clamped))) {
          k = run_steady_x2<OBS, K, FORM_C>(L, J, c, 0.0, 0.0, k, wl, thr_k, ctx.impact_exit);
        } else if (past && __all((!L[0].active || L[0].free_lane) &&
                                 (!L[1].active || L[1].free_lane))) {
          const double cmd0 = k >= c[0].nd ? c[0].a_cmd : 0.0;
          const double cmd1 = k >= c[1].nd ? c[1].a_cmd : 0.0;
          k = run_steady_x2<OBS, K, FORM_F>(L, J, c, cmd0, cmd1, k, wl, thr_k, ctx.impact_exit);
        } else {
          run_block64x2<OBS, K>(L, J, c, k, wnd, ctx.impact_exit);
          k += K;
        }
      } else if (KM > KS && k + KM <= wl &&
                 !__any((L[0].active && L[0].s.v <= thr_m[0]) ||
                        (L[1].active && L[1].s.v <= thr_m[1]))) {
        run_block64x2<OBS, KM>(L, J, c, k, wnd, ctx.impact_exit);
        k += KM;
      } else if (k + KS <= wl && !__any((L[0].active && L[0].s.v <= thr_s[0]) ||
                                        (L[1].active && L[1].s.v <= thr_s[1]))) {
        run_block64x2<OBS, KS>(L, J, c, k, wnd, ctx.impact_exit);
        k += KS;
      } else {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          if (!L[q].active) continue;
          const double cmd = k >= c[q].nd ? c[q].a_cmd : 0.0;
          step64<false, AEB_EULER>(L[q].s, L[q].l, J[q], 0.0, c[q].dt, cmd);
          if (k >= c[q].nd) L[q].clamped = L[q].clamped || (L[q].limited && L[q].s.a <= J[q].alim);
          const bool impact = OBS == AEB_OBS_STATIONARY && L[q].s.x > J[q].gap;
          if (impact && !L[q].collided) {
            L[q].collided = true;
            vimp[q] = static_cast<float>(L[q].s.v);
          }
          if (impact && ctx.impact_exit) {
            L[q].active = false;
            end[q] = AEB_END_IMPACT;
            steps[q] = k + 1;
            dist[q] = L[q].s.x;
          }
          if (L[q].active) {
            if (L[q].s.v <= 0.0) {
              L[q].active = false;
              end[q] = AEB_END_STOP;
              steps[q] = k + 1;
              dist[q] = L[q].s.x;
            } else if (k + 1 == c[q].nmax) {
              L[q].active = false;
              end[q] = AEB_END_HORIZON;
              steps[q] = k + 1;
              dist[q] = L[q].s.x;
            }
          }
        }
        k += 1;
      }
    }
    // replay the block in which each pending sample passed the obstacle (see
    // k_roll_fp64), one sample of the lane after the other
    if (OBS == AEB_OBS_STATIONARY) {
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if (!__any(L[q].pend)) continue;
        St64 r = L[q].sv;
        Ld64 rl{};
        int kr = L[q].sk;
        constexpr int RB = 8;
        const double cmd = kr >= c[q].nd ? c[q].a_cmd : 0.0;
        if (K > RB) {
          bool skip = L[q].pend;
          for (int it = 0; it < K / RB; ++it) {
            skip = skip && kr + RB <= L[q].se;
            if (!__any(skip)) break;
            if (skip) {
              St64 t = r;
              block64<FORM_G, RB, false, AEB_EULER>(t, rl, J[q], 0.0, c[q].dt, cmd);
              if (t.x > J[q].gap) {
                skip = false;
              } else {
                r = t;
                kr += RB;
              }
            }
          }
        }
        for (int it = 0; it <= K; ++it) {
          if (!__any(L[q].pend)) break;
          if (L[q].pend) {
            const double cm = kr >= c[q].nd ? c[q].a_cmd : 0.0;
            step64<false, AEB_EULER>(r, rl, J[q], 0.0, c[q].dt, cm);
            ++kr;
            if (r.x > J[q].gap) {
              L[q].pend = false;
              vimp[q] = static_cast<float>(r.v);
              if (ctx.impact_exit) {
                end[q] = AEB_END_IMPACT;
                steps[q] = kr;
                dist[q] = r.x;
              }
            }
          }
        }
        if (L[q].pend) vimp[q] = __builtin_nanf("");  // unreachable; makes a broken replay visible
      }
    }
    if (ctx.lanes) count_lanes(ctx.lanes, k, 128);
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      if (!valid[q]) continue;
      const double mg = J[q].gap - dist[q];
      margin[q] = mg < J[q].gap ? mg : J[q].gap;
      int64_t i;
      const OutCols o = lane_out<BATCH>(ctx, J[q], g[q], i);
      o.dist[i] = dist[q];
      o.margin[i] = margin[q];
      o.steps[i] = steps[q];
      o.status[i] = static_cast<uint8_t>(end[q] | (L[q].collided ? AEB_COLLIDED : 0));
      o.vimp[i] = L[q].collided ? vimp[q] : 0.0f;
    }
  }
}

// ---------------------------------------------------------------------------
// FP32 compensated block forms.  State: speed (a float, or with SPLIT a float
// base plus an in-block increment carried exactly at block ends), actuator
// deviation e = a - cmd, in-block position sum p and a Kahan pair X that
// absorbs p at every block end.  Forms as in FP64:
//   G: m = max(e + (a_cmd - c), alim - c), e decays;  F: m = e + (a_cmd - c);
//   C: m = alim - c;  D: m = max(-c, alim - c) (e = 0 during the dead time).
// ---------------------------------------------------------------------------
struct L32 {
  float dt, nkd, nkt, alc, tb, td, tdm, ejump, thr, gapf;
};

struct St32 {
  float vb, vi, e, p;
  Kahan32 X;
};

template <bool SPLIT>
__device__ inline float speed32(const St32& s) {
  return SPLIT ? s.vb + s.vi : s.vb;
}

template <int FORM, int K, bool SPLIT>
__device__ inline void block32(St32& s, const L32& c, float tk) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const float v = speed32<SPLIT>(s);
    const float q = v * v;
    float m;
    if (FORM == FORM_G)
      m = fmaxf(s.e + tk, c.alc);
    else if (FORM == FORM_F)
      m = s.e + tk;
    else if (FORM == FORM_C)
      m = c.alc;
    else
      m = c.tdm;
    const float acc = fmaf(c.nkd, q, m);
    s.p = fmaf(c.dt, v, s.p);
    if (SPLIT)
      s.vi = fmaf(c.dt, acc, s.vi);
    else
      s.vb = fmaf(c.dt, acc, s.vb);
    if (FORM == FORM_G || FORM == FORM_F) s.e = fmaf(c.nkt, s.e, s.e);
  }
}

// Every 64 steps (by step index, so the rounding of a lane never depends on
// how its wavefront grouped the steps) the speed base absorbs its increment
// and the position's block sum goes into the Kahan pair.
constexpr int FLUSH = 64;

__device__ inline void flush32(St32& s, bool split) {
  if (split) {
    const float t = s.vb + s.vi;
    s.vi = s.vi - (t - s.vb);
    s.vb = t;
  }
  s.X.add(s.p);
  s.p = 0.0f;
}

template <bool SPLIT>
__device__ inline void step32(St32& s, const L32& c, bool braking) {
  const float v = speed32<SPLIT>(s);
  const float q = v * v;
  const float m = fmaxf(s.e + (braking ? c.tb : c.td), c.alc);
  const float acc = fmaf(c.nkd, q, m);
  s.p = fmaf(c.dt, v, s.p);
  if (SPLIT)
    s.vi = fmaf(c.dt, acc, s.vi);
  else
    s.vb = fmaf(c.dt, acc, s.vb);
  s.e = fmaf(c.nkt, s.e, s.e);
}

// Without compensation the speed's rounding grows with the step count; a
// lane predicted to run longer than this carries it.
constexpr double SPLIT_STEPS = 6000.0;

// Speed compensation is a per-lane property (its predicted length), so a
// lane's arithmetic never depends on its wavefront; a wavefront holding both
// kinds runs each form under its lane mask.
template <int FORM, int K>
__device__ inline void block32_any(St32& s, const L32& c, float tk, bool split) {
  if (__all(split)) {
    block32<FORM, K, true>(s, c, tk);
  } else if (__all(!split)) {
    block32<FORM, K, false>(s, c, tk);
  } else {
    if (split) block32<FORM, K, true>(s, c, tk);
    if (!split) block32<FORM, K, false>(s, c, tk);
  }
}

struct Lane32 {
  St32 s, sv;  // state, and start state of the block where the obstacle was passed
  int sk, sb;  // step index at that block start, and the block's length
  bool active, crossed, pend, clamped, free_lane;
};

template <int OBS, int B>
__device__ inline void run_block32(Lane32& L, const L32& c, bool split, int nd, int k, int wnd,
                                   int impact_exit) {
  if (OBS == AEB_OBS_STATIONARY && !L.crossed) {
    L.sv = L.s;
    L.sk = k;
    L.sb = B;
  }
  // blocks never straddle nd: the lane's target is fixed for the block
  const float tk = k >= nd ? c.tb : c.td;
  if (k + B <= wnd) {
    block32_any<FORM_D, B>(L.s, c, tk, split);
  } else if (__all(!L.active || L.clamped)) {
    block32_any<FORM_C, B>(L.s, c, tk, split);
  } else if (__all(!L.active || L.free_lane)) {
    block32_any<FORM_F, B>(L.s, c, tk, split);
  } else {
    block32_any<FORM_G, B>(L.s, c, tk, split);
    L.clamped = L.clamped || (k + B > nd && L.s.e + c.tb <= c.alc);
  }
  if ((k + B) % FLUSH == 0) flush32(L.s, split);
  if (OBS == AEB_OBS_STATIONARY && L.active && !L.crossed &&
      (L.s.X.hi - L.s.X.lo) + L.s.p > c.gapf) {
    L.crossed = true;
    L.pend = true;
    if (impact_exit) L.active = false;
  }
}

// Consecutive K-step blocks in one steady form and one speed representation
// (as run_steady of the FP64 kernel), with the flush at every flush point.
template <int OBS, int K, int FORM, bool SPLIT>
__device__ inline int run_steady32(Lane32& L, const L32& c, float tk, int k, int wl,
                                   int impact_exit) {
  do {
    const St32 b = L.s;
#pragma unroll
    for (int q = 0; q < K / 16; ++q) {
      block32<FORM, 16, SPLIT>(L.s, c, tk);
      asm volatile("" : "+v"(L.s.p));  // no position update sunk to the end of the run
    }
    if ((k + K) % FLUSH == 0) flush32(L.s, SPLIT);
    if (OBS == AEB_OBS_STATIONARY && L.active && !L.crossed &&
        (L.s.X.hi - L.s.X.lo) + L.s.p > c.gapf) {
      L.sv = b;
      L.sk = k;
      L.sb = K;
      L.crossed = true;
      L.pend = true;
      if (impact_exit) L.active = false;
    }
    k += K;
  } while (k + K <= wl && __any(L.active) && !__any(L.active && speed32<SPLIT>(L.s) <= c.thr));
  return k;
}

template <int OBS, int K, bool BATCH>
__global__ __launch_bounds__(256) void k_roll_fp32c(const Job* __restrict__ jobs,
                                                    const uint32_t* __restrict__ perm, int64_t n,
                                                    Ctx ctx, double band_abs, double band_rel,
                                                    uint32_t* fix, unsigned long long* counter,
                                                    int persistent) {
  if (ctx.hdr) n = ctx.hdr->total;  // a recorded mix: its size from the device header
  constexpr int KS = 4;
  constexpr int KM = K >= 64 ? 16 : KS;  // middle level of the block ladder
  static_assert(FLUSH % K == 0 && K % KM == 0 && KM % KS == 0,
                "flush points must fall on block ends");
  for (int pass = 0;; ++pass) {
    const int64_t base = next_chunk(counter, persistent, pass, n);
    if (base >= n) break;
    const int64_t pos = base + (threadIdx.x & 63);
    const bool valid = pos < n;
    const uint32_t g = valid ? perm[pos] : 0u;
    Job J;
    if (valid) {
      J = jobs[g];
    } else {
      J = Job{1.0, 0.0, 0.0, -1.0, 0.5, 1e30, 1.0, 0.0f, 0u};
    }
    // the scenario's constants and limits as lane values, also for one scenario
    // (the limits then take the per-lane path: the same values in every lane)
    const LaneScn sc = BATCH ? lane_scn<BATCH>(ctx, J, valid, g)
                             : lane_values(lane_scn<BATCH>(ctx, J, valid, g));
    const int nd = sc.nd, nmax = sc.nmax;
    const bool varnd = true;
    const int wnd = __builtin_amdgcn_readfirstlane(varnd ? wave_min(valid ? nd : INT_MAX) : nd);
    L32 c;  // (the speed read below is base + increment; the increment is 0 without compensation)
    c.dt = static_cast<float>(sc.dt);
    c.nkd = static_cast<float>(J.nkd);
    c.nkt = static_cast<float>(-J.kt);
    c.alc = static_cast<float>(J.alim - J.c);
    c.tb = static_cast<float>(sc.a_cmd - J.c);
    c.td = static_cast<float>(0.0 - J.c);
    c.tdm = fmaxf(c.td, c.alc);
    c.ejump = static_cast<float>(-sc.a_cmd);
    c.thr = static_cast<float>(static_cast<double>(K) * sc.dt * J.dmax);
    c.gapf = static_cast<float>(J.gap);
    const float thr_m = static_cast<float>(static_cast<double>(KM) * sc.dt * J.dmax);
    const float thr_s = static_cast<float>(static_cast<double>(KS) * sc.dt * J.dmax);
    const double band = band_abs + band_rel * fabs(J.gap);
    const bool split = J.pred > SPLIT_STEPS;  // per lane
    Lane32 L;
    L.s.vb = static_cast<float>(J.v0);
    L.s.vi = split ? static_cast<float>(J.v0 - static_cast<double>(L.s.vb)) : 0.0f;
    L.s.e = 0.0f;
    L.s.p = 0.0f;
    L.sv = L.s;
    L.sk = 0;
    L.sb = K;
    L.active = valid;
    L.crossed = L.pend = L.clamped = false;
    L.free_lane = J.alim < sc.a_cmd - 1e-6;
    const int impact_exit = ctx.impact_exit;
    bool boundary = false;
    int end = 0, steps = 0;
    double dist = 0.0;
    float vimp = 0.0f;
    int k = 0, wl = -1;
    for (;;) {
      // the step index is the same in every lane: keep it (and the branches on it) scalar
      k = __builtin_amdgcn_readfirstlane(k);
      if (!__any(L.active)) break;
      if (!varnd || k >= wl) wl = wave_lim(varnd, L.active, k, nd, nmax);
      // the command switches on at step nd: e = a - cmd jumps by -a_cmd.  Blocks
      // never straddle nd, so every lane passes through k == nd at a loop top.
      if (k == nd) L.s.e += c.ejump;
      const float v_now = speed32<true>(L.s);
      // blocks start on multiples of their length, so flush points fall on block ends
      if (k % K == 0 && k + K <= wl && !__any(L.active && v_now <= c.thr)) {
        // past every lane's dead time, in a form no later block changes, no
        // lane with the compensated speed: a run of blocks.  Without an
        // obstacle only (measured: with one the run loses to single blocks,
        // and runs for compensated-speed lanes cost more registers than they
        // save)
        const bool past = OBS == AEB_OBS_NONE && k + K > wnd;
        const bool no_split = __all(!split);
        const bool steady_c = past && __all(!L.active || L.clamped);
        const bool steady_f = past && !steady_c && __all(!L.active || L.free_lane);
        const float tk = k >= nd ? c.tb : c.td;
        if (steady_c && no_split) {
          k = run_steady32<OBS, K, FORM_C, false>(L, c, tk, k, wl, impact_exit);
        } else if (steady_f && no_split) {
          k = run_steady32<OBS, K, FORM_F, false>(L, c, tk, k, wl, impact_exit);
        } else {
          run_block32<OBS, K>(L, c, split, nd, k, wnd, impact_exit);
          k += K;
        }
      } else if (KM > KS && k % KM == 0 && k + KM <= wl &&
                 !__any(L.active && v_now <= thr_m)) {
        run_block32<OBS, KM>(L, c, split, nd, k, wnd, impact_exit);
        k += KM;
      } else if (k % KS == 0 && k + KS <= wl && !__any(L.active && v_now <= thr_s)) {
        run_block32<OBS, KS>(L, c, split, nd, k, wnd, impact_exit);
        k += KS;
      } else {
        if (L.active) {
          const float vb = v_now;
          if (split) step32<true>(L.s, c, k >= nd);
          if (!split) step32<false>(L.s, c, k >= nd);
          if ((k + 1) % FLUSH == 0) flush32(L.s, split);
          if (k >= nd) L.clamped = L.clamped || (L.s.e + c.tb <= c.alc);
          const float v = speed32<true>(L.s);
          if (OBS == AEB_OBS_STATIONARY && !L.crossed && (L.s.X.hi - L.s.X.lo) + L.s.p > c.gapf) {
            L.crossed = true;
            vimp = v;
            if (impact_exit) {
              L.active = false;
              end = AEB_END_IMPACT;
              steps = k + 1;
              dist = L.s.X.value(L.s.p);
              const double step_len = static_cast<double>(c.dt) * static_cast<double>(vb);
              boundary = fabs(dist - J.gap) < band || fabs(J.gap - (dist - step_len)) < band;
            }
          }
          if (L.active) {
            if (v <= 0.0f) {
              L.active = false;
              end = AEB_END_STOP;
              steps = k + 1;
              dist = L.s.X.value(L.s.p);
            } else if (k + 1 == nmax) {
              L.active = false;
              end = AEB_END_HORIZON;
              steps = k + 1;
              dist = L.s.X.value(L.s.p);
            }
          }
        }
        k += 1;
      }
    }
    // replay the block in which each pending lane passed the obstacle, single
    // steps with the per-step test; the crossing recurs within the block (at its
    // last step at the latest, where the block-end test fired)
    if (OBS == AEB_OBS_STATIONARY && __any(L.pend)) {
      St32 r = L.sv;
      int kr = L.sk;
      for (int it = 0; it < K; ++it) {
        if (!__any(L.pend)) break;
        if (L.pend) {
          const float vb = speed32<true>(r);
          if (split) step32<true>(r, c, kr >= nd);
          if (!split) step32<false>(r, c, kr >= nd);
          ++kr;
          if (kr % FLUSH == 0) flush32(r, split);
          const float v = speed32<true>(r);
          if ((r.X.hi - r.X.lo) + r.p > c.gapf || it == L.sb - 1) {
            L.pend = false;
            vimp = v;
            if (impact_exit) {
              end = AEB_END_IMPACT;
              steps = kr;
              dist = r.X.value(r.p);
              const double step_len = static_cast<double>(c.dt) * static_cast<double>(vb);
              boundary = fabs(dist - J.gap) < band || fabs(J.gap - (dist - step_len)) < band;
            }
          }
        }
      }
    }
    bool collided = L.crossed;
    if (OBS == AEB_OBS_STATIONARY && !impact_exit) {
      // the flag is decided in FP64 on the compensated distance
      collided = dist > J.gap;
      boundary = fabs(J.gap - dist) < band;
      if (collided != L.crossed) vimp = 0.0f;
    } else if (OBS == AEB_OBS_STATIONARY && !L.crossed) {
      boundary = J.gap - dist < band;
    }
    if (ctx.lanes) count_lanes(ctx.lanes, k, 64);
    if (valid) {
      const double mg = J.gap - dist;
      int64_t i;
      const OutCols o = lane_out<BATCH>(ctx, J, g, i);
      o.dist[i] = dist;
      o.margin[i] = mg < J.gap ? mg : J.gap;
      o.steps[i] = steps;
      o.status[i] = static_cast<uint8_t>(end | (collided ? AEB_COLLIDED : 0) |
                                         (boundary ? AEB_BOUNDARY : 0));
      o.vimp[i] = collided ? vimp : 0.0f;
      if (boundary && fix) {
        const uint32_t slot = atomicAdd(fix, 1u);
        fix[1 + slot] = g;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// FP32 compensated form with a lead vehicle.  The clearance is integrated
// directly, c' = c + dt (v_lead - v), as an in-block sum plus a Kahan pair,
// so no two large positions are ever subtracted; both speeds are a float
// base plus an in-block increment.  A lane's clearance after a step is read
// after that step's flush (every 64 steps by index) in every path, and its
// running minimum is the margin.  A crossing inside a block (minimum below
// zero) is replayed from the block's start state; the rollout ends there.
// ---------------------------------------------------------------------------
struct Ld32 {
  float vb, vi;  // lead speed: base + increment (read clamped at 0)
  float pg;      // in-block clearance sum
  Kahan32 G;     // clearance
  float gmin;    // running minimum of the clearance after each step
};

__device__ inline float lead_speed(const Ld32& l) { return fmaxf(l.vb + l.vi, 0.0f); }
__device__ inline float clearance(const Ld32& l) { return (l.G.hi - l.G.lo) + l.pg; }

__device__ inline void flush32l(St32& s, Ld32& l) {
  flush32(s, true);
  const float t = l.vb + l.vi;
  l.vi = l.vi - (t - l.vb);
  l.vb = t;
  l.G.add(l.pg);
  l.pg = 0.0f;
}

// one step of ego and lead (the ego's form as in block32, speed always split)
template <int FORM>
__device__ inline void step32l(St32& s, Ld32& l, const L32& c, float tk, float al) {
  const float v = s.vb + s.vi;
  const float vl = lead_speed(l);
  const float q = v * v;
  float m;
  if (FORM == FORM_G)
    m = fmaxf(s.e + tk, c.alc);
  else if (FORM == FORM_F)
    m = s.e + tk;
  else if (FORM == FORM_C)
    m = c.alc;
  else
    m = c.tdm;
  const float acc = fmaf(c.nkd, q, m);
  s.p = fmaf(c.dt, v, s.p);
  l.pg = fmaf(c.dt, vl - v, l.pg);
  l.vi = fmaf(-c.dt, al, l.vi);
  s.vi = fmaf(c.dt, acc, s.vi);
  if (FORM == FORM_G || FORM == FORM_F) s.e = fmaf(c.nkt, s.e, s.e);
}

template <int FORM, int K>
__device__ inline void block32l(St32& s, Ld32& l, const L32& c, float tk, float al,
                                bool flush_end) {
  float ghl = l.G.hi - l.G.lo;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    step32l<FORM>(s, l, c, tk, al);
    if (j == K - 1 && flush_end) {
      flush32l(s, l);
      ghl = l.G.hi - l.G.lo;
    }
    l.gmin = fminf(l.gmin, ghl + l.pg);
  }
}

struct Lane32L {
  St32 s, sv;
  Ld32 l, lv;
  int sk;
  bool active, pend, clamped, free_lane;
};

template <int B>
__device__ inline void run_block32l(Lane32L& L, const L32& c, float al, int nd, int k, int wnd) {
  // a lane that has ended keeps the start state of the block it ended in
  if (L.active) {
    L.sv = L.s;
    L.lv = L.l;
    L.sk = k;
  }
  const float tk = k >= nd ? c.tb : c.td;
  const bool fl = (k + B) % FLUSH == 0;
  if (k + B <= wnd) {
    block32l<FORM_D, B>(L.s, L.l, c, tk, al, fl);
  } else if (__all(!L.active || L.clamped)) {
    block32l<FORM_C, B>(L.s, L.l, c, tk, al, fl);
  } else if (__all(!L.active || L.free_lane)) {
    block32l<FORM_F, B>(L.s, L.l, c, tk, al, fl);
  } else {
    block32l<FORM_G, B>(L.s, L.l, c, tk, al, fl);
    L.clamped = L.clamped || (k + B > nd && L.s.e + c.tb <= c.alc);
  }
  if (L.active && L.l.gmin < 0.0f) {  // the lead was reached inside the block
    L.pend = true;
    L.active = false;
  }
}

template <int K, bool BATCH>
__global__ __launch_bounds__(256) void k_roll_fp32c_lead(const Job* __restrict__ jobs,
                                                         const LeadJob* __restrict__ leads,
                                                         const uint32_t* __restrict__ perm,
                                                         int64_t n, Ctx ctx, double band_abs,
                                                         double band_rel, uint32_t* fix,
                                                         unsigned long long* counter,
                                                         int persistent) {
  if (ctx.hdr) n = ctx.hdr->total;  // a recorded mix: its size from the device header
  constexpr int KS = 4;
  constexpr int KM = K >= 64 ? 16 : KS;  // middle level of the block ladder
  static_assert(FLUSH % K == 0 && K % KM == 0 && KM % KS == 0,
                "flush points must fall on block ends");
  for (int pass = 0;; ++pass) {
    const int64_t base = next_chunk(counter, persistent, pass, n);
    if (base >= n) break;
    const int64_t pos = base + (threadIdx.x & 63);
    const bool valid = pos < n;
    const uint32_t g = valid ? perm[pos] : 0u;
    Job J;
    if (valid) {
      J = jobs[g];
    } else {
      J = Job{1.0, 0.0, 0.0, -1.0, 0.5, 1e30, 1.0, 0.0f, 0u};
    }
    const float al = valid ? static_cast<float>(leads[g].decel) : 0.0f;
    const LaneScn sc = lane_scn<BATCH>(ctx, J, valid, g);
    const int nd = sc.nd, nmax = sc.nmax;
    const bool varnd = BATCH || ctx.nds;
    const int wnd = __builtin_amdgcn_readfirstlane(varnd ? wave_min(valid ? nd : INT_MAX) : nd);
    L32 c;
    c.dt = static_cast<float>(sc.dt);
    c.nkd = static_cast<float>(J.nkd);
    c.nkt = static_cast<float>(-J.kt);
    c.alc = static_cast<float>(J.alim - J.c);
    c.tb = static_cast<float>(sc.a_cmd - J.c);
    c.td = static_cast<float>(0.0 - J.c);
    c.tdm = fmaxf(c.td, c.alc);
    c.ejump = static_cast<float>(-sc.a_cmd);
    c.thr = static_cast<float>(static_cast<double>(K) * sc.dt * J.dmax);
    c.gapf = static_cast<float>(J.gap);
    const float thr_m = static_cast<float>(static_cast<double>(KM) * sc.dt * J.dmax);
    const float thr_s = static_cast<float>(static_cast<double>(KS) * sc.dt * J.dmax);
    const double band = band_abs + band_rel * fabs(J.gap);
    Lane32L L;
    L.s.vb = static_cast<float>(J.v0);
    L.s.vi = static_cast<float>(J.v0 - static_cast<double>(L.s.vb));
    L.s.e = 0.0f;
    L.s.p = 0.0f;
    L.l.vb = L.s.vb;
    L.l.vi = L.s.vi;
    L.l.pg = 0.0f;
    L.l.G.hi = c.gapf;
    L.l.G.lo = static_cast<float>(static_cast<double>(c.gapf) - J.gap);
    L.l.gmin = clearance(L.l);
    L.sv = L.s;
    L.lv = L.l;
    L.sk = 0;
    L.active = valid;
    L.pend = L.clamped = false;
    L.free_lane = J.alim < sc.a_cmd - 1e-6;
    bool boundary = false, collided = false;
    int end = 0, steps = 0;
    double dist = 0.0;
    float vimp = 0.0f;
    float gprev = L.l.gmin;
    float gm_end = L.l.gmin;  // running minimum of the clearance when the lane ended
    int k = 0, wl = -1;
    for (;;) {
      k = __builtin_amdgcn_readfirstlane(k);
      if (!__any(L.active)) break;
      if (!varnd || k >= wl) wl = wave_lim(varnd, L.active, k, nd, nmax);
      if (k == nd) L.s.e += c.ejump;
      const float v_now = L.s.vb + L.s.vi;
      if (k % K == 0 && k + K <= wl && !__any(L.active && v_now <= c.thr)) {
        run_block32l<K>(L, c, al, nd, k, wnd);
        k += K;
      } else if (KM > KS && k % KM == 0 && k + KM <= wl &&
                 !__any(L.active && v_now <= thr_m)) {
        run_block32l<KM>(L, c, al, nd, k, wnd);
        k += KM;
      } else if (k % KS == 0 && k + KS <= wl && !__any(L.active && v_now <= thr_s)) {
        run_block32l<KS>(L, c, al, nd, k, wnd);
        k += KS;
      } else {
        if (L.active) {
          const float gp = clearance(L.l);
          step32l<FORM_G>(L.s, L.l, c, k >= nd ? c.tb : c.td, al);
          if ((k + 1) % FLUSH == 0) flush32l(L.s, L.l);
          if (k >= nd) L.clamped = L.clamped || (L.s.e + c.tb <= c.alc);
          const float gk = clearance(L.l);
          L.l.gmin = fminf(L.l.gmin, gk);
          const float v = L.s.vb + L.s.vi;
          if (gk < 0.0f) {
            L.active = false;
            collided = true;
            vimp = v - lead_speed(L.l);
            end = AEB_END_IMPACT;
            steps = k + 1;
            dist = L.s.X.value(L.s.p);
            boundary = fabs(static_cast<double>(gp)) < band || fabs(static_cast<double>(gk)) < band;
          } else if (v <= 0.0f) {
            L.active = false;
            end = AEB_END_STOP;
            steps = k + 1;
            dist = L.s.X.value(L.s.p);
          } else if (k + 1 == nmax) {
            L.active = false;
            end = AEB_END_HORIZON;
            steps = k + 1;
            dist = L.s.X.value(L.s.p);
          }
          if (!L.active) gm_end = L.l.gmin;
        }
        k += 1;
      }
    }
    // replay the block in which each pending lane reached the lead: the same
    // steps one at a time, with the clearance read after each (post-flush)
    if (__any(L.pend)) {
      St32 r = L.sv;
      Ld32 rl = L.lv;
      int kr = L.sk;
      gprev = clearance(rl);
      for (int it = 0; it < K; ++it) {
        if (!__any(L.pend)) break;
        if (L.pend) {
          step32l<FORM_G>(r, rl, c, kr >= nd ? c.tb : c.td, al);
          ++kr;
          if (kr % FLUSH == 0) flush32l(r, rl);
          const float gk = clearance(rl);
          rl.gmin = fminf(rl.gmin, gk);
          if (gk < 0.0f) {
            L.pend = false;
            collided = true;
            vimp = (r.vb + r.vi) - lead_speed(rl);
            end = AEB_END_IMPACT;
            steps = kr;
            dist = r.X.value(r.p);
            boundary = fabs(static_cast<double>(gprev)) < band || fabs(static_cast<double>(gk)) < band;
            gm_end = rl.gmin;
          }
          gprev = gk;
        }
      }
    }
    if (L.pend) vimp = __builtin_nanf("");  // unreachable; makes a broken replay visible
    if (!collided) boundary = static_cast<double>(gm_end) < band;
    if (ctx.lanes) count_lanes(ctx.lanes, k, 64);
    if (valid) {
      int64_t i;
      const OutCols o = lane_out<BATCH>(ctx, J, g, i);
      o.dist[i] = dist;
      o.margin[i] = static_cast<double>(gm_end);
      o.steps[i] = steps;
      o.status[i] = static_cast<uint8_t>(end | (collided ? AEB_COLLIDED : 0) |
                                         (boundary ? AEB_BOUNDARY : 0));
      o.vimp[i] = collided ? vimp : 0.0f;
      if (boundary && fix) {
        const uint32_t slot = atomicAdd(fix, 1u);
        fix[1 + slot] = g;
      }
    }
  }
}

}  // namespace

// The block path counts steps in int and tests k + (block length) and
// k + (command delay): the horizon and the dead time together stay this far
// below 2^31 (longer runs take the checked FP64 kernel, which counts in 64 bits).
bool block_steps_ok(const aeb_scenario& s) {
  return horizon_steps(s) + dead_steps(s) <= BLOCK_STEP_MAX;
}

bool fast_path_applies(const aeb_scenario& s, int precision) {
  if (!block_steps_ok(s)) return false;
  // the controller: FP64 only (explicit Euler, fused or unfused, or RK4)
  if (control_on(s)) return precision == AEB_FP64;
  if (precision == AEB_FP64) return s.obstacle != AEB_OBS_LEAD || s.integrator != AEB_RK4;
  if (s.integrator != AEB_EULER) return false;
  return precision == AEB_FP32C || precision == AEB_FP32C_FIXUP;
}

namespace {

// Launch shape of the integration kernel from the tuning table: workgroup
// size, and either one pass over ceil(n / block) workgroups or a persistent
// grid of `waves_per_simd` wavefronts per SIMD claiming work from the counter.
struct Shape {
  unsigned grid, block;
  int persistent;
};

// spt: samples per lane of the kernel launched (a one-pass grid covers
// n / spt lanes)
Shape shape(const TuneCfg& t, int64_t n, int spt = 1) {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      cus = 256;
  }
  Shape sh;
  sh.block = static_cast<unsigned>(t.block);
  const int64_t per = static_cast<int64_t>(t.block) * spt;
  const int64_t need = (n + per - 1) / per;
  if (t.waves_per_simd > 0) {
    const int64_t grid = static_cast<int64_t>(cus) * 4 * t.waves_per_simd * 64 / t.block;
    sh.grid = static_cast<unsigned>(need < grid ? need : grid);
    sh.persistent = 1;
  } else {
    sh.grid = static_cast<unsigned>(need);
    sh.persistent = 0;
  }
  return sh;
}

struct Bufs {
  Job* jobs;
  LeadJob* leads;
  uint32_t* keys;
  uint32_t* perm;
  int32_t* nds;
  uint32_t* fix;  // FP32C fix-up list: count, then sample indices
  uint32_t* hist;
  unsigned long long* counter;
  ScnDev* tab;
  aeb_scenario* scns;
};

// scratch: jobs | leads | keys | perm | command steps | fix-up list |
// histogram | counter | scenario tables
size_t bufs_layout(int64_t n, int n_scn, bool lead, char* base, Bufs* b) {
  auto up = [](size_t x) { return (x + 255) & ~size_t(255); };
  const size_t off_jobs = 0;
  const size_t off_leads = up(off_jobs + sizeof(Job) * n);
  const size_t off_keys = up(off_leads + (lead ? sizeof(LeadJob) * n : 0));
  const size_t off_perm = up(off_keys + sizeof(uint32_t) * n);
  const size_t off_nds = up(off_perm + sizeof(uint32_t) * n);
  const size_t off_fix = up(off_nds + sizeof(int32_t) * n);
  const size_t off_hist = up(off_fix + sizeof(uint32_t) * (n + 1));
  const size_t off_cnt = up(off_hist + sizeof(uint32_t) * NBINS_CTL);
  const size_t off_tab = up(off_cnt + sizeof(unsigned long long));
  const size_t off_scn = up(off_tab + sizeof(ScnDev) * n_scn);
  const size_t total = up(off_scn + sizeof(aeb_scenario) * n_scn);
  if (b) {
    b->jobs = reinterpret_cast<Job*>(base + off_jobs);
    b->leads = lead ? reinterpret_cast<LeadJob*>(base + off_leads) : nullptr;
    b->keys = reinterpret_cast<uint32_t*>(base + off_keys);
    b->perm = reinterpret_cast<uint32_t*>(base + off_perm);
    b->nds = reinterpret_cast<int32_t*>(base + off_nds);
    b->fix = reinterpret_cast<uint32_t*>(base + off_fix);
    b->hist = reinterpret_cast<uint32_t*>(base + off_hist);
    b->counter = reinterpret_cast<unsigned long long*>(base + off_cnt);
    b->tab = reinterpret_cast<ScnDev*>(base + off_tab);
    b->scns = reinterpret_cast<aeb_scenario*>(base + off_scn);
  }
  return total;
}

// sort the prepared keys into the permutation (the scan zeroes the claim counter)
// (hdr: a recorded mix, n its capacity and the actual count on the device)
// (hist: the key histogram still to be taken; the plain method's prep takes it)
template <int NB = NBINS>
void sort_keys(const Bufs& b, int64_t n, hipStream_t st, const BatchHdr* hdr = nullptr,
               bool hist = true) {
  const unsigned pblk = static_cast<unsigned>((n + PREP_SAMPLES - 1) / PREP_SAMPLES);
  if (hist)
    hipLaunchKernelGGL(k_hist<NB>, dim3(pblk), dim3(PREP_BLOCK), 0, st, b.keys, n, b.hist, hdr);
  hipLaunchKernelGGL(k_scan<NB>, dim3(1), dim3(PREP_BLOCK), 0, st, b.hist, b.counter);
  hipLaunchKernelGGL(k_scatter<NB>, dim3(pblk), dim3(PREP_BLOCK), 0, st, b.keys, n, b.hist,
                     b.perm, hdr);
}

template <int OBS, int K, bool BATCH, int INTEG = AEB_EULER, bool CTL = false>
void go64(const Shape& sh, const Bufs& b, int64_t n, const Ctx& ctx, hipStream_t st) {
  hipLaunchKernelGGL((k_roll_fp64<OBS, K, BATCH, INTEG, CTL>), dim3(sh.grid), dim3(sh.block), 0,
                     st, b.jobs, b.leads, b.perm, n, ctx, b.counter, sh.persistent);
}

template <int OBS, int K, bool BATCH>
void go64x2(const Shape& sh, const Bufs& b, int64_t n, const Ctx& ctx, hipStream_t st) {
  hipLaunchKernelGGL((k_roll_fp64x2<OBS, K, BATCH>), dim3(sh.grid), dim3(sh.block), 0, st, b.jobs,
                     b.perm, n, ctx, b.counter, sh.persistent);
}

template <int OBS, bool BATCH>
void go64x2k(int k, const Shape& sh, const Bufs& b, int64_t n, const Ctx& ctx, hipStream_t st) {
  if (k == 16)
    go64x2<OBS, 16, BATCH>(sh, b, n, ctx, st);
  else if (k == 64)
    go64x2<OBS, 64, BATCH>(sh, b, n, ctx, st);
  else if (k == 128)
    go64x2<OBS, 128, BATCH>(sh, b, n, ctx, st);
  else
    go64x2<OBS, 32, BATCH>(sh, b, n, ctx, st);
}

template <int OBS, bool BATCH>
void go64k(int k, const Shape& sh, const Bufs& b, int64_t n, const Ctx& ctx, hipStream_t st) {
  if (k == 16)
    go64<OBS, 16, BATCH>(sh, b, n, ctx, st);
  else if (k == 64)
    go64<OBS, 64, BATCH>(sh, b, n, ctx, st);
  else if (k == 128)
    go64<OBS, 128, BATCH>(sh, b, n, ctx, st);
  else
    go64<OBS, 32, BATCH>(sh, b, n, ctx, st);
}

template <int OBS, bool BATCH>
void go32k(int k, const Shape& sh, const Bufs& b, int64_t n, const Ctx& ctx, double band_abs,
           double band_rel, uint32_t* fix, hipStream_t st) {
  if (k == 16)
    hipLaunchKernelGGL((k_roll_fp32c<OBS, 16, BATCH>), dim3(sh.grid), dim3(sh.block), 0, st,
                       b.jobs, b.perm, n, ctx, band_abs, band_rel, fix, b.counter, sh.persistent);
  else if (k == 64)
    hipLaunchKernelGGL((k_roll_fp32c<OBS, 64, BATCH>), dim3(sh.grid), dim3(sh.block), 0, st,
                       b.jobs, b.perm, n, ctx, band_abs, band_rel, fix, b.counter, sh.persistent);
  else
    hipLaunchKernelGGL((k_roll_fp32c<OBS, 32, BATCH>), dim3(sh.grid), dim3(sh.block), 0, st,
                       b.jobs, b.perm, n, ctx, band_abs, band_rel, fix, b.counter, sh.persistent);
}

// With timing enabled, the lane accounting of the launch that follows
// (zeroed first, by a kernel so that the sequence stays recordable).
inline void arm_lanes(Ctx& ctx, hipStream_t st) {
  ctx.lanes = timing_lanes();
  if (ctx.lanes)
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, reinterpret_cast<uint32_t*>(ctx.lanes),
                       int64_t(2));
}

template <bool BATCH>
int integrate(const aeb_scenario& s0, int precision, const Bufs& b, int64_t n, const Ctx& ctx_in,
              const ParamSrc* src, hipStream_t st) {
  const int obs = s0.obstacle;
  Ctx ctx = ctx_in;
  const TuneCfg t = tune_get(precision == AEB_FP64 ? AEB_FP64 : AEB_FP32C, obs);
  const Shape sh = shape(t, n);
  if (!BATCH && control_on(s0)) {
    // the controller decides every ctl_period and blocks stay within a
    // decision period: the top level is a block size that divides the period
    // where one is built (50 steps: 20 and 10 Hz at 1 ms; 40: 25 Hz), else 48
    // (a 50-step period would take a 48-step and a 2-step block); FP64 only
    const int64_t per = ctl_args(s0).period;
    arm_lanes(ctx, st);
    timing_begin(st);
    if (s0.integrator == AEB_RK4)
      go64<AEB_OBS_STATIONARY, 16, false, AEB_RK4, true>(sh, b, n, ctx, st);
    else if (s0.nofma && obs == AEB_OBS_LEAD)  // the unfused form
      per % 50 == 0   ? go64<AEB_OBS_LEAD, 50, false, EULER_NOFMA, true>(sh, b, n, ctx, st)
      : per % 40 == 0 ? go64<AEB_OBS_LEAD, 40, false, EULER_NOFMA, true>(sh, b, n, ctx, st)
                      : go64<AEB_OBS_LEAD, 48, false, EULER_NOFMA, true>(sh, b, n, ctx, st);
    else if (s0.nofma)
      per % 50 == 0   ? go64<AEB_OBS_STATIONARY, 50, false, EULER_NOFMA, true>(sh, b, n, ctx, st)
      : per % 40 == 0 ? go64<AEB_OBS_STATIONARY, 40, false, EULER_NOFMA, true>(sh, b, n, ctx, st)
                      : go64<AEB_OBS_STATIONARY, 48, false, EULER_NOFMA, true>(sh, b, n, ctx, st);
    else if (obs == AEB_OBS_LEAD)
      per % 50 == 0   ? go64<AEB_OBS_LEAD, 50, false, AEB_EULER, true>(sh, b, n, ctx, st)
      : per % 40 == 0 ? go64<AEB_OBS_LEAD, 40, false, AEB_EULER, true>(sh, b, n, ctx, st)
                      : go64<AEB_OBS_LEAD, 48, false, AEB_EULER, true>(sh, b, n, ctx, st);
    else
      per % 50 == 0   ? go64<AEB_OBS_STATIONARY, 50, false, AEB_EULER, true>(sh, b, n, ctx, st)
      : per % 40 == 0 ? go64<AEB_OBS_STATIONARY, 40, false, AEB_EULER, true>(sh, b, n, ctx, st)
                      : go64<AEB_OBS_STATIONARY, 48, false, AEB_EULER, true>(sh, b, n, ctx, st);
    timing_end(st);
    AEB_HIP(hipGetLastError());
    return AEB_OK;
  }
  if (precision == AEB_FP64 && s0.integrator == AEB_RK4) {
    // an RK4 step costs about eight Euler steps: short blocks keep the tail small
    arm_lanes(ctx, st);
    timing_begin(st);
    if (obs == AEB_OBS_STATIONARY)
      go64<AEB_OBS_STATIONARY, 16, BATCH, AEB_RK4>(sh, b, n, ctx, st);
    else
      go64<AEB_OBS_NONE, 16, BATCH, AEB_RK4>(sh, b, n, ctx, st);
    timing_end(st);
    AEB_HIP(hipGetLastError());
    return AEB_OK;
  }
  if (precision == AEB_FP64 && s0.nofma) {
    // the unfused form: 128-step blocks, the launch shape of the table
    arm_lanes(ctx, st);
    timing_begin(st);
    if (obs == AEB_OBS_STATIONARY)
      go64<AEB_OBS_STATIONARY, 128, BATCH, EULER_NOFMA>(sh, b, n, ctx, st);
    else if (obs == AEB_OBS_LEAD)
      go64<AEB_OBS_LEAD, 128, BATCH, EULER_NOFMA>(sh, b, n, ctx, st);
    else
      go64<AEB_OBS_NONE, 128, BATCH, EULER_NOFMA>(sh, b, n, ctx, st);
    timing_end(st);
    AEB_HIP(hipGetLastError());
    return AEB_OK;
  }
  if (precision == AEB_FP64 && t.spt == 2 && obs != AEB_OBS_LEAD) {
    // two samples per lane (the tuned FP64 shape)
    const Shape sh2 = shape(t, n, 2);
    arm_lanes(ctx, st);
    timing_begin(st);
    if (obs == AEB_OBS_STATIONARY)
      go64x2k<AEB_OBS_STATIONARY, BATCH>(t.k, sh2, b, n, ctx, st);
    else
      go64x2k<AEB_OBS_NONE, BATCH>(t.k, sh2, b, n, ctx, st);
    timing_end(st);
    AEB_HIP(hipGetLastError());
    return AEB_OK;
  }
  if (precision == AEB_FP64) {
    arm_lanes(ctx, st);
    timing_begin(st);
    if (obs == AEB_OBS_STATIONARY)
      go64k<AEB_OBS_STATIONARY, BATCH>(t.k, sh, b, n, ctx, st);
    else if (obs == AEB_OBS_LEAD)
      go64k<AEB_OBS_LEAD, BATCH>(t.k, sh, b, n, ctx, st);
    else
      go64k<AEB_OBS_NONE, BATCH>(t.k, sh, b, n, ctx, st);
    timing_end(st);
    AEB_HIP(hipGetLastError());
    return AEB_OK;
  }
  uint32_t* fix = nullptr;
  if (precision == AEB_FP32C_FIXUP) {
    if (BATCH) return fail(AEB_EINVAL, "the FP64 fix-up mode is not available for batches");
    fix = b.fix;
    hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, fix, int64_t(1));
  }
  // The form's stated distance tolerance is 1e-4 relative; at the obstacle the
  // distance is the gap, so outcomes within 1 mm + 1e-4 of the gap of the
  // boundary are flagged (and, in the fix-up mode, recomputed in FP64): as
  // long as the distance error stays below that band, every flag outside it
  // equals the FP64 one.
  const double band_abs = 1e-3, band_rel = 1e-4;
  arm_lanes(ctx, st);
  timing_begin(st);
  if (obs == AEB_OBS_LEAD) {
    if (t.k == 16)
      hipLaunchKernelGGL((k_roll_fp32c_lead<16, BATCH>), dim3(sh.grid), dim3(sh.block), 0, st,
                         b.jobs, b.leads, b.perm, n, ctx, band_abs, band_rel, fix, b.counter,
                         sh.persistent);
    else if (t.k == 64)
      hipLaunchKernelGGL((k_roll_fp32c_lead<64, BATCH>), dim3(sh.grid), dim3(sh.block), 0, st,
                         b.jobs, b.leads, b.perm, n, ctx, band_abs, band_rel, fix, b.counter,
                         sh.persistent);
    else
      hipLaunchKernelGGL((k_roll_fp32c_lead<32, BATCH>), dim3(sh.grid), dim3(sh.block), 0, st,
                         b.jobs, b.leads, b.perm, n, ctx, band_abs, band_rel, fix, b.counter,
                         sh.persistent);
  } else if (obs == AEB_OBS_STATIONARY)
    go32k<AEB_OBS_STATIONARY, BATCH>(t.k, sh, b, n, ctx, band_abs, band_rel, fix, st);
  else
    go32k<AEB_OBS_NONE, BATCH>(t.k, sh, b, n, ctx, band_abs, band_rel, fix, st);
  timing_end(st);
  AEB_HIP(hipGetLastError());
  if (fix) return launch_fixup(s0, src, ctx.out, fix, st);
  return AEB_OK;
}

}  // namespace

size_t rollout_scratch_bytes(const aeb_scenario& s, int64_t n) {
  return bufs_layout(n, 0, s.obstacle == AEB_OBS_LEAD, nullptr, nullptr);
}

int launch_rollout_fast_into(const aeb_scenario& s, const ParamSrc* src, int precision,
                             const OutCols& out, int64_t n, void* scratch_base, hipStream_t st) {
  const int64_t nd = dead_steps(s), nmax = horizon_steps(s);
  if (!block_steps_ok(s))
    return fail(AEB_EINVAL, "horizon plus dead time beyond 2^31 - 4096 steps on the block path");
  const bool lead = s.obstacle == AEB_OBS_LEAD;
  Bufs b;
  bufs_layout(n, 0, lead, static_cast<char*>(scratch_base), &b);
  const unsigned pblk = prep_grid(n);
  const bool ctl = control_on(s);
  const int nb = ctl ? NBINS_CTL : NBINS;
  hipLaunchKernelGGL(k_zero, dim3(nb / 256), dim3(256), 0, st, b.hist, int64_t(nb));
  PrepArgs pa{};
  pa.s = s;
  pa.src = src ? *src : ParamSrc{};
  pa.n = n;
  pa.nd = static_cast<int>(nd);
  pa.nmax = static_cast<int>(nmax);
  pa.cap = static_cast<float>(nmax);
  pa.nds = perception_on(s) ? b.nds : nullptr;
  pa.ctl = ctl ? 1 : 0;
  pa.weight = out.weight;
  const unsigned cblk = static_cast<unsigned>((n + PREP_SAMPLES - 1) / PREP_SAMPLES);
  if (src && ctl)
    hipLaunchKernelGGL(k_prep_cols<NBINS_CTL>, dim3(cblk), dim3(PREP_BLOCK), 0, st, pa, b.jobs,
                       b.leads, b.keys, b.hist);
  else if (src)
    hipLaunchKernelGGL(k_prep_cols<NBINS>, dim3(cblk), dim3(PREP_BLOCK), 0, st, pa, b.jobs,
                       b.leads, b.keys, b.hist);
  else
    hipLaunchKernelGGL((k_prep<true, false>), dim3(pblk), dim3(PREP_BLOCK), 0, st, pa, b.jobs,
                       b.leads, b.keys);
  if (ctl)
    sort_keys<NBINS_CTL>(b, n, st, nullptr, !src);
  else
    sort_keys(b, n, st, nullptr, !src);
  Ctx ctx{};
  ctx.dt = s.dt;
  ctx.a_cmd = s.a_cmd;
  ctx.nd = static_cast<int>(nd);
  ctx.nmax = static_cast<int>(nmax);
  ctx.impact_exit = s.impact_exit;
  ctx.out = out;
  ctx.tab = nullptr;
  ctx.nds = pa.nds;
  ctx.ca = ctl_args(s);
  return integrate<false>(s, precision, b, n, ctx, src, st);
}

int launch_rollout_fast(const aeb_scenario& s, const ParamSrc* src, int precision,
                        const OutCols& out, int64_t n, hipStream_t st) {
  void* base = pool_block(rollout_scratch_bytes(s, n), st);
  if (!base) return AEB_ENOMEM;
  return launch_rollout_fast_into(s, src, precision, out, n, base, st);
}

size_t batch_scratch_bytes(int64_t total, int n_scn, bool lead) {
  return bufs_layout(total, n_scn, lead, nullptr, nullptr);
}

int fill_batch_table(const aeb_scenario* scns, int n_scn, const OutCols* outs, ScnDev* tab,
                     int64_t* total_out, int64_t* cap_out) {
  int64_t total = 0, cap = 1, padded = 0;
  for (int j = 0; j < n_scn; ++j) {
    const int64_t nd = dead_steps(scns[j]), nmax = horizon_steps(scns[j]);
    if (!block_steps_ok(scns[j]))
      return fail(AEB_EINVAL, "horizon plus dead time beyond 2^31 - 4096 steps on the block path");
    tab[j].dt = scns[j].dt;
    tab[j].a_cmd = scns[j].a_cmd;
    tab[j].nd = static_cast<int>(nd);
    tab[j].nmax = static_cast<int>(nmax);
    tab[j].off = total;
    tab[j].poff = padded;
    tab[j].out = outs[j];
    total += scns[j].n_samples;
    padded += (scns[j].n_samples + 63) & ~int64_t(63);
    if (nmax > cap) cap = nmax;
  }
  if (total > 0xffffffffLL) return fail(AEB_EINVAL, "a batch holds at most 2^32 - 1 samples");
  *total_out = total;
  *cap_out = cap;
  return AEB_OK;
}

int launch_batch_fast_into(const aeb_scenario* scns, int n_scn, int precision,
                           const ScnDev* tab, int64_t total, int64_t cap, void* scratch_base,
                           hipStream_t st) {
  const bool lead = scns[0].obstacle == AEB_OBS_LEAD;
  Bufs b;
  bufs_layout(total, n_scn, lead, static_cast<char*>(scratch_base), &b);
  AEB_HIP(hipMemcpyAsync(b.tab, tab, sizeof(ScnDev) * n_scn, hipMemcpyHostToDevice, st));
  AEB_HIP(hipMemcpyAsync(b.scns, scns, sizeof(aeb_scenario) * n_scn, hipMemcpyHostToDevice, st));
  // the prep's index space: each scenario padded to a multiple of 64 samples
  const int64_t padded = tab[n_scn - 1].poff + ((scns[n_scn - 1].n_samples + 63) & ~int64_t(63));
  const unsigned pblk = prep_grid(padded);
  hipLaunchKernelGGL(k_zero, dim3(NBINS / 256), dim3(256), 0, st, b.hist, int64_t(NBINS));
  PrepArgs pa{};
  pa.n = total;
  pa.cap = static_cast<float>(cap);
  pa.scns = b.scns;
  pa.tab = b.tab;
  pa.n_scn = n_scn;
  bool perc = false;
  for (int j = 0; j < n_scn; ++j) perc = perc || perception_on(scns[j]);
  pa.nds = perc ? b.nds : nullptr;
  hipLaunchKernelGGL((k_prep<true, true>), dim3(pblk), dim3(PREP_BLOCK), 0, st, pa, b.jobs,
                     b.leads, b.keys);
  sort_keys(b, total, st);
  Ctx ctx{};
  ctx.impact_exit = scns[0].impact_exit;
  ctx.tab = b.tab;
  ctx.nds = pa.nds;
  return integrate<true>(scns[0], precision, b, total, ctx, nullptr, st);
}

int launch_batch_fast_dev(const aeb_scenario& kind, bool perception, int precision,
                          const BatchHdr* hdr, const ScnDev* tab, const aeb_scenario* scns,
                          int cap_scn, int64_t cap_total, void* scratch_base, hipStream_t st) {
  const bool lead = kind.obstacle == AEB_OBS_LEAD;
  Bufs b;
  bufs_layout(cap_total, 0, lead, static_cast<char*>(scratch_base), &b);
  // the prep's index space for any mix within the capacity (each scenario
  // padded to a multiple of 64 samples)
  const unsigned pblk = prep_grid(cap_total + 63 * static_cast<int64_t>(cap_scn));
  hipLaunchKernelGGL(k_zero, dim3(NBINS / 256), dim3(256), 0, st, b.hist, int64_t(NBINS));
  PrepArgs pa{};
  pa.n = cap_total;
  pa.cap = 1.0f;
  pa.scns = scns;
  pa.tab = tab;
  pa.n_scn = cap_scn;
  pa.nds = perception ? b.nds : nullptr;
  pa.hdr = hdr;
  hipLaunchKernelGGL((k_prep<true, true>), dim3(pblk), dim3(PREP_BLOCK), 0, st, pa, b.jobs,
                     b.leads, b.keys);
  sort_keys(b, cap_total, st, hdr);
  Ctx ctx{};
  ctx.impact_exit = kind.impact_exit;
  ctx.tab = tab;
  ctx.nds = pa.nds;
  ctx.hdr = hdr;
  return integrate<true>(kind, precision, b, cap_total, ctx, nullptr, st);
}

int launch_batch_fast(const aeb_scenario* scns, int n_scn, int precision, const OutCols* outs,
                      hipStream_t st) {
  std::vector<ScnDev> tab(n_scn);
  int64_t total = 0, cap = 1;
  int rc = fill_batch_table(scns, n_scn, outs, tab.data(), &total, &cap);
  if (rc != AEB_OK) return rc;
  const bool lead = scns[0].obstacle == AEB_OBS_LEAD;
  void* base = pool_block(batch_scratch_bytes(total, n_scn, lead), st);
  if (!base) return AEB_ENOMEM;
  rc = launch_batch_fast_into(scns, n_scn, precision, tab.data(), total, cap, base, st);
  if (rc != AEB_OK) return rc;
  // the tables are copied from pageable host memory: keep them valid until
  // the copies have run
  AEB_HIP(hipStreamSynchronize(st));
  return AEB_OK;
}

}  // namespace aeb
