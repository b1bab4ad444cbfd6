// kernels_fast.hip -- the throughput path of the explicit-Euler rollout for a
// stationary obstacle or none (the configurations of Sec. IV with dead time
// and rolling resistance), FP64 and FP32-compensated.
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
//     the dead-time switch inside the block (guaranteed by per-lane bounds);
//     otherwise single steps with every test.  Inside a block the step takes
//     the cheapest form that gives bit-identical results in the current
//     phase: dead time (a = 0), generic, never-limited (max(a, alim) = a) or
//     friction-limited (max(a, alim) = alim for good, actuator update dead).
//     A crossing of the obstacle inside a block is found afterwards by
//     replaying that block from its saved start state.
#include <hip/hip_runtime.h>

#include "aeb_common.h"
#include "aeb_runtime.h"
#include "fast_path.h"
#include "rollout_steps.h"

namespace aeb {

namespace {

constexpr int NBINS = 8192;  // sort keys: 64 coarse x 2 classes x 64 fine
constexpr int PREP_BLOCK = 1024;
constexpr int PREP_PER = 4;  // samples per thread in prep and scatter

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

template <bool DEVRNG>
__global__ __launch_bounds__(PREP_BLOCK) void k_prep(aeb_scenario s, ParamSrc src, int64_t n,
                                                     int64_t nd, int64_t nmax, Job* jobs,
                                                     uint32_t* keys, uint32_t* ghist) {
  __shared__ uint32_t hist[NBINS];
  for (int j = threadIdx.x; j < NBINS; j += PREP_BLOCK) hist[j] = 0;
  __syncthreads();
  for (int r = 0; r < PREP_PER; ++r) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * (PREP_BLOCK * PREP_PER) +
                      r * PREP_BLOCK + threadIdx.x;
    if (i >= n) break;
    double v0, mu, mass, sg, cg, cda, crr, tau, gap;
    if (DEVRNG) {
      Sample q = draw_sample(s, static_cast<uint64_t>(i));
      v0 = q.v0; mu = q.mu; mass = q.mass; sg = q.sin_grade; cg = q.cos_grade;
      cda = q.cda; crr = q.crr; tau = q.tau; gap = q.gap;
    } else {
      v0 = src.v0[i]; mu = src.mu[i]; mass = src.mass[i]; sg = src.sin_g[i]; cg = src.cos_g[i];
      cda = src.cda[i]; crr = src.crr[i]; tau = src.tau[i]; gap = src.gap[i];
    }
    const Consts k = derive(s, mu, mass, sg, cg, cda, crr);
    Job J;
    J.v0 = v0;
    J.nkd = -k.kd;
    J.c = k.c;
    J.alim = k.alim;
    J.kt = s.dt / tau;
    J.gap = gap;
    // |acc| <= min(|a_cmd|, |alim|) + kd vmax^2 + |c|, with vmax the largest
    // speed the sample can reach (only a downhill pull can raise it)
    const double creach = k.c < 0.0 ? -k.c : 0.0;
    const double vmax = fabs(v0) + s.horizon * creach;
    const double brake = fmin(fabs(s.a_cmd), fabs(k.alim));
    J.dmax = (brake + fabs(k.kd) * vmax * vmax + fabs(k.c)) * 1.0001 + 1e-9;
    // classify and predict
    const bool limited = !(k.alim < s.a_cmd - 1e-6);
    const float t = predict_stop_time(static_cast<float>(v0), static_cast<float>(k.kd),
                                      static_cast<float>(k.c), static_cast<float>(k.alim),
                                      static_cast<float>(tau), static_cast<float>(s.a_cmd),
                                      static_cast<float>(nd) * static_cast<float>(s.dt));
    float steps = t / static_cast<float>(s.dt);
    const float cap = static_cast<float>(nmax);
    if (!(steps < cap)) steps = cap;
    if (!(steps > 0.0f)) steps = 0.0f;
    J.pred = static_cast<double>(steps);
    jobs[i] = J;
    const uint32_t u = static_cast<uint32_t>(steps * (4096.0f / (cap + 1.0f)));
    const uint32_t ud = 4095u - (u > 4095u ? 4095u : u);  // longest first
    const uint32_t key = ((ud >> 6) << 7) | (limited ? 0u : 64u) | (ud & 63u);
    keys[i] = key;
    atomicAdd(&hist[key], 1u);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < NBINS; j += PREP_BLOCK)
    if (hist[j]) atomicAdd(&ghist[j], hist[j]);
}

// exclusive scan of the key histogram into bucket offsets (one block)
__global__ __launch_bounds__(1024) void k_scan(uint32_t* hist) {
  __shared__ uint32_t part[1024];
  constexpr int PER = NBINS / 1024;
  uint32_t loc[PER];
  uint32_t sum = 0;
  for (int j = 0; j < PER; ++j) {
    loc[j] = hist[threadIdx.x * PER + j];
    sum += loc[j];
  }
  part[threadIdx.x] = sum;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
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
__global__ __launch_bounds__(PREP_BLOCK) void k_scatter(const uint32_t* keys, int64_t n,
                                                        uint32_t* offs, uint32_t* perm) {
  __shared__ uint32_t cnt[NBINS];
  for (int j = threadIdx.x; j < NBINS; j += PREP_BLOCK) cnt[j] = 0;
  __syncthreads();
  uint32_t key[PREP_PER], rank[PREP_PER];
  const int64_t base_i = static_cast<int64_t>(blockIdx.x) * (PREP_BLOCK * PREP_PER);
  for (int r = 0; r < PREP_PER; ++r) {
    const int64_t i = base_i + r * PREP_BLOCK + threadIdx.x;
    key[r] = i < n ? keys[i] : 0u;
    rank[r] = i < n ? atomicAdd(&cnt[key[r]], 1u) : 0u;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < NBINS; j += PREP_BLOCK) {
    const uint32_t c = cnt[j];
    cnt[j] = c ? atomicAdd(&offs[j], c) : 0u;
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

template <int FORM, int K>
__device__ inline void block64(St64& s, const Job& J, double dt, double cmd) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const double q = s.v * s.v;
    double acc;
    if (FORM == FORM_G) {
      acc = fma(J.nkd, q, fmax(s.a, J.alim)) - J.c;
      s.a = fma(J.kt, cmd - s.a, s.a);
    } else if (FORM == FORM_F) {
      acc = fma(J.nkd, q, s.a) - J.c;
      s.a = fma(J.kt, cmd - s.a, s.a);
    } else if (FORM == FORM_C) {
      acc = fma(J.nkd, q, J.alim) - J.c;
    } else {  // FORM_D
      acc = fma(J.nkd, q, 0.0) - J.c;
    }
    s.x = fma(dt, s.v, s.x);
    s.v = fma(dt, acc, s.v);
  }
}

__device__ inline void step64(St64& s, const Job& J, double dt, double cmd) {
  const double q = s.v * s.v;
  const double acc = fma(J.nkd, q, fmax(s.a, J.alim)) - J.c;
  s.a = fma(J.kt, cmd - s.a, s.a);
  s.x = fma(dt, s.v, s.x);
  s.v = fma(dt, acc, s.v);
}

template <int OBS, int K>
__global__ __launch_bounds__(256) void k_roll_fp64(const Job* __restrict__ jobs,
                                                   const uint32_t* __restrict__ perm, int64_t n,
                                                   double dt, double a_cmd, int nd, int nmax,
                                                   int impact_exit, OutCols out) {
  const int64_t pos = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const bool valid = pos < n;
  const uint32_t idx = valid ? perm[pos] : 0u;
  Job J;
  if (valid) {
    J = jobs[idx];
  } else {
    J = Job{1.0, 0.0, 0.0, -1.0, 0.5, 1e30, 1.0, 0.0};
  }
  // never limited: a >= a_cmd - (rounding) > alim, so max(a, alim) = a
  const bool lane_free = J.alim < a_cmd - 1e-6;
  // limited for good once a <= alim: a never climbs above max(a, a_cmd) < alim
  const bool lane_limited = J.alim > a_cmd + 1e-9;
  const double thr = static_cast<double>(K) * dt * J.dmax;   // v above this cannot reach 0 in K steps
  St64 s{0.0, J.v0, 0.0};
  bool active = valid, collided = false, pend = false, clamped = false;
  St64 sv{0.0, 0.0, 0.0};
  int sk = 0;
  int end = 0, steps = 0;
  double dist = 0.0;
  float vimp = 0.0f;
  int k = 0;
  // every lane has ended by step nmax (the horizon test fires at k + 1 == nmax)
  while (k < nmax) {
    if (!__any(active)) break;
    const bool near = active && (s.v <= thr);
    const bool straddle = (k < nd) && (k + K > nd);
    const bool horizon = k + K >= nmax;  // a block never ends on the last step
    if (!straddle && !horizon && !__any(near)) {
      const double cmd = k >= nd ? a_cmd : 0.0;
      // keep the start state of a block in which the lane may pass the obstacle
      if (OBS == AEB_OBS_STATIONARY && !collided) {
        sv = s;
        sk = k;
      }
      if (k + K <= nd) {
        block64<FORM_D, K>(s, J, dt, cmd);
      } else if (__all(!active || clamped)) {
        block64<FORM_C, K>(s, J, dt, cmd);
      } else if (__all(!active || lane_free)) {
        block64<FORM_F, K>(s, J, dt, cmd);
      } else {
        block64<FORM_G, K>(s, J, dt, cmd);
        clamped = clamped || (lane_limited && s.a <= J.alim);
      }
      k += K;
      if (OBS == AEB_OBS_STATIONARY && active && !collided && s.x > J.gap) {
        collided = true;
        pend = true;
        if (impact_exit) active = false;
      }
    } else {
      const double cmd = k >= nd ? a_cmd : 0.0;
      if (active) {
        step64(s, J, dt, cmd);
        if (k >= nd) clamped = clamped || (lane_limited && s.a <= J.alim);
        if (OBS == AEB_OBS_STATIONARY && !collided && s.x > J.gap) {
          collided = true;
          vimp = static_cast<float>(s.v);
          if (impact_exit) {
            active = false;
            end = AEB_END_IMPACT;
            steps = k + 1;
            dist = s.x;
          }
        }
        if (active) {
          if (s.v <= 0.0) {
            active = false;
            end = AEB_END_STOP;
            steps = k + 1;
            dist = s.x;
          } else if (k + 1 == nmax) {
            active = false;
            end = AEB_END_HORIZON;
            steps = k + 1;
            dist = s.x;
          }
        }
      }
      k += 1;
    }
  }
  if (active) {  // unreachable: kept so that no lane can leave without a result
    end = AEB_END_HORIZON;
    steps = k;
    dist = s.x;
  }
  // replay the block in which each pending lane passed the obstacle
  if (OBS == AEB_OBS_STATIONARY && __any(pend)) {
    St64 r = sv;
    int kr = sk;
    // the replay is bit-identical to the block, so the crossing recurs within K steps
    for (int it = 0; it <= K; ++it) {
      if (!__any(pend)) break;
      if (pend) {
        const double cmd = kr >= nd ? a_cmd : 0.0;
        step64(r, J, dt, cmd);
        ++kr;
        if (r.x > J.gap) {
          pend = false;
          vimp = static_cast<float>(r.v);
          if (impact_exit) {
            end = AEB_END_IMPACT;
            steps = kr;
            dist = r.x;
          }
        }
      }
    }
  }
  if (pend) vimp = __builtin_nanf("");  // unreachable; makes a broken replay visible
  if (valid) {
    const double mg = J.gap - dist;
    out.dist[idx] = dist;
    out.margin[idx] = mg < J.gap ? mg : J.gap;
    out.steps[idx] = steps;
    out.status[idx] = static_cast<uint8_t>(end | (collided ? AEB_COLLIDED : 0));
    out.vimp[idx] = collided ? vimp : 0.0f;
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
__device__ inline void block32(St32& s, const L32& c) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const float v = speed32<SPLIT>(s);
    const float q = v * v;
    float m;
    if (FORM == FORM_G)
      m = fmaxf(s.e + c.tb, c.alc);
    else if (FORM == FORM_F)
      m = s.e + c.tb;
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
  if (SPLIT) {
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
// wavefront whose lanes are predicted to run longer than this carries it.
constexpr double SPLIT_STEPS = 6000.0;

template <int FORM, int K>
__device__ inline void block32_any(St32& s, const L32& c, bool split) {
  if (split)
    block32<FORM, K, true>(s, c);
  else
    block32<FORM, K, false>(s, c);
}

template <int OBS, int K>
__global__ __launch_bounds__(256) void k_roll_fp32c(const Job* __restrict__ jobs,
                                                    const uint32_t* __restrict__ perm, int64_t n,
                                                    double dt, double a_cmd, int nd, int nmax,
                                                    int impact_exit, double band_abs,
                                                    double band_rel, OutCols out, uint32_t* fix) {
  const int64_t pos = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  const bool valid = pos < n;
  const uint32_t idx = valid ? perm[pos] : 0u;
  Job J;
  if (valid) {
    J = jobs[idx];
  } else {
    J = Job{1.0, 0.0, 0.0, -1.0, 0.5, 1e30, 1.0, 0.0};
  }
  L32 c;  // (the speed read below is base + increment; the increment is 0 without compensation)
  c.dt = static_cast<float>(dt);
  c.nkd = static_cast<float>(J.nkd);
  c.nkt = static_cast<float>(-J.kt);
  c.alc = static_cast<float>(J.alim - J.c);
  c.tb = static_cast<float>(a_cmd - J.c);
  c.td = static_cast<float>(0.0 - J.c);
  c.tdm = fmaxf(c.td, c.alc);
  c.ejump = static_cast<float>(-a_cmd);
  c.thr = static_cast<float>(static_cast<double>(K) * dt * J.dmax);
  c.gapf = static_cast<float>(J.gap);
  const double band = band_abs + band_rel * fabs(J.gap);
  const bool lane_free = J.alim < a_cmd - 1e-6;
  const bool split = __any(valid && J.pred > SPLIT_STEPS);  // wave-uniform
  St32 s;
  s.vb = static_cast<float>(J.v0);
  s.vi = split ? static_cast<float>(J.v0 - static_cast<double>(s.vb)) : 0.0f;
  s.e = 0.0f;
  s.p = 0.0f;
  bool active = valid, crossed = false, clamped = false, boundary = false, pend = false;
  St32 sv = s;  // start state of the block in which the lane passed the obstacle
  int sk = 0;
  int end = 0, steps = 0;
  double dist = 0.0;
  float vimp = 0.0f;
  int k = 0;
  while (k < nmax) {
    if (!__any(active)) break;
    // the command switches on at step nd: e = a - cmd jumps by -a_cmd.  Blocks
    // never straddle nd, so every lane passes through k == nd at a loop top.
    if (k == nd) s.e += c.ejump;
    const bool near = active && (speed32<true>(s) <= c.thr);
    const bool straddle = (k < nd) && (k + K > nd);
    const bool horizon = k + K >= nmax;
    if (!straddle && !horizon && !__any(near)) {
      if (OBS == AEB_OBS_STATIONARY && !crossed) {
        sv = s;
        sk = k;
      }
      if (k + K <= nd) {
        block32_any<FORM_D, K>(s, c, split);
      } else if (__all(!active || clamped)) {
        block32_any<FORM_C, K>(s, c, split);
      } else if (__all(!active || lane_free)) {
        block32_any<FORM_F, K>(s, c, split);
      } else {
        block32_any<FORM_G, K>(s, c, split);
        clamped = clamped || (s.e + c.tb <= c.alc);
      }
      k += K;
      if (OBS == AEB_OBS_STATIONARY && active && !crossed && s.X.hi - s.X.lo > c.gapf) {
        crossed = true;
        pend = true;
        if (impact_exit) active = false;
      }
    } else {
      if (active) {
        const float vb = speed32<true>(s);
        if (split)
          step32<true>(s, c, k >= nd);
        else
          step32<false>(s, c, k >= nd);
        if (k >= nd) clamped = clamped || (s.e + c.tb <= c.alc);
        const float v = speed32<true>(s);
        if (OBS == AEB_OBS_STATIONARY && !crossed && (s.X.hi - s.X.lo) + s.p > c.gapf) {
          crossed = true;
          vimp = v;
          if (impact_exit) {
            active = false;
            end = AEB_END_IMPACT;
            steps = k + 1;
            dist = s.X.value(s.p);
            const double step_len = static_cast<double>(c.dt) * static_cast<double>(vb);
            boundary = (dist - J.gap < band) || (J.gap - (dist - step_len) < band);
          }
        }
        if (active) {
          if (v <= 0.0f) {
            active = false;
            end = AEB_END_STOP;
            steps = k + 1;
            dist = s.X.value(s.p);
          } else if (k + 1 == nmax) {
            active = false;
            end = AEB_END_HORIZON;
            steps = k + 1;
            dist = s.X.value(s.p);
          }
        }
      }
      k += 1;
    }
  }
  if (active) {  // unreachable: kept so that no lane can leave without a result
    end = AEB_END_HORIZON;
    steps = k;
    dist = s.X.value(s.p);
  }
  // replay the block in which each pending lane passed the obstacle, single
  // steps with the per-step test; the crossing recurs within the block (at its
  // last step at the latest, where the block-end test fired)
  if (OBS == AEB_OBS_STATIONARY && __any(pend)) {
    St32 r = sv;
    int kr = sk;
    for (int it = 0; it < K; ++it) {
      if (!__any(pend)) break;
      if (pend) {
        const float vb = speed32<true>(r);
        if (split)
          step32<true>(r, c, kr >= nd);
        else
          step32<false>(r, c, kr >= nd);
        ++kr;
        const float v = speed32<true>(r);
        if ((r.X.hi - r.X.lo) + r.p > c.gapf || it == K - 1) {
          pend = false;
          vimp = v;
          if (impact_exit) {
            end = AEB_END_IMPACT;
            steps = kr;
            dist = r.X.value(r.p);
            const double step_len = static_cast<double>(c.dt) * static_cast<double>(vb);
            boundary = (dist - J.gap < band) || (J.gap - (dist - step_len) < band);
          }
        }
      }
    }
  }
  bool collided = crossed;
  if (OBS == AEB_OBS_STATIONARY && !impact_exit) {
    // the flag is decided in FP64 on the compensated distance
    collided = dist > J.gap;
    boundary = fabs(J.gap - dist) < band;
    if (collided != crossed) vimp = 0.0f;
  } else if (OBS == AEB_OBS_STATIONARY && !crossed) {
    boundary = J.gap - dist < band;
  }
  if (valid) {
    const double mg = J.gap - dist;
    out.dist[idx] = dist;
    out.margin[idx] = mg < J.gap ? mg : J.gap;
    out.steps[idx] = steps;
    out.status[idx] = static_cast<uint8_t>(end | (collided ? AEB_COLLIDED : 0) |
                                           (boundary ? AEB_BOUNDARY : 0));
    out.vimp[idx] = collided ? vimp : 0.0f;
    if (boundary && fix) {
      const uint32_t slot = atomicAdd(fix, 1u);
      fix[1 + slot] = idx;
    }
  }
}

}  // namespace

bool fast_path_applies(const aeb_scenario& s, int precision) {
  if (s.integrator != AEB_EULER || s.obstacle == AEB_OBS_LEAD) return false;
  if (precision == AEB_FP64) return !s.nofma;
  return precision == AEB_FP32C || precision == AEB_FP32C_FIXUP;
}

int launch_rollout_fast(const aeb_scenario& s, const ParamSrc* src, int precision,
                        const OutCols& out, int64_t n, hipStream_t st) {
  (void)precision;
  const int64_t nd = dead_steps(s), nmax = horizon_steps(s);
  if (nmax > 0x7fffffff || nd > 0x7fffffff)
    return fail(AEB_EINVAL, "step counts beyond 2^31");
  // scratch: jobs | keys | perm | histogram
  const size_t off_jobs = 0;
  const size_t off_keys = (off_jobs + sizeof(Job) * n + 255) & ~size_t(255);
  const size_t off_perm = (off_keys + sizeof(uint32_t) * n + 255) & ~size_t(255);
  const size_t off_hist = (off_perm + sizeof(uint32_t) * n + 255) & ~size_t(255);
  const size_t total = off_hist + sizeof(uint32_t) * NBINS;
  char* base = static_cast<char*>(scratch(total, st));
  if (!base) return AEB_ENOMEM;
  Job* jobs = reinterpret_cast<Job*>(base + off_jobs);
  uint32_t* keys = reinterpret_cast<uint32_t*>(base + off_keys);
  uint32_t* perm = reinterpret_cast<uint32_t*>(base + off_perm);
  uint32_t* hist = reinterpret_cast<uint32_t*>(base + off_hist);
  const unsigned nblk = static_cast<unsigned>((n + 255) / 256);
  const unsigned pblk = static_cast<unsigned>((n + PREP_BLOCK * PREP_PER - 1) / (PREP_BLOCK * PREP_PER));
  hipLaunchKernelGGL(k_zero, dim3(NBINS / 256), dim3(256), 0, st, hist, int64_t(NBINS));
  ParamSrc p = src ? *src : ParamSrc{};
  if (src)
    hipLaunchKernelGGL(k_prep<false>, dim3(pblk), dim3(PREP_BLOCK), 0, st, s, p, n, nd, nmax, jobs,
                       keys, hist);
  else
    hipLaunchKernelGGL(k_prep<true>, dim3(pblk), dim3(PREP_BLOCK), 0, st, s, p, n, nd, nmax, jobs,
                       keys, hist);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, hist);
  hipLaunchKernelGGL(k_scatter, dim3(pblk), dim3(PREP_BLOCK), 0, st, keys, n, hist, perm);
  constexpr int K = 32;
  const int ind = static_cast<int>(nd), inmax = static_cast<int>(nmax);
  if (precision != AEB_FP64) {
    uint32_t* fix = nullptr;
    if (precision == AEB_FP32C_FIXUP) {
      fix = static_cast<uint32_t*>(scratch_fix(sizeof(uint32_t) * (n + 1), st));
      if (!fix) return AEB_ENOMEM;
      hipLaunchKernelGGL(k_zero, dim3(1), dim3(64), 0, st, fix, int64_t(1));
    }
    // FP32 errors stay below ~1e-4 m; outcomes within 1 mm (+1e-5 of the gap)
    // of the boundary are flagged (and, in the fix-up mode, recomputed in FP64)
    const double band_abs = 1e-3, band_rel = 1e-5;
    timing_begin(st);
    if (s.obstacle == AEB_OBS_STATIONARY)
      hipLaunchKernelGGL((k_roll_fp32c<AEB_OBS_STATIONARY, K>), dim3(nblk), dim3(256), 0, st, jobs,
                         perm, n, s.dt, s.a_cmd, ind, inmax, s.impact_exit, band_abs, band_rel, out,
                         fix);
    else
      hipLaunchKernelGGL((k_roll_fp32c<AEB_OBS_NONE, K>), dim3(nblk), dim3(256), 0, st, jobs, perm,
                         n, s.dt, s.a_cmd, ind, inmax, s.impact_exit, band_abs, band_rel, out, fix);
    timing_end(st);
    if (fix) {
      int rc = launch_fixup(s, src, out, fix, st);
      if (rc != AEB_OK) return rc;
    }
    AEB_HIP(hipGetLastError());
    return AEB_OK;
  }
  timing_begin(st);
  if (s.obstacle == AEB_OBS_STATIONARY)
    hipLaunchKernelGGL((k_roll_fp64<AEB_OBS_STATIONARY, K>), dim3(nblk), dim3(256), 0, st, jobs,
                       perm, n, s.dt, s.a_cmd, ind, inmax, s.impact_exit, out);
  else
    hipLaunchKernelGGL((k_roll_fp64<AEB_OBS_NONE, K>), dim3(nblk), dim3(256), 0, st, jobs, perm, n,
                       s.dt, s.a_cmd, ind, inmax, s.impact_exit, out);
  timing_end(st);
  AEB_HIP(hipGetLastError());
  return AEB_OK;
}

}  // namespace aeb
