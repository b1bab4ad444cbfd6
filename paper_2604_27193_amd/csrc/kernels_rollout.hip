// kernels_rollout.hip -- the Monte Carlo rollout (Sec. V): one sample per
// lane, parameters loaded from SoA columns (coalesced) or drawn in registers
// from the counter generator, outputs stored SoA.
#include <hip/hip_runtime.h>

#include "aeb_common.h"
#include "aeb_runtime.h"
#include "fast_path.h"
#include "rollout_steps.h"

namespace aeb {

// sample i's parameters from the columns or the generator
template <bool DEVRNG>
__device__ inline Lane load_lane(const aeb_scenario& s, const ParamSrc& src, int64_t i) {
  Lane L;
  double mu, mass, sg, cg, cda, crr;
  if (DEVRNG) {
    Sample q = draw_sample(s, static_cast<uint64_t>(i));
    L.v0 = q.v0;
    mu = q.mu;
    mass = q.mass;
    sg = q.sin_grade;
    cg = q.cos_grade;
    cda = q.cda;
    crr = q.crr;
    L.tau = q.tau;
    L.gap = q.gap;
    L.lead = q.lead_decel;
    L.trig = q.trigger;
    L.log_w = q.log_w;
  } else {
    L.v0 = src.v0[i];
    mu = src.mu[i];
    mass = src.mass[i];
    sg = src.sin_g[i];
    cg = src.cos_g[i];
    cda = src.cda[i];
    crr = src.crr[i];
    L.tau = src.tau[i];
    L.gap = src.gap[i];
    L.lead = src.lead[i];
    L.trig = src.trig ? src.trig[i] : 0.0;
    L.log_w = src.logw ? src.logw[i] : 0.0;
  }
  L.k = derive(s, mu, mass, sg, cg, cda, crr);
  L.index = static_cast<uint64_t>(i);
  return L;
}

__device__ inline void store(const OutCols& o, int64_t i, const Result& r) {
  o.dist[i] = r.dist;
  o.margin[i] = r.margin;
  o.steps[i] = r.steps;
  o.status[i] = r.status;
  o.vimp[i] = r.vimp;
}

template <int INTEG, int OBS, bool NOFMA, bool DEVRNG, bool CTL>
__global__ __launch_bounds__(256) void k_rollout_fp64(aeb_scenario s, ParamSrc src, OutCols out,
                                                      int64_t n, int64_t nd, int64_t nmax,
                                                      CtlArgs ca) {
  int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Lane L = load_lane<DEVRNG>(s, src, i);
  // with perception the command step is the sample's own
  if (perception_on(s)) nd = command_step(s, L.trig, nmax);
  Result r = (INTEG == AEB_EULER)
                 ? euler_fp64<OBS, NOFMA, CTL>(L, s.dt, s.a_cmd, nd, nmax, s.impact_exit, &ca)
                 : rk4_fp64<OBS, CTL>(L, s.dt, s.a_cmd, nd, nmax, s.impact_exit, &ca);
  store(out, i, r);
  if (out.weight) out.weight[i] = exp(L.log_w);
}

// FP64 recomputation of the samples listed in fix[1 .. fix[0]]; clears the
// boundary bit
template <int OBS, bool DEVRNG>
__global__ __launch_bounds__(256) void k_fixup_fp64(aeb_scenario s, ParamSrc src, OutCols out,
                                                    int64_t nd, int64_t nmax, const uint32_t* fix) {
  const uint32_t cnt = fix[0];
  for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < cnt; j += gridDim.x * blockDim.x) {
    int64_t i = fix[1 + j];
    Lane L = load_lane<DEVRNG>(s, src, i);
    const int64_t ndl = perception_on(s) ? command_step(s, L.trig, nmax) : nd;
    Result r = s.nofma ? euler_fp64<OBS, true>(L, s.dt, s.a_cmd, ndl, nmax, s.impact_exit)
                       : euler_fp64<OBS, false>(L, s.dt, s.a_cmd, ndl, nmax, s.impact_exit);
    store(out, i, r);
  }
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <int INTEG, int OBS, bool NOFMA, bool CTL = false>
static void go_fp64(const aeb_scenario& s, const ParamSrc* src, const OutCols& out, int64_t n,
                    int64_t nd, int64_t nmax, hipStream_t st) {
  dim3 grid(static_cast<unsigned>((n + 255) / 256)), block(256);
  ParamSrc p = src ? *src : ParamSrc{};
  const CtlArgs ca = ctl_args(s);
  if (src)
    hipLaunchKernelGGL((k_rollout_fp64<INTEG, OBS, NOFMA, false, CTL>), grid, block, 0, st, s, p,
                       out, n, nd, nmax, ca);
  else
    hipLaunchKernelGGL((k_rollout_fp64<INTEG, OBS, NOFMA, true, CTL>), grid, block, 0, st, s, p,
                       out, n, nd, nmax, ca);
}

// the closed-loop controller outside the block path (horizons beyond its step
// limit): FP64, one checked lane per sample
static int go_control(const aeb_scenario& s, const ParamSrc* src, int precision,
                      const OutCols& out, int64_t n, int64_t nd, int64_t nmax, hipStream_t st) {
  if (precision != AEB_FP64)
    return fail(AEB_EINVAL, "the closed-loop controller runs in FP64 only");
  timing_begin(st);
  if (s.integrator == AEB_RK4)
    go_fp64<AEB_RK4, AEB_OBS_STATIONARY, false, true>(s, src, out, n, nd, nmax, st);
  else if (s.obstacle == AEB_OBS_LEAD)
    s.nofma ? go_fp64<AEB_EULER, AEB_OBS_LEAD, true, true>(s, src, out, n, nd, nmax, st)
            : go_fp64<AEB_EULER, AEB_OBS_LEAD, false, true>(s, src, out, n, nd, nmax, st);
  else
    s.nofma ? go_fp64<AEB_EULER, AEB_OBS_STATIONARY, true, true>(s, src, out, n, nd, nmax, st)
            : go_fp64<AEB_EULER, AEB_OBS_STATIONARY, false, true>(s, src, out, n, nd, nmax, st);
  timing_end(st);
  AEB_HIP(hipGetLastError());
  return AEB_OK;
}

template <int OBS>
static void go_fixup(const aeb_scenario& s, const ParamSrc* src, const OutCols& out,
                     const uint32_t* fix, hipStream_t st) {
  const int64_t nd = dead_steps(s), nmax = horizon_steps(s);
  ParamSrc p = src ? *src : ParamSrc{};
  if (src)
    hipLaunchKernelGGL((k_fixup_fp64<OBS, false>), dim3(64), dim3(256), 0, st, s, p, out, nd, nmax,
                       fix);
  else
    hipLaunchKernelGGL((k_fixup_fp64<OBS, true>), dim3(64), dim3(256), 0, st, s, p, out, nd, nmax,
                       fix);
}

int launch_fixup(const aeb_scenario& s, const ParamSrc* src, const OutCols& out,
                 const uint32_t* fix, hipStream_t st) {
  switch (s.obstacle) {
    case AEB_OBS_NONE: go_fixup<AEB_OBS_NONE>(s, src, out, fix, st); break;
    case AEB_OBS_STATIONARY: go_fixup<AEB_OBS_STATIONARY>(s, src, out, fix, st); break;
    default: go_fixup<AEB_OBS_LEAD>(s, src, out, fix, st); break;
  }
  AEB_HIP(hipGetLastError());
  return AEB_OK;
}

// Batches the batched block-structured launch cannot take (the unfused Euler
// form, the closed-loop controller, the fix-up mode) run scenario by scenario.
int launch_batch(const aeb_scenario* scns, int n_scn, int precision, const OutCols* outs,
                 hipStream_t st) {
  bool fast = precision != AEB_FP32C_FIXUP;
  for (int j = 0; j < n_scn && fast; ++j)
    fast = fast_path_applies(scns[j], precision) && !control_on(scns[j]);
  if (fast) return launch_batch_fast(scns, n_scn, precision, outs, st);
  for (int j = 0; j < n_scn; ++j) {
    const int rc = launch_rollout(scns[j], nullptr, precision, outs[j], scns[j].n_samples, st);
    if (rc != AEB_OK) return rc;
  }
  return AEB_OK;
}

int launch_rollout(const aeb_scenario& s, const ParamSrc* src, int precision, const OutCols& out,
                   int64_t n, hipStream_t st) {
  const int64_t nd = dead_steps(s), nmax = horizon_steps(s);
  if (fast_path_applies(s, precision)) return launch_rollout_fast(s, src, precision, out, n, st);
  if (control_on(s)) return go_control(s, src, precision, out, n, nd, nmax, st);
  if (precision == AEB_FP32C || precision == AEB_FP32C_FIXUP) {
    // every Euler case within the block path's step limit takes it
    return fail(AEB_EINVAL,
                "the FP32 compensated form needs the explicit Euler integrator and a horizon "
                "plus dead time below 2^31 - 4096 steps");
  } else if (s.integrator == AEB_RK4) {
    timing_begin(st);
    if (s.obstacle == AEB_OBS_NONE)
      go_fp64<AEB_RK4, AEB_OBS_NONE, false>(s, src, out, n, nd, nmax, st);
    else
      go_fp64<AEB_RK4, AEB_OBS_STATIONARY, false>(s, src, out, n, nd, nmax, st);
    timing_end(st);
  } else if (s.nofma) {
    timing_begin(st);
    switch (s.obstacle) {
      case AEB_OBS_NONE: go_fp64<AEB_EULER, AEB_OBS_NONE, true>(s, src, out, n, nd, nmax, st); break;
      case AEB_OBS_STATIONARY: go_fp64<AEB_EULER, AEB_OBS_STATIONARY, true>(s, src, out, n, nd, nmax, st); break;
      default: go_fp64<AEB_EULER, AEB_OBS_LEAD, true>(s, src, out, n, nd, nmax, st); break;
    }
    timing_end(st);
  } else {
    timing_begin(st);
    switch (s.obstacle) {
      case AEB_OBS_NONE: go_fp64<AEB_EULER, AEB_OBS_NONE, false>(s, src, out, n, nd, nmax, st); break;
      case AEB_OBS_STATIONARY: go_fp64<AEB_EULER, AEB_OBS_STATIONARY, false>(s, src, out, n, nd, nmax, st); break;
      default: go_fp64<AEB_EULER, AEB_OBS_LEAD, false>(s, src, out, n, nd, nmax, st); break;
    }
    timing_end(st);
  }
  AEB_HIP(hipGetLastError());
  return AEB_OK;
}

}  // namespace aeb
