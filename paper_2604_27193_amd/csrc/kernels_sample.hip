// kernels_sample.hip -- device side of the counter-based sampler (Sec. IV-B):
// raw uniforms and parameter columns drawn in a kernel, one sample per lane,
// coalesced SoA stores.
#include <hip/hip_runtime.h>

#include "aeb_common.h"
#include "aeb_runtime.h"

namespace aeb {

__global__ __launch_bounds__(256) void k_uniforms(uint64_t seed, uint64_t sid, int64_t first,
                                                  int64_t count, uint32_t slot, uint32_t attempt,
                                                  double* __restrict__ out) {
  int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= count) return;
  U2 u = uniform2(seed, sid, static_cast<uint64_t>(first + k), slot, attempt);
  reinterpret_cast<double2*>(out)[k] = make_double2(u.a, u.b);
}

__global__ __launch_bounds__(256) void k_sample(aeb_scenario s, int64_t first, int64_t count,
                                                aeb_params p) {
  int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= count) return;
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

int launch_uniforms(uint64_t seed, uint64_t sid, int64_t first, int64_t count, uint32_t slot,
                    uint32_t attempt, double* out, hipStream_t stream) {
  if ((reinterpret_cast<uintptr_t>(out) & 15) != 0)
    return fail(AEB_EINVAL, "aeb_uniforms: device output must be 16-byte aligned");
  int64_t blocks = (count + 255) / 256;
  hipLaunchKernelGGL(k_uniforms, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, seed,
                     sid, first, count, slot, attempt, out);
  AEB_HIP(hipGetLastError());
  return AEB_OK;
}

int launch_sample(const aeb_scenario& s, int64_t first, int64_t count, const aeb_params& out,
                  hipStream_t stream) {
  int64_t blocks = (count + 255) / 256;
  hipLaunchKernelGGL(k_sample, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, stream, s, first,
                     count, out);
  AEB_HIP(hipGetLastError());
  return AEB_OK;
}

}  // namespace aeb
