// approx_check.hip -- self-checks of the controller's decision arithmetic.
// Measures, on the device, the largest errors of the
// single-precision hardware approximations the controller's decision screen
// uses (rollout_steps.h, ctl_fast), over every input that can reach them:
//   log2:  v_log_f32(a) against log2(a), relative to max(1, |log2 a|), for
//          every float a in [2^-53, 1] (the uniforms' range, rounded);
//   sqrt:  v_sqrt_f32(x) against sqrt(x), relative, for every float x in
//          [2^-24, 80] (the squared radius; below 2^-24 only 0 occurs);
//   sin, cos: v_sin_f32(b), v_cos_f32(b) against sin(2 pi b), cos(2 pi b),
//          absolute, for every float b in [2^-53, 1].
// References in double precision (log2, sqrt, sinpi and cospi of 2b: no
// rounded multiple of pi).  One thread per input, grid-stride; the maxima of
// non-negative doubles are kept as their bit patterns (which order the same).
// Also evaluates the exact stage's own log, sine and cosine at given
// arguments, so that a test can hold the device's results against the host's,
// and runs a kernel of known instruction counts for checking the VALU
// counters' accounting.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "aeb_runtime.h"
#include "rollout_steps.h"

namespace aeb {
namespace {

constexpr uint32_t LO_U = 0x25000000u;    // 2^-53
constexpr uint32_t HI_U = 0x3F800000u;    // 1.0
constexpr uint32_t LO_S = 0x33800000u;    // 2^-24
constexpr uint32_t HI_S = 0x42A00000u;    // 80.0

__device__ inline double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

__device__ inline void block_max(double v, unsigned long long* out) {
  __shared__ double part[4];
  v = wave_max(v);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = part[0];
    for (int w = 1; w < 4; ++w) m = fmax(m, part[w]);
    atomicMax(out, static_cast<unsigned long long>(__double_as_longlong(m)));
  }
}

__global__ __launch_bounds__(256) void k_check_uniform_range(unsigned long long* out) {
  double el = 0.0, es = 0.0, ec = 0.0;
  const uint32_t count = HI_U - LO_U + 1;
  for (uint32_t k = blockIdx.x * 256u + threadIdx.x; k < count; k += gridDim.x * 256u) {
    const float x = __uint_as_float(LO_U + k);
    const double xd = x;
    const double l = log2(xd);
    const double e = fabs(static_cast<double>(__builtin_amdgcn_logf(x)) - l) / fmax(1.0, fabs(l));
    el = fmax(el, e);
    es = fmax(es, fabs(static_cast<double>(__builtin_amdgcn_sinf(x)) - sinpi(2.0 * xd)));
    ec = fmax(ec, fabs(static_cast<double>(__builtin_amdgcn_cosf(x)) - cospi(2.0 * xd)));
  }
  block_max(el, out + 0);
  block_max(es, out + 2);
  block_max(ec, out + 3);
}

__global__ __launch_bounds__(256) void k_check_sqrt(unsigned long long* out) {
  double er = 0.0;
  const uint32_t count = HI_S - LO_S + 1;
  for (uint32_t k = blockIdx.x * 256u + threadIdx.x; k < count; k += gridDim.x * 256u) {
    const float x = __uint_as_float(LO_S + k);
    const double r = sqrt(static_cast<double>(x));
    er = fmax(er, fabs(static_cast<double>(__builtin_amdgcn_sqrtf(x)) - r) / r);
  }
  // sqrt(0) is 0 exactly or the error is unbounded
  if (blockIdx.x == 0 && threadIdx.x == 0 && __builtin_amdgcn_sqrtf(0.0f) != 0.0f) er = INFINITY;
  block_max(er, out + 1);
}

// the exact stage's log, sine and cosine at given arguments (ctl_math.h)
__global__ __launch_bounds__(256) void k_ctl_math(const double* a, const double* x, int64_t n,
                                                  double* la, double* sx, double* cx) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (i >= n) return;
  la[i] = ctl_log(a[i]);
  ctl_sincos(x[i], &sx[i], &cx[i]);
}

// Counter check: a kernel of known instruction counts, to verify how the
// VALU counters account fused multiply-adds, adds and multiplies before they
// are used on the rollout kernels.  Every lane runs `iters` rounds of CH
// independent fused multiply-adds, then adds its CH values up (CH - 1 adds);
// its initial values are integer conversions, no floating-point arithmetic.
constexpr int PROBE_CH = 8;

template <typename T>
__global__ __launch_bounds__(256) void k_valu_probe(T* out, int iters, T a, T b) {
  T x[PROBE_CH];
#pragma unroll
  for (int c = 0; c < PROBE_CH; ++c) x[c] = static_cast<T>(static_cast<int>(threadIdx.x) + c);
  for (int i = 0; i < iters; ++i) {
#pragma unroll
    for (int c = 0; c < PROBE_CH; ++c) x[c] = fma(x[c], a, b);
  }
  T s = x[0];
#pragma unroll
  for (int c = 1; c < PROBE_CH; ++c) s = s + x[c];
  out[static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x] = s;
}

}  // namespace

int launch_valu_probe(int fp32, int64_t threads, int iters, void* out, hipStream_t st) {
  const dim3 grid(static_cast<unsigned>(threads / 256));
  if (fp32)
    hipLaunchKernelGGL(k_valu_probe<float>, grid, dim3(256), 0, st, static_cast<float*>(out),
                       iters, 0.999f, 1e-3f);
  else
    hipLaunchKernelGGL(k_valu_probe<double>, grid, dim3(256), 0, st, static_cast<double*>(out),
                       iters, 0.999, 1e-3);
  AEB_HIP(hipGetLastError());
  return AEB_OK;
}

int launch_ctl_math(const double* a, const double* x, int64_t n, double* la, double* sx,
                    double* cx, hipStream_t st) {
  if (n > 0)
    hipLaunchKernelGGL(k_ctl_math, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, st,
                       a, x, n, la, sx, cx);
  AEB_HIP(hipGetLastError());
  return AEB_OK;
}

int launch_approx_check(double* measured, double* bounds, hipStream_t st) {
  unsigned long long* d = nullptr;
  AEB_HIP(hipMalloc(&d, 4 * sizeof(unsigned long long)));
  int rc = AEB_OK;
  unsigned long long h[4] = {0, 0, 0, 0};
  if (hipMemsetAsync(d, 0, sizeof(h), st) != hipSuccess) rc = AEB_EDEVICE;
  if (rc == AEB_OK) {
    hipLaunchKernelGGL(k_check_uniform_range, dim3(4096), dim3(256), 0, st, d);
    hipLaunchKernelGGL(k_check_sqrt, dim3(4096), dim3(256), 0, st, d);
    if (hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(h, d, sizeof(h), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      rc = AEB_EDEVICE;
  }
  (void)hipFree(d);
  if (rc != AEB_OK) return fail(rc, "aeb_ctl_approx_check: a HIP call failed");
  std::memcpy(measured, h, sizeof(h));
  bounds[0] = CTL_EL;
  bounds[1] = CTL_ES;
  bounds[2] = CTL_ET;
  bounds[3] = CTL_ET;
  return AEB_OK;
}

}  // namespace aeb
