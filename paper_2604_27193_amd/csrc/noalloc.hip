// noalloc.hip -- aeb_rollout_noalloc: the rollout of aeb_rollout on a fixed,
// library-owned device scratch array instead of the growable pool, for
// callers that cannot allocate device memory while they run.
//
// The scratch (job records, sort keys and permutation, per-sample command
// steps, the FP32 fix-up list, the length histogram and the claim counter of
// the sorted block-structured path) lives in one file-scope device array.
// Host code never passes the array's name to a kernel: at a device's first
// call the entry point looks up the array's device address with
// hipGetSymbolAddress, with that device current, and keeps it per device.
// Every call on a device shares that device's array; the kernels clear what
// must start at zero (histogram, counter, fix-up count) with fill kernels, so
// no call depends on what the previous one left.  Calls that overlap on one
// device race on the array.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "aeb.h"
#include "aeb_runtime.h"
#include "fast_path.h"

namespace {

static __device__ __align__(256) unsigned char scratch[AEB_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEV = 64;
std::mutex g_mu;
void* g_ptr[MAX_DEV] = {nullptr};

// device address of this device's array (looked up once per device)
int scratch_ptr(void** out) {
  int dev = -1;
  AEB_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEV)
    return aeb::fail(AEB_EDEVICE, "aeb_rollout_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    AEB_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return aeb::fail(AEB_EDEVICE, "aeb_rollout_noalloc: scratch symbol has no address");
    g_ptr[dev] = p;
  }
  *out = g_ptr[dev];
  return AEB_OK;
}

}  // namespace

extern "C" int aeb_rollout_noalloc(const aeb_scenario* scn, const aeb_params* params,
                                   int precision, const aeb_outputs* out, void* stream) {
  using namespace aeb;
  ParamSrc src{};
  int rc = rollout_args(scn, params, precision, out, &src);
  if (rc != AEB_OK) return rc;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  OutCols oc{out->dist, out->status, out->steps, out->margin, out->v_impact, out->weight};
  const ParamSrc* ps = params ? &src : nullptr;
  if (!fast_path_applies(*scn, precision)) {
    // the checked kernels (horizons beyond the block path, or a controller
    // outside it) use no scratch
    return launch_rollout(*scn, ps, precision, oc, scn->n_samples, st);
  }
  const size_t need = rollout_scratch_bytes(*scn, scn->n_samples);
  if (need > static_cast<size_t>(AEB_NOALLOC_SCRATCH_BYTES))
    return fail(AEB_ENOMEM, "aeb_rollout_noalloc: " + std::to_string(scn->n_samples) +
                                " samples need " + std::to_string(need) +
                                " bytes of scratch, more than the fixed " +
                                std::to_string(static_cast<long long>(AEB_NOALLOC_SCRATCH_BYTES)) +
                                "-byte array; use aeb_rollout");
  void* base = nullptr;
  rc = scratch_ptr(&base);
  if (rc != AEB_OK) return rc;
  // the timing hooks (aeb_timing_enable) would create events and a counter
  // buffer on first use: off inside this call
  const bool was = timing_suspend(true);
  rc = launch_rollout_fast_into(*scn, ps, precision, oc, scn->n_samples, base, st);
  timing_resume(was);
  return rc;
}
