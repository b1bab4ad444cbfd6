// aeb_runtime.h -- internal declarations of the library: error reporting,
// the per-device scratch arena, scenario validation and the kernel launchers
// that the C ABI (abi.cpp) calls.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "aeb.h"
#include "aeb_common.h"

namespace aeb {

// thread-local message behind aeb_last_error()
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);

#define AEB_HIP(call)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return ::aeb::fail(AEB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

// Grow-only device scratch, per device and slot; never shrinks before exit.
// Returns nullptr (with the error set) if the allocation fails.  Slot 0 holds
// the rollout's job records and sort buffers and the reduction's partials;
// slot 1 the FP32 fix-up list, which lives alongside slot 0.
void* scratch_slot(int slot, size_t bytes, hipStream_t stream);
inline void* scratch(size_t bytes, hipStream_t stream) { return scratch_slot(0, bytes, stream); }
inline void* scratch_fix(size_t bytes, hipStream_t stream) { return scratch_slot(1, bytes, stream); }

// events around the integration kernel (aeb_timing_enable)
void timing_begin(hipStream_t stream);
void timing_end(hipStream_t stream);
// switch the hooks off on this thread (returns the previous state) / back on
bool timing_suspend(bool off);
void timing_resume(bool was);

int validate(const aeb_scenario& s);

// llround(horizon/dt), llround(dead_time/dt)
int64_t horizon_steps(const aeb_scenario& s);
int64_t dead_steps(const aeb_scenario& s);

// Kernel-side view of the parameter source: device columns or the generator.
struct ParamSrc {
  const double *v0, *mu, *mass, *sin_g, *cos_g, *cda, *crr, *tau, *gap, *lead;
  const double* trig;  // perception delay; null reads as 0
  const double* logw;  // importance-sampling log likelihood ratio; null reads as 0
};

struct OutCols {
  double* dist;
  uint8_t* status;
  int32_t* steps;
  double* margin;
  float* vimp;
  double* weight;  // optional importance-sampling weights (null: not written)
};

// launchers (kernels_*.hip); all asynchronous on `stream`
int launch_uniforms(uint64_t seed, uint64_t sid, int64_t first, int64_t count, uint32_t slot,
                    uint32_t attempt, double* out, hipStream_t stream);
int launch_sample(const aeb_scenario& s, int64_t first, int64_t count, const aeb_params& out,
                  hipStream_t stream);
int launch_rollout(const aeb_scenario& s, const ParamSrc* src, int precision, const OutCols& out,
                   int64_t n, hipStream_t stream);
int launch_batch(const aeb_scenario* scns, int n_scn, int precision, const OutCols* outs,
                 hipStream_t stream);
int launch_fixup(const aeb_scenario& s, const ParamSrc* src, const OutCols& out,
                 const uint32_t* fix, hipStream_t stream);
int launch_reduce(const OutCols& out, int64_t n, const aeb_reduce_req& req, aeb_stats* host_out,
                  hipStream_t stream);

// The reduction in two parts on caller-provided scratch (reduce_scratch_bytes):
// reduce_enqueue queues the kernels and the copy of the statistics into
// host_out (pinned memory keeps it asynchronous); once the stream has run
// them, a non-zero host_out->reserved asks for reduce_fallback (synchronous),
// which recomputes the order statistics by radix select.
size_t reduce_scratch_bytes(int64_t n, const aeb_reduce_req& req);
int reduce_enqueue(const OutCols& out, int64_t n, const aeb_reduce_req& req, void* scratch_base,
                   aeb_stats* host_out, hipStream_t stream);
int reduce_fallback(const OutCols& out, int64_t n, const aeb_reduce_req& req, void* scratch_base,
                    aeb_stats* host_out, hipStream_t stream);
int check_reduce_req(const aeb_reduce_req& req);

}  // namespace aeb
