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

// Device scratch of one library call.  Each ABI entry point that enqueues
// work on scratch opens a ScratchScope on its stream; scratch_slot() inside
// it hands out blocks of a per-device pool that no other live scope holds.
// When the scope ends, an event recorded on the stream fences each block, so
// a later call on another stream reuses it only after that work (or waits
// for it on the device), and a block is freed to grow it only after its
// event has completed.  Calls on different streams or threads therefore
// never share scratch that is in flight.  A call holds one block per slot
// (slot 0: the rollout's job records, sort buffers and fix-up list, or the
// reduction's partials).  Returns nullptr (with the error set) if the
// allocation fails, outside a scope, or on a stream that is being captured
// into a graph.
class ScratchScope {
 public:
  static constexpr int SLOTS = 1;
  explicit ScratchScope(hipStream_t st);
  ~ScratchScope();
  ScratchScope(const ScratchScope&) = delete;
  ScratchScope& operator=(const ScratchScope&) = delete;

 private:
  friend void* scratch_slot(int slot, size_t bytes, hipStream_t stream);
  hipStream_t st_;
  int dev_ = -1;
  ScratchScope* outer_;
  void* held_[SLOTS] = {nullptr};
};
void* scratch_slot(int slot, size_t bytes, hipStream_t stream);
inline void* pool_block(size_t bytes, hipStream_t stream) { return scratch_slot(0, bytes, stream); }

// events around the integration kernel (aeb_timing_enable)
void timing_begin(hipStream_t stream);
// the lane counters the next timed integration kernel accumulates into (null
// when timing is off)
unsigned long long* timing_lanes();
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
// Largest errors of the controller screen's single-precision approximations
// over their whole input ranges (measured[4]) and the bounds the screen
// assumes for them (bounds[4]): log2, sqrt, sin, cos.  Synchronises `st`.
int launch_valu_probe(int fp32, int64_t threads, int iters, void* out, hipStream_t st);
int launch_ctl_math(const double* a, const double* x, int64_t n, double* la, double* sx,
                    double* cx, hipStream_t st);
int launch_approx_check(double* measured, double* bounds, hipStream_t st);

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
// statistics of nseg output sets (segmented launches on one pool block; waits)
int launch_batch_reduce(const OutCols* outs, const int64_t* ns, int nseg,
                        const aeb_reduce_req& req, aeb_stats* host_out, hipStream_t stream);

// The reduction in two parts on caller-provided scratch (reduce_scratch_bytes):
// reduce_enqueue queues the kernels and the copy of the statistics into
// host_out (pinned memory keeps it asynchronous); once the stream has run
// them, a non-zero host_out->reserved asks for reduce_fallback (synchronous),
// which recomputes the order statistics by radix select into the set's
// device statistics `dstats` and copies them to host_out.  reduce_enqueue
// keeps the statistics at the start of the scratch (dstats = scratch).
size_t reduce_scratch_bytes(int64_t n, const aeb_reduce_req& req);
// a bound on the sum of reduce_scratch_bytes (each rounded up to 256 bytes)
// over any cap_sets sets of cap_samples samples in all
size_t reduce_scratch_bytes_cap(int cap_sets, int64_t cap_samples, const aeb_reduce_req& req);
int reduce_enqueue(const OutCols& out, int64_t n, const aeb_reduce_req& req, void* scratch_base,
                   aeb_stats* host_out, hipStream_t stream);
int reduce_fallback(const OutCols& out, int64_t n, const aeb_reduce_req& req, void* scratch_base,
                    aeb_stats* dstats, aeb_stats* host_out, hipStream_t stream);
// reduce_fallback calls since the library was loaded
unsigned long long reduce_fallback_count();

// The reduction of nseg output sets as one launch sequence (every kernel of
// it covers all sets): set j has its own scratch at bases[j]
// (reduce_scratch_bytes(ns[j])); `table_dev` (device) and `table_host` (host,
// pinned for an asynchronous call, unchanged until the stream has copied it)
// hold reduce_table_bytes(nseg, ns) bytes: the set table, copied to the
// device by the call, and the sets' device statistics, at
// reduce_table_stats(table_dev, nseg, ns) + j, copied to host_out[j].  The
// fallback of set j then takes that device statistics pointer.
size_t reduce_table_bytes(int nseg, const int64_t* ns);
aeb_stats* reduce_table_stats(void* table_dev, int nseg, const int64_t* ns);
int reduce_enqueue_sets(const OutCols* outs, const int64_t* ns, int nseg,
                        const aeb_reduce_req& req, char* const* bases, void* table_dev,
                        void* table_host, aeb_stats* host_out, hipStream_t stream);

// The same launch sequence laid out for a capacity -- up to cap_sets sets of
// cap_samples samples in all -- so that one recording serves any such mix:
// reduce_fill_sets_cap writes a mix into the host table (before each replay),
// reduce_enqueue_sets_cap queues the table copy, kernels whose grids cover
// the capacity (blocks past the mix return at once) and the copy of
// cap_sets statistics to host_out (the first nseg are the mix's).  The
// table needs reduce_table_bytes_cap bytes on both sides; the statistics of
// set j on the device are reduce_table_stats_cap(table_dev, ...) + j.
size_t reduce_table_bytes_cap(int cap_sets, int64_t cap_samples);
aeb_stats* reduce_table_stats_cap(void* table_dev, int cap_sets, int64_t cap_samples);
int reduce_fill_sets_cap(const OutCols* outs, const int64_t* ns, int nseg, int cap_sets,
                         int64_t cap_samples, char* const* bases, void* table_dev,
                         void* table_host);
int reduce_enqueue_sets_cap(int cap_sets, int64_t cap_samples, const aeb_reduce_req& req,
                            bool weighted, void* table_dev, const void* table_host,
                            aeb_stats* host_out, hipStream_t stream);
int check_reduce_req(const aeb_reduce_req& req);

// Argument checks of aeb_rollout (scenario, precision, column lengths) and the
// kernel view of the parameter columns (all null for the in-kernel generator).
int rollout_args(const aeb_scenario* scn, const aeb_params* params, int precision,
                 const aeb_outputs* out, ParamSrc* src);

}  // namespace aeb
