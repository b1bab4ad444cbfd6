// fast_path.h -- job records and entry points of the sorted, block-structured
// explicit-Euler rollout (kernels_fast.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "aeb.h"
#include "aeb_runtime.h"

namespace aeb {

// Per-sample record written by the prep stage (64 bytes: one half cache line).
struct Job {
  double v0;      // initial speed
  double nkd;     // -kd
  double c;       // grade plus rolling resistance
  double alim;    // friction limit (negative)
  double kt;      // dt / tau (explicit Euler) or 1 / tau (RK4)
  double gap;     // initial gap to the obstacle
  double dmax;    // bound on |dv/dt| over the whole rollout
  float pred;     // predicted number of steps
  uint32_t scn;   // scenario of the sample in a batched launch
};

// Lead-vehicle data of a sample (lead-vehicle scenarios only).
struct LeadJob {
  double decel;   // lead deceleration
};

// Sizes of a batched launch on device tables (a recorded mix reads them here).
struct BatchHdr {
  long long total;  // samples
  float cap;        // largest step count of the mix's scenarios (sort-key scale)
  int n_scn;        // scenarios
};

// Per-scenario constants of a batched launch.
struct ScnDev {
  double dt, a_cmd;
  int nd, nmax;
  long long off;   // first global sample index of the scenario
  long long poff;  // its first index in the batched prep's index space, where
                   // every scenario starts on a multiple of 64 (one scenario
                   // per wavefront)
  OutCols out;
};

enum { FORM_G = 0, FORM_F = 1, FORM_C = 2, FORM_D = 3 };

// horizon plus dead time, in steps, that the block path accepts
constexpr int64_t BLOCK_STEP_MAX = 0x7fffffffLL - 4096;
bool block_steps_ok(const aeb_scenario& s);
bool fast_path_applies(const aeb_scenario& s, int precision);
int launch_rollout_fast(const aeb_scenario& s, const ParamSrc* src, int precision,
                        const OutCols& out, int64_t n, hipStream_t st);
// the same on caller-provided device scratch of rollout_scratch_bytes(s, n)
// bytes (precision AEB_FP64 or AEB_FP32C)
size_t rollout_scratch_bytes(const aeb_scenario& s, int64_t n);
int launch_rollout_fast_into(const aeb_scenario& s, const ParamSrc* src, int precision,
                             const OutCols& out, int64_t n, void* scratch_base, hipStream_t st);
// all samples of several scenarios in one sorted launch (parameters drawn in-kernel)
int launch_batch_fast(const aeb_scenario* scns, int n_scn, int precision, const OutCols* outs,
                      hipStream_t st);

// The same launch on caller-provided device scratch (batch_scratch_bytes) with
// the scenario table already filled (fill_batch_table).  `scns` and `tab` are
// copied to the device asynchronously: they must stay valid until the stream
// has run the copies (pinned host memory lets the caller keep going).
size_t batch_scratch_bytes(int64_t total, int n_scn, bool lead);

// The batched launch on device tables the caller keeps (a recorded graph
// refreshes them by a copy node before these kernels): every grid covers
// cap_total samples and cap_scn scenarios, and the kernels read the actual
// sizes from *hdr.  kind gives the integrator, obstacle, impact_exit and
// nofma that all scenarios share; perception: whether any has it.
int launch_batch_fast_dev(const aeb_scenario& kind, bool perception, int precision,
                          const BatchHdr* hdr, const ScnDev* tab, const aeb_scenario* scns,
                          int cap_scn, int64_t cap_total, void* scratch_base, hipStream_t st);
int fill_batch_table(const aeb_scenario* scns, int n_scn, const OutCols* outs, ScnDev* tab,
                     int64_t* total, int64_t* cap);
int launch_batch_fast_into(const aeb_scenario* scns, int n_scn, int precision,
                           const ScnDev* tab, int64_t total, int64_t cap, void* scratch_base,
                           hipStream_t st);

}  // namespace aeb
