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
  double kt;      // dt / tau
  double gap;     // initial gap to the obstacle
  double dmax;    // bound on |dv/dt| over the whole rollout
  double pred;    // predicted number of steps
};

enum { FORM_G = 0, FORM_F = 1, FORM_C = 2, FORM_D = 3 };

bool fast_path_applies(const aeb_scenario& s, int precision);
int launch_rollout_fast(const aeb_scenario& s, const ParamSrc* src, int precision,
                        const OutCols& out, int64_t n, hipStream_t st);

}  // namespace aeb
