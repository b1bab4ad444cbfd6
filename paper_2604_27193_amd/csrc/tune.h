// tune.h -- launch-shape table of the block-structured integration kernels,
// per precision (FP64 / FP32C) and obstacle kind, filled with defaults,
// a JSON cache, or the autotuner (tune.cpp).
#pragma once

#include <vector>

namespace aeb {

struct TuneCfg {
  int k;               // steps per unchecked block (16, 32, 64; FP64 also 128)
  int block;           // threads per workgroup (64, 128, 256)
  int waves_per_simd;  // 0: one pass, one workgroup per `block` samples; else a persistent
                       // grid of this many wavefronts per SIMD claiming 64-sample chunks
  int spt = 1;         // samples per thread: 1, or 2 (FP64 explicit Euler without a lead
                       // vehicle or controller: each lane integrates two sorted samples)
};

// One timed candidate of the last autotuner sweep.
struct TuneResult {
  TuneCfg t;
  float ms;
};

// candidates of the last sweep for (precision, obstacle), fastest first
std::vector<TuneResult> tune_results(int precision, int obstacle);

// precision: AEB_FP64 or AEB_FP32C (the fix-up mode uses the FP32C entry)
TuneCfg tune_get(int precision, int obstacle);
bool tune_valid(int precision, const TuneCfg& t, int obstacle);
void tune_set(int precision, int obstacle, const TuneCfg& t);

}  // namespace aeb
