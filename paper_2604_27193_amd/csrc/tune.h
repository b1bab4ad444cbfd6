// tune.h -- launch-shape table of the block-structured integration kernels,
// per precision (FP64 / FP32C) and obstacle kind, filled with defaults,
// a JSON cache, or the autotuner (tune.cpp).
#pragma once

namespace aeb {

struct TuneCfg {
  int k;               // steps per unchecked block (16, 32, 64)
  int block;           // threads per workgroup (64, 128, 256)
  int waves_per_simd;  // 0: one pass, one workgroup per `block` samples; else a persistent
                       // grid of this many wavefronts per SIMD claiming 64-sample chunks
};

// precision: AEB_FP64 or AEB_FP32C (the fix-up mode uses the FP32C entry)
TuneCfg tune_get(int precision, int obstacle);
bool tune_valid(int precision, const TuneCfg& t);
void tune_set(int precision, int obstacle, const TuneCfg& t);

}  // namespace aeb
