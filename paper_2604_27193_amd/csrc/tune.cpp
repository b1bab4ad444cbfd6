// tune.cpp -- the launch-shape table (tune.h), its JSON cache and the
// autotuner: for a calibration scenario it times every candidate shape of
// the integration kernel (steps per block, workgroup size, one-pass or
// persistent grid) on the device and keeps the fastest.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "aeb_runtime.h"
#include "fast_path.h"
#include "tune.h"

namespace aeb {
namespace {

std::mutex g_mu;
std::once_flag g_env_once;
// [precision 0 FP64, 1 FP32C][obstacle none, stationary, lead]
// defaults measured on MI355X (1,048,576-sample workloads, launch shapes
// timed in one process, interleaved): FP64 256 threads and 4 persistent
// wavefronts per SIMD, 128-step blocks with an obstacle and 64-step blocks
// without; FP32C 64-step blocks, 256 threads, one pass
TuneCfg g_tab[2][3] = {
    {{64, 256, 4, 1}, {128, 256, 4, 1}, {128, 256, 4, 1}},
    {{64, 256, 0, 1}, {64, 256, 0, 1}, {64, 256, 0, 1}},
};
std::vector<TuneResult> g_res[2][3];  // the last sweep's candidates

int pidx(int precision) { return precision == AEB_FP64 ? 0 : 1; }

// Entries of the cache: one object per line,
//   {"precision": P, "obstacle": O, "k": K, "block": B, "waves_per_simd": W, "ms": T}
int load_file(const char* path) {
  std::ifstream f(path);
  if (!f) return fail(AEB_EINVAL, std::string("cannot read tuning cache ") + path);
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string txt = ss.str();
  auto field = [](const std::string& obj, const char* key, long* out) {
    const std::string k = std::string("\"") + key + "\"";
    size_t p = obj.find(k);
    if (p == std::string::npos) return false;
    p = obj.find(':', p + k.size());
    if (p == std::string::npos) return false;
    char* end = nullptr;
    *out = std::strtol(obj.c_str() + p + 1, &end, 10);
    return end != obj.c_str() + p + 1;
  };
  struct Entry {
    int p, o;
    TuneCfg t;
  };
  std::vector<Entry> got;
  size_t pos = txt.find("\"entries\"");
  if (pos == std::string::npos) return fail(AEB_EINVAL, "tuning cache without entries");
  for (;;) {
    const size_t a = txt.find('{', pos);
    if (a == std::string::npos) break;
    const size_t b = txt.find('}', a);
    if (b == std::string::npos) break;
    const std::string obj = txt.substr(a, b - a + 1);
    pos = b + 1;
    long prec, obs, k, block, w, spt = 1;
    if (!field(obj, "precision", &prec) || !field(obj, "obstacle", &obs) || !field(obj, "k", &k) ||
        !field(obj, "block", &block) || !field(obj, "waves_per_simd", &w))
      return fail(AEB_EINVAL, "malformed tuning cache entry: " + obj);
    (void)field(obj, "samples_per_thread", &spt);  // absent in caches of format 1: one
    const TuneCfg t{static_cast<int>(k), static_cast<int>(block), static_cast<int>(w),
                    static_cast<int>(spt)};
    if ((prec != AEB_FP64 && prec != AEB_FP32C) || obs < 0 || obs > 2 ||
        !tune_valid(static_cast<int>(prec), t, static_cast<int>(obs)))
      return fail(AEB_EINVAL, "invalid tuning cache entry: " + obj);
    got.push_back(Entry{pidx(static_cast<int>(prec)), static_cast<int>(obs), t});
  }
  if (got.empty()) return fail(AEB_EINVAL, "tuning cache holds no entries");
  std::lock_guard<std::mutex> g(g_mu);
  for (const Entry& e : got) g_tab[e.p][e.o] = e.t;
  return AEB_OK;
}

int save_file(const char* path, const float ms[2][3]) {
  std::ofstream f(path);
  if (!f) return fail(AEB_EINVAL, std::string("cannot write tuning cache ") + path);
  f << "{\"format\": 2, \"entries\": [\n";
  std::lock_guard<std::mutex> g(g_mu);
  for (int p = 0; p < 2; ++p)
    for (int o = 0; o < 3; ++o) {
      const TuneCfg& t = g_tab[p][o];
      f << "  {\"precision\": " << (p == 0 ? AEB_FP64 : AEB_FP32C) << ", \"obstacle\": " << o
        << ", \"k\": " << t.k << ", \"block\": " << t.block
        << ", \"waves_per_simd\": " << t.waves_per_simd
        << ", \"samples_per_thread\": " << t.spt << ", \"ms\": " << ms[p][o] << "}"
        << (p == 1 && o == 2 ? "\n" : ",\n");
    }
  f << "]}\n";
  return f ? AEB_OK : fail(AEB_EINVAL, "write failed");
}

void load_env() {
  const char* p = std::getenv("AEB_TUNE_CACHE");
  if (p && *p) (void)load_file(p);
}

float g_ms[2][3] = {};

}  // namespace

bool tune_valid(int precision, const TuneCfg& t, int obstacle) {
  // FP32C blocks must divide its 64-step flush period; FP64 also takes 128
  const bool k_ok = t.k == 16 || t.k == 32 || t.k == 64 || (t.k == 128 && precision == AEB_FP64);
  const bool b_ok = t.block == 64 || t.block == 128 || t.block == 256;
  // two samples per thread: the FP64 kernel without a lead vehicle
  const bool s_ok = t.spt == 1 || (t.spt == 2 && precision == AEB_FP64 && obstacle != AEB_OBS_LEAD);
  return k_ok && b_ok && s_ok && t.waves_per_simd >= 0 && t.waves_per_simd <= 32;
}

std::vector<TuneResult> tune_results(int precision, int obstacle) {
  std::lock_guard<std::mutex> g(g_mu);
  return g_res[pidx(precision)][obstacle < 0 || obstacle > 2 ? 0 : obstacle];
}

TuneCfg tune_get(int precision, int obstacle) {
  std::call_once(g_env_once, load_env);
  std::lock_guard<std::mutex> g(g_mu);
  return g_tab[pidx(precision)][obstacle < 0 || obstacle > 2 ? 0 : obstacle];
}

void tune_set(int precision, int obstacle, const TuneCfg& t) {
  std::call_once(g_env_once, load_env);
  std::lock_guard<std::mutex> g(g_mu);
  g_tab[pidx(precision)][obstacle] = t;
}

}  // namespace aeb

using namespace aeb;

extern "C" {

int aeb_tune_get(int precision, int obstacle, aeb_tune_shape* shape) {
  if ((precision != AEB_FP64 && precision != AEB_FP32C) || obstacle < 0 || obstacle > 2 || !shape)
    return fail(AEB_EINVAL, "aeb_tune_get: bad argument");
  const TuneCfg t = tune_get(precision, obstacle);
  shape->k = t.k;
  shape->block = t.block;
  shape->waves_per_simd = t.waves_per_simd;
  shape->samples_per_thread = t.spt;
  return AEB_OK;
}

int aeb_tune_set(int precision, int obstacle, const aeb_tune_shape* shape) {
  if (!shape) return fail(AEB_EINVAL, "aeb_tune_set: null shape");
  const TuneCfg t{shape->k, shape->block, shape->waves_per_simd, shape->samples_per_thread};
  if ((precision != AEB_FP64 && precision != AEB_FP32C) || obstacle < 0 || obstacle > 2 ||
      !tune_valid(precision, t, obstacle))
    return fail(AEB_EINVAL, "aeb_tune_set: unsupported shape");
  tune_set(precision, obstacle, t);
  return AEB_OK;
}

int aeb_tune_results(int precision, int obstacle, aeb_tune_shape* shapes, float* ms, int max,
                     int* count) {
  if ((precision != AEB_FP64 && precision != AEB_FP32C) || obstacle < 0 || obstacle > 2 ||
      !count || max < 0 || (max > 0 && (!shapes || !ms)))
    return fail(AEB_EINVAL, "aeb_tune_results: bad argument");
  const std::vector<TuneResult> r = tune_results(precision, obstacle);
  *count = static_cast<int>(r.size());
  for (int j = 0; j < max && j < static_cast<int>(r.size()); ++j) {
    shapes[j].k = r[j].t.k;
    shapes[j].block = r[j].t.block;
    shapes[j].waves_per_simd = r[j].t.waves_per_simd;
    shapes[j].samples_per_thread = r[j].t.spt;
    ms[j] = r[j].ms;
  }
  return AEB_OK;
}

int aeb_tune_load(const char* path) {
  if (!path) return fail(AEB_EINVAL, "aeb_tune_load: null path");
  std::call_once(g_env_once, load_env);
  return load_file(path);
}

int aeb_autotune(const aeb_scenario* calib, int precision, const char* cache_path, void* stream,
                 float* best_ms) {
  if (!calib) return fail(AEB_EINVAL, "aeb_autotune: null scenario");
  int rc = validate(*calib);
  if (rc != AEB_OK) return rc;
  if (precision != AEB_FP64 && precision != AEB_FP32C)
    return fail(AEB_EINVAL, "aeb_autotune: precision must be AEB_FP64 or AEB_FP32C");
  // the tuned table serves explicit Euler in the fused form; RK4, the unfused
  // form and the controller run fixed block sizes, so their timings would
  // overwrite the Euler entry with noise
  if (!fast_path_applies(*calib, precision) || control_on(*calib) ||
      calib->integrator != AEB_EULER || (precision == AEB_FP64 && calib->nofma))
    return fail(AEB_EINVAL, "aeb_autotune: the scenario does not take the tuned block-structured path");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t n = calib->n_samples;
  // temporary outputs, released before returning
  char* mem = nullptr;
  const size_t col = (static_cast<size_t>(n) * 8 + 255) & ~size_t(255);
  AEB_HIP(hipMalloc(reinterpret_cast<void**>(&mem), 5 * col));
  OutCols out{reinterpret_cast<double*>(mem), reinterpret_cast<uint8_t*>(mem + col),
              reinterpret_cast<int32_t*>(mem + 2 * col), reinterpret_cast<double*>(mem + 3 * col),
              reinterpret_cast<float*>(mem + 4 * col)};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  (void)hipEventCreate(&e0);
  (void)hipEventCreate(&e1);
  const TuneCfg keep = tune_get(precision, calib->obstacle);
  std::vector<TuneCfg> cands;
  for (int sp : {1, 2})
    for (int k : {16, 32, 64, 128})
      for (int b : {64, 128, 256})
        for (int w : {0, 4, 8}) {
          const TuneCfg t{k, b, w, sp};
          if (tune_valid(precision, t, calib->obstacle)) cands.push_back(t);
        }
  std::vector<TuneResult> res;
  TuneCfg best = keep;
  float best_t = 1e30f;
  rc = AEB_OK;
  for (const TuneCfg& t : cands) {
    tune_set(precision, calib->obstacle, t);
    std::vector<float> ms;
    for (int r = 0; r < 4 && rc == AEB_OK; ++r) {
      if (hipEventRecord(e0, st) != hipSuccess) rc = fail(AEB_EDEVICE, "event record failed");
      if (rc == AEB_OK) {
        ScratchScope scope(st);
        rc = launch_rollout_fast(*calib, nullptr, precision, out, n, st);
      }
      if (rc == AEB_OK && hipEventRecord(e1, st) != hipSuccess)
        rc = fail(AEB_EDEVICE, "event record failed");
      if (rc == AEB_OK && hipEventSynchronize(e1) != hipSuccess)
        rc = fail(AEB_EDEVICE, "event wait failed");
      float x = 0.0f;
      if (rc == AEB_OK && r > 0 && hipEventElapsedTime(&x, e0, e1) == hipSuccess)
        ms.push_back(x);
    }
    if (rc != AEB_OK) break;
    std::sort(ms.begin(), ms.end());
    const float med = ms[ms.size() / 2];
    res.push_back(TuneResult{t, med});
    if (med < best_t) {
      best_t = med;
      best = t;
    }
  }
  tune_set(precision, calib->obstacle, rc == AEB_OK ? best : keep);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(mem);
  if (rc != AEB_OK) return rc;
  g_ms[pidx(precision)][calib->obstacle] = best_t;
  std::stable_sort(res.begin(), res.end(),
                   [](const TuneResult& a, const TuneResult& b) { return a.ms < b.ms; });
  {
    std::lock_guard<std::mutex> g(g_mu);
    g_res[pidx(precision)][calib->obstacle] = res;
  }
  if (best_ms) *best_ms = best_t;
  if (cache_path) return save_file(cache_path, g_ms);
  return AEB_OK;
}

}  // extern "C"
