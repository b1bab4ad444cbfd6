// serve.cpp -- the device executor of the serving path and its C ABI
// (aeb_server_*, aeb_serve_*).
//
// A launch ("tick") runs the admitted requests of one kind as one sorted
// multi-scenario rollout (parameters drawn in-kernel from each request's seed
// and id, so nothing per sample crosses PCIe) followed by one segmented
// reduction over all of its requests, all on one of the server's streams; the
// statistics land in pinned host memory and an event marks the tick's end.
// A tick replays a HIP graph recorded once per stream and bucket (kind,
// perception, scenario count and samples rounded up to powers of two): the
// host writes the tick's scenario and set tables into pinned memory and the
// graph's first nodes copy them to the device, so the mix changes from tick
// to tick while the recording stays the same.  All device memory comes from
// the caller's arena: per stream, the rollout's job records and sort buffers
// for max_tick_samples samples and the device tables; per request, its
// output columns and the reduction's scratch.
#include <hip/hip_runtime.h>

#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "aeb_runtime.h"
#include "fast_path.h"
#include "mixgraph.h"
#include "serve_sched.h"

namespace aeb {
namespace {

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

// per request: dist | margin | v_impact | steps | status, then reduce scratch
size_t out_bytes(int64_t n) {
  const size_t m = static_cast<size_t>(n);
  return up256(8 * m) + up256(8 * m) + up256(4 * m) + up256(4 * m) + up256(m);
}

OutCols out_cols(char* base, int64_t n) {
  const size_t m = static_cast<size_t>(n);
  OutCols o;
  o.dist = reinterpret_cast<double*>(base);
  o.margin = reinterpret_cast<double*>(base + up256(8 * m));
  o.vimp = reinterpret_cast<float*>(base + 2 * up256(8 * m));
  o.steps = reinterpret_cast<int32_t*>(base + 2 * up256(8 * m) + up256(4 * m));
  o.status = reinterpret_cast<uint8_t*>(base + 2 * up256(8 * m) + 2 * up256(4 * m));
  return o;
}

size_t table_bytes(const aeb_server_cfg& c) {
  return up256(reduce_table_bytes_cap(c.max_slots, c.max_tick_samples));
}

size_t stream_bytes(const aeb_server_cfg& c) {
  return up256(batch_scratch_bytes(c.max_tick_samples, c.max_slots, true)) + table_bytes(c) +
         up256(mix_table_bytes(c.max_slots));
}

size_t request_bytes(const aeb_server_cfg& c, int64_t n) {
  return out_bytes(n) + up256(reduce_scratch_bytes(n, c.req));
}

int check_cfg(const aeb_server_cfg* c) {
  if (!c) return fail(AEB_EINVAL, "server: null configuration");
  if (c->max_slots < 1 || c->max_slots > 1024) return fail(AEB_EINVAL, "max_slots outside 1..1024");
  if (c->precision != AEB_FP64 && c->precision != AEB_FP32C)
    return fail(AEB_EINVAL, "server precision must be AEB_FP64 or AEB_FP32C");
  if (c->n_streams < 1 || c->n_streams > 8) return fail(AEB_EINVAL, "n_streams outside 1..8");
  if (c->tick_us < 0 || c->tick_us > 1000000) return fail(AEB_EINVAL, "tick_us outside 0..1e6");
  if (c->max_queue < 1) return fail(AEB_EINVAL, "max_queue must be >= 1");
  if (c->max_tick_samples < 1 || c->max_tick_samples > 0x7fffffffLL)
    return fail(AEB_EINVAL, "max_tick_samples outside 1..2^31-1");
  if (c->flags & ~AEB_SERVE_EAGER) return fail(AEB_EINVAL, "unknown server flags");
  return check_reduce_req(c->req);
}

struct StreamCtx {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  char* scratch = nullptr;          // device: rollout scratch of one launch
  char* rtab = nullptr;             // device: the reduction's set table
  ScnDev* tab = nullptr;            // pinned: scenario table of the launch
  aeb_scenario* scns = nullptr;     // pinned: its scenarios
  char* rtab_host = nullptr;        // pinned: host side of the reduction's set table
  char* mtab = nullptr;             // device: scenario tables of a recorded launch
  char* mtab_host = nullptr;        // pinned: host side of those tables
  aeb_stats* stats = nullptr;       // pinned: statistics of the launch's requests
  std::vector<int64_t> ns;          // sample counts of the launch's requests
  MixShape last;                    // bucket of the last launch (if recorded)
  bool last_recorded = false;
  std::map<uint64_t, MixGraph> graphs;  // recordings by bucket
  hipError_t status = hipSuccess;   // completion status of the last launch
};

class HipExecutor final : public serve::Executor {
 public:
  HipExecutor(const aeb_server_cfg& cfg, int dev) : cfg_(cfg), dev_(dev) {}

  ~HipExecutor() override { release(); }

  int init() {
    char* arena = static_cast<char*>(cfg_.arena);
    const size_t sb = stream_bytes(cfg_);
    streams_.resize(cfg_.n_streams);
    for (int s = 0; s < cfg_.n_streams; ++s) {
      StreamCtx& S = streams_[s];
      AEB_HIP(hipStreamCreateWithFlags(&S.st, hipStreamNonBlocking));
      AEB_HIP(hipEventCreateWithFlags(&S.ev, hipEventDisableTiming));
      S.scratch = arena + sb * s;
      S.mtab = S.scratch + (sb - up256(mix_table_bytes(cfg_.max_slots)));
      S.rtab = S.mtab - table_bytes(cfg_);
      AEB_HIP(hipHostMalloc(reinterpret_cast<void**>(&S.tab), sizeof(ScnDev) * cfg_.max_slots,
                            hipHostMallocDefault));
      AEB_HIP(hipHostMalloc(reinterpret_cast<void**>(&S.scns),
                            sizeof(aeb_scenario) * cfg_.max_slots, hipHostMallocDefault));
      AEB_HIP(hipHostMalloc(reinterpret_cast<void**>(&S.rtab_host), table_bytes(cfg_),
                            hipHostMallocDefault));
      AEB_HIP(hipHostMalloc(reinterpret_cast<void**>(&S.mtab_host),
                            mix_table_bytes(cfg_.max_slots), hipHostMallocDefault));
      AEB_HIP(hipHostMalloc(reinterpret_cast<void**>(&S.stats),
                            sizeof(aeb_stats) * cfg_.max_slots, hipHostMallocDefault));
    }
    req_base_ = arena + sb * cfg_.n_streams;
    return AEB_OK;
  }

  void release() {
    for (StreamCtx& S : streams_) {
      if (S.st) (void)hipStreamSynchronize(S.st);
      if (S.ev) (void)hipEventDestroy(S.ev);
      if (S.st) (void)hipStreamDestroy(S.st);
      if (S.tab) (void)hipHostFree(S.tab);
      if (S.scns) (void)hipHostFree(S.scns);
      if (S.rtab_host) (void)hipHostFree(S.rtab_host);
      if (S.mtab_host) (void)hipHostFree(S.mtab_host);
      for (auto& kv : S.graphs) mix_release(&kv.second);
      if (S.stats) (void)hipHostFree(S.stats);
      S = StreamCtx{};
    }
  }

  uint64_t footprint(const aeb_scenario& s) const override {
    return request_bytes(cfg_, s.n_samples);
  }

  int check(const aeb_scenario& s) const override {
    const int rc = validate(s);
    if (rc != AEB_OK) return rc;
    if (s.is_mask)
      return fail(AEB_EINVAL, "serving returns unweighted statistics: no importance sampling");
    if (!fast_path_applies(s, cfg_.precision) || control_on(s))
      return fail(AEB_EINVAL,
                  "serving runs the batched block-structured path (not RK4 in FP32C, not "
                  "the closed-loop controller, at most 2^31 - 4096 steps)");
    return AEB_OK;
  }

  void bind_thread() override { (void)hipSetDevice(dev_); }

  int launch(int stream, const std::vector<serve::Request*>& tick) override {
    const int rc = enqueue(stream, tick);
    // on failure part of the tick may already be queued: let it drain before
    // the scheduler hands the requests' memory to others
    if (rc != AEB_OK) (void)hipStreamSynchronize(streams_[stream].st);
    return rc;
  }

  // The tick's bucket: its kind, capacities rounded up to powers of two.
  MixShape shape_of(const std::vector<serve::Request*>& tick) const {
    MixShape m;
    m.kind = tick[0]->scn;
    m.precision = cfg_.precision;
    int64_t total = 0;
    for (const serve::Request* r : tick) {
      m.perception = m.perception || perception_on(r->scn);
      total += r->scn.n_samples;
    }
    int c = 1;
    while (c < static_cast<int>(tick.size())) c <<= 1;
    m.cap_scn = c < cfg_.max_slots ? c : cfg_.max_slots;
    int64_t t = int64_t(1) << 15;
    while (t < total) t <<= 1;
    m.cap_total = t < cfg_.max_tick_samples ? t : cfg_.max_tick_samples;
    m.reduce = true;
    m.weighted = false;
    m.req = cfg_.req;
    return m;
  }

  static uint64_t key_of(const MixShape& m) {
    return static_cast<uint64_t>(m.kind.integrator) | static_cast<uint64_t>(m.kind.obstacle) << 1 |
           static_cast<uint64_t>(m.kind.impact_exit) << 3 | static_cast<uint64_t>(m.kind.nofma) << 4 |
           static_cast<uint64_t>(m.perception) << 5 | static_cast<uint64_t>(m.cap_scn) << 6 |
           static_cast<uint64_t>(m.cap_total) << 20;
  }

  MixBufs bufs(const StreamCtx& S) const {
    MixBufs b;
    b.dtab = S.mtab;
    b.htab = S.mtab_host;
    b.scratch = S.scratch;
    b.drtab = S.rtab;
    b.hrtab = S.rtab_host;
    b.hstats = S.stats;
    return b;
  }

  int enqueue(int stream, const std::vector<serve::Request*>& tick) {
    StreamCtx& S = streams_[stream];
    const int n = static_cast<int>(tick.size());
    std::vector<OutCols> oc(n);
    std::vector<aeb_scenario> scns(n);
    std::vector<char*> bases(n);
    S.ns.resize(n);
    for (int j = 0; j < n; ++j) {
      scns[j] = tick[j]->scn;
      S.ns[j] = tick[j]->scn.n_samples;
      oc[j] = out_cols(req_base_ + tick[j]->off, S.ns[j]);
      bases[j] = req_base_ + tick[j]->off + out_bytes(S.ns[j]);
    }
    int rc;
    if (cfg_.flags & AEB_SERVE_EAGER) {
      // the copies and kernels one by one, tables laid out for this tick
      std::memcpy(S.scns, scns.data(), sizeof(aeb_scenario) * n);
      int64_t total = 0, cap = 1;
      rc = fill_batch_table(S.scns, n, oc.data(), S.tab, &total, &cap);
      if (rc != AEB_OK) return rc;
      rc = launch_batch_fast_into(S.scns, n, cfg_.precision, S.tab, total, cap, S.scratch, S.st);
      if (rc != AEB_OK) return rc;
      rc = reduce_enqueue_sets(oc.data(), S.ns.data(), n, cfg_.req, bases.data(), S.rtab,
                               S.rtab_host, S.stats, S.st);
      if (rc != AEB_OK) return rc;
      S.last_recorded = false;
    } else {
      const MixShape m = shape_of(tick);
      const MixBufs b = bufs(S);
      rc = mix_fill(m, scns.data(), n, oc.data(), bases.data(), b);
      if (rc != AEB_OK) return rc;
      const uint64_t key = key_of(m);
      auto it = S.graphs.find(key);
      if (it == S.graphs.end()) {
        MixGraph g;
        rc = mix_record(m, b, &g);
        if (rc != AEB_OK) return rc;
        it = S.graphs.emplace(key, g).first;
      }
      AEB_HIP(hipGraphLaunch(it->second.exec, S.st));
      S.last = m;
      S.last_recorded = true;
    }
    AEB_HIP(hipEventRecord(S.ev, S.st));
    return AEB_OK;
  }

  bool done(int stream) override {
    StreamCtx& S = streams_[stream];
    const hipError_t e = hipEventQuery(S.ev);
    if (e == hipErrorNotReady) return false;
    S.status = e;
    return true;
  }

  void finish(int stream, const std::vector<serve::Request*>& tick) override {
    StreamCtx& S = streams_[stream];
    const int n = static_cast<int>(tick.size());
    for (int j = 0; j < n; ++j) {
      serve::Request* r = tick[j];
      if (S.status != hipSuccess) {
        r->rc = fail(AEB_EDEVICE, std::string("serving launch: ") + hipGetErrorString(S.status));
        continue;
      }
      aeb_stats& st = S.stats[j];
      if (st.reserved) {
        // rare: a selection bin too crowded for the in-LDS sort
        char* base = req_base_ + r->off;
        char* red = base + out_bytes(r->scn.n_samples);
        aeb_stats* dst =
            S.last_recorded ? reduce_table_stats_cap(S.rtab, S.last.cap_scn, S.last.cap_total) + j
                            : reduce_table_stats(S.rtab, n, S.ns.data()) + j;
        r->rc = reduce_fallback(out_cols(base, r->scn.n_samples), r->scn.n_samples, cfg_.req,
                                red, dst, &st, S.st);
      }
      st.reserved = 0;
      r->stats = st;
    }
  }

 private:
  aeb_server_cfg cfg_;
  int dev_;
  std::vector<StreamCtx> streams_;
  char* req_base_ = nullptr;    // device: the request part of the arena
};

}  // namespace
}  // namespace aeb

struct aeb_server {
  std::unique_ptr<aeb::HipExecutor> ex;
  std::unique_ptr<aeb::serve::Scheduler> sched;
  uint64_t fixed = 0, request_part = 0;
};

using namespace aeb;

extern "C" {

int aeb_server_fixed_bytes(const aeb_server_cfg* cfg, uint64_t* bytes) {
  const int rc = check_cfg(cfg);
  if (rc != AEB_OK) return rc;
  if (!bytes) return fail(AEB_EINVAL, "null output");
  *bytes = stream_bytes(*cfg) * static_cast<uint64_t>(cfg->n_streams);
  return AEB_OK;
}

int aeb_serve_footprint(const aeb_server_cfg* cfg, int64_t n_samples, uint64_t* bytes) {
  const int rc = check_cfg(cfg);
  if (rc != AEB_OK) return rc;
  if (!bytes || n_samples < 1 || n_samples > 0x7fffffffLL)
    return fail(AEB_EINVAL, "n_samples outside 1..2^31-1");
  *bytes = serve::Arena::round(request_bytes(*cfg, n_samples));
  return AEB_OK;
}

int aeb_server_create(const aeb_server_cfg* cfg, aeb_server** out) {
  if (!out) return fail(AEB_EINVAL, "aeb_server_create: null output");
  *out = nullptr;
  int rc = check_cfg(cfg);
  if (rc != AEB_OK) return rc;
  if (!cfg->arena || (reinterpret_cast<uintptr_t>(cfg->arena) & 255u) != 0)
    return fail(AEB_EINVAL, "the arena must be a non-null, 256-byte aligned device pointer");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(AEB_EDEVICE, "no current HIP device");
  const uint64_t fixed = stream_bytes(*cfg) * static_cast<uint64_t>(cfg->n_streams);
  const uint64_t one = serve::Arena::round(request_bytes(*cfg, cfg->max_tick_samples));
  if (cfg->arena_bytes < fixed + one)
    return fail(AEB_ENOMEM, "arena of " + std::to_string(cfg->arena_bytes) +
                                " bytes; the server needs " + std::to_string(fixed + one) +
                                " (streams plus one request of max_tick_samples)");
  auto srv = std::unique_ptr<aeb_server>(new (std::nothrow) aeb_server);
  if (!srv) return fail(AEB_ENOMEM, "host allocation failed");
  srv->ex.reset(new (std::nothrow) HipExecutor(*cfg, dev));
  if (!srv->ex) return fail(AEB_ENOMEM, "host allocation failed");
  rc = srv->ex->init();
  if (rc != AEB_OK) return rc;
  serve::Config sc;
  sc.arena_bytes = cfg->arena_bytes - fixed;
  sc.max_slots = cfg->max_slots;
  sc.n_streams = cfg->n_streams;
  sc.tick_us = cfg->tick_us;
  sc.max_queue = cfg->max_queue;
  sc.max_tick_samples = cfg->max_tick_samples;
  srv->fixed = fixed;
  srv->request_part = sc.arena_bytes;
  srv->sched.reset(new (std::nothrow) serve::Scheduler(sc, srv->ex.get()));
  if (!srv->sched) return fail(AEB_ENOMEM, "host allocation failed");
  srv->sched->start();
  *out = srv.release();
  return AEB_OK;
}

int aeb_server_destroy(aeb_server* srv) {
  if (!srv) return AEB_OK;
  srv->sched->wait_idle();
  srv->sched->stop();
  srv->sched.reset();
  srv->ex.reset();
  delete srv;
  return AEB_OK;
}

int aeb_serve_submit(aeb_server* srv, const aeb_scenario* scn, double deadline_s,
                     uint64_t* ticket) {
  if (!srv || !scn || !ticket) return fail(AEB_EINVAL, "aeb_serve_submit: null argument");
  if (!(deadline_s > 0.0)) return fail(AEB_EINVAL, "deadline must be positive");
  const int rc = srv->sched->submit(*scn, deadline_s, ticket);
  if (rc == AEB_ENOMEM) return fail(rc, "request larger than the arena or max_tick_samples");
  if (rc == AEB_EAGAIN) return fail(rc, "queue full");
  return rc;
}

int aeb_serve_poll(aeb_server* srv, uint64_t ticket, aeb_stats* out, aeb_req_timing* timing) {
  if (!srv || !out) return fail(AEB_EINVAL, "aeb_serve_poll: null argument");
  const int rc = srv->sched->poll(ticket, out, timing);
  if (rc == AEB_ENOTFOUND) return fail(rc, "unknown ticket");
  return rc;
}

int aeb_server_info_get(aeb_server* srv, aeb_server_info* out) {
  if (!srv || !out) return fail(AEB_EINVAL, "aeb_server_info_get: null argument");
  const serve::Counters c = srv->sched->counters();
  out->submitted = c.submitted;
  out->completed = c.completed;
  out->failed = c.failed;
  out->missed = c.missed;
  out->ticks = c.ticks;
  out->queued = c.queued;
  out->admitted = c.admitted;
  out->running = c.running;
  out->arena_in_use = c.arena_in_use;
  out->arena_peak = c.arena_peak;
  out->arena_request_bytes = srv->request_part;
  out->fixed_bytes = srv->fixed;
  return AEB_OK;
}

}  // extern "C"
