// serve_fake.cpp -- test shim: the serving scheduler driven by a host
// stand-in for the device executor, so admission, packing, stream rotation,
// completion and accounting can be checked on the CPU.  Built by the tests
// with g++ (no HIP); not part of the library.
#include <cstdint>
#include <cstring>
#include <memory>
#include <vector>

#include "serve_sched.h"

using aeb::serve::Arena;
using aeb::serve::Config;
using aeb::serve::Counters;
using aeb::serve::Executor;
using aeb::serve::Request;
using aeb::serve::Scheduler;

namespace {

class FakeExecutor final : public Executor {
 public:
  FakeExecutor(int n_streams, uint64_t bytes_per_sample, int auto_polls)
      : per_(bytes_per_sample), auto_polls_(auto_polls), left_(n_streams, -1),
        ticks_(n_streams), fail_next_(0) {}

  uint64_t footprint(const aeb_scenario& s) const override {
    return per_ * static_cast<uint64_t>(s.n_samples);
  }
  int check(const aeb_scenario& s) const override {
    if (s.n_samples < 1) return AEB_EINVAL;
    if (s.integrator != AEB_EULER) return AEB_EINVAL;
    return AEB_OK;
  }
  int launch(int stream, const std::vector<Request*>& tick) override {
    ticks_[stream].clear();
    for (Request* r : tick) ticks_[stream].push_back(r->ticket);
    ++launches_;
    if (fail_next_) {
      fail_next_ = 0;
      return AEB_EDEVICE;
    }
    left_[stream] = auto_polls_;  // -1: complete only on fake_complete
    return AEB_OK;
  }
  bool done(int stream) override {
    if (left_[stream] == 0) return true;
    if (left_[stream] > 0) --left_[stream];
    return left_[stream] == 0;
  }
  void finish(int stream, const std::vector<Request*>& tick) override {
    for (Request* r : tick) {
      std::memset(&r->stats, 0, sizeof(r->stats));
      r->stats.n = r->scn.n_samples;
      r->stats.n_collide = static_cast<int64_t>(r->ticket);  // lets tests match results
      r->stats.n_stop = stream;
    }
    left_[stream] = -1;
  }
  void complete(int stream) { left_[stream] = 0; }

  uint64_t per_;
  int auto_polls_;
  std::vector<int> left_;
  std::vector<std::vector<uint64_t>> ticks_;
  int fail_next_;
  int launches_ = 0;
};

struct Fake {
  std::unique_ptr<FakeExecutor> ex;
  std::unique_ptr<Scheduler> sched;
};

aeb_scenario make(int64_t n, int integrator, int obstacle) {
  aeb_scenario s;
  std::memset(&s, 0, sizeof(s));
  s.n_samples = n;
  s.integrator = integrator;
  s.obstacle = obstacle;
  return s;
}

}  // namespace

extern "C" {

// ---- arena ----
void* arena_new(uint64_t cap) { return new Arena(cap); }
void arena_delete(void* a) { delete static_cast<Arena*>(a); }
int64_t arena_alloc(void* a, uint64_t bytes) { return static_cast<Arena*>(a)->alloc(bytes); }
int arena_release(void* a, int64_t off) { return static_cast<Arena*>(a)->release(off) ? 1 : 0; }
void arena_state(void* a, uint64_t* out4) {
  const Arena* A = static_cast<Arena*>(a);
  out4[0] = A->in_use();
  out4[1] = A->peak();
  out4[2] = A->largest_free();
  out4[3] = A->n_free_ranges();
}

// ---- scheduler with the stand-in executor ----
void* fake_create(uint64_t arena_bytes, int max_slots, int n_streams, int tick_us, int max_queue,
                  int64_t max_tick_samples, uint64_t bytes_per_sample, int auto_polls) {
  Config c;
  c.arena_bytes = arena_bytes;
  c.max_slots = max_slots;
  c.n_streams = n_streams;
  c.tick_us = tick_us;
  c.max_queue = max_queue;
  c.max_tick_samples = max_tick_samples;
  auto* f = new Fake;
  f->ex.reset(new FakeExecutor(n_streams, bytes_per_sample, auto_polls));
  f->sched.reset(new Scheduler(c, f->ex.get()));
  return f;
}

void fake_destroy(void* h) {
  auto* f = static_cast<Fake*>(h);
  f->sched->stop();
  delete f;
}

int fake_submit(void* h, int64_t n, int integrator, int obstacle, double deadline,
                uint64_t* ticket) {
  return static_cast<Fake*>(h)->sched->submit(make(n, integrator, obstacle), deadline, ticket);
}

// out3: stats.n, stats.n_collide (the ticket), stats.n_stop (the stream)
int fake_poll(void* h, uint64_t ticket, int64_t* out3, aeb_req_timing* tm) {
  aeb_stats* st = new aeb_stats;
  const int rc = static_cast<Fake*>(h)->sched->poll(ticket, st, tm);
  if (rc == AEB_OK || rc == AEB_EDEVICE) {
    out3[0] = st->n;
    out3[1] = st->n_collide;
    out3[2] = st->n_stop;
  }
  delete st;
  return rc;
}

int fake_step(void* h) { return static_cast<Fake*>(h)->sched->step() ? 1 : 0; }
void fake_complete(void* h, int stream) { static_cast<Fake*>(h)->ex->complete(stream); }
void fake_fail_next(void* h) { static_cast<Fake*>(h)->ex->fail_next_ = 1; }
int fake_launches(void* h) { return static_cast<Fake*>(h)->ex->launches_; }

// tickets of the tick last launched on `stream`
int fake_tick(void* h, int stream, uint64_t* out, int cap) {
  const auto& t = static_cast<Fake*>(h)->ex->ticks_[stream];
  const int n = static_cast<int>(t.size());
  for (int j = 0; j < n && j < cap; ++j) out[j] = t[j];
  return n;
}

// submitted, completed, failed, missed, ticks, queued, admitted, running, in_use, peak
void fake_counters(void* h, uint64_t* out10) {
  const Counters c = static_cast<Fake*>(h)->sched->counters();
  const uint64_t v[10] = {c.submitted, c.completed, c.failed, c.missed, c.ticks,
                          c.queued,    c.admitted,  c.running, c.arena_in_use, c.arena_peak};
  std::memcpy(out10, v, sizeof(v));
}

void fake_start(void* h) { static_cast<Fake*>(h)->sched->start(); }
void fake_wait_idle(void* h) { static_cast<Fake*>(h)->sched->wait_idle(); }
void fake_stop(void* h) { static_cast<Fake*>(h)->sched->stop(); }
void fake_drain(void* h) { static_cast<Fake*>(h)->sched->drain(); }

}  // extern "C"
