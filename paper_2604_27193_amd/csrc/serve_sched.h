// serve_sched.h -- the request scheduler of the serving path (continuous
// batching of Monte Carlo evaluations under the collision-avoidance time
// budget of Sec. VI), independent of the device.
//
// Requests arrive at any time (submit, thread-safe).  A worker admits them in
// arrival order while their device footprint fits the free part of a
// caller-provided memory arena and a slot is free, packs the admitted requests
// of one kind into a "tick" and hands the tick to an executor, which runs it
// on one of several streams.  Ticks on different streams overlap on the
// device; a stream takes its next tick once its last one has completed.
// Completed requests release their memory and slot, and their statistics and
// timestamps wait for the client's poll.  Strict arrival-order admission: a
// request that does not fit waits for memory rather than being overtaken, so
// no request starves.
//
// The executor interface lets the same scheduler drive the device (the HIP
// executor of the library) or a host stand-in in tests.
#pragma once

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>

#include <sys/prctl.h>
#include <unordered_map>
#include <vector>

#include "aeb.h"

namespace aeb {
namespace serve {

// First-fit allocator of byte ranges in [0, capacity), in 256-byte units,
// with coalescing of neighbouring free ranges.
class Arena {
 public:
  static constexpr uint64_t ALIGN = 256;

  explicit Arena(uint64_t capacity = 0) { reset(capacity); }

  void reset(uint64_t capacity) {
    cap_ = capacity & ~(ALIGN - 1);
    free_.clear();
    used_.clear();
    in_use_ = peak_ = 0;
    if (cap_) free_[0] = cap_;
  }

  static uint64_t round(uint64_t b) { return (b + ALIGN - 1) & ~(ALIGN - 1); }

  // offset of a new range of `bytes` (rounded up), or -1 if no free range fits
  int64_t alloc(uint64_t bytes) {
    const uint64_t need = round(bytes ? bytes : 1);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < need) continue;
      const uint64_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > need) free_[off + need] = len - need;
      used_[off] = need;
      in_use_ += need;
      peak_ = std::max(peak_, in_use_);
      return static_cast<int64_t>(off);
    }
    return -1;
  }

  // give back a range returned by alloc; false for an unknown offset
  bool release(int64_t off) {
    auto u = used_.find(static_cast<uint64_t>(off));
    if (off < 0 || u == used_.end()) return false;
    uint64_t start = u->first, len = u->second;
    in_use_ -= len;
    used_.erase(u);
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
    return true;
  }

  uint64_t capacity() const { return cap_; }
  uint64_t in_use() const { return in_use_; }
  uint64_t peak() const { return peak_; }
  uint64_t largest_free() const {
    uint64_t m = 0;
    for (const auto& f : free_) m = std::max(m, f.second);
    return m;
  }
  size_t n_free_ranges() const { return free_.size(); }

 private:
  uint64_t cap_ = 0, in_use_ = 0, peak_ = 0;
  std::map<uint64_t, uint64_t> free_;  // offset -> length
  std::map<uint64_t, uint64_t> used_;  // offset -> length
};

enum State { QUEUED = 0, ADMITTED = 1, RUNNING = 2, DONE = 3 };

struct Request {
  uint64_t ticket = 0;
  aeb_scenario scn{};
  double deadline = 0.0;    // seconds after arrival
  uint64_t footprint = 0;   // arena bytes
  int64_t off = -1;         // arena range while admitted or running
  int slot = -1;
  int state = QUEUED;
  int rc = AEB_OK;          // outcome of the execution
  double t_arrive = 0, t_admit = 0, t_start = 0, t_done = 0;
  aeb_stats stats{};
};

// Requests of one kind can share a launch.
inline bool same_kind(const aeb_scenario& a, const aeb_scenario& b) {
  return a.integrator == b.integrator && a.obstacle == b.obstacle &&
         a.impact_exit == b.impact_exit && a.nofma == b.nofma;
}

class Executor {
 public:
  virtual ~Executor() = default;
  // device bytes one request needs from the arena while admitted
  virtual uint64_t footprint(const aeb_scenario& s) const = 0;
  // AEB_OK if the executor can run the scenario, else an error (message set)
  virtual int check(const aeb_scenario& s) const = 0;
  // enqueue the tick on `stream` (requests hold their arena offset and slot)
  virtual int launch(int stream, const std::vector<Request*>& tick) = 0;
  // the stream's last tick has completed on the device
  virtual bool done(int stream) = 0;
  // collect the results of the stream's completed tick into the requests
  virtual void finish(int stream, const std::vector<Request*>& tick) = 0;
  // called once on the worker thread before its first step
  virtual void bind_thread() {}
};

struct Config {
  uint64_t arena_bytes = 0;   // part of the arena left for request footprints
  int max_slots = 64;         // requests admitted or running at once
  int n_streams = 2;
  int tick_us = 200;          // packing window while the device is busy
  int max_queue = 4096;       // waiting requests
  int64_t max_tick_samples = 1 << 22;
};

struct Counters {
  uint64_t submitted = 0, completed = 0, failed = 0, missed = 0, ticks = 0;
  uint64_t queued = 0, admitted = 0, running = 0;
  uint64_t arena_in_use = 0, arena_peak = 0;
};

class Scheduler {
 public:
  Scheduler(const Config& cfg, Executor* ex)
      : cfg_(cfg), ex_(ex), arena_(cfg.arena_bytes), running_(cfg.n_streams),
        t0_(std::chrono::steady_clock::now()) {
    for (int s = 0; s < cfg_.max_slots; ++s) free_slots_.push_back(cfg_.max_slots - 1 - s);
  }

  ~Scheduler() { stop(); }

  // seconds since the scheduler was created (steady clock)
  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0_).count();
  }

  int submit(const aeb_scenario& s, double deadline, uint64_t* ticket) {
    const int rc = ex_->check(s);
    if (rc != AEB_OK) return rc;
    const uint64_t fp = Arena::round(ex_->footprint(s));
    std::lock_guard<std::mutex> g(mu_);
    if (fp > arena_.capacity()) return AEB_ENOMEM;
    if (s.n_samples > cfg_.max_tick_samples) return AEB_ENOMEM;
    if (static_cast<int>(queue_.size()) >= cfg_.max_queue) return AEB_EAGAIN;
    auto r = std::make_unique<Request>();
    r->ticket = ++last_ticket_;
    r->scn = s;
    r->deadline = deadline;
    r->footprint = fp;
    r->t_arrive = now();
    *ticket = r->ticket;
    queue_.push_back(r.get());
    reqs_.emplace(r->ticket, std::move(r));
    ++cnt_.submitted;
    cv_.notify_all();
    return AEB_OK;
  }

  // AEB_OK (and the request is forgotten) once done; AEB_EAGAIN while pending;
  // AEB_ENOTFOUND for a ticket never issued or already collected.  A request
  // whose execution failed returns that error (and is forgotten as well).
  int poll(uint64_t ticket, aeb_stats* st, aeb_req_timing* tm) {
    std::lock_guard<std::mutex> g(mu_);
    auto it = reqs_.find(ticket);
    if (it == reqs_.end()) return AEB_ENOTFOUND;
    Request* r = it->second.get();
    if (r->state != DONE) return AEB_EAGAIN;
    const int rc = r->rc;
    if (st) *st = r->stats;
    if (tm) {
      tm->arrive = r->t_arrive;
      tm->admit = r->t_admit;
      tm->start = r->t_start;
      tm->done = r->t_done;
      tm->missed = (r->t_done - r->t_arrive) > r->deadline ? 1 : 0;
      tm->reserved = 0;
    }
    reqs_.erase(it);
    return rc;
  }

  Counters counters() const {
    std::lock_guard<std::mutex> g(mu_);
    Counters c = cnt_;
    c.queued = queue_.size();
    c.admitted = admitted_.size();
    c.running = 0;
    for (const auto& t : running_) c.running += t.size();
    c.arena_in_use = arena_.in_use();
    c.arena_peak = arena_.peak();
    return c;
  }

  // One scheduling round: collect completed ticks, admit, launch.  Returns
  // true if anything changed.
  bool step() {
    std::lock_guard<std::mutex> g(mu_);
    bool any = reap();
    any = admit() || any;
    any = launch() || any;
    return any;
  }

  // true while requests are queued, admitted or running
  bool busy() const {
    std::lock_guard<std::mutex> g(mu_);
    if (!queue_.empty() || !admitted_.empty()) return true;
    for (const auto& t : running_)
      if (!t.empty()) return true;
    return false;
  }

  // run step() on a worker thread until stop()
  void start() {
    if (worker_.joinable()) return;
    quit_ = false;
    worker_ = std::thread([this] { loop(); });
  }

  void stop() {
    {
      std::lock_guard<std::mutex> g(mu_);
      quit_ = true;
      cv_.notify_all();
    }
    if (worker_.joinable()) worker_.join();
  }

  // finish every queued and running request (the worker must not be running)
  void drain() {
    while (busy()) {
      if (!step()) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }

  // with the worker running: wait until every accepted request is done
  void wait_idle() {
    while (busy()) std::this_thread::sleep_for(std::chrono::microseconds(100));
  }

  const Arena& arena() const { return arena_; }

 private:
  void loop() {
    ex_->bind_thread();
    // the polls below sleep a few microseconds; the default timer slack
    // (50 us) would stretch each into tens of microseconds of latency
    (void)prctl(PR_SET_TIMERSLACK, 1UL, 0UL, 0UL, 0UL);
    for (;;) {
      bool in_flight;
      {
        std::unique_lock<std::mutex> lk(mu_);
        if (quit_) break;
        in_flight = false;
        for (const auto& t : running_) in_flight = in_flight || !t.empty();
        if (!in_flight && queue_.empty() && admitted_.empty()) {
          cv_.wait(lk, [this] { return quit_ || !queue_.empty(); });
          if (quit_) break;
        }
      }
      if (!step()) {
        // device work in flight or a packing window open: poll again shortly
        std::this_thread::sleep_for(std::chrono::microseconds(in_flight ? 10 : 50));
      }
    }
  }

  void release(Request* r) {
    arena_.release(r->off);
    r->off = -1;
    free_slots_.push_back(r->slot);
    r->slot = -1;
  }

  bool reap() {
    bool any = false;
    for (int s = 0; s < cfg_.n_streams; ++s) {
      auto& tick = running_[s];
      if (tick.empty() || !ex_->done(s)) continue;
      ex_->finish(s, tick);
      const double t = now();
      for (Request* r : tick) {
        r->t_done = t;
        r->state = DONE;
        release(r);
        if (r->rc != AEB_OK) ++cnt_.failed;
        ++cnt_.completed;
        if (r->t_done - r->t_arrive > r->deadline) ++cnt_.missed;
      }
      tick.clear();
      any = true;
    }
    return any;
  }

  bool admit() {
    bool any = false;
    while (!queue_.empty() && !free_slots_.empty()) {
      Request* r = queue_.front();
      const int64_t off = arena_.alloc(r->footprint);
      if (off < 0) break;  // wait for memory; later requests do not overtake
      queue_.pop_front();
      r->off = off;
      r->slot = free_slots_.back();
      free_slots_.pop_back();
      r->state = ADMITTED;
      r->t_admit = now();
      admitted_.push_back(r);
      any = true;
    }
    return any;
  }

  bool launch() {
    if (admitted_.empty()) return false;
    int idle = -1, busy_streams = 0;
    for (int s = 0; s < cfg_.n_streams; ++s) {
      if (running_[s].empty()) {
        if (idle < 0) idle = s;
      } else {
        ++busy_streams;
      }
    }
    if (idle < 0) return false;
    // with the device busy, wait up to one packing window for more requests
    const double waited = now() - admitted_.front()->t_admit;
    int64_t pending = 0;
    for (Request* r : admitted_) pending += r->scn.n_samples;
    if (busy_streams > 0 && waited * 1e6 < cfg_.tick_us && pending < cfg_.max_tick_samples)
      return false;
    // pack: the oldest admitted request and the following ones of its kind
    std::vector<Request*> tick;
    int64_t samples = 0;
    const aeb_scenario& kind = admitted_.front()->scn;
    for (auto it = admitted_.begin(); it != admitted_.end();) {
      Request* r = *it;
      if (!same_kind(r->scn, kind) || (!tick.empty() && samples + r->scn.n_samples >
                                                            cfg_.max_tick_samples)) {
        ++it;
        continue;
      }
      samples += r->scn.n_samples;
      tick.push_back(r);
      it = admitted_.erase(it);
    }
    const double t = now();
    for (Request* r : tick) {
      r->t_start = t;
      r->state = RUNNING;
    }
    const int rc = ex_->launch(idle, tick);
    ++cnt_.ticks;
    if (rc != AEB_OK) {
      for (Request* r : tick) {
        r->rc = rc;
        r->t_done = t;
        r->state = DONE;
        release(r);
        ++cnt_.failed;
        ++cnt_.completed;
        if (r->t_done - r->t_arrive > r->deadline) ++cnt_.missed;
      }
      return true;
    }
    running_[idle] = std::move(tick);
    return true;
  }

  Config cfg_;
  Executor* ex_;
  Arena arena_;
  mutable std::mutex mu_;
  std::condition_variable cv_;
  std::thread worker_;
  bool quit_ = false;
  uint64_t last_ticket_ = 0;
  std::deque<Request*> queue_;
  std::deque<Request*> admitted_;
  std::vector<std::vector<Request*>> running_;
  std::vector<int> free_slots_;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs_;
  Counters cnt_;
  std::chrono::steady_clock::time_point t0_;
};

}  // namespace serve
}  // namespace aeb
