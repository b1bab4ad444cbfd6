// sanitize_sched.cpp -- the serving scheduler under ThreadSanitizer: four
// client threads submit 600 requests while the worker thread admits,
// launches and completes them (a stand-in executor) and two more threads
// poll concurrently; every request must come back with its own result.
// Built and run by tests/test_sanitizers.py with g++ -fsanitize=thread; exit
// status 0 when every check holds (a data race makes TSan report and exit
// with its own status).
#include <atomic>
#include <cstdio>
#include <random>
#include <thread>
#include <vector>

#include "serve_fake.cpp"

int main() {
  void* h = fake_create(4000, 6, 3, 100, 100000, 1000000, 1, 3);
  fake_start(h);
  std::mt19937 rng(3);
  const int64_t choice[3] = {100, 400, 1500};
  std::vector<int64_t> sizes(600);
  for (auto& s : sizes) s = choice[rng() % 3];
  std::vector<uint64_t> tickets(sizes.size(), 0);
  std::vector<std::atomic<int>> got(sizes.size());
  for (auto& g : got) g = 0;
  std::atomic<int> bad{0};
  std::vector<std::thread> th;
  for (int c = 0; c < 4; ++c)
    th.emplace_back([&, c] {
      for (size_t k = c; k < sizes.size(); k += 4) {
        uint64_t t = 0;
        if (fake_submit(h, sizes[k], 0, 1, 10.0, &t) != 0) ++bad;
        tickets[k] = t;
      }
    });
  for (auto& t : th) t.join();
  th.clear();
  // two pollers split the requests between them while the worker runs
  for (int p = 0; p < 2; ++p)
    th.emplace_back([&, p] {
      for (size_t k = p; k < sizes.size(); k += 2) {
        for (;;) {
          int64_t out[3] = {0, 0, 0};
          aeb_req_timing tm;
          const int rc = fake_poll(h, tickets[k], out, &tm);
          if (rc == AEB_EAGAIN) {
            std::this_thread::yield();
            continue;
          }
          if (rc != AEB_OK || out[0] != sizes[k] || static_cast<uint64_t>(out[1]) != tickets[k] ||
              !(tm.arrive <= tm.admit && tm.admit <= tm.start && tm.start <= tm.done))
            ++bad;
          ++got[k];
          break;
        }
      }
    });
  for (auto& t : th) t.join();
  fake_wait_idle(h);
  uint64_t c[10] = {0};
  fake_counters(h, c);
  fake_stop(h);
  fake_destroy(h);
  for (auto& g : got)
    if (g != 1) ++bad;
  if (c[1] != sizes.size()) ++bad;  // completed
  std::printf("requests %zu, completed %llu, bad %d\n", sizes.size(),
              static_cast<unsigned long long>(c[1]), bad.load());
  return bad == 0 ? 0 : 1;
}
