// sanitize_sampler.cpp -- the library's host-side arithmetic under
// AddressSanitizer and UndefinedBehaviorSanitizer: the parameter draws of
// the plain method (generator, distributions, perception trigger, importance
// weights) and the per-sample constants, for argv[2] samples of every
// scenario in the file named by argv[1] (raw aeb_scenario records), on four
// threads as the host sampler runs them.  Built and run by
// tests/test_sanitizers.py (clang++ -fsanitize=address,undefined, plain C++
// against the HIP headers); exit status 0 when every draw is finite where
// its distribution is (the trigger may be +inf: never confirmed).
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "aeb_common.h"

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  const int64_t n = std::atoll(argv[2]);
  aeb_scenario s;
  int k = 0, bad = 0;
  while (std::fread(&s, sizeof(s), 1, f) == 1) {
    std::vector<int> err(4, 0);
    std::vector<double> sum(4, 0.0);
    std::vector<std::thread> th;
    for (int t = 0; t < 4; ++t)
      th.emplace_back([&, t] {
        for (int64_t i = t; i < n; i += 4) {
          const aeb::Sample p = aeb::draw_sample(s, static_cast<uint64_t>(i));
          const aeb::Consts c =
              aeb::derive(s, p.mu, p.mass, p.sin_grade, p.cos_grade, p.cda, p.crr);
          const double v[] = {p.v0, p.mu, p.mass, p.grade, p.sin_grade, p.cos_grade, p.cda,
                              p.crr, p.tau, p.gap, p.lead_decel, p.log_w, c.kd, c.c, c.alim};
          for (double x : v)
            if (!std::isfinite(x)) ++err[t];
          if (std::isnan(p.trigger)) ++err[t];
          sum[t] += p.v0;
        }
      });
    for (auto& t : th) t.join();
    for (int t = 0; t < 4; ++t) bad += err[t];
    std::printf("scenario %d: mean v0 %.4f\n", k, (sum[0] + sum[1] + sum[2] + sum[3]) / n);
    ++k;
  }
  std::fclose(f);
  std::printf("scenarios %d, bad draws %d\n", k, bad);
  return (bad == 0 && k > 0) ? 0 : 1;
}
