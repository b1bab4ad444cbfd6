/* sanitize_oracle.c -- the FP64 reference under AddressSanitizer and
 * UndefinedBehaviorSanitizer: for every scenario in the file named by argv[1]
 * (raw orc_scenario records), validation, the parameter columns, the
 * rollouts and the sort-based statistics (and the weighted estimates) of
 * argv[2] samples.  Built and run by tests/test_sanitizers.py with gcc
 * -fsanitize=address,undefined; exit status 0 when everything ran and every
 * call returned success. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "aeb_oracle.h"

int main(int argc, char** argv) {
  if (argc < 3) return 2;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  const int64_t n = atoll(argv[2]);
  orc_scenario s;
  int k = 0, bad = 0;
  while (fread(&s, sizeof(s), 1, f) == 1) {
    if (orc_validate(&s) != 0) {
      ++bad;
      continue;
    }
    double* cols[13];
    for (int c = 0; c < 13; ++c) cols[c] = malloc(sizeof(double) * n);
    if (orc_sample_range(&s, 0, n, cols) != 0) ++bad;
    double* dist = malloc(sizeof(double) * n);
    double* margin = malloc(sizeof(double) * n);
    uint8_t* status = malloc(n);
    int32_t* steps = malloc(sizeof(int32_t) * n);
    float* vimp = malloc(sizeof(float) * n);
    if (orc_run_range(&s, 0, n, dist, status, steps, margin, vimp) != 0) ++bad;
    if (orc_rollout_given(&s, (const double* const*)cols, n, 0, dist, status, steps, margin,
                          vimp) != 0)
      ++bad;
    orc_reduce_req req = {0};
    req.n_risk = 3;
    req.risk[0] = 0.05;
    req.risk[1] = 0.01;
    req.risk[2] = 0.0;
    req.n_margin_q = 2;
    req.margin_q[0] = 0.0;
    req.margin_q[1] = 0.5;
    req.n_grid = 64;
    req.grid_lo = 20.0;
    req.grid_hi = 140.0;
    orc_stats* st = malloc(sizeof(orc_stats));
    if (orc_reduce(dist, status, margin, vimp, n, &req, st) != 0) ++bad;
    double* w = malloc(sizeof(double) * n);
    for (int64_t i = 0; i < n; ++i) w[i] = exp(cols[12][i]);
    double p[64], se[64], pc, pcs;
    if (orc_weighted_risk(dist, status, w, n, 20.0, 140.0, 64, p, se, &pc, &pcs) != 0) ++bad;
    printf("scenario %d: P(collision) %.4f, mean %.3f\n", k, st->p_collision, st->mean_dist);
    for (int c = 0; c < 13; ++c) free(cols[c]);
    free(dist);
    free(margin);
    free(status);
    free(steps);
    free(vimp);
    free(st);
    free(w);
    ++k;
  }
  fclose(f);
  printf("scenarios %d, failures %d\n", k, bad);
  return (bad == 0 && k > 0) ? 0 : 1;
}
