// mixgraph.cpp -- the launch sequence of a mix of scenarios laid out for a
// capacity, its host-side table filling and its recording as a HIP graph.
#include "mixgraph.h"

#include <cstring>
#include <string>
#include <vector>

namespace aeb {
namespace {

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

struct TabOffs {
  size_t tab, scns, total;
};

TabOffs tab_offs(int cap_scn) {
  TabOffs o;
  o.tab = up256(sizeof(BatchHdr));
  o.scns = up256(o.tab + sizeof(ScnDev) * cap_scn);
  o.total = up256(o.scns + sizeof(aeb_scenario) * cap_scn);
  return o;
}

}  // namespace

size_t mix_table_bytes(int cap_scn) { return tab_offs(cap_scn).total; }

size_t mix_scratch_bytes(const MixShape& m) {
  return batch_scratch_bytes(m.cap_total, 0, m.kind.obstacle == AEB_OBS_LEAD);
}

bool mix_fits(const MixShape& m, const aeb_scenario& s) {
  return s.integrator == m.kind.integrator && s.obstacle == m.kind.obstacle &&
         s.impact_exit == m.kind.impact_exit && s.nofma == m.kind.nofma &&
         (m.perception || !perception_on(s)) && (m.weighted || s.is_mask == 0);
}

int mix_fill(const MixShape& m, const aeb_scenario* scns, int n_scn, const OutCols* outs,
             char* const* red_bases, const MixBufs& b) {
  if (n_scn < 1 || n_scn > m.cap_scn) return fail(AEB_EINVAL, "mix: scenario count beyond capacity");
  for (int j = 0; j < n_scn; ++j)
    if (!mix_fits(m, scns[j]))
      return fail(AEB_EINVAL, "mix: scenario " + std::to_string(j) + " is of another kind");
  const TabOffs o = tab_offs(m.cap_scn);
  BatchHdr* hdr = reinterpret_cast<BatchHdr*>(b.htab);
  ScnDev* tab = reinterpret_cast<ScnDev*>(b.htab + o.tab);
  aeb_scenario* hs = reinterpret_cast<aeb_scenario*>(b.htab + o.scns);
  std::memcpy(hs, scns, sizeof(aeb_scenario) * n_scn);
  int64_t total = 0, cap = 1;
  int rc = fill_batch_table(hs, n_scn, outs, tab, &total, &cap);
  if (rc != AEB_OK) return rc;
  if (total > m.cap_total) return fail(AEB_EINVAL, "mix: more samples than the capacity");
  hdr->total = total;
  hdr->cap = static_cast<float>(cap);
  hdr->n_scn = n_scn;
  if (!m.reduce) return AEB_OK;
  std::vector<int64_t> ns(n_scn);
  for (int j = 0; j < n_scn; ++j) ns[j] = scns[j].n_samples;
  return reduce_fill_sets_cap(outs, ns.data(), n_scn, m.cap_scn, m.cap_total, red_bases, b.drtab,
                              b.hrtab);
}

int mix_enqueue(const MixShape& m, const MixBufs& b, hipStream_t st) {
  const TabOffs o = tab_offs(m.cap_scn);
  // the header and scenario table, then the scenarios (only the capacity's
  // entries that a mix can use)
  AEB_HIP(hipMemcpyAsync(b.dtab, b.htab, o.total, hipMemcpyHostToDevice, st));
  int rc = launch_batch_fast_dev(m.kind, m.perception, m.precision,
                                 reinterpret_cast<const BatchHdr*>(b.dtab),
                                 reinterpret_cast<const ScnDev*>(b.dtab + o.tab),
                                 reinterpret_cast<const aeb_scenario*>(b.dtab + o.scns), m.cap_scn,
                                 m.cap_total, b.scratch, st);
  if (rc != AEB_OK || !m.reduce) return rc;
  return reduce_enqueue_sets_cap(m.cap_scn, m.cap_total, m.req, m.weighted, b.drtab, b.hrtab,
                                 b.hstats, st);
}

int mix_record(const MixShape& m, const MixBufs& b, MixGraph* g) {
  hipStream_t st = nullptr;
  AEB_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  const bool was = timing_suspend(true);
  int rc = AEB_OK;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = fail(AEB_EDEVICE, "hipStreamBeginCapture failed");
  } else {
    rc = mix_enqueue(m, b, st);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc == AEB_OK && e != hipSuccess)
      rc = fail(AEB_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    g->graph = graph;
  }
  timing_resume(was);
  (void)hipStreamDestroy(st);
  if (rc == AEB_OK && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
    rc = fail(AEB_EDEVICE, "hipGraphInstantiate failed");
  if (rc != AEB_OK) mix_release(g);
  return rc;
}

void mix_release(MixGraph* g) {
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  g->exec = nullptr;
  g->graph = nullptr;
}

}  // namespace aeb
