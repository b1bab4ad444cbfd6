// graph.cpp -- recorded launch sequences (aeb_graph_*): a steady-state rollout
// plus reduction of one scenario, or of a fixed mix of scenarios in one
// batched launch, captured once into a HIP graph and replayed with one
// launch.  The graph owns its device scratch (allocated at creation, so no
// later call can move it) and, for batches, pinned copies of the scenario
// tables that its copy nodes read at every replay.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "aeb_runtime.h"
#include "fast_path.h"
#include "mixgraph.h"

struct aeb_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  char* scratch = nullptr;           // device: rollout scratch, then one reduce scratch per set
  aeb::ScnDev* tab = nullptr;        // pinned (batches)
  aeb_scenario* scns = nullptr;      // pinned (batches)
  std::vector<aeb::OutCols> outs;
  std::vector<int64_t> ns;
  std::vector<size_t> red_off;       // offset of each set's reduce scratch
  size_t tab_off = 0;                // batches: offset of the reduction's set table
  char* rtab_host = nullptr;         // batches: pinned host copy of that table
  aeb_stats* host_stats = nullptr;   // caller's pinned statistics, one per set
  bool reduce = false;
  aeb_reduce_req req{};
  // a recording for changing mixes (aeb_graph_create_mix)
  bool mix = false;
  aeb::MixShape shape;
  aeb::MixBufs mb;
  aeb::MixGraph mg;
  char* mix_dev = nullptr;           // device: tables, rollout and reduction scratch
  char* red_base = nullptr;          // device: the reduction scratch of the sets
  int last_n = 0;                    // the last launched mix
  aeb_stats* last_stats = nullptr;   // where its statistics go (caller's host memory)
};

namespace aeb {
namespace {

size_t up256(size_t b) { return (b + 255) & ~size_t(255); }

bool outputs_ok(const aeb_outputs* o) {
  return o && o->dist && o->status && o->steps && o->margin && o->v_impact;
}

void destroy(aeb_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  if (g->scratch) (void)hipFree(g->scratch);
  if (g->tab) (void)hipHostFree(g->tab);
  if (g->scns) (void)hipHostFree(g->scns);
  if (g->rtab_host) (void)hipHostFree(g->rtab_host);
  if (g->mix) {
    aeb::mix_release(&g->mg);
    if (g->mix_dev) (void)hipFree(g->mix_dev);
    if (g->mb.htab) (void)hipHostFree(g->mb.htab);
    if (g->mb.hrtab) (void)hipHostFree(g->mb.hrtab);
    if (g->mb.hstats) (void)hipHostFree(g->mb.hstats);
  }
  delete g;
}

bool pinned(const void* p) {
  unsigned flags = 0;
  return hipHostGetFlags(&flags, const_cast<void*>(p)) == hipSuccess;
}

// Capture `enqueue` (which queues work on the given stream) into g's graph.
template <typename F>
int capture(aeb_graph* g, F enqueue) {
  hipStream_t st = nullptr;
  AEB_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
  const bool was = timing_suspend(true);
  int rc = AEB_OK;
  if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    rc = fail(AEB_EDEVICE, "hipStreamBeginCapture failed");
  } else {
    rc = enqueue(st);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(st, &graph);
    if (rc == AEB_OK && e != hipSuccess)
      rc = fail(AEB_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    g->graph = graph;
  }
  timing_resume(was);
  (void)hipStreamDestroy(st);
  if (rc != AEB_OK) return rc;
  AEB_HIP(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
  return AEB_OK;
}

// One set: its own reduction.  Several: one segmented reduction over all of
// them (its set table copied from pinned memory by a node of the graph).
int enqueue_reduces(aeb_graph* g, hipStream_t st) {
  if (!g->reduce) return AEB_OK;
  if (g->outs.size() == 1)
    return reduce_enqueue(g->outs[0], g->ns[0], g->req, g->scratch + g->red_off[0],
                          &g->host_stats[0], st);
  std::vector<char*> bases;
  for (size_t j = 0; j < g->outs.size(); ++j) bases.push_back(g->scratch + g->red_off[j]);
  return reduce_enqueue_sets(g->outs.data(), g->ns.data(), static_cast<int>(g->outs.size()),
                             g->req, bases.data(), g->scratch + g->tab_off, g->rtab_host,
                             g->host_stats, st);
}

// the device statistics of set j (where the fallback writes)
aeb_stats* set_stats(aeb_graph* g, size_t j) {
  if (g->outs.size() == 1) return reinterpret_cast<aeb_stats*>(g->scratch + g->red_off[0]);
  return reduce_table_stats(g->scratch + g->tab_off, static_cast<int>(g->outs.size()),
                            g->ns.data()) + j;
}

// lay out the reduce scratch (and, for several sets, the set table) after
// `base` bytes; returns the total (0 if the pinned table cannot be had)
size_t plan_reduces(aeb_graph* g, size_t base) {
  size_t off = up256(base);
  g->red_off.clear();
  if (g->reduce && g->outs.size() > 1) {
    const size_t tb = reduce_table_bytes(static_cast<int>(g->outs.size()), g->ns.data());
    g->tab_off = off;
    off += up256(tb);
    if (hipHostMalloc(reinterpret_cast<void**>(&g->rtab_host), tb, hipHostMallocDefault) !=
        hipSuccess)
      return 0;
  }
  for (size_t j = 0; j < g->outs.size(); ++j) {
    g->red_off.push_back(off);
    if (g->reduce) off += up256(reduce_scratch_bytes(g->ns[j], g->req));
  }
  return off;
}

int check_common(int precision, const aeb_reduce_req* req, aeb_stats* host_stats, bool batch) {
  if (precision != AEB_FP64 && precision != AEB_FP32C && (batch || precision != AEB_FP32C_FIXUP))
    return fail(AEB_EINVAL, batch ? "batched graphs take AEB_FP64 or AEB_FP32C"
                                  : "graphs take AEB_FP64, AEB_FP32C or AEB_FP32C_FIXUP");
  if (req) {
    const int rc = check_reduce_req(*req);
    if (rc != AEB_OK) return rc;
    if (!host_stats || !pinned(host_stats))
      return fail(AEB_EINVAL, "graph statistics need pinned host memory (hipHostMalloc)");
  }
  return AEB_OK;
}

}  // namespace
}  // namespace aeb

using namespace aeb;

extern "C" {

int aeb_graph_create(const aeb_scenario* scn, const aeb_params* params, int precision,
                     const aeb_outputs* out, const aeb_reduce_req* req, aeb_stats* host_stats,
                     aeb_graph** out_graph) {
  if (!out_graph) return fail(AEB_EINVAL, "aeb_graph_create: null output");
  *out_graph = nullptr;
  if (!scn || !outputs_ok(out)) return fail(AEB_EINVAL, "aeb_graph_create: null argument");
  int rc = validate(*scn);
  if (rc != AEB_OK) return rc;
  rc = check_common(precision, req, host_stats, false);
  if (rc != AEB_OK) return rc;
  if (!fast_path_applies(*scn, precision))
    return fail(AEB_EINVAL, "graphs record the block-structured path (not RK4 or the "
                            "closed-loop controller in FP32C, at most 2^31 - 4096 steps)");
  if (out->n != scn->n_samples) return fail(AEB_EINVAL, "outputs length differs from n_samples");
  ParamSrc src{};
  if (params) {
    if (!params->v0 || !params->mu || !params->mass || !params->sin_grade ||
        !params->cos_grade || !params->cda || !params->crr || !params->tau || !params->gap ||
        !params->lead_decel || params->n != scn->n_samples)
      return fail(AEB_EINVAL, "aeb_graph_create: incomplete parameter columns");
    if (scn->is_mask && !params->log_weight)
      return fail(AEB_EINVAL, "aeb_graph_create: importance sampling needs the log_weight column");
    if (perception_on(*scn) && !params->trigger)
      return fail(AEB_EINVAL, "aeb_graph_create: a scenario with perception needs the trigger column");
    src = ParamSrc{params->v0, params->mu,  params->mass, params->sin_grade, params->cos_grade,
                   params->cda, params->crr, params->tau, params->gap, params->lead_decel,
                   params->trigger, params->log_weight};
  }
  aeb_graph* g = new (std::nothrow) aeb_graph;
  if (!g) return fail(AEB_ENOMEM, "host allocation failed");
  g->outs.push_back(OutCols{out->dist, out->status, out->steps, out->margin, out->v_impact,
                                   out->weight});
  g->ns.push_back(scn->n_samples);
  g->reduce = req != nullptr;
  if (req) g->req = *req;
  g->host_stats = host_stats;
  const size_t roll = rollout_scratch_bytes(*scn, scn->n_samples);
  const size_t total = plan_reduces(g, roll);
  if (total == 0 || hipMalloc(reinterpret_cast<void**>(&g->scratch), total) != hipSuccess) {
    destroy(g);
    return fail(AEB_ENOMEM, "graph scratch allocation failed");
  }
  const aeb_scenario s = *scn;
  rc = capture(g, [&](hipStream_t st) {
    int r = launch_rollout_fast_into(s, params ? &src : nullptr, precision, g->outs[0],
                                     s.n_samples, g->scratch, st);
    if (r != AEB_OK) return r;
    return enqueue_reduces(g, st);
  });
  if (rc != AEB_OK) {
    destroy(g);
    return rc;
  }
  *out_graph = g;
  return AEB_OK;
}

int aeb_graph_create_batch(const aeb_scenario* scns, int n_scn, int precision,
                           const aeb_outputs* outs, const aeb_reduce_req* req,
                           aeb_stats* host_stats, aeb_graph** out_graph) {
  if (!out_graph) return fail(AEB_EINVAL, "aeb_graph_create_batch: null output");
  *out_graph = nullptr;
  if (!scns || !outs || n_scn < 1) return fail(AEB_EINVAL, "aeb_graph_create_batch: empty batch");
  int rc = check_common(precision, req, host_stats, true);
  if (rc != AEB_OK) return rc;
  for (int j = 0; j < n_scn; ++j) {
    rc = validate(scns[j]);
    if (rc != AEB_OK) return rc;
    if (!outputs_ok(&outs[j]) || outs[j].n != scns[j].n_samples)
      return fail(AEB_EINVAL, "outputs of scenario " + std::to_string(j) + " do not match it");
    if (scns[j].integrator != scns[0].integrator || scns[j].obstacle != scns[0].obstacle ||
        scns[j].impact_exit != scns[0].impact_exit || scns[j].nofma != scns[0].nofma)
      return fail(AEB_EINVAL, "batched scenarios must share integrator, obstacle, impact_exit, nofma");
  }
  for (int j = 0; j < n_scn; ++j)
    if (!fast_path_applies(scns[j], precision) || control_on(scns[j]))
      return fail(AEB_EINVAL, "batched graphs record the batched block-structured path (not "
                              "RK4 in FP32C, not the closed-loop controller, at most 2^31 - 4096 "
                              "steps)");
  aeb_graph* g = new (std::nothrow) aeb_graph;
  if (!g) return fail(AEB_ENOMEM, "host allocation failed");
  for (int j = 0; j < n_scn; ++j) {
    g->outs.push_back(
        OutCols{outs[j].dist, outs[j].status, outs[j].steps, outs[j].margin, outs[j].v_impact,
                    outs[j].weight});
    g->ns.push_back(scns[j].n_samples);
  }
  g->reduce = req != nullptr;
  if (req) g->req = *req;
  g->host_stats = host_stats;
  if (hipHostMalloc(reinterpret_cast<void**>(&g->tab), sizeof(ScnDev) * n_scn,
                    hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&g->scns), sizeof(aeb_scenario) * n_scn,
                    hipHostMallocDefault) != hipSuccess) {
    destroy(g);
    return fail(AEB_ENOMEM, "pinned table allocation failed");
  }
  std::memcpy(g->scns, scns, sizeof(aeb_scenario) * n_scn);
  int64_t total = 0, cap = 1;
  rc = fill_batch_table(g->scns, n_scn, g->outs.data(), g->tab, &total, &cap);
  if (rc != AEB_OK) {
    destroy(g);
    return rc;
  }
  const bool lead = scns[0].obstacle == AEB_OBS_LEAD;
  const size_t roll = batch_scratch_bytes(total, n_scn, lead);
  const size_t bytes = plan_reduces(g, roll);
  if (bytes == 0 || hipMalloc(reinterpret_cast<void**>(&g->scratch), bytes) != hipSuccess) {
    destroy(g);
    return fail(AEB_ENOMEM, "graph scratch allocation failed");
  }
  rc = capture(g, [&](hipStream_t st) {
    int r = launch_batch_fast_into(g->scns, n_scn, precision, g->tab, total, cap, g->scratch, st);
    if (r != AEB_OK) return r;
    return enqueue_reduces(g, st);
  });
  if (rc != AEB_OK) {
    destroy(g);
    return rc;
  }
  *out_graph = g;
  return AEB_OK;
}

int aeb_graph_create_mix(const aeb_scenario* kind, int precision, int max_scn,
                         int64_t max_samples, const aeb_reduce_req* req, aeb_graph** out_graph) {
  if (!out_graph) return fail(AEB_EINVAL, "aeb_graph_create_mix: null output");
  *out_graph = nullptr;
  if (!kind) return fail(AEB_EINVAL, "aeb_graph_create_mix: null kind");
  if (precision != AEB_FP64 && precision != AEB_FP32C)
    return fail(AEB_EINVAL, "mix graphs take AEB_FP64 or AEB_FP32C");
  if (max_scn < 1 || max_scn > 65536 || max_samples < 1 || max_samples > 0xffffffffLL)
    return fail(AEB_EINVAL, "mix capacity outside 1..65536 scenarios, 1..2^32-1 samples");
  int rc = validate(*kind);
  if (rc != AEB_OK) return rc;
  if (!fast_path_applies(*kind, precision) || control_on(*kind))
    return fail(AEB_EINVAL, "mix graphs record the batched block-structured path (not RK4 "
                            "in FP32C, not the closed-loop controller)");
  if (req) {
    rc = check_reduce_req(*req);
    if (rc != AEB_OK) return rc;
  }
  aeb_graph* g = new (std::nothrow) aeb_graph;
  if (!g) return fail(AEB_ENOMEM, "host allocation failed");
  g->mix = true;
  MixShape& m = g->shape;
  m.kind = *kind;
  m.perception = perception_on(*kind);
  m.precision = precision;
  m.cap_scn = max_scn;
  m.cap_total = max_samples;
  m.reduce = req != nullptr;
  m.weighted = kind->is_mask != 0;
  if (req) m.req = *req;
  const size_t tb = up256(mix_table_bytes(max_scn));
  const size_t sb = up256(mix_scratch_bytes(m));
  const size_t rb = req ? up256(reduce_table_bytes_cap(max_scn, max_samples)) : 0;
  const size_t rs = req ? up256(reduce_scratch_bytes_cap(max_scn, max_samples, *req)) : 0;
  if (hipMalloc(reinterpret_cast<void**>(&g->mix_dev), tb + sb + rb + rs) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&g->mb.htab), tb, hipHostMallocDefault) !=
          hipSuccess ||
      (req && (hipHostMalloc(reinterpret_cast<void**>(&g->mb.hrtab), rb, hipHostMallocDefault) !=
                   hipSuccess ||
               hipHostMalloc(reinterpret_cast<void**>(&g->mb.hstats),
                             sizeof(aeb_stats) * max_scn, hipHostMallocDefault) != hipSuccess))) {
    destroy(g);
    return fail(AEB_ENOMEM, "mix graph allocation failed");
  }
  g->mb.dtab = g->mix_dev;
  g->mb.scratch = g->mix_dev + tb;
  g->mb.drtab = req ? g->mix_dev + tb + sb : nullptr;
  g->red_base = req ? g->mix_dev + tb + sb + rb : nullptr;
  rc = mix_record(m, g->mb, &g->mg);
  if (rc != AEB_OK) {
    destroy(g);
    return rc;
  }
  *out_graph = g;
  return AEB_OK;
}

int aeb_graph_launch_mix(aeb_graph* g, const aeb_scenario* scns, int n_scn,
                         const aeb_outputs* outs, aeb_stats* host_stats, void* stream) {
  if (!g || !g->mix) return fail(AEB_EINVAL, "aeb_graph_launch_mix: not a mix graph");
  if (!scns || !outs || n_scn < 1) return fail(AEB_EINVAL, "aeb_graph_launch_mix: empty mix");
  if (g->shape.reduce && !host_stats)
    return fail(AEB_EINVAL, "aeb_graph_launch_mix: the graph computes statistics: host_stats");
  if (g->last_n != 0)
    return fail(AEB_EINVAL, "aeb_graph_launch_mix: the previous replay was not finished "
                            "(aeb_graph_finish) and may still read the tables");
  std::vector<OutCols> oc(n_scn);
  std::vector<int64_t> ns(n_scn);
  std::vector<char*> bases(n_scn);
  char* p = g->red_base;
  for (int j = 0; j < n_scn; ++j) {
    int rc = validate(scns[j]);
    if (rc != AEB_OK) return fail(rc, "scenario " + std::to_string(j) + ": " + aeb_last_error());
    if (!outputs_ok(&outs[j]) || outs[j].n != scns[j].n_samples)
      return fail(AEB_EINVAL, "outputs of scenario " + std::to_string(j) + " do not match it");
    if (control_on(scns[j]) || !fast_path_applies(scns[j], g->shape.precision))
      return fail(AEB_EINVAL, "scenario " + std::to_string(j) + " does not take the batched path");
    oc[j] = OutCols{outs[j].dist, outs[j].status, outs[j].steps, outs[j].margin, outs[j].v_impact,
                    outs[j].weight};
    ns[j] = scns[j].n_samples;
    bases[j] = p;
    if (g->shape.reduce) p += up256(reduce_scratch_bytes(ns[j], g->shape.req));
  }
  // the graph's previous replay must have finished reading the pinned tables
  // (aeb_graph_finish, or any sync of its stream, orders that)
  int rc = mix_fill(g->shape, scns, n_scn, oc.data(), bases.data(), g->mb);
  if (rc != AEB_OK) return rc;
  AEB_HIP(hipGraphLaunch(g->mg.exec, static_cast<hipStream_t>(stream)));
  g->outs = oc;
  g->ns = ns;
  g->red_off.clear();
  for (int j = 0; j < n_scn; ++j) g->red_off.push_back(static_cast<size_t>(bases[j] - g->red_base));
  g->last_n = n_scn;
  g->last_stats = host_stats;
  return AEB_OK;
}

int aeb_graph_launch(aeb_graph* g, void* stream) {
  if (g && g->mix) return fail(AEB_EINVAL, "aeb_graph_launch: a mix graph takes aeb_graph_launch_mix");
  if (!g || !g->exec) return fail(AEB_EINVAL, "aeb_graph_launch: null graph");
  AEB_HIP(hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream)));
  return AEB_OK;
}

int aeb_graph_finish(aeb_graph* g, void* stream) {
  if (!g) return fail(AEB_EINVAL, "aeb_graph_finish: null graph");
  hipStream_t st = static_cast<hipStream_t>(stream);
  AEB_HIP(hipStreamSynchronize(st));
  if (g->mix) {
    if (!g->shape.reduce) return AEB_OK;
    aeb_stats* dst = reduce_table_stats_cap(g->mb.drtab, g->shape.cap_scn, g->shape.cap_total);
    for (int j = 0; j < g->last_n; ++j) {
      aeb_stats& s = g->mb.hstats[j];
      if (s.reserved) {
        const int rc = reduce_fallback(g->outs[j], g->ns[j], g->shape.req,
                                       g->red_base + g->red_off[j], dst + j, &s, st);
        if (rc != AEB_OK) return rc;
      }
      s.reserved = 0;
      g->last_stats[j] = s;
    }
    g->last_n = 0;
    return AEB_OK;
  }
  if (!g->reduce) return AEB_OK;
  for (size_t j = 0; j < g->outs.size(); ++j) {
    aeb_stats& s = g->host_stats[j];
    if (s.reserved) {
      const int rc = reduce_fallback(g->outs[j], g->ns[j], g->req, g->scratch + g->red_off[j],
                                     set_stats(g, j), &s, st);
      if (rc != AEB_OK) return rc;
    }
    s.reserved = 0;
  }
  return AEB_OK;
}

int aeb_graph_destroy(aeb_graph* g) {
  destroy(g);
  return AEB_OK;
}

}  // extern "C"
