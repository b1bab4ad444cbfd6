// mixgraph.h -- one recorded launch sequence for changing mixes of scenarios.
//
// A mix is up to cap_scn scenarios of one kind (integrator, obstacle,
// impact_exit, nofma) with cap_total samples in all (a mix recorded with
// per-sample command steps also takes scenarios without perception):
// the batched rollout of all of them, then (optionally) the segmented
// reduction of their outputs.  Every kernel's grid covers the capacity and
// reads the mix's actual sizes from device tables, and the tables themselves
// are copied from pinned host memory by the first nodes of the sequence, so
// one recording (a HIP graph) replays any mix that fits: the host rewrites
// the pinned tables, then launches the graph.  Results equal those of the
// eager batched launch (and of each scenario alone) bit for bit.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "aeb_runtime.h"
#include "fast_path.h"

namespace aeb {

// Buffers of a mix launch (all sized for the capacity; the library never
// frees them here).
struct MixBufs {
  char* dtab = nullptr;        // device: BatchHdr | ScnDev[cap] | aeb_scenario[cap]
  char* htab = nullptr;        // pinned host: the same layout
  char* scratch = nullptr;     // device: mix_scratch_bytes
  char* drtab = nullptr;       // device: reduction table (reduce_table_bytes_cap)
  char* hrtab = nullptr;       // pinned host: the same
  aeb_stats* hstats = nullptr; // pinned host: cap statistics
};

struct MixShape {
  aeb_scenario kind{};   // integrator, obstacle, impact_exit, nofma of the mix
  bool perception = false;   // per-sample command steps (any scenario with perception)
  int precision = AEB_FP64;
  int cap_scn = 1;
  int64_t cap_total = 1;
  bool reduce = false;
  bool weighted = false;
  aeb_reduce_req req{};
};

size_t mix_table_bytes(int cap_scn);
size_t mix_scratch_bytes(const MixShape& m);

// Write a mix into the pinned tables (scenario table, and with a reduction
// its set table, set j's reduction scratch at red_bases[j]).
int mix_fill(const MixShape& m, const aeb_scenario* scns, int n_scn, const OutCols* outs,
             char* const* red_bases, const MixBufs& b);

// Queue the whole sequence on `st` (capturable: copies from pinned memory
// and kernel launches only).
int mix_enqueue(const MixShape& m, const MixBufs& b, hipStream_t st);

// A recording of mix_enqueue.
struct MixGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};
int mix_record(const MixShape& m, const MixBufs& b, MixGraph* g);
void mix_release(MixGraph* g);

// Whether a scenario can join a mix of this shape.
bool mix_fits(const MixShape& m, const aeb_scenario& s);

}  // namespace aeb
