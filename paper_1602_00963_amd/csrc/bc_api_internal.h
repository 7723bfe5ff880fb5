// Internal entry points shared by the C ABI and the serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/bc.h"
#include "bc_host.h"

namespace bcx {

bc_status fail(bc_status st, const std::string& msg);

// Launch state of one caller: an event pool that times each kernel launch
// on its stream, and pinned host staging for the batches' lane tables.  A
// graph owns one for bc_compute / bc_trace / bc_autotune (which run under
// the graph's lock), each server worker owns its own.  It is released
// explicitly by its owner, never by a static or thread-local destructor:
// those run at process exit, after the HIP runtime (or a profiler attached
// to it) may already have shut down.
struct Exec {
  std::vector<hipEvent_t> ev;
  size_t used = 0;
  char* stage = nullptr;
  size_t stage_bytes = 0;
  hipError_t mark(hipStream_t st);     // records the next event of the pool on st
  hipError_t collect(double* ms);      // after the stream was waited for: adds the pairs' durations
  bc_status tables(size_t bytes, char** out);  // pinned staging of at least `bytes`
  void release();
};

// Options after defaults and checks.
struct Resolved {
  int mode, B, K, block, grid_per_cu, sigma_mode;
  bool deg1, deg2;
  double alpha;
  double beta = 0.0;    // bottom-up hysteresis (0 = none)
  int cap_factor = 32;  // batched level-list capacity: n * min(B, cap_factor) entries
  int max_slots = 1;    // result slots one batch may feed (the server packs up to 64)
  int grid_total = 0;   // cap on the persistent grid's workgroups (the server's share of the device); 0 = none
  bool trace = false;   // parity traces: per-lane levels are kept (extra n * B int32)
  bool no_alloc = false;  // bc_compute_noalloc: no events, counters cleared by a fill kernel
  int graph_launches = 0;  // plain form: per-source launches captured per HIP graph (0 = none)
};
bc_status resolve_opts(const bc_graph* g, const bc_compute_opts* o, Resolved* r);
void graph_groups(const bc_graph* g, const Resolved& r, const int32_t* sources, int64_t k, std::vector<Group>* groups,
                  int64_t* credited);
bc_status compute_groups(bc_graph* g, const Resolved& r, std::vector<Group>& groups, int64_t credited,
                         void* workspace, size_t ws_bytes, hipStream_t st, double* const* slots, int nslots,
                         Exec* ex, bc_run_stats* stats);
int64_t graph_n(const bc_graph* g);
int context_device(const bc_context* c);
int context_cus(const bc_context* c);
// A score array from the library's internal vertex order to the caller's, in place.
void scores_to_caller(const bc_graph* g, double* a);
// Closed-form scores of the vertices removed by the iterated reduction for a
// source list (caller ids), in the caller's order; empty unless the graph
// was loaded with BC_LOAD_PRUNE_TREES.
void tree_scores_caller(const bc_graph* g, const int32_t* sources, int64_t k, std::vector<double>* out);
bool graph_pruned(const bc_graph* g);
int64_t graph_nnz(const bc_graph* g);
int graph_device(const bc_graph* g);
size_t graph_ws_bytes(const bc_graph* g, const Resolved& r);
// Workgroups per CU the batched kernel can keep resident (both count forms).
int batch_occupancy(int K);

// The entry point that allocates nothing (bc_static.hip): the size of its
// fixed device scratch array, the per-device lookup of that array's address,
// a fill kernel that clears device memory, and the compute path it runs
// (the plain form, workspace = the scratch array).
constexpr size_t kNoAllocScratchBytes = 64ull << 20;
hipError_t noalloc_scratch_init(int device);
hipError_t zero_async(void* p, size_t bytes, hipStream_t st);
bc_status compute_noalloc(bc_graph* g, const int32_t* sources, int64_t k, const bc_compute_opts* opts, void* scratch,
                          size_t scratch_bytes, hipStream_t st, bc_run_stats* stats);

}  // namespace bcx
