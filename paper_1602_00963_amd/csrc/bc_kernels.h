// Kernel argument blocks and launchers (host-visible).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bc_common.h"

namespace bcx {

// Global run counters accumulated by the kernels (device, uint64 each).
enum StatIdx : int {
  kStLevels = 0,
  kStBuLevels = 1,
  kStReached = 2,
  kStReachedNnz = 3,
  kStDag = 4,
  kStLaunches = 5,
  kStCount = 8
};

struct PlainArgs {
  int32_t n;
  int64_t nnz;
  const int32_t* rp;
  const int32_t* ci;
  const int32_t* omega;       // pendants per vertex, or null
  const int2* gu;             // static units (vertex, chunk) of every vertex with edges
  int32_t ngu;
  int32_t* d;
  uint64_t* sig;              // exact counts
  double* sm;                 // extended counts: significand
  int32_t* se;                //                  exponent
  double* psi;                // (1 + delta + omega) / sigma  (extended: over the significand)
  int32_t* Q;
  Unit* U;
  int32_t* qoff;
  int32_t* uoff;
  LevelCtr* lc;
  double* part_m;
  int32_t* part_e;
  int32_t* arrive;
  int32_t* gmulti;
  int32_t* err;
  int32_t* ovf_now;           // set when a count wraps in this launch
  int32_t* ovf_list;          // sources that wrapped (host reruns them extended)
  int32_t* ovf_count;
  uint64_t* ns;               // component size accumulator (1-degree own term)
  unsigned long long* stats;  // StatIdx counters
  GridBar* bar;
  uint64_t bar_limit;         // wall-clock ticks a grid-barrier wait may last
  double* bc;
  double* delta_out;          // per-vertex delta of this source (trace), or null
  int32_t src;
  int32_t own;                // folded sources (pendants, tree vertices) represented by this launch
  double tsub;                // sum over them of the size of src's subtree that holds them
  double weight;              // sources represented by src's sweep
  double alpha;
  double beta;                // stay bottom-up while frontier vertices * beta >= n (0: no hysteresis)
  int32_t cap_entries, cap_units, cap_parts, cap_multi, cap_levels;
};

// Level lists of the batched kernel hold (vertex, word) entries: entry
// (v, k) is in level l's list when some lane of word k has v on level l.
// Q entries are k << 32 | v.
__host__ __device__ inline uint64_t bentry(int32_t v, int k) { return ((uint64_t)k << 32) | (uint32_t)v; }

// A work unit of the batched kernel: edges [beg, end) of vertex v (degree
// deg), for the 64 sources of word k, belonging to level-list entry e;
// an entry of degree > 256 spans several units (chunk c) that combine their
// partial sums in slots pb + c.
struct BUnit {
  int32_t v, beg, end, deg;
  int32_t k, c, e, pb;
};

struct BatchArgs {
  int32_t n;
  int64_t nnz;
  int32_t K;                  // 64-lane words per vertex (batch = 64 K)
  const int32_t* rp;
  const int32_t* ci;
  const int32_t* omega;
  const int2* gu;             // static units (vertex, chunk) for bottom-up levels
  int32_t ngu;
  int32_t* lv;                // [n][64K] level per (vertex, lane), kept for traces only
  int32_t keep_lv;            // write lv (traces)
  uint64_t* sig;              // [n][64K] exact counts; psi overwrites them in the backward sweep
  double* sm;                 // [n][64K] extended significand (psi overwrites)
  int32_t* se;                // [n][64K] extended exponent
  uint64_t* vis;              // [n][K] lanes that reached the vertex
  uint64_t* fm;               // [4][n][K] rotating per-level lane masks
  uint64_t* Q;                // (vertex, word) entries, level after level
  BUnit* U;                   // their work units
  int32_t* qoff;              // [levels] first entry of each level
  int32_t* uoff;              // [levels] first unit of each level
  LevelCtr* lc;               // [levels] append counters
  double* part_m;             // [slot][64] partial sums of split entries (slots level-relative)
  int32_t* part_e;
  int32_t* arrive;            // [entries] arrival counters of split entries
  uint64_t* emask;            // [entries] lanes of the entry's word on its level, set when counted
  int32_t* err;
  uint32_t* lane_ovf;         // [64K] lanes whose count wrapped
  int32_t* ovf_list;          // sources of wrapped lanes, appended per batch (host reruns them)
  int32_t* ovf_count;
  int32_t* fail_list;         // sources of batches that hit a list capacity (host reruns them)
  int32_t* fail_count;
  unsigned long long* lane_ns;// [64K] component sizes (1-degree own term)
  unsigned long long* stats;
  double* delta_out;          // trace: [64K][n] dependencies, or null
  uint64_t* sig_out;          // trace: [64K][n] counts copied before the backward sweep, or null
  double* sm_out;             // trace (extended)
  int32_t* se_out;
  // batch description (device arrays, 64K entries each)
  const int32_t* lane_src;    // source vertex of each lane, -1 = inactive
  const double* lane_w;       // sources represented by the lane's sweep
  const int32_t* lane_own;    // folded sources represented (own term)
  const double* lane_tsub;    // sum over them of the size of the lane source's subtree that holds them
  const int8_t* lane_pa;      // derived lanes: partner lanes (same word), -1 if traversed
  const int8_t* lane_pb;
  double* const* slot_bc;     // per-slot score arrays (device), up to 64
  const int16_t* lane_pair;   // [64K] (word, slot) pair of each lane
  const int8_t* pair_slot;    // [npairs] slot of each pair; pairs are numbered in word order
  int32_t npairs, cap_pairs;
  double* pair_bc;            // [cap_pairs][n] per-pair sums of one launch, zero between launches
  const uint64_t* edge_lanes; // [K] lanes that propagate along edges (active, not derived)
  const uint64_t* derived_lanes; // [K] lanes derived from two partner lanes of their word
  uint64_t* dla;              // [n][K] derived lanes c with d_a(v) <= d_b(v) at v (a, b: c's partners)
  uint64_t* dlb;              // [n][K] derived lanes c with d_b(v) <= d_a(v)
  int32_t has_derived;        // any lane derived from two partner lanes
  int32_t has_own;            // any lane with pendant sources (component sizes needed)
  unsigned long long* fulledges; // edges x words whose word's edge lanes have all reached the vertex
  GridBar* bar;
  uint64_t bar_limit;         // wall-clock ticks a grid-barrier wait may last
  int32_t clear_at_end;       // clear the masks before returning (off for traces)
  double alpha;
  double beta;                // stay bottom-up while frontier entries * beta >= n * words (0: no hysteresis)
  int32_t cap_entries, cap_units, cap_parts, cap_levels;
};

constexpr int kBatchChunk = 256;
constexpr int kMaxWords = 16;    // batches of up to 1024 sources
constexpr int kBatchBlock = 1024; // threads per workgroup of the batched kernel (one per CU)
constexpr int kPlainChunkHost = 64;

// One source per launch with the paper's active-edge mapping (prefix sum of
// frontier degrees + binary search per edge, prefix sums reused backward).
struct ScanArgs {
  int32_t n;
  const int32_t* rp;
  const int32_t* ci;
  int32_t* d;
  uint64_t* sig;
  double* psi;                // (1 + delta) / sigma of finished vertices
  double* acc;                // backward accumulators
  int32_t* Q;                 // frontiers, level after level
  int32_t* qoff;              // [levels + 2] level starts; qoff[l + 2] counts level l+1's appends meanwhile
  int64_t* cd;                // [n] exclusive prefix sum of degrees within each level (aligned with Q)
  int64_t* tot;               // [levels] edges of each level's frontier
  int64_t* bsum;              // [grid] chunk totals of the scan
  int32_t* err;
  int32_t* ovf_now;
  int32_t* ovf_list;
  int32_t* ovf_count;
  unsigned long long* stats;
  GridBar* bar;
  uint64_t bar_limit;
  double* bc;
  double* delta_out;
  int32_t src;
  double weight;
};

hipError_t launch_plain(const PlainArgs& a, bool ext, int grid, int block, hipStream_t st);
hipError_t launch_scan(const ScanArgs& a, int grid, hipStream_t st);
hipError_t scan_max_grid(int* blocks_per_cu);
hipError_t plain_max_grid(bool ext, int block, int* blocks_per_cu);

hipError_t launch_batch(const BatchArgs& a, bool ext, int grid, int block, hipStream_t st);
hipError_t batch_max_grid(bool ext, int block, int* blocks_per_cu);

}  // namespace bcx
