// One source per workgroup (BC_MODE_PER_WORKGROUP): launch arguments and
// entry points of the per-workgroup kernel.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace bcx {

// Packed adjacency slot per vertex (kEllWidth ints, 32-byte aligned): the
// degree, then the neighbours in row order when there are at most
// kEllWidth - 1 of them, else the row's start in the CSR column array.
constexpr int kEllWidth = 8;

// Per-source state of one vertex, one 16-byte record so that a neighbour
// test and its count or dependency share one cache line: lvl = level + 1
// (0: not reached), e = exponent of the extended count, val = the count
// (uint64, or the fp64 significand of the extended form) until the backward
// sweep replaces it with psi = (1 + delta + omega) / sigma (fp64 bits).
struct alignas(16) WgVert {
  int32_t lvl;
  int32_t e;
  uint64_t val;
};

// Per-workgroup slices: n vertex records, the stacked level queue (n
// entries of {vertex, successor mask}) and its n + 2 level offsets; the
// sources and their weights for the launch.
struct WgArgs {
  int32_t n;
  const int32_t* ell;         // [n][kEllWidth] packed adjacency
  const int32_t* ci;          // CSR columns (rows longer than kEllWidth - 1)
  const int32_t* omega;
  WgVert* vs;                 // [grid][n], all zero between sources
  int2* Q;                    // [grid][n]: vertex and a neighbour mask: bit j (j < 31) for
                              // the j-th neighbour being a predecessor (extended counts,
                              // from the pull) until the vertex's claim pass, a successor
                              // after it (bit 31: a successor at some j >= 31)
  int32_t* qoff;              // [grid][n + 2]
  const int32_t* src;         // [nsrc] sources, weights, own counts and subtree sums
  const double* w;
  const int32_t* own;
  const double* tsub;
  int64_t nsrc;
  double* const* sbc;         // [nsrc] the score array each source's contributions go to
  int32_t* ovf_list;          // [nsrc] sources whose exact count wrapped
  int32_t* ovf_count;
  unsigned long long* stats;  // kSt* counters
};

hipError_t launch_wg(const WgArgs& a, bool ext, int grid, hipStream_t st);
hipError_t wg_max_grid(int* blocks_per_cu);  // resident workgroups per CU, both count forms

}  // namespace bcx
