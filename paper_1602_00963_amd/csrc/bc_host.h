// Host-side graph preparation (no device code).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace bcx {

enum VertexKind : int32_t { kKept = 0, kPendant = 1, kK2 = 2, kIsolated = 3 };

// Result of the 1-degree reduction: omega (pendants per vertex), the kind of
// every vertex, the neighbour of each pendant, and the residual graph G' on
// the original ids (pruned vertices keep empty rows).
struct Pruned {
  std::vector<int32_t> omega, kind, hub, rp, ci;
};

// A traversal source: vertex v of the traversed graph, the number of
// requested sources its sweep stands for (itself and/or its pendants), and
// how many of those are pendants (the own term omega * (n_v - 2) per pendant).
struct Group {
  int32_t v;
  double w;
  int32_t own;
  int32_t slot = 0;  // result array the sweep's contributions go to
};

// A 2-degree vertex c whose sweep is derived from its neighbours a and b
// (indices into the group list).
struct Triple {
  int32_t a, b, c;
};

bool validate_csr(int32_t n, const int32_t* rp, const int32_t* ci, int64_t nnz, std::string* why);
void prune_deg1(int32_t n, const int32_t* rp, const int32_t* ci, Pruned* out);
// src == nullptr means every vertex 0..k-1.  `credited` = requested
// sources that are not isolated.
void map_sources(int32_t n, const int32_t* rp, const Pruned* pr, const int32_t* src, int64_t k,
                 std::vector<Group>* groups, int64_t* credited);
// Locality ranking of the vertices for batching: breadth-first discovery
// order, starting from the highest-degree vertex, then each remaining
// component.  Sources adjacent in this order are close in the graph, so the
// 64 sources of a word sit on nearby levels of every vertex.
std::vector<int32_t> locality_rank(int32_t n, const int32_t* rp, const int32_t* ci);

// Orders groups by (result slot, rank of their vertex).
void order_groups(const std::vector<int32_t>& rank, std::vector<Group>& groups);

void choose_deg2(int32_t n, const int32_t* rp, const int32_t* ci, std::vector<Group>& groups,
                 std::vector<Triple>* triples);

}  // namespace bcx
