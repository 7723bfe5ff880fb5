// Host-side graph preparation (no device code).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace bcx {

enum VertexKind : int32_t { kKept = 0, kPendant = 1, kK2 = 2, kIsolated = 3, kTree = 4 };

// Result of the 1-degree reduction: omega (vertices folded into each kept
// vertex), the kind of every vertex, the neighbour of each pendant, and the
// residual graph G' on the same ids (pruned vertices keep empty rows).
//
// With `trees` (the reduction iterated until no degree-1 vertex is left) a
// removed vertex u hangs from parent[u]; its subtree (u and everything that
// hangs below it) has sub[u] vertices; core[u] is the kept vertex at the
// top of its tree and top[u] the child of core[u] whose subtree holds u.
// Components that are trees are removed whole (core = -1, top = the tree's
// root, which has parent -1).  omega(v) of a kept vertex is the size of the forest hanging
// from it; comp[v] is the size of v's component in the original graph.
struct Pruned {
  std::vector<int32_t> omega, kind, hub, rp, ci;
  bool trees = false;
  std::vector<int32_t> parent, core, top, order;  // order: removed vertices, children before parents
  std::vector<int64_t> sub, comp;
};

// A traversal source: vertex v of the traversed graph, the number of
// requested sources its sweep stands for (itself and/or sources folded into
// it), how many of those are folded vertices, and the sum over those of the
// size of the subtree of v's that holds them (1 per pendant).  The sweep's
// own term is own * (n_v - 1) - tsub: each folded source a reaches every
// vertex of v's component through v except v and its own subtree.
struct Group {
  int32_t v;
  double w;
  int32_t own;
  int32_t slot = 0;  // result array the sweep's contributions go to
  double tsub = 0.0;
};

// A 2-degree vertex c whose sweep is derived from its neighbours a and b
// (indices into the group list).
struct Triple {
  int32_t a, b, c;
};

bool validate_csr(int32_t n, const int32_t* rp, const int32_t* ci, int64_t nnz, std::string* why);
void prune_deg1(int32_t n, const int32_t* rp, const int32_t* ci, Pruned* out);
// The reduction iterated: degree-1 vertices are peeled until none is left.
void prune_trees(int32_t n, const int32_t* rp, const int32_t* ci, Pruned* out);
// RAW scores of the removed vertices of an iterated reduction for a source
// multiset (src == nullptr: every vertex), added to out[n]: a removed vertex
// is a cut vertex, so it lies on every shortest path between two of the
// components it separates and on no other.
void tree_scores(int32_t n, const Pruned& p, const int32_t* src, int64_t k, double* out);
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
