// Host-side graph preparation: CSR validation, the 1-degree reduction
// (Sec. 3.4.1, Alg. 6), mapping requested sources onto traversal sources
// with weights (Sec. 2.2, Eq. (4)-(5)), and the choice of 2-degree vertices
// whose forward sweep is derived from their neighbours' (Sec. 3.4.2).
#include "bc_host.h"

#include <algorithm>
#include <cstdio>
#include <cstring>

namespace bcx {

bool validate_csr(int32_t n, const int32_t* rp, const int32_t* ci, int64_t nnz, std::string* why) {
  char buf[256];
  if (n < 0) { *why = "n < 0"; return false; }
  if (nnz < 0 || nnz > INT32_MAX) { *why = "nnz out of range (must fit int32)"; return false; }
  if (rp[0] != 0) { *why = "row_ptr[0] != 0"; return false; }
  if ((int64_t)rp[n] != nnz) {
    snprintf(buf, sizeof buf, "row_ptr[n] = %d but nnz = %lld", rp[n], (long long)nnz);
    *why = buf;
    return false;
  }
  for (int32_t v = 0; v < n; ++v) {
    if (rp[v + 1] < rp[v]) {
      snprintf(buf, sizeof buf, "row_ptr decreases at vertex %d", v);
      *why = buf;
      return false;
    }
  }
  for (int32_t v = 0; v < n; ++v) {
    for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
      const int32_t w = ci[e];
      if (w < 0 || w >= n) {
        snprintf(buf, sizeof buf, "vertex %d has neighbour id %d outside [0, n)", v, w);
        *why = buf;
        return false;
      }
      if (w == v) {
        snprintf(buf, sizeof buf, "self-loop at vertex %d", v);
        *why = buf;
        return false;
      }
    }
  }
  // duplicates: sort a copy of each row; symmetry: every (v, w) has (w, v)
  std::vector<int32_t> row;
  std::vector<int64_t> fill(rp, rp + n);  // cursor per vertex for the transpose
  std::vector<int32_t> tr((size_t)nnz);
  for (int32_t v = 0; v < n; ++v) {
    row.assign(ci + rp[v], ci + rp[v + 1]);
    std::sort(row.begin(), row.end());
    for (size_t i = 1; i < row.size(); ++i) {
      if (row[i] == row[i - 1]) {
        snprintf(buf, sizeof buf, "duplicate edge (%d, %d)", v, row[i]);
        *why = buf;
        return false;
      }
    }
    for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
      const int32_t w = ci[e];
      if (fill[w] >= rp[w + 1]) {
        snprintf(buf, sizeof buf, "asymmetric: vertex %d has more in-edges than out-edges", w);
        *why = buf;
        return false;
      }
      tr[(size_t)fill[w]++] = v;
    }
  }
  // the transpose rows must equal the rows as sets
  for (int32_t v = 0; v < n; ++v) {
    row.assign(ci + rp[v], ci + rp[v + 1]);
    std::vector<int32_t> t(tr.begin() + rp[v], tr.begin() + rp[v + 1]);
    std::sort(row.begin(), row.end());
    std::sort(t.begin(), t.end());
    if (row != t) {
      snprintf(buf, sizeof buf, "asymmetric adjacency at vertex %d", v);
      *why = buf;
      return false;
    }
  }
  return true;
}

void prune_deg1(int32_t n, const int32_t* rp, const int32_t* ci, Pruned* out) {
  out->omega.assign((size_t)n, 0);
  out->kind.assign((size_t)n, 0);
  out->hub.assign((size_t)n, -1);
  auto deg = [&](int32_t v) { return rp[v + 1] - rp[v]; };
  for (int32_t u = 0; u < n; ++u) {
    const int32_t du = deg(u);
    if (du == 0) { out->kind[u] = kIsolated; continue; }
    if (du != 1) continue;
    const int32_t v = ci[rp[u]];
    if (deg(v) >= 2) {
      out->kind[u] = kPendant;
      out->hub[u] = v;
      out->omega[v] += 1;
    } else {
      out->kind[u] = kK2;
    }
  }
  out->rp.assign((size_t)n + 1, 0);
  out->ci.clear();
  out->ci.reserve((size_t)rp[n]);
  for (int32_t v = 0; v < n; ++v) {
    if (out->kind[v] == kKept) {
      for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
        const int32_t w = ci[e];
        if (out->kind[w] == kKept) out->ci.push_back(w);
      }
    }
    out->rp[v + 1] = (int32_t)out->ci.size();
  }
}

void prune_trees(int32_t n, const int32_t* rp, const int32_t* ci, Pruned* out) {
  out->trees = true;
  out->omega.assign((size_t)n, 0);
  out->kind.assign((size_t)n, kKept);
  out->hub.assign((size_t)n, -1);
  out->parent.assign((size_t)n, -1);
  out->core.assign((size_t)n, -1);
  out->top.assign((size_t)n, -1);
  out->sub.assign((size_t)n, 1);
  out->comp.assign((size_t)n, 0);
  out->order.clear();
  std::vector<int32_t> deg((size_t)n), queue;
  for (int32_t v = 0; v < n; ++v) {
    deg[v] = rp[v + 1] - rp[v];
    if (deg[v] == 0) out->kind[v] = kIsolated;
    if (deg[v] == 1) queue.push_back(v);
  }
  // peel: a vertex left with one neighbour hangs from it; a vertex left with
  // none is the last vertex of a tree component (its root)
  for (size_t h = 0; h < queue.size(); ++h) {
    const int32_t u = queue[h];
    if (out->kind[u] != kKept || deg[u] != 1) continue;
    int32_t p = -1;
    for (int32_t e = rp[u]; e < rp[u + 1]; ++e)
      if (out->kind[ci[e]] == kKept) { p = ci[e]; break; }
    out->kind[u] = kTree;
    out->parent[u] = p;
    out->order.push_back(u);
    out->sub[p] += out->sub[u];
    if (--deg[p] == 1) queue.push_back(p);
    if (deg[p] == 0) {
      out->kind[p] = kTree;  // root of a tree component
      out->order.push_back(p);
    }
  }
  // component sizes of the original graph
  std::vector<int32_t> stack;
  std::vector<char> seen((size_t)n, 0);
  std::vector<int32_t> members;
  for (int32_t s = 0; s < n; ++s) {
    if (seen[s]) continue;
    members.clear();
    stack.assign(1, s);
    seen[s] = 1;
    while (!stack.empty()) {
      const int32_t v = stack.back();
      stack.pop_back();
      members.push_back(v);
      for (int32_t e = rp[v]; e < rp[v + 1]; ++e)
        if (!seen[ci[e]]) { seen[ci[e]] = 1; stack.push_back(ci[e]); }
    }
    for (int32_t v : members) out->comp[v] = (int64_t)members.size();
  }
  // the kept vertex each tree hangs from, and the top child holding each
  // removed vertex (parents before children: reverse removal order)
  for (size_t i = out->order.size(); i-- > 0;) {
    const int32_t u = out->order[i];
    const int32_t p = out->parent[u];
    if (p < 0) {  // root of a tree component: top names it for every vertex of that tree
      out->top[u] = u;
    } else if (out->kind[p] == kKept) {
      out->core[u] = p;
      out->top[u] = u;
    } else {
      out->core[u] = out->core[p];
      out->top[u] = out->top[p];
    }
  }
  for (int32_t v = 0; v < n; ++v)
    if (out->kind[v] == kKept) out->omega[v] = (int32_t)(out->sub[v] - 1);
  out->rp.assign((size_t)n + 1, 0);
  out->ci.clear();
  out->ci.reserve((size_t)rp[n]);
  for (int32_t v = 0; v < n; ++v) {
    if (out->kind[v] == kKept)
      for (int32_t e = rp[v]; e < rp[v + 1]; ++e)
        if (out->kind[ci[e]] == kKept) out->ci.push_back(ci[e]);
    out->rp[v + 1] = (int32_t)out->ci.size();
  }
}

void tree_scores(int32_t n, const Pruned& p, const int32_t* src, int64_t k, double* out) {
  // cnt[v]: requested sources in v's subtree (v's own multiplicity included)
  std::vector<double> cnt((size_t)n, src ? 0.0 : 1.0);
  if (src)
    for (int64_t i = 0; i < k; ++i) cnt[src[i]] += 1.0;
  // requested sources per component, keyed by a representative: the kept
  // vertex a tree hangs from, or a tree component's root
  auto rep = [&](int32_t v) { return p.kind[v] == kKept ? v : (p.core[v] >= 0 ? p.core[v] : p.top[v]); };
  std::vector<double> in_comp((size_t)n, 0.0);
  if (src) {
    // per component: sum over its vertices; kept vertices of one component
    // are connected through kept vertices only, so label them first
    std::vector<int32_t> lab((size_t)n, -1), stack;
    for (int32_t s = 0; s < n; ++s) {
      if (p.kind[s] != kKept || lab[s] >= 0) continue;
      lab[s] = s;
      stack.assign(1, s);
      while (!stack.empty()) {
        const int32_t v = stack.back();
        stack.pop_back();
        for (int32_t e = p.rp[v]; e < p.rp[v + 1]; ++e)
          if (lab[p.ci[e]] < 0) { lab[p.ci[e]] = s; stack.push_back(p.ci[e]); }
      }
    }
    for (int64_t i = 0; i < k; ++i) {
      const int32_t v = src[i];
      if (p.kind[v] == kIsolated) continue;
      const int32_t r = rep(v);
      in_comp[p.kind[r] == kKept ? lab[r] : r] += 1.0;
    }
    for (int32_t v = 0; v < n; ++v)
      if (p.kind[v] == kKept) in_comp[v] = in_comp[lab[v]];
  }
  for (int32_t u : p.order) {
    const int32_t par = p.parent[u];
    if (par >= 0) cnt[par] += cnt[u];
  }
  // sum over the children c of each removed vertex of cnt[c] (N - 1 - sub[c])
  std::vector<double> child((size_t)n, 0.0);
  for (int32_t u : p.order) {
    const int32_t par = p.parent[u];
    if (par >= 0 && p.kind[par] == kTree) child[par] += cnt[u] * (double)(p.comp[u] - 1 - p.sub[u]);
  }
  for (int32_t u : p.order) {
    const double N = (double)p.comp[u];
    double total;
    if (!src) {
      total = N;  // every vertex of the component is a source
    } else {
      total = in_comp[rep(u)];
    }
    // sources outside u's subtree reach the sub[u] - 1 vertices below u through it
    const double outside = total - cnt[u];
    out[u] += outside * (double)(p.sub[u] - 1) + child[u];
  }
}

void map_sources(int32_t n, const int32_t* rp, const Pruned* pr, const int32_t* src, int64_t k,
                 std::vector<Group>* groups, int64_t* credited) {
  std::vector<double> w((size_t)n, 0.0), tsub((size_t)n, 0.0);
  std::vector<int32_t> own((size_t)n, 0);
  std::vector<char> seen((size_t)n, 0);
  std::vector<int32_t> order;
  int64_t cred = 0;
  auto add = [&](int32_t v, double wt, int32_t ow, double ts) {
    if (!seen[v]) { seen[v] = 1; order.push_back(v); }
    w[v] += wt;
    own[v] += ow;
    tsub[v] += ts;
  };
  for (int64_t i = 0; i < k; ++i) {
    const int32_t s = src ? src[i] : (int32_t)i;
    if (rp[s + 1] == rp[s]) continue;  // isolated: no pairs
    ++cred;
    if (!pr) { add(s, 1.0, 0, 0.0); continue; }
    switch (pr->kind[s]) {
      case kKept: add(s, 1.0, 0, 0.0); break;
      case kPendant: add(pr->hub[s], 1.0, 1, 1.0); break;
      case kTree:
        // served by the sweep of the kept vertex its tree hangs from; a tree
        // component is scored on the host alone
        if (pr->core[s] >= 0) add(pr->core[s], 1.0, 1, (double)pr->sub[pr->top[s]]);
        break;
      default: break;  // ends of 2-vertex components: no inner vertices
    }
  }
  groups->clear();
  groups->reserve(order.size());
  for (int32_t v : order) groups->push_back(Group{v, w[v], own[v], 0, tsub[v]});
  *credited = cred;
}

void choose_deg2(int32_t n, const int32_t* rp, const int32_t* ci, std::vector<Group>& groups,
                 std::vector<Triple>* triples) {
  triples->clear();
  // Derived vertices: c of degree 2 whose two neighbours are requested
  // sources of the same result slot that are traversed (never derived
  // themselves).  A neighbour may serve several derived vertices; every
  // cluster (derived vertices and their partners, joined through shared
  // partners) must fit one 64-lane word.  Greedy in source order.
  int nslot = 1;
  for (const auto& gr : groups) nslot = std::max(nslot, gr.slot + 1);
  const size_t G = groups.size();
  std::vector<int32_t> gi((size_t)n, -1), uf(G), size(G, 1);
  std::vector<char> role(G, 0);  // 1 partner, 2 derived
  for (size_t i = 0; i < G; ++i) uf[i] = (int32_t)i;
  auto find = [&](int32_t x) {
    while (uf[x] != x) x = uf[x] = uf[uf[x]];
    return x;
  };
  for (int sl = 0; sl < nslot; ++sl) {
    for (size_t i = 0; i < G; ++i)
      if (groups[i].slot == sl) gi[groups[i].v] = (int32_t)i;
    for (size_t i = 0; i < G; ++i) {
      if (groups[i].slot != sl || role[i] != 0) continue;
      const int32_t c = groups[i].v;
      if (rp[c + 1] - rp[c] != 2) continue;
      const int32_t ia = gi[ci[rp[c]]], ib = gi[ci[rp[c] + 1]];
      if (ia < 0 || ib < 0 || role[ia] == 2 || role[ib] == 2) continue;
      const int32_t ra = find(ia), rb = find(ib);
      const int32_t merged = (ra == rb ? size[ra] : size[ra] + size[rb]) + 1;
      if (merged > 64) continue;
      role[i] = 2;
      role[ia] = role[ib] = 1;
      uf[ra] = (int32_t)i;
      if (rb != ra) uf[rb] = (int32_t)i;
      size[i] = merged;
      triples->push_back(Triple{ia, ib, (int32_t)i});
    }
    for (size_t i = 0; i < G; ++i)
      if (groups[i].slot == sl) gi[groups[i].v] = -1;
  }
}

std::vector<int32_t> locality_rank(int32_t n, const int32_t* rp, const int32_t* ci) {
  std::vector<int32_t> rank((size_t)n, -1), queue;
  queue.reserve((size_t)n);
  int32_t next = 0;
  auto bfs = [&](int32_t s) {
    rank[s] = next++;
    size_t head = queue.size();
    queue.push_back(s);
    while (head < queue.size()) {
      const int32_t v = queue[head++];
      for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
        const int32_t x = ci[e];
        if (rank[x] < 0) {
          rank[x] = next++;
          queue.push_back(x);
        }
      }
    }
  };
  int32_t hub = 0;
  for (int32_t v = 1; v < n; ++v)
    if (rp[v + 1] - rp[v] > rp[hub + 1] - rp[hub]) hub = v;
  if (n > 0) bfs(hub);
  for (int32_t v = 0; v < n; ++v)
    if (rank[v] < 0) bfs(v);
  return rank;
}

void order_groups(const std::vector<int32_t>& rank, std::vector<Group>& groups) {
  std::stable_sort(groups.begin(), groups.end(), [&](const Group& a, const Group& b) {
    if (a.slot != b.slot) return a.slot < b.slot;
    return rank[a.v] < rank[b.v];
  });
}

}  // namespace bcx
