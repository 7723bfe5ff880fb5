// C ABI of the library: graph residency, workspace layout, the plain and
// batched launchers, parity traces and host-side checks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <array>
#include <atomic>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bc.h"
#include "bc_api_internal.h"
#include "bc_host.h"
#include "bc_kernels.h"
#include "bc_plain.h"
#include "bc_wg.h"

using namespace bcx;

static thread_local std::string g_err;

bc_status bcx::fail(bc_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HIPCHK(x)                                                                             \
  do {                                                                                        \
    hipError_t e_ = (x);                                                                      \
    if (e_ != hipSuccess) return fail(BC_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
  } while (0)

namespace {

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Sequential carving of a workspace; with base == nullptr it only sizes.
struct Carve {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

constexpr int kTableBatches = 256;  // lane tables uploaded per group of batches

int64_t plain_cap_units(int64_t n, int64_t nnz) { return n + nnz / kPlainChunkHost + 64; }
int64_t plain_cap_parts(int64_t n, int64_t nnz) { return n + nnz / kPlainChunkHost + 64; }

struct PlainWs {
  int32_t *d, *se, *Q, *qoff, *uoff, *part_e, *arrive, *gmulti, *err, *ovf_now, *ovf_list, *ovf_count;
  uint64_t *sig, *ns;
  double *sm, *psi, *part_m, *delta, *bc_tmp;
  Unit* U;
  LevelCtr* lc;
  unsigned long long* stats;
  GridBar* bar;
  size_t ctl_bytes;  // bytes from `lc` through the control scalars (zeroed per call)
  char* ctl_begin;
};

size_t plain_layout(int64_t n, int64_t nnz, char* base, PlainWs* w) {
  Carve c{base};
  PlainWs t{};
  t.d = c.take<int32_t>(n);
  t.sig = c.take<uint64_t>(n);
  t.sm = c.take<double>(n);
  t.se = c.take<int32_t>(n);
  t.psi = c.take<double>(n);
  t.Q = c.take<int32_t>(n);
  t.U = c.take<Unit>(plain_cap_units(n, nnz));
  t.qoff = c.take<int32_t>(n + 3);
  t.uoff = c.take<int32_t>(n + 3);
  t.part_m = c.take<double>(plain_cap_parts(n, nnz));
  t.part_e = c.take<int32_t>(plain_cap_parts(n, nnz));
  t.arrive = c.take<int32_t>(n);
  t.ovf_list = c.take<int32_t>(n + 1);
  t.delta = c.take<double>(n);
  t.bc_tmp = c.take<double>(n);
  c.off = align_up(c.off, 256);
  const size_t ctl0 = c.off;
  t.lc = c.take<LevelCtr>(n + 3);
  t.gmulti = c.take<int32_t>(1);
  t.err = c.take<int32_t>(1);
  t.ovf_now = c.take<int32_t>(1);
  t.ovf_count = c.take<int32_t>(1);
  t.ns = c.take<uint64_t>(1);
  t.stats = c.take<unsigned long long>(kStCount);
  t.bar = c.take<GridBar>(1);
  c.off = align_up(c.off, 256);
  t.ctl_bytes = c.off - ctl0;
  t.ctl_begin = base ? base + ctl0 : nullptr;
  if (w) *w = t;
  return c.off;
}

struct ScanWs {
  int32_t *d, *Q, *qoff, *err, *ovf_now, *ovf_list, *ovf_count;
  uint64_t* sig;
  double *psi, *acc, *delta, *bc_tmp;
  int64_t *cd, *tot, *bsum;
  unsigned long long* stats;
  GridBar* bar;
  size_t ctl_bytes;
  char* ctl_begin;
};

constexpr int kScanMaxGrid = 4096;

size_t scan_layout(int64_t n, char* base, ScanWs* w) {
  Carve c{base};
  ScanWs t{};
  t.d = c.take<int32_t>(n);
  t.sig = c.take<uint64_t>(n);
  t.psi = c.take<double>(n);
  t.acc = c.take<double>(n);
  t.Q = c.take<int32_t>(n);
  t.qoff = c.take<int32_t>(n + 3);
  t.cd = c.take<int64_t>(n);
  t.tot = c.take<int64_t>(n + 1);
  t.bsum = c.take<int64_t>(kScanMaxGrid);
  t.ovf_list = c.take<int32_t>(n + 1);
  t.delta = c.take<double>(n);
  t.bc_tmp = c.take<double>(n);
  c.off = align_up(c.off, 256);
  const size_t ctl0 = c.off;
  t.err = c.take<int32_t>(1);
  t.ovf_now = c.take<int32_t>(1);
  t.ovf_count = c.take<int32_t>(1);
  t.stats = c.take<unsigned long long>(kStCount);
  t.bar = c.take<GridBar>(1);
  c.off = align_up(c.off, 256);
  t.ctl_bytes = c.off - ctl0;
  t.ctl_begin = base ? base + ctl0 : nullptr;
  if (w) *w = t;
  return c.off;
}

// Per-workgroup workspace: grid slices of the per-source state, the call's
// source table, the overflow list and counters.
struct WgWs {
  WgVert* vs;
  int2* Q;
  int32_t *qoff, *src, *own, *ovf_list, *ovf_count;
  double *w, *tsub;
  double** sbc;  // per source: the score array its contributions go to
  unsigned long long* stats;
  size_t ctl_bytes;
  char* ctl_begin;
};

constexpr size_t kWgStateBudget = 64ull << 30;  // bytes of per-workgroup state at most

// Workgroups of the per-workgroup mode: per_cu per compute unit (default:
// as many as fit), fewer when their state would pass kWgStateBudget.
int wg_grid(int64_t n, int cus, int per_cu, int total) {
  int bpc = 1;
  if (wg_max_grid(&bpc) != hipSuccess || bpc < 1) bpc = 1;
  const int want = per_cu > 0 ? std::min(per_cu, bpc) : bpc;
  const size_t per = (sizeof(WgVert) + sizeof(int2) + 4) * (size_t)n + 64;
  const int64_t fit = (int64_t)std::max<size_t>(1, kWgStateBudget / per);
  int64_t grid = std::min<int64_t>((int64_t)cus * want, fit);
  if (total > 0) grid = std::min<int64_t>(grid, total);  // a server worker's share
  return (int)std::max<int64_t>(1, grid);
}

size_t wg_layout(int64_t n, int grid, int64_t nsrc, char* base, WgWs* w) {
  Carve c{base};
  WgWs t{};
  const size_t gn = (size_t)grid * (size_t)n;
  t.vs = c.take<WgVert>(gn);
  t.Q = c.take<int2>(gn);
  t.qoff = c.take<int32_t>((size_t)grid * (size_t)(n + 2));
  t.src = c.take<int32_t>(std::max<int64_t>(nsrc, 1));
  t.own = c.take<int32_t>(std::max<int64_t>(nsrc, 1));
  t.w = c.take<double>(std::max<int64_t>(nsrc, 1));
  t.tsub = c.take<double>(std::max<int64_t>(nsrc, 1));
  t.sbc = c.take<double*>(std::max<int64_t>(nsrc, 1));
  t.ovf_list = c.take<int32_t>(std::max<int64_t>(nsrc, 1));
  c.off = align_up(c.off, 256);
  const size_t ctl0 = c.off;
  t.ovf_count = c.take<int32_t>(1);
  t.stats = c.take<unsigned long long>(kStCount);
  c.off = align_up(c.off, 256);
  t.ctl_bytes = c.off - ctl0;
  t.ctl_begin = base ? base + ctl0 : nullptr;
  if (w) *w = t;
  return c.off;
}

struct BatchCaps {
  int64_t entries, units, parts, multi;
};

// Level-list capacities of the batched kernel.  A (vertex, word) entry sits
// on at most min(64, depth + 1) levels (one per distinct distance of the
// word's sources); lists are sized for min(64, cap_factor) of them, and a
// batch that runs out is rerun with the worst case.
BatchCaps batch_caps(int64_t n, int64_t nnz, int B, int cap_factor) {
  const int64_t K = B / 64;
  const int64_t f = std::min<int64_t>(64, cap_factor);
  BatchCaps c;
  c.entries = std::min<int64_t>(n * K * f + 1024, (int64_t)INT32_MAX / 2);
  c.units = std::min<int64_t>(c.entries + nnz * K * f / kBatchChunk + 1024, (int64_t)INT32_MAX / 2);
  c.parts = std::min<int64_t>(K * (2 * nnz / kBatchChunk) + 1024, (int64_t)INT32_MAX / 2);  // per level
  c.multi = c.entries;
  return c;
}

struct BatchWs {
  int32_t *lv, *se, *qoff, *uoff, *part_e, *arrive, *err, *ovf_list, *ovf_count;
  int32_t *fail_list, *fail_count;
  uint64_t *sig, *vis, *fm, *Q, *emask;
  double *part_m, *pair_bc;
  BUnit* U;
  LevelCtr* lc;
  uint32_t* lane_ovf;
  unsigned long long *lane_ns, *stats, *fulledges;
  GridBar* bar;
  size_t mask_bytes;   // vis + fm + dla + dlb, cleared per call
  uint64_t *dla, *dlb;
  int32_t cap_pairs;   // (word, slot) pair arrays
  char* tables;        // kTableBatches lane tables
  size_t table_bytes;  // bytes of one table
  size_t ctl_bytes;
  char* ctl_begin;
  BatchCaps caps;
};

// One batch's lane table: lane_src[B], lane_own[B], l0[B] (int32), lane_w[B],
// lane_tsub[B] (double), lane_pair[B] (int16), lane_pa[B], lane_pb[B], lane_slot[B]
// (int8), pair_slot[kMaxPairs] (int8), then 8-aligned edge_lanes[16], derived_lanes[16]
// (uint64) and slot_bc[64] (device pointers).
constexpr int kMaxSlots = 64;
constexpr int kMaxPairs = kMaxWords + kMaxSlots;
size_t table_bytes(int B) {
  return align_up((size_t)B * (4 + 4 + 4 + 8 + 8 + 2 + 1 + 1 + 1) + kMaxPairs + 8 + 16 * kMaxWords + 8 * kMaxSlots, 256);
}

// Lanes are packed slot by slot, so the slots met along the words are
// non-decreasing and a batch has at most K + slots - 1 (word, slot) pairs.
int32_t cap_pairs_for(int K, int max_slots) { return K + std::min(max_slots, kMaxSlots) - 1; }

size_t batch_layout(int64_t n, int64_t nnz, int B, int cap_factor, int max_slots, bool with_lv, char* base,
                    BatchWs* w) {
  const int K = B / 64;
  Carve c{base};
  BatchWs t{};
  t.caps = batch_caps(n, nnz, B, cap_factor);
  t.lv = with_lv ? c.take<int32_t>((size_t)n * B) : nullptr;  // per-lane levels: traces only
  t.sig = c.take<uint64_t>((size_t)n * B);
  t.se = c.take<int32_t>((size_t)n * B);
  t.vis = c.take<uint64_t>((size_t)n * K * 7);  // vis, the four level-mask arrays, dla, dlb
  t.fm = t.vis ? t.vis + (size_t)n * K : nullptr;
  t.dla = t.vis ? t.vis + (size_t)n * K * 5 : nullptr;
  t.dlb = t.vis ? t.vis + (size_t)n * K * 6 : nullptr;
  t.mask_bytes = sizeof(uint64_t) * (size_t)n * K * 7;
  t.Q = c.take<uint64_t>(t.caps.entries);
  t.U = c.take<BUnit>(t.caps.units);
  t.qoff = c.take<int32_t>(n + 3);
  t.uoff = c.take<int32_t>(n + 3);
  t.part_m = c.take<double>((size_t)t.caps.parts * 64);
  t.part_e = c.take<int32_t>((size_t)t.caps.parts * 64);
  t.arrive = c.take<int32_t>(t.caps.entries);
  t.emask = c.take<uint64_t>(t.caps.entries);
  t.cap_pairs = cap_pairs_for(K, max_slots);
  t.pair_bc = c.take<double>((size_t)t.cap_pairs * n);
  t.ovf_list = c.take<int32_t>(n + 1);
  t.fail_list = c.take<int32_t>(n + 1);
  t.table_bytes = table_bytes(B);
  t.tables = c.take<char>(t.table_bytes * kTableBatches);
  c.off = align_up(c.off, 256);
  const size_t ctl0 = c.off;
  t.lc = c.take<LevelCtr>(n + 3);
  t.err = c.take<int32_t>(1);
  t.ovf_count = c.take<int32_t>(1);
  t.fail_count = c.take<int32_t>(1);
  t.lane_ovf = c.take<uint32_t>(B);
  t.lane_ns = c.take<unsigned long long>(B);
  t.fulledges = c.take<unsigned long long>(1);
  t.stats = c.take<unsigned long long>(kStCount);
  t.bar = c.take<GridBar>(1);
  c.off = align_up(c.off, 256);
  t.ctl_bytes = c.off - ctl0;
  t.ctl_begin = base ? base + ctl0 : nullptr;
  if (w) *w = t;
  return c.off;
}

}  // namespace

// ------------------------------------------------------------------ objects

// A batched-mode setting chosen by bc_autotune.
struct TunedSet {
  int32_t batch = 0, grid = 0;
  double alpha = 0.0, beta = 0.0;
};
using ShapeKey = std::array<int64_t, 5>;

struct bc_context {
  int device = 0;
  int cus = 0;
  std::string arch;
  uint64_t bar_ticks = 0;  // longest grid-barrier wait, in ticks of the device's wall clock
  std::mutex tune_mu;
  std::map<ShapeKey, TunedSet> tune_cache;  // bc_autotune results by graph shape
};

struct bc_graph {
  bc_context* ctx = nullptr;
  int32_t n = 0;
  int64_t nnz = 0;
  bool pruned = false;
  std::vector<int32_t> h_rp, h_ci;  // the graph on internal ids (host copy)
  // internal id of each caller vertex id (empty: the caller's order is kept)
  std::vector<int32_t> perm;
  Pruned pr;
  // device: original graph and (if pruned) the residual graph G'
  int32_t *d_rp = nullptr, *d_ci = nullptr, *d_rrp = nullptr, *d_rci = nullptr, *d_omega = nullptr;
  int2 *d_gu_p = nullptr, *d_gu_b = nullptr, *d_rgu_p = nullptr, *d_rgu_b = nullptr;
  int32_t ngu_p = 0, ngu_b = 0, nrgu_p = 0, nrgu_b = 0;
  double* d_bc = nullptr;
  std::atomic<int64_t> resident{0};  // device bytes held (read by bc_graph_stats_get without the lock)
  int64_t max_degree = 0, isolated = 0, pendants = 0, k2 = 0, deg2 = 0, rnnz = 0, tree = 0;
  int64_t bfs_depth = 0;  // eccentricity of a highest-degree vertex (a lower bound on the diameter)
  // scores of the vertices removed by the iterated reduction (host, internal
  // order), accumulated like the device scores until bc_scores_reset
  std::vector<double> h_tree;
  // library-owned cached workspace
  void* ws = nullptr;
  size_t ws_bytes = 0;
  // batched-mode setting chosen by bc_autotune
  bool tuned = false;
  int32_t tuned_batch = 0, tuned_grid = 0;
  double tuned_alpha = 0.0, tuned_beta = 0.0;
  // batching order of sources (computed on the first batched call)
  std::vector<int32_t> rank;
  std::once_flag rank_once;
  std::atomic<bool> ext_hint{false};   // an exact-count probe on this graph found most sources wrapping
  std::mutex ell_mu;                   // packed adjacency of the full / residual graph, built on first use
  int32_t* d_ell[2] = {nullptr, nullptr};
  Exec exec;  // launch timing and lane-table staging of calls made under `mu`
  std::mutex mu;
};

namespace bcx {

// Static units (vertex, chunk) of every vertex with edges.
static std::vector<int2> static_units(int32_t n, const int32_t* rp, int chunk) {
  std::vector<int2> u;
  for (int32_t v = 0; v < n; ++v) {
    const int32_t dg = rp[v + 1] - rp[v];
    if (dg == 0) continue;
    const int32_t nu = (dg + chunk - 1) / chunk;
    for (int32_t c = 0; c < nu; ++c) u.push_back(make_int2(v, c));
  }
  return u;
}

template <class T>
static bc_status upload(const std::vector<T>& h, T** d, std::atomic<int64_t>* resident) {
  const size_t bytes = std::max<size_t>(h.size(), 1) * sizeof(T);
  HIPCHK(hipMalloc((void**)d, bytes));
  if (!h.empty()) HIPCHK(hipMemcpy(*d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  *resident += (int64_t)bytes;
  return BC_OK;
}

// Number of levels below v in a breadth-first search from v.
static int64_t bfs_depth_from(int32_t n, const int32_t* rp, const int32_t* ci, int32_t v) {
  std::vector<int32_t> lvl((size_t)n, -1), q;
  q.reserve((size_t)n);
  q.push_back(v);
  lvl[v] = 0;
  for (size_t h = 0; h < q.size(); ++h)
    for (int32_t e = rp[q[h]]; e < rp[q[h] + 1]; ++e)
      if (lvl[ci[e]] < 0) {
        lvl[ci[e]] = lvl[q[h]] + 1;
        q.push_back(ci[e]);
      }
  return lvl[q.back()];
}

// Rewrites the CSR in the vertex order `order` (order[i] = the vertex placed
// at position i); perm[caller id] = internal id.  Rows stay sorted.
static void relabel(int32_t n, std::vector<int32_t>& rp, std::vector<int32_t>& ci, const std::vector<int32_t>& order,
                    std::vector<int32_t>* perm) {
  perm->assign((size_t)n, 0);
  for (int32_t i = 0; i < n; ++i) (*perm)[order[i]] = i;
  std::vector<int32_t> nrp((size_t)n + 1, 0), nci(ci.size());
  for (int32_t i = 0; i < n; ++i) {
    const int32_t v = order[i];
    int32_t o = nrp[i];
    for (int32_t e = rp[v]; e < rp[v + 1]; ++e) nci[o++] = (*perm)[ci[e]];
    std::sort(nci.begin() + nrp[i], nci.begin() + o);
    nrp[i + 1] = o;
  }
  rp.swap(nrp);
  ci.swap(nci);
}

// The default internal order: decreasing degree, ties by the caller's id.
// The vertices touched most often (hubs: every edge to them reads their
// level masks and counts) then share cache lines at the low ids instead of
// being spread over the arrays.
static std::vector<int32_t> degree_order(int32_t n, const std::vector<int32_t>& rp) {
  std::vector<int32_t> order((size_t)n);
  for (int32_t v = 0; v < n; ++v) order[v] = v;
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return rp[a + 1] - rp[a] > rp[b + 1] - rp[b]; });
  return order;
}

// Reverse Cuthill-McKee: per connected component a breadth-first order from
// a pseudo-peripheral vertex (George-Liu: repeat a BFS from a least-degree
// vertex of the last level while the eccentricity grows), neighbours taken
// by increasing degree; the whole sequence reversed.  Vertices adjacent in
// the graph land close together, which on long-diameter graphs keeps large
// runs of a BFS wavefront in consecutive records.
static std::vector<int32_t> rcm_order(int32_t n, const std::vector<int32_t>& rp, const std::vector<int32_t>& ci) {
  auto deg = [&](int32_t v) { return rp[v + 1] - rp[v]; };
  std::vector<int32_t> by_deg((size_t)n);
  for (int32_t v = 0; v < n; ++v) by_deg[v] = v;
  std::stable_sort(by_deg.begin(), by_deg.end(), [&](int32_t a, int32_t b) { return deg(a) < deg(b); });
  std::vector<char> placed((size_t)n, 0);
  std::vector<int32_t> lvl((size_t)n, -1), q, order, nb;
  order.reserve((size_t)n);
  for (int32_t s0 : by_deg) {
    if (placed[s0]) continue;
    int32_t root = s0, ecc = -1;
    for (int it = 0; it < 8; ++it) {  // pseudo-peripheral root
      q.assign(1, root);
      lvl[root] = 0;
      for (size_t h = 0; h < q.size(); ++h)
        for (int32_t e = rp[q[h]]; e < rp[q[h] + 1]; ++e)
          if (lvl[ci[e]] < 0) {
            lvl[ci[e]] = lvl[q[h]] + 1;
            q.push_back(ci[e]);
          }
      const int32_t depth = lvl[q.back()];
      int32_t best = q.back();
      for (size_t h = q.size(); h-- > 0 && lvl[q[h]] == depth;)
        if (deg(q[h]) < deg(best) || (deg(q[h]) == deg(best) && q[h] < best)) best = q[h];
      for (int32_t v : q) lvl[v] = -1;
      if (depth <= ecc) break;
      ecc = depth;
      root = best;
    }
    const size_t start = order.size();
    order.push_back(root);
    placed[root] = 1;
    for (size_t h = start; h < order.size(); ++h) {
      const int32_t v = order[h];
      nb.clear();
      for (int32_t e = rp[v]; e < rp[v + 1]; ++e)
        if (!placed[ci[e]]) {
          placed[ci[e]] = 1;
          nb.push_back(ci[e]);
        }
      std::sort(nb.begin(), nb.end(), [&](int32_t a, int32_t b) { return deg(a) != deg(b) ? deg(a) < deg(b) : a < b; });
      order.insert(order.end(), nb.begin(), nb.end());
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

// Caller ids -> internal ids.
static std::vector<int32_t> to_internal(const bc_graph* g, const int32_t* src, int64_t k) {
  std::vector<int32_t> out(src, src + k);
  if (!g->perm.empty())
    for (auto& v : out) v = g->perm[v];
  return out;
}

// Each of `rows` rows of n values from internal to caller order, in place.
template <class T>
static void rows_to_caller(const bc_graph* g, T* a, int64_t rows) {
  if (g->perm.empty() || !a) return;
  const int64_t n = g->n;
  std::vector<T> tmp((size_t)n);
  for (int64_t r = 0; r < rows; ++r) {
    T* row = a + r * n;
    for (int64_t v = 0; v < n; ++v) tmp[v] = row[g->perm[v]];
    std::copy(tmp.begin(), tmp.end(), row);
  }
}

void scores_to_caller(const bc_graph* g, double* a) { rows_to_caller(g, a, 1); }

// Scores of the vertices the iterated reduction removed (closed form, host),
// for internal source ids (nullptr: all), added to the graph's accumulator.
static void add_tree_scores(bc_graph* g, const Resolved& r, const int32_t* isrc, int64_t k) {
  if (!r.deg1 || !g->pr.trees) return;
  if (g->h_tree.empty()) g->h_tree.assign((size_t)g->n, 0.0);
  tree_scores(g->n, g->pr, isrc, isrc ? k : g->n, g->h_tree.data());
}

void tree_scores_caller(const bc_graph* g, const int32_t* sources, int64_t k, std::vector<double>* out) {
  out->clear();
  if (!g->pruned || !g->pr.trees) return;
  const std::vector<int32_t> isrc = to_internal(g, sources, k);
  out->assign((size_t)g->n, 0.0);
  tree_scores(g->n, g->pr, isrc.data(), k, out->data());
  scores_to_caller(g, out->data());
}

// A graph's shape for the tuning cache: log2 of its non-isolated vertices,
// of its mean and of its largest degree, whether it is deep (BC_MODE_AUTO's
// test), and whether the call uses the 1-degree reduction.
static ShapeKey shape_key(const bc_graph* g, bool deg1);

// The tuned batched setting in effect for a graph: its own bc_autotune
// result, else one tuned on a graph of the same shape in the context.
static bool tuned_params(const bc_graph* g, bool deg1, TunedSet* t);

}  // namespace bcx

extern "C" {

const char* bc_status_string(bc_status st) {
  switch (st) {
    case BC_OK: return "ok";
    case BC_E_INVALID_ARG: return "invalid argument";
    case BC_E_INVALID_GRAPH: return "invalid graph";
    case BC_E_OUT_OF_MEMORY: return "out of memory";
    case BC_E_DEVICE: return "device error";
    case BC_E_BUSY: return "busy";
    case BC_E_NOT_FOUND: return "not found";
    case BC_E_TIMEOUT: return "timeout";
    case BC_E_REJECTED: return "rejected";
    case BC_E_CAPACITY: return "capacity exceeded";
  }
  return "unknown status";
}

const char* bc_last_error(void) { return g_err.c_str(); }

bc_status bc_context_create(int device, bc_context** out) {
  if (!out) return fail(BC_E_INVALID_ARG, "out is null");
  int count = 0;
  HIPCHK(hipGetDeviceCount(&count));
  if (device < 0 || device >= count) return fail(BC_E_INVALID_ARG, "device id out of range");
  HIPCHK(hipSetDevice(device));
  HIPCHK(noalloc_scratch_init(device));
  hipDeviceProp_t p;
  HIPCHK(hipGetDeviceProperties(&p, device));
  auto* c = new bc_context;
  c->device = device;
  c->cus = p.multiProcessorCount;
  c->arch = p.gcnArchName;
  // A persistent grid whose workgroups cannot all be resident (other
  // persistent work holding the CUs) gives up at a barrier after this long
  // instead of waiting forever; BC_BARRIER_TIMEOUT_MS overrides 20 s.
  int khz = 0;
  if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, device) != hipSuccess || khz <= 0) khz = 100000;
  double ms = 20000.0;
  if (const char* e = getenv("BC_BARRIER_TIMEOUT_MS")) ms = std::max(0.0, atof(e));
  c->bar_ticks = (uint64_t)(ms * (double)khz);
  *out = c;
  return BC_OK;
}

bc_status bc_context_destroy(bc_context* ctx) {
  delete ctx;
  return BC_OK;
}

bc_status bc_validate_csr(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int64_t nnz) {
  if (!row_ptr || (nnz > 0 && !col_idx)) return fail(BC_E_INVALID_ARG, "null CSR array");
  std::string why;
  if (!validate_csr(n, row_ptr, col_idx, nnz, &why)) return fail(BC_E_INVALID_GRAPH, why);
  return BC_OK;
}

bc_status bc_prune_deg1_host(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int32_t* omega,
                             int32_t* kind, int32_t* hub, int32_t* res_row_ptr, int32_t* res_col_idx,
                             int64_t* res_nnz) {
  if (!row_ptr || !col_idx || n < 0) return fail(BC_E_INVALID_ARG, "null CSR array");
  Pruned p;
  prune_deg1(n, row_ptr, col_idx, &p);
  if (omega) memcpy(omega, p.omega.data(), sizeof(int32_t) * n);
  if (kind) memcpy(kind, p.kind.data(), sizeof(int32_t) * n);
  if (hub) memcpy(hub, p.hub.data(), sizeof(int32_t) * n);
  if (res_row_ptr) memcpy(res_row_ptr, p.rp.data(), sizeof(int32_t) * (n + 1));
  if (res_col_idx) memcpy(res_col_idx, p.ci.data(), sizeof(int32_t) * p.ci.size());
  if (res_nnz) *res_nnz = (int64_t)p.ci.size();
  return BC_OK;
}

bc_status bc_prune_trees_host(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const int32_t* sources,
                              int64_t k, int32_t* omega, int32_t* kind, double* scores, int64_t* res_nnz) {
  if (!row_ptr || !col_idx || n < 0 || k < 0 || (k > 0 && !sources)) return fail(BC_E_INVALID_ARG, "bad arguments");
  for (int64_t i = 0; i < k; ++i)
    if (sources[i] < 0 || sources[i] >= n) return fail(BC_E_INVALID_ARG, "source id out of range");
  Pruned p;
  prune_trees(n, row_ptr, col_idx, &p);
  if (omega) memcpy(omega, p.omega.data(), sizeof(int32_t) * n);
  if (kind) memcpy(kind, p.kind.data(), sizeof(int32_t) * n);
  if (scores) {
    std::fill(scores, scores + n, 0.0);
    tree_scores(n, p, k ? sources : nullptr, k ? k : n, scores);
  }
  if (res_nnz) *res_nnz = (int64_t)p.ci.size();
  return BC_OK;
}

bc_status bc_vertex_order_host(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint32_t load_flags,
                               int32_t* perm, int64_t* bfs_depth) {
  if (!row_ptr || !col_idx || n <= 0 || !perm) return fail(BC_E_INVALID_ARG, "bad arguments");
  if (row_ptr[0] != 0) return fail(BC_E_INVALID_GRAPH, "row_ptr[0] must be 0");
  for (int32_t v = 0; v < n; ++v)
    if (row_ptr[v + 1] < row_ptr[v]) return fail(BC_E_INVALID_GRAPH, "row_ptr must be non-decreasing");
  std::vector<int32_t> rp(row_ptr, row_ptr + n + 1), ci(col_idx, col_idx + row_ptr[n]);
  for (int32_t u : ci)
    if (u < 0 || u >= n) return fail(BC_E_INVALID_GRAPH, "column index out of range");
  int32_t hub = 0;
  int64_t maxd = -1;
  for (int32_t v = 0; v < n; ++v)
    if (rp[v + 1] - rp[v] > maxd) {
      maxd = rp[v + 1] - rp[v];
      hub = v;
    }
  if (bfs_depth) *bfs_depth = bfs_depth_from(n, rp.data(), ci.data(), hub);
  if (load_flags & BC_LOAD_KEEP_ORDER) {
    for (int32_t v = 0; v < n; ++v) perm[v] = v;
    return BC_OK;
  }
  const std::vector<int32_t> order = (load_flags & BC_LOAD_ORDER_RCM) ? rcm_order(n, rp, ci) : degree_order(n, rp);
  for (int32_t i = 0; i < n; ++i) perm[order[i]] = i;
  return BC_OK;
}

bc_status bc_coverage_host(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint32_t load_flags,
                           uint32_t heuristics, int64_t* out) {
  if (!row_ptr || !col_idx || n < 0 || !out) return fail(BC_E_INVALID_ARG, "bad arguments");
  const bool prune = (load_flags & (BC_LOAD_PRUNE_DEG1 | BC_LOAD_PRUNE_TREES)) && (heuristics & BC_H_DEG1);
  Pruned p;
  if (prune) {
    if (load_flags & BC_LOAD_PRUNE_TREES) prune_trees(n, row_ptr, col_idx, &p);
    else prune_deg1(n, row_ptr, col_idx, &p);
  }
  std::vector<Group> groups;
  int64_t credited = 0;
  map_sources(n, row_ptr, prune ? &p : nullptr, nullptr, n, &groups, &credited);
  const int32_t* trp = prune ? p.rp.data() : row_ptr;
  const int32_t* tci = prune ? p.ci.data() : col_idx;
  int64_t cand = 0;
  for (const auto& gr : groups) cand += trp[gr.v + 1] - trp[gr.v] == 2;
  std::vector<Triple> triples;
  if (heuristics & BC_H_DEG2) {
    const std::vector<int32_t> rank = locality_rank(n, row_ptr, col_idx);
    order_groups(rank, groups);
    choose_deg2(n, trp, tci, groups, &triples);
  }
  out[0] = credited;                                              // non-isolated sources
  out[1] = (int64_t)groups.size() - (int64_t)triples.size();      // sweeps traversed
  out[2] = credited - (int64_t)groups.size();                     // served by the 1-degree reduction
  out[3] = (int64_t)triples.size();                               // derived (2-degree)
  out[4] = cand;                                                  // degree-2 vertices among the sweeps
  return BC_OK;
}

bc_status bc_graph_load(bc_context* ctx, int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                        int64_t nnz, uint32_t flags, bc_graph** out) {
  if (!ctx || !out || n <= 0 || !row_ptr || (nnz > 0 && !col_idx)) return fail(BC_E_INVALID_ARG, "bad arguments");
  if (nnz < 0 || nnz > INT32_MAX) return fail(BC_E_INVALID_GRAPH, "nnz must fit int32");
  HIPCHK(hipSetDevice(ctx->device));
  auto g = new bc_graph;
  g->ctx = ctx;
  g->n = n;
  g->nnz = nnz;
  g->h_rp.resize((size_t)n + 1);
  g->h_ci.resize((size_t)nnz);
  if (flags & BC_LOAD_DEVICE_PTRS) {
    if (hipMemcpy(g->h_rp.data(), row_ptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost) != hipSuccess ||
        (nnz && hipMemcpy(g->h_ci.data(), col_idx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost) != hipSuccess)) {
      delete g;
      return fail(BC_E_DEVICE, "copy of device CSR failed");
    }
  } else {
    memcpy(g->h_rp.data(), row_ptr, sizeof(int32_t) * (n + 1));
    if (nnz) memcpy(g->h_ci.data(), col_idx, sizeof(int32_t) * nnz);
  }
  const int32_t* rp = g->h_rp.data();
  const int32_t* ci = g->h_ci.data();
  if (flags & BC_LOAD_VALIDATE) {
    std::string why;
    if (!validate_csr(n, rp, ci, nnz, &why)) { delete g; return fail(BC_E_INVALID_GRAPH, why); }
  } else if (rp[0] != 0 || rp[n] != nnz) {
    delete g;
    return fail(BC_E_INVALID_GRAPH, "row_ptr[0] must be 0 and row_ptr[n] must equal nnz");
  }
  int32_t hub = 0;
  for (int32_t v = 0; v < n; ++v) {
    const int64_t dg = rp[v + 1] - rp[v];
    if (dg > g->max_degree) hub = v;
    g->max_degree = std::max(g->max_degree, dg);
    g->isolated += dg == 0;
  }
  g->bfs_depth = bfs_depth_from(n, rp, ci, hub);
  if (!(flags & BC_LOAD_KEEP_ORDER)) {
    const std::vector<int32_t> order =
        (flags & BC_LOAD_ORDER_RCM) ? rcm_order(n, g->h_rp, g->h_ci) : degree_order(n, g->h_rp);
    relabel(n, g->h_rp, g->h_ci, order, &g->perm);
    rp = g->h_rp.data();
    ci = g->h_ci.data();
  }
  bc_status st = BC_OK;
  st = upload(g->h_rp, &g->d_rp, &g->resident);
  if (st == BC_OK) st = upload(g->h_ci, &g->d_ci, &g->resident);
  if (st == BC_OK) {
    auto up = static_units(n, rp, kPlainChunkHost), ub = static_units(n, rp, kBatchChunk);
    g->ngu_p = (int32_t)up.size();
    g->ngu_b = (int32_t)ub.size();
    st = upload(up, &g->d_gu_p, &g->resident);
    if (st == BC_OK) st = upload(ub, &g->d_gu_b, &g->resident);
  }
  const int32_t* trp = rp;
  if (st == BC_OK && (flags & (BC_LOAD_PRUNE_DEG1 | BC_LOAD_PRUNE_TREES))) {
    g->pruned = true;
    if (flags & BC_LOAD_PRUNE_TREES) prune_trees(n, rp, ci, &g->pr);
    else prune_deg1(n, rp, ci, &g->pr);
    for (int32_t v = 0; v < n; ++v) {
      g->pendants += g->pr.kind[v] == kPendant;
      g->k2 += g->pr.kind[v] == kK2;
      g->tree += g->pr.kind[v] == kTree;
    }
    g->rnnz = (int64_t)g->pr.ci.size();
    st = upload(g->pr.rp, &g->d_rrp, &g->resident);
    if (st == BC_OK) st = upload(g->pr.ci, &g->d_rci, &g->resident);
    if (st == BC_OK) st = upload(g->pr.omega, &g->d_omega, &g->resident);
    if (st == BC_OK) {
      auto up = static_units(n, g->pr.rp.data(), kPlainChunkHost), ub = static_units(n, g->pr.rp.data(), kBatchChunk);
      g->nrgu_p = (int32_t)up.size();
      g->nrgu_b = (int32_t)ub.size();
      st = upload(up, &g->d_rgu_p, &g->resident);
      if (st == BC_OK) st = upload(ub, &g->d_rgu_b, &g->resident);
    }
    trp = g->pr.rp.data();
  } else {
    g->rnnz = nnz;
  }
  for (int32_t v = 0; v < n; ++v) g->deg2 += (trp[v + 1] - trp[v]) == 2;
  if (st == BC_OK) {
    if (hipMalloc((void**)&g->d_bc, sizeof(double) * n) != hipSuccess) st = fail(BC_E_OUT_OF_MEMORY, "score array");
    else if (hipMemset(g->d_bc, 0, sizeof(double) * n) != hipSuccess) st = fail(BC_E_DEVICE, "memset");
    g->resident += (int64_t)sizeof(double) * n;
  }
  if (st != BC_OK) {
    bc_graph_free(g);
    return st;
  }
  *out = g;
  return BC_OK;
}

bc_status bc_graph_stats_get(const bc_graph* g, bc_graph_stats* out) {
  if (!g || !out) return fail(BC_E_INVALID_ARG, "null argument");
  out->n = g->n;
  out->nnz = g->nnz;
  out->m = g->nnz / 2;
  out->isolated = g->isolated;
  out->pendants = g->pendants;
  out->k2_vertices = g->k2;
  out->residual_nnz = g->rnnz;
  out->deg2_vertices = g->deg2;
  out->max_degree = g->max_degree;
  out->tree_vertices = g->tree;
  out->bfs_depth = g->bfs_depth;
  TunedSet tp;
  out->tuned_batch = bcx::tuned_params(g, g->pruned, &tp) ? tp.batch : 0;
  out->resident_bytes = g->resident.load();
  return BC_OK;
}

bc_status bc_graph_free(bc_graph* g) {
  if (!g) return BC_OK;
  (void)hipSetDevice(g->ctx->device);
  for (void* p : {(void*)g->d_rp, (void*)g->d_ci, (void*)g->d_rrp, (void*)g->d_rci, (void*)g->d_omega,
                  (void*)g->d_gu_p, (void*)g->d_gu_b, (void*)g->d_rgu_p, (void*)g->d_rgu_b, (void*)g->d_bc,
                  (void*)g->d_ell[0], (void*)g->d_ell[1], g->ws})
    if (p) (void)hipFree(p);
  g->exec.release();
  delete g;
  return BC_OK;
}

}  // extern "C"

// ---------------------------------------------------------------- compute

namespace bcx {

// BC_MODE_AUTO: graphs whose breadth-first depth from a highest-degree
// vertex exceeds this run one source per workgroup (R-MAT graphs stay near
// ten levels, road networks and lattices reach hundreds to thousands).
constexpr int64_t kLongDepth = 64;

static bc_status resolve(const bc_graph* g, const bc_compute_opts* o, Resolved* r) {
  bc_compute_opts d{};
  if (!o) o = &d;
  r->mode = o->mode;
  if (r->mode == BC_MODE_AUTO)  // long diameters (thousands of levels) go one source per workgroup
    r->mode = (g->bfs_depth > kLongDepth && !(o->heuristics & BC_H_DEG2)) ? BC_MODE_PER_WORKGROUP : BC_MODE_BATCHED;
  if (r->mode != BC_MODE_PLAIN && r->mode != BC_MODE_BATCHED && r->mode != BC_MODE_PLAIN_SCAN &&
      r->mode != BC_MODE_PER_WORKGROUP)
    return fail(BC_E_INVALID_ARG, "unknown mode");
  TunedSet tp;
  const bool tuned = tuned_params(g, (o->heuristics & BC_H_DEG1) != 0, &tp);
  r->B = o->batch ? o->batch : (tuned ? tp.batch : 256);
  if (r->B % 64 != 0 || r->B < 64 || r->B > 64 * kMaxWords)
    return fail(BC_E_INVALID_ARG, "batch must be a multiple of 64 from 64 to 1024");
  r->K = r->B / 64;
  const int blk = (r->mode == BC_MODE_BATCHED || r->mode == BC_MODE_PER_WORKGROUP) ? kBatchBlock : 256;
  r->block = o->block ? o->block : blk;
  if (r->block != blk)
    return fail(BC_E_INVALID_ARG, "block must be 1024 (batched, per_workgroup) or 256 (plain, plain_scan)");
  r->grid_per_cu = o->grid_per_cu ? o->grid_per_cu : (tuned && !o->batch ? tp.grid : 0);
  r->sigma_mode = o->sigma_mode;
  if (r->sigma_mode < 0 || r->sigma_mode > 2) return fail(BC_E_INVALID_ARG, "unknown sigma mode");
  r->deg1 = (o->heuristics & BC_H_DEG1) != 0;
  r->deg2 = (o->heuristics & BC_H_DEG2) != 0;
  if (r->deg1 && !g->pruned) return fail(BC_E_INVALID_ARG, "BC_H_DEG1 needs a graph loaded with BC_LOAD_PRUNE_DEG1");
  if (r->deg2 && r->mode != BC_MODE_BATCHED) return fail(BC_E_INVALID_ARG, "BC_H_DEG2 needs the batched mode");
  if (r->deg2 && r->mode == BC_MODE_PER_WORKGROUP) return fail(BC_E_INVALID_ARG, "BC_H_DEG2 needs the batched mode");
  if (r->mode == BC_MODE_PLAIN_SCAN && (r->deg1 || r->sigma_mode == BC_SIGMA_EXTENDED))
    return fail(BC_E_INVALID_ARG, "BC_MODE_PLAIN_SCAN takes no heuristics and exact counts");
  if (o->alpha > 0) r->alpha = o->alpha;
  else if (o->alpha < 0) r->alpha = 0.0;  // never bottom-up
  else if (tuned && !o->batch && r->mode == BC_MODE_BATCHED) r->alpha = tp.alpha;
  else r->alpha = 0.0;  // top-down only: bottom-up levels were slower on every graph measured
  if (o->beta < 0) return fail(BC_E_INVALID_ARG, "beta must be >= 0");
  r->beta = o->beta > 0 ? o->beta : (tuned && !o->batch && r->mode == BC_MODE_BATCHED ? tp.beta : 0.0);
  if (o->graph_launches < 0 || (o->graph_launches > 0 && r->mode != BC_MODE_PLAIN))
    return fail(BC_E_INVALID_ARG, "graph_launches must be >= 0 and is for BC_MODE_PLAIN only");
  r->graph_launches = o->graph_launches;
  return BC_OK;
}

static ShapeKey shape_key(const bc_graph* g, bool deg1) {
  auto lg = [](int64_t x) {
    int64_t b = 0;
    while (x > 1) { x >>= 1; ++b; }
    return b;
  };
  const int64_t nv = std::max<int64_t>(1, g->n - g->isolated);
  const int64_t nnz = deg1 ? g->rnnz : g->nnz;
  return ShapeKey{lg(nv), lg(std::max<int64_t>(1, nnz / nv)), lg(g->max_degree + 1), g->bfs_depth > kLongDepth ? 1 : 0,
                  deg1 ? 1 : 0};
}

static bool tuned_params(const bc_graph* g, bool deg1, TunedSet* t) {
  if (g->tuned) {
    *t = TunedSet{g->tuned_batch, g->tuned_grid, g->tuned_alpha, g->tuned_beta};
    return true;
  }
  std::lock_guard<std::mutex> lk(g->ctx->tune_mu);
  const auto it = g->ctx->tune_cache.find(shape_key(g, deg1));
  if (it == g->ctx->tune_cache.end()) return false;
  *t = it->second;
  return true;
}

size_t ws_bytes_for(const bc_graph* g, const Resolved& r, int cap_factor) {
  cap_factor = std::max(cap_factor, r.cap_factor);
  if (r.mode == BC_MODE_PLAIN) return plain_layout(g->n, g->nnz, nullptr, nullptr);
  if (r.mode == BC_MODE_PLAIN_SCAN)  // wrapped sources rerun in the plain workspace
    return std::max(scan_layout(g->n, nullptr, nullptr), plain_layout(g->n, g->nnz, nullptr, nullptr));
  if (r.mode == BC_MODE_PER_WORKGROUP)  // sized for as many sources as vertices
    return wg_layout(g->n, wg_grid(g->n, g->ctx->cus, r.grid_per_cu, r.grid_total), g->n, nullptr, nullptr);
  return batch_layout(g->n, g->nnz, r.B, cap_factor, r.max_slots, r.trace, nullptr, nullptr);
}

struct TravGraph {
  const int32_t *rp, *ci, *omega;
  const int2 *gu_p, *gu_b;
  int32_t ngu_p, ngu_b;
  int64_t nnz;
  const int32_t* h_rp;
  const int32_t* h_ci;
};

static TravGraph trav(const bc_graph* g, bool deg1) {
  if (deg1)
    return TravGraph{g->d_rrp, g->d_rci, g->d_omega, g->d_rgu_p, g->d_rgu_b, g->nrgu_p, g->nrgu_b,
                     (int64_t)g->pr.ci.size(), g->pr.rp.data(), g->pr.ci.data()};
  return TravGraph{g->d_rp, g->d_ci, nullptr, g->d_gu_p, g->d_gu_b, g->ngu_p, g->ngu_b, g->nnz,
                   g->h_rp.data(), g->h_ci.data()};
}

// Plain-form graphs with at least this many traversed directed edges run
// four workgroups per CU (wide levels hide more latency), smaller ones one
// (fewer workgroups make the per-level barrier cheaper); measured on the
// scale-16 (1 best) and scale-20 (4-6 best) R-MAT graphs.
constexpr int64_t kPlainWideNnz = int64_t(1) << 24;

static int grid_for(const bc_graph* g, const Resolved& r, bool ext, bool batched) {
  int bpc = 1;
  hipError_t e = batched ? batch_max_grid(ext, r.block, &bpc) : plain_max_grid(ext, r.block, &bpc);
  if (e != hipSuccess || bpc < 1) bpc = 1;
  // The occupancy query's last workgroup per CU did not always fit beside the
  // others (the plain kernel at 7 per CU never became wholly resident, and a
  // persistent grid that is not cannot pass its first barrier): stay below it.
  const int cap = bpc > 1 ? bpc - 1 : 1;
  const int64_t tnnz = r.deg1 ? g->rnnz : g->nnz;
  const int want = r.grid_per_cu > 0 ? r.grid_per_cu : (batched ? cap : (tnnz >= kPlainWideNnz ? 4 : 1));
  const int grid = g->ctx->cus * std::min(want, cap);
  return r.grid_total > 0 ? std::min(grid, r.grid_total) : grid;
}

// Lane packing of one call: a list of batches, each with per-lane group
// indices (-1 = empty) and derived-lane partners.
struct Packing {
  int B;
  std::vector<int32_t> lane_group;  // nbatches * B
  std::vector<int8_t> pa, pb;       // nbatches * B
  int64_t nbatches = 0;
  int64_t derived = 0;
};

static void pack_lanes(const std::vector<Group>& groups, const std::vector<Triple>& triples, int B, Packing* p) {
  p->B = B;
  const size_t G = groups.size();
  // clusters: derived vertices with their partners, joined through shared
  // partners (each fits one 64-lane word by construction)
  std::vector<int32_t> uf(G);
  for (size_t i = 0; i < G; ++i) uf[i] = (int32_t)i;
  auto find = [&](int32_t x) {
    while (uf[x] != x) x = uf[x] = uf[uf[x]];
    return x;
  };
  std::vector<char> in_cluster(G, 0);
  std::vector<std::pair<int32_t, int32_t>> partners(G, {-1, -1});
  for (const auto& t : triples) {
    in_cluster[t.a] = in_cluster[t.b] = in_cluster[t.c] = 1;
    partners[t.c] = {t.a, t.b};
    uf[find(t.a)] = find(t.c);
    uf[find(t.b)] = find(t.c);
  }
  std::vector<std::vector<int32_t>> members(G);
  std::vector<int32_t> roots;
  for (size_t i = 0; i < G; ++i) {
    if (!in_cluster[i]) continue;
    const int32_t r = find((int32_t)i);
    if (members[r].empty()) roots.push_back(r);
    members[r].push_back((int32_t)i);
  }
  std::vector<int32_t> lanes, pos(G, -1);
  std::vector<int8_t> pa, pb;
  auto pad_to_word = [&](size_t need) {
    const size_t used = lanes.size() % 64;
    if (used + need > 64) {
      while (lanes.size() % 64) { lanes.push_back(-1); pa.push_back(-1); pb.push_back(-1); }
    }
  };
  // slot by slot (a cluster's members share one slot): its clusters, then its other groups
  int nslot = 1;
  for (const auto& gr : groups) nslot = std::max(nslot, gr.slot + 1);
  for (int sl = 0; sl < nslot; ++sl) {
    for (int32_t r : roots) {
      if (groups[r].slot != sl) continue;
      pad_to_word(members[r].size());
      for (int32_t m : members[r]) {  // partners first, then the derived lanes that point at them
        if (partners[m].first >= 0) continue;
        pos[m] = (int32_t)(lanes.size() % 64);
        lanes.push_back(m); pa.push_back(-1); pb.push_back(-1);
      }
      for (int32_t m : members[r]) {
        if (partners[m].first < 0) continue;
        lanes.push_back(m);
        pa.push_back((int8_t)pos[partners[m].first]);
        pb.push_back((int8_t)pos[partners[m].second]);
      }
    }
    for (size_t i = 0; i < G; ++i) {
      if (in_cluster[i] || groups[i].slot != sl) continue;
      lanes.push_back((int32_t)i); pa.push_back(-1); pb.push_back(-1);
    }
  }
  while (lanes.size() % B) { lanes.push_back(-1); pa.push_back(-1); pb.push_back(-1); }
  p->lane_group = std::move(lanes);
  p->pa = std::move(pa);
  p->pb = std::move(pb);
  p->nbatches = (int64_t)(p->lane_group.size() / B);
  p->derived = (int64_t)triples.size();
}

struct TablePtrs {
  int32_t *lane_src, *lane_own, *l0;
  double *lane_w, *lane_tsub;
  int16_t* pair;
  int8_t *pa, *pb, *slot, *pair_slot;
  uint64_t *el, *dl;
  double** slot_bc;
};

static TablePtrs table_at(char* t, int B) {
  TablePtrs p;
  p.lane_src = (int32_t*)t;
  p.lane_own = p.lane_src + B;
  p.l0 = p.lane_own + B;
  p.lane_w = (double*)(p.l0 + B);
  p.lane_tsub = p.lane_w + B;
  p.pair = (int16_t*)(p.lane_tsub + B);
  p.pa = (int8_t*)(p.pair + B);
  p.pb = p.pa + B;
  p.slot = p.pb + B;
  p.pair_slot = p.slot + B;
  p.el = (uint64_t*)(((uintptr_t)(p.pair_slot + kMaxPairs) + 7) & ~(uintptr_t)7);
  p.dl = p.el + kMaxWords;
  p.slot_bc = (double**)(p.dl + kMaxWords);
  return p;
}

struct TableInfo {
  int32_t nl0;     // distinct source vertices
  int32_t npairs;  // (word, slot) pairs
  bool derived;    // any derived lane
};

// Fills one batch's table.  Pairs are numbered word by word in order of
// first appearance; the per-pair sums of a launch are folded in that order.
static TableInfo fill_table(char* dst, const Packing& pk, int64_t b, const std::vector<Group>& groups, int B,
                            double* const* slot_ptrs, int nslots) {
  TablePtrs t = table_at(dst, B);
  for (int k = 0; k < kMaxWords; ++k) t.el[k] = t.dl[k] = 0;
  for (int s = 0; s < kMaxSlots; ++s) t.slot_bc[s] = s < nslots ? slot_ptrs[s] : nullptr;
  for (int p = 0; p < kMaxPairs; ++p) t.pair_slot[p] = 0;
  TableInfo info{0, 0, false};
  std::vector<int32_t> distinct;
  int cur_word = -1, cur_slot = -1;
  for (int j = 0; j < B; ++j) {
    const int32_t gi = pk.lane_group[(size_t)b * B + j];
    t.pa[j] = pk.pa[(size_t)b * B + j];
    t.pb[j] = pk.pb[(size_t)b * B + j];
    t.slot[j] = 0;
    t.pair[j] = (int16_t)std::max(info.npairs - 1, 0);
    if (gi < 0) { t.lane_src[j] = -1; t.lane_own[j] = 0; t.lane_w[j] = 0.0; t.lane_tsub[j] = 0.0; continue; }
    t.lane_src[j] = groups[gi].v;
    t.lane_own[j] = groups[gi].own;
    t.lane_tsub[j] = groups[gi].tsub;
    t.lane_w[j] = groups[gi].w;
    t.slot[j] = (int8_t)groups[gi].slot;
    if ((j >> 6) != cur_word || groups[gi].slot != cur_slot) {
      cur_word = j >> 6;
      cur_slot = groups[gi].slot;
      t.pair_slot[info.npairs] = (int8_t)cur_slot;
      ++info.npairs;
    }
    t.pair[j] = (int16_t)(info.npairs - 1);
    distinct.push_back(groups[gi].v);
    if (t.pa[j] < 0) {
      t.el[j >> 6] |= 1ull << (j & 63);
    } else {
      t.dl[j >> 6] |= 1ull << (j & 63);
      info.derived = true;
    }
  }
  std::sort(distinct.begin(), distinct.end());
  distinct.erase(std::unique(distinct.begin(), distinct.end()), distinct.end());
  for (int j = 0; j < B; ++j) t.l0[j] = j < (int)distinct.size() ? distinct[j] : -1;
  info.nl0 = (int32_t)distinct.size();
  return info;
}

static void table_ptrs(char* dev, int B, BatchArgs* a) {
  TablePtrs t = table_at(dev, B);
  a->lane_src = t.lane_src;
  a->lane_own = t.lane_own;
  a->lane_tsub = t.lane_tsub;
  a->lane_w = t.lane_w;
  a->lane_pa = t.pa;
  a->lane_pb = t.pb;
  a->edge_lanes = t.el;
  a->derived_lanes = t.dl;
  a->slot_bc = t.slot_bc;
  a->lane_pair = t.pair;
  a->pair_slot = t.pair_slot;
}

struct CallOut {
  std::vector<int32_t> ovf;   // overflowed traversal sources
  std::vector<int32_t> fail;  // sources of batches that exceeded a list capacity
  unsigned long long st[kStCount] = {0};
  double kernel_ms = 0.0;     // summed launch durations
  int err = 0;
  void merge(const CallOut& o) {
    for (int i = 0; i < kStCount; ++i) st[i] += o.st[i];
    kernel_ms += o.kernel_ms;
  }
};

// Launch timing: an event pair recorded on the launch stream around each
// kernel launch; durations are summed when the host next waits for the
// stream.
hipError_t Exec::mark(hipStream_t st) {
  if (used == ev.size()) {
    hipEvent_t e;
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) return r;
    ev.push_back(e);
  }
  return hipEventRecord(ev[used++], st);
}

hipError_t Exec::collect(double* ms) {
  for (size_t i = 0; i + 1 < used; i += 2) {
    float f = 0.f;
    hipError_t r = hipEventElapsedTime(&f, ev[i], ev[i + 1]);
    if (r != hipSuccess) return r;
    *ms += f;
  }
  used = 0;
  return hipSuccess;
}

bc_status Exec::tables(size_t bytes, char** out) {
  if (stage_bytes < bytes) {
    if (stage) (void)hipHostFree(stage);
    stage = nullptr;
    stage_bytes = 0;
    HIPCHK(hipHostMalloc((void**)&stage, bytes, hipHostMallocDefault));
    stage_bytes = bytes;
  }
  *out = stage;
  return BC_OK;
}

void Exec::release() {
  for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  ev.clear();
  used = 0;
  if (stage) (void)hipHostFree(stage);
  stage = nullptr;
  stage_bytes = 0;
}

// Trace destinations (device) for a batch, or nulls.
struct TraceDev {
  double* delta = nullptr;
  uint64_t* sig = nullptr;
  double* sm = nullptr;
  int32_t* se = nullptr;
  double* bc = nullptr;  // scratch score array
};

// Runs all groups through the batched kernel.  Scores go to `bc`.
bc_status run_batched(bc_graph* g, const Resolved& r, bool ext, const TravGraph& tg,
                      const std::vector<Group>& groups, const std::vector<Triple>& triples, char* wsbase,
                      int cap_factor, hipStream_t st, double* const* slot_ptrs, int nslots, const TraceDev* tr,
                      Exec* ex, CallOut* out, std::vector<int32_t>* trace_lane_vertex) {
  ex->used = 0;
  BatchWs w;
  batch_layout(g->n, g->nnz, r.B, cap_factor, r.max_slots, r.trace, wsbase, &w);
  HIPCHK(hipMemsetAsync(w.ctl_begin, 0, w.ctl_bytes, st));
  HIPCHK(hipMemsetAsync(w.vis, 0, w.mask_bytes, st));
  HIPCHK(hipMemsetAsync(w.pair_bc, 0, sizeof(double) * (size_t)w.cap_pairs * g->n, st));
  Packing pk;
  pack_lanes(groups, triples, r.B, &pk);
  // a trace call owns trace rows for one launch of B lanes only
  if (tr && pk.nbatches > 1) return fail(BC_E_INVALID_ARG, "a trace call must pack into one launch");
  if (trace_lane_vertex) trace_lane_vertex->assign(pk.lane_group.begin(), pk.lane_group.end());
  char* stage = nullptr;
  bc_status s = ex->tables(w.table_bytes * kTableBatches, &stage);
  if (s != BC_OK) return s;
  const int grid = grid_for(g, r, ext, true);
  BatchArgs a{};
  a.n = g->n;
  a.nnz = tg.nnz;
  a.K = r.K;
  a.rp = tg.rp;
  a.ci = tg.ci;
  a.omega = tg.omega;
  a.gu = tg.gu_b;
  a.ngu = tg.ngu_b;
  a.lv = w.lv;
  a.sig = w.sig;
  a.sm = (double*)w.sig;
  a.se = w.se;
  a.vis = w.vis;
  a.fm = w.fm;
  a.dla = w.dla;
  a.dlb = w.dlb;
  a.Q = w.Q;
  a.U = w.U;
  a.qoff = w.qoff;
  a.uoff = w.uoff;
  a.lc = w.lc;
  a.part_m = w.part_m;
  a.part_e = w.part_e;
  a.arrive = w.arrive;
  a.emask = w.emask;
  a.err = w.err;
  a.lane_ovf = w.lane_ovf;
  a.ovf_list = w.ovf_list;
  a.ovf_count = w.ovf_count;
  a.lane_ns = w.lane_ns;
  a.stats = w.stats;
  a.fail_list = w.fail_list;
  a.fail_count = w.fail_count;
  a.fulledges = w.fulledges;
  a.bar = w.bar;
  a.bar_limit = g->ctx->bar_ticks;
  a.clear_at_end = tr ? 0 : 1;
  a.keep_lv = (tr && w.lv) ? 1 : 0;
  a.alpha = r.alpha;
  a.beta = r.beta;
  a.cap_entries = (int32_t)w.caps.entries;
  a.cap_units = (int32_t)w.caps.units;
  a.cap_parts = (int32_t)w.caps.parts;
  a.cap_levels = g->n + 3;
  a.cap_pairs = w.cap_pairs;
  a.pair_bc = w.pair_bc;
  bool any_own = false;
  for (const auto& gr : groups) any_own |= gr.own > 0;
  a.has_own = any_own ? 1 : 0;
  for (int64_t b0 = 0; b0 < pk.nbatches; b0 += kTableBatches) {
    const int64_t nb = std::min<int64_t>(kTableBatches, pk.nbatches - b0);
    std::vector<TableInfo> info(nb);
    for (int64_t b = 0; b < nb; ++b) {
      info[b] = fill_table(stage + b * w.table_bytes, pk, b0 + b, groups, r.B, slot_ptrs, nslots);
      if (info[b].npairs > w.cap_pairs) return fail(BC_E_CAPACITY, "batch has more (word, slot) pairs than sized");
    }
    HIPCHK(hipMemcpyAsync(w.tables, stage, nb * w.table_bytes, hipMemcpyHostToDevice, st));
    for (int64_t b = 0; b < nb; ++b) {
      char* t = w.tables + b * w.table_bytes;
      table_ptrs(t, r.B, &a);
      a.npairs = info[b].npairs;
      a.has_derived = info[b].derived ? 1 : 0;
      if (tr) {
        const size_t off = (size_t)b * r.B * g->n;
        a.delta_out = tr->delta ? tr->delta + off : nullptr;
        a.sig_out = (!ext && tr->sig) ? tr->sig + off : nullptr;
        a.sm_out = (ext && tr->sm) ? tr->sm + off : nullptr;
        a.se_out = (ext && tr->se) ? tr->se + off : nullptr;
      }
      HIPCHK(ex->mark(st));
      HIPCHK(launch_batch(a, ext, grid, r.block, st));
      HIPCHK(ex->mark(st));
    }
    HIPCHK(hipStreamSynchronize(st));  // staging buffer reused by the next group
    HIPCHK(ex->collect(&out->kernel_ms));
  }
  int32_t cnt = 0, err = 0, fcnt = 0;
  HIPCHK(hipMemcpyAsync(&cnt, w.ovf_count, sizeof cnt, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&fcnt, w.fail_count, sizeof fcnt, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&err, w.err, sizeof err, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(out->st, w.stats, sizeof(out->st), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (err & kErrBarrier) return fail(BC_E_DEVICE, "grid-barrier wait gave up: the persistent grid was not resident");
  out->err = err;
  out->ovf.resize(std::min<int32_t>(cnt, g->n + 1));
  out->fail.resize(std::min<int32_t>(fcnt, g->n + 1));
  if (!out->ovf.empty())
    HIPCHK(hipMemcpy(out->ovf.data(), w.ovf_list, sizeof(int32_t) * out->ovf.size(), hipMemcpyDeviceToHost));
  if (!out->fail.empty())
    HIPCHK(hipMemcpy(out->fail.data(), w.fail_list, sizeof(int32_t) * out->fail.size(), hipMemcpyDeviceToHost));
  return BC_OK;
}

// The plain form's per-source launches from a HIP graph: k identical
// launches captured once, replayed while k sources remain, each launch
// taking the next source of a device list (the remainder runs as single
// launches of the same form).  Returns after the stream has drained, since
// the list is freed on the way out.
static bc_status plain_replayed(const PlainArgs& a, bool ext, int grid, int block, const std::vector<Group>& groups,
                                int k, hipStream_t st, Exec* ex, CallOut* out) {
  const int64_t G = (int64_t)groups.size();
  if (G > INT32_MAX) return fail(BC_E_INVALID_ARG, "too many sources for one device list");
  std::vector<PlainSrc> h((size_t)G);
  for (int64_t i = 0; i < G; ++i) h[i] = PlainSrc{groups[i].v, groups[i].own, groups[i].tsub, groups[i].w};
  const size_t rec = (sizeof(PlainSrc) * (size_t)G + 255) / 256 * 256;
  struct Held {
    hipStream_t st;
    hipStream_t cs = nullptr;
    hipGraph_t gr = nullptr;
    hipGraphExec_t ge = nullptr;
    char* buf = nullptr;
    ~Held() {
      (void)hipStreamSynchronize(st);
      if (ge) (void)hipGraphExecDestroy(ge);
      if (gr) (void)hipGraphDestroy(gr);
      if (cs) (void)hipStreamDestroy(cs);
      if (buf) (void)hipFree(buf);
    }
  } held{st};
  HIPCHK(hipMalloc(&held.buf, rec + 256));
  const PlainFeed f{(const PlainSrc*)held.buf, (int32_t*)(held.buf + rec), (int32_t)G};
  HIPCHK(hipMemcpyAsync(held.buf, h.data(), sizeof(PlainSrc) * (size_t)G, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(f.cursor, 0, sizeof(int32_t), st));
  // captured on a stream of its own (the caller's may be the null stream)
  HIPCHK(hipStreamCreateWithFlags(&held.cs, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(held.cs, hipStreamCaptureModeRelaxed));
  hipError_t e = hipSuccess;
  for (int i = 0; i < k && e == hipSuccess; ++i) e = launch_plain_fed(a, f, ext, grid, block, held.cs);
  const hipError_t e_end = hipStreamEndCapture(held.cs, &held.gr);
  HIPCHK(e);
  HIPCHK(e_end);
  HIPCHK(hipGraphInstantiate(&held.ge, held.gr, nullptr, nullptr, 0));
  const int64_t replays = G / k;
  for (int64_t i = 0; i < replays + (G - replays * k); ++i) {
    if (ex) HIPCHK(ex->mark(st));
    if (i < replays) HIPCHK(hipGraphLaunch(held.ge, st));
    else HIPCHK(launch_plain_fed(a, f, ext, grid, block, st));
    if (!ex) continue;
    HIPCHK(ex->mark(st));
    if (ex->used >= 512) {
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(ex->collect(&out->kernel_ms));
    }
  }
  HIPCHK(hipStreamSynchronize(st));
  return BC_OK;
}

bc_status run_plain(bc_graph* g, const Resolved& r, bool ext, const TravGraph& tg, const std::vector<Group>& groups,
                    char* wsbase, hipStream_t st, double* bc, double* delta_out, Exec* ex, CallOut* out) {
  if (ex) ex->used = 0;
  PlainWs w;
  plain_layout(g->n, g->nnz, wsbase, &w);
  if (r.no_alloc) HIPCHK(zero_async(w.ctl_begin, w.ctl_bytes, st));
  else HIPCHK(hipMemsetAsync(w.ctl_begin, 0, w.ctl_bytes, st));
  const int grid = grid_for(g, r, ext, false);
  PlainArgs a{};
  a.n = g->n;
  a.nnz = tg.nnz;
  a.rp = tg.rp;
  a.ci = tg.ci;
  a.omega = tg.omega;
  a.gu = tg.gu_p;
  a.ngu = tg.ngu_p;
  a.d = w.d;
  a.sig = w.sig;
  a.sm = w.sm;
  a.se = w.se;
  a.psi = w.psi;
  a.Q = w.Q;
  a.U = w.U;
  a.qoff = w.qoff;
  a.uoff = w.uoff;
  a.lc = w.lc;
  a.part_m = w.part_m;
  a.part_e = w.part_e;
  a.arrive = w.arrive;
  a.gmulti = w.gmulti;
  a.err = w.err;
  a.ovf_now = w.ovf_now;
  a.ovf_list = w.ovf_list;
  a.ovf_count = w.ovf_count;
  a.ns = w.ns;
  a.stats = w.stats;
  a.bar = w.bar;
  a.bar_limit = g->ctx->bar_ticks;
  a.bc = bc;
  a.delta_out = delta_out;
  a.alpha = r.alpha;
  a.beta = r.beta;
  a.cap_entries = g->n;
  a.cap_units = (int32_t)plain_cap_units(g->n, g->nnz);
  a.cap_parts = (int32_t)plain_cap_parts(g->n, g->nnz);
  a.cap_multi = g->n;
  a.cap_levels = g->n + 3;
  const bool replay = r.graph_launches > 0 && (int64_t)groups.size() >= r.graph_launches && !r.no_alloc;
  if (replay) {
    const bc_status s = plain_replayed(a, ext, grid, r.block, groups, r.graph_launches, st, ex, out);
    if (s != BC_OK) return s;
  }
  for (size_t i = 0; !replay && i < groups.size(); ++i) {
    const Group& gr = groups[i];
    a.src = gr.v;
    a.weight = gr.w;
    a.own = gr.own;
    a.tsub = gr.tsub;
    if (ex) HIPCHK(ex->mark(st));
    HIPCHK(launch_plain(a, ext, grid, r.block, st));
    if (!ex) continue;
    HIPCHK(ex->mark(st));
    if (ex->used >= 512) {
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(ex->collect(&out->kernel_ms));
    }
  }
  int32_t cnt = 0, err = 0;
  HIPCHK(hipMemcpyAsync(&cnt, w.ovf_count, sizeof cnt, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&err, w.err, sizeof err, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(out->st, w.stats, sizeof(out->st), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (ex) HIPCHK(ex->collect(&out->kernel_ms));
  if (err & kErrBarrier) return fail(BC_E_DEVICE, "grid-barrier wait gave up: the persistent grid was not resident");
  out->err = err;
  out->ovf.resize(std::min<int32_t>(cnt, g->n + 1));
  if (cnt) HIPCHK(hipMemcpy(out->ovf.data(), w.ovf_list, sizeof(int32_t) * out->ovf.size(), hipMemcpyDeviceToHost));
  return BC_OK;
}

// One source per launch with the paper's prefix-sum / binary-search mapping.
bc_status run_scan(bc_graph* g, const Resolved& r, const TravGraph& tg, const std::vector<Group>& groups,
                   char* wsbase, hipStream_t st, double* bc, Exec* ex, CallOut* out) {
  if (ex) ex->used = 0;
  ScanWs w;
  scan_layout(g->n, wsbase, &w);
  HIPCHK(hipMemsetAsync(w.ctl_begin, 0, w.ctl_bytes, st));
  int bpc = 1;
  if (scan_max_grid(&bpc) != hipSuccess || bpc < 1) bpc = 1;
  const int grid = std::min(kScanMaxGrid, g->ctx->cus * std::min(bpc, 2));
  ScanArgs a{};
  a.n = g->n;
  a.rp = tg.rp;
  a.ci = tg.ci;
  a.d = w.d;
  a.sig = w.sig;
  a.psi = w.psi;
  a.acc = w.acc;
  a.Q = w.Q;
  a.qoff = w.qoff;
  a.cd = w.cd;
  a.tot = w.tot;
  a.bsum = w.bsum;
  a.err = w.err;
  a.ovf_now = w.ovf_now;
  a.ovf_list = w.ovf_list;
  a.ovf_count = w.ovf_count;
  a.stats = w.stats;
  a.bar = w.bar;
  a.bar_limit = g->ctx->bar_ticks;
  a.bc = bc;
  a.delta_out = nullptr;
  for (const auto& gr : groups) {
    a.src = gr.v;
    a.weight = gr.w;
    if (ex) HIPCHK(ex->mark(st));
    HIPCHK(launch_scan(a, grid, st));
    if (!ex) continue;
    HIPCHK(ex->mark(st));
    if (ex->used >= 512) {
      HIPCHK(hipStreamSynchronize(st));
      HIPCHK(ex->collect(&out->kernel_ms));
    }
  }
  int32_t cnt = 0, err = 0;
  HIPCHK(hipMemcpyAsync(&cnt, w.ovf_count, sizeof cnt, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(&err, w.err, sizeof err, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(out->st, w.stats, sizeof(out->st), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (ex) HIPCHK(ex->collect(&out->kernel_ms));
  if (err & kErrBarrier) return fail(BC_E_DEVICE, "grid-barrier wait gave up: the persistent grid was not resident");
  out->ovf.resize(std::min<int32_t>(cnt, g->n + 1));
  if (cnt) HIPCHK(hipMemcpy(out->ovf.data(), w.ovf_list, sizeof(int32_t) * out->ovf.size(), hipMemcpyDeviceToHost));
  return BC_OK;
}

// Packed adjacency for the per-workgroup kernel: kEllWidth ints per vertex,
// the degree then up to kEllWidth - 1 neighbours in row order, or (larger
// degree) the row start in the CSR; one aligned 32-byte slot, so a vertex's
// bounds and (usually) all its neighbours arrive in one line.
static std::vector<int32_t> build_ell(int32_t n, const int32_t* rp, const int32_t* ci) {
  std::vector<int32_t> e((size_t)n * kEllWidth, 0);
  for (int32_t v = 0; v < n; ++v) {
    int32_t* s = &e[(size_t)v * kEllWidth];
    const int32_t d = rp[v + 1] - rp[v];
    s[0] = d;
    if (d <= kEllWidth - 1) std::copy(ci + rp[v], ci + rp[v + 1], s + 1);
    else s[1] = rp[v];
  }
  return e;
}

static bc_status ensure_ell(bc_graph* g, bool deg1, const TravGraph& tg, const int32_t** out) {
  const int i = deg1 ? 1 : 0;
  std::lock_guard<std::mutex> lk(g->ell_mu);
  if (!g->d_ell[i]) {  // a failed build leaves it null, and the next call tries again
    int32_t* d = nullptr;
    const bc_status s = upload(build_ell(g->n, tg.h_rp, tg.h_ci), &d, &g->resident);
    if (s != BC_OK) {
      if (d) (void)hipFree(d);
      return s;
    }
    g->d_ell[i] = d;
  }
  *out = g->d_ell[i];
  return BC_OK;
}

// All groups in one launch: each workgroup walks its share of the sources.
bc_status run_wg(bc_graph* g, const Resolved& r, bool ext, const TravGraph& tg, const std::vector<Group>& groups,
                 char* wsbase, hipStream_t st, double* const* slots, int nslots, Exec* ex, CallOut* out) {
  if (ex) ex->used = 0;
  const int grid = wg_grid(g->n, g->ctx->cus, r.grid_per_cu, r.grid_total);
  const int64_t ns_all = (int64_t)groups.size();
  if (ns_all > g->n) {  // the source table holds n groups: run the rest in further launches
    for (int64_t b = 0; b < ns_all; b += g->n) {
      const std::vector<Group> part(groups.begin() + b, groups.begin() + std::min<int64_t>(ns_all, b + g->n));
      CallOut o;
      bc_status s = run_wg(g, r, ext, tg, part, wsbase, st, slots, nslots, ex, &o);
      if (s != BC_OK) return s;
      out->merge(o);
      out->ovf.insert(out->ovf.end(), o.ovf.begin(), o.ovf.end());
    }
    return BC_OK;
  }
  const int64_t ns = ns_all;
  WgWs w;
  wg_layout(g->n, grid, g->n, wsbase, &w);
  HIPCHK(hipMemsetAsync(w.ctl_begin, 0, w.ctl_bytes, st));
  HIPCHK(hipMemsetAsync(w.vs, 0, sizeof(WgVert) * (size_t)grid * g->n, st));  // not reached
  if (ns == 0) return BC_OK;
  std::vector<int32_t> hs((size_t)ns), ho((size_t)ns);
  std::vector<double> hw((size_t)ns), ht((size_t)ns);
  std::vector<double*> hb((size_t)ns);
  for (int64_t i = 0; i < ns; ++i) {
    hs[i] = groups[i].v;
    ho[i] = groups[i].own;
    hw[i] = groups[i].w;
    ht[i] = groups[i].tsub;
    if (groups[i].slot < 0 || groups[i].slot >= nslots) return fail(BC_E_INVALID_ARG, "source group without a result slot");
    hb[i] = slots[groups[i].slot];
  }
  HIPCHK(hipMemcpyAsync(w.sbc, hb.data(), sizeof(double*) * ns, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(w.src, hs.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(w.own, ho.data(), sizeof(int32_t) * ns, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(w.w, hw.data(), sizeof(double) * ns, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(w.tsub, ht.data(), sizeof(double) * ns, hipMemcpyHostToDevice, st));
  WgArgs a{};
  a.n = g->n;
  bc_status es = ensure_ell(g, tg.omega != nullptr, tg, &a.ell);
  if (es != BC_OK) return es;
  a.ci = tg.ci;
  a.omega = tg.omega;
  a.vs = w.vs;
  a.Q = w.Q;
  a.qoff = w.qoff;
  a.src = w.src;
  a.w = w.w;
  a.own = w.own;
  a.tsub = w.tsub;
  a.nsrc = ns;
  a.sbc = w.sbc;
  a.ovf_list = w.ovf_list;
  a.ovf_count = w.ovf_count;
  a.stats = w.stats;
  if (ex) HIPCHK(ex->mark(st));
  HIPCHK(launch_wg(a, ext, (int)std::min<int64_t>(grid, ns), st));
  if (ex) HIPCHK(ex->mark(st));
  int32_t cnt = 0;
  HIPCHK(hipMemcpyAsync(&cnt, w.ovf_count, sizeof cnt, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(out->st, w.stats, sizeof(out->st), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (ex) HIPCHK(ex->collect(&out->kernel_ms));
  out->ovf.resize(std::min<int64_t>(cnt, ns));
  if (cnt) HIPCHK(hipMemcpy(out->ovf.data(), w.ovf_list, sizeof(int32_t) * out->ovf.size(), hipMemcpyDeviceToHost));
  return BC_OK;
}

static void add_stats(bc_run_stats* s, const CallOut& o) {
  s->levels += (int64_t)o.st[kStLevels];
  s->bottom_up_levels += (int64_t)o.st[kStBuLevels];
  s->reached += (int64_t)o.st[kStReached];
  s->reached_nnz += (int64_t)o.st[kStReachedNnz];
  s->dag_edges += (int64_t)o.st[kStDag];
  s->launches += (int64_t)o.st[kStLaunches];
  s->kernel_ms += o.kernel_ms;
}

// Workspace: the caller's, or the graph's cached one (grown on demand).
static bc_status get_ws(bc_graph* g, size_t need, void* user, size_t user_bytes, char** out) {
  if (user) {
    if (user_bytes < need) return fail(BC_E_OUT_OF_MEMORY, "workspace smaller than bc_workspace_size()");
    *out = (char*)user;
    return BC_OK;
  }
  if (g->ws_bytes < need) {
    if (g->ws) HIPCHK(hipFree(g->ws));
    g->ws = nullptr;
    g->ws_bytes = 0;
    if (hipMalloc(&g->ws, need) != hipSuccess) return fail(BC_E_OUT_OF_MEMORY, "workspace allocation failed");
    g->ws_bytes = need;
  }
  *out = (char*)g->ws;
  return BC_OK;
}

// The groups whose vertex is listed (every group of that vertex: several
// result slots may traverse the same vertex).
static std::vector<Group> groups_at(int32_t n, const std::vector<Group>& groups, const std::vector<int32_t>& vs) {
  std::vector<char> mark((size_t)n, 0);
  for (int32_t v : vs) if (v >= 0 && v < n) mark[v] = 1;
  std::vector<Group> out;
  for (const auto& gr : groups) if (mark[gr.v]) out.push_back(gr);
  return out;
}

// Runs groups in the chosen mode; in batched mode, batches that exceed a
// list capacity (they add nothing) are rerun once with worst-case lists.
static bc_status run_groups(bc_graph* g, const Resolved& r, bool ext, const TravGraph& tg,
                            const std::vector<Group>& groups, const std::vector<Triple>& triples, void* user_ws,
                            size_t user_bytes, hipStream_t st, double* const* slots, int nslots, Exec* ex,
                            CallOut* out) {
  char* ws = nullptr;
  bc_status s = get_ws(g, ws_bytes_for(g, r, r.cap_factor), user_ws, user_bytes, &ws);
  if (s != BC_OK) return s;
  if (r.mode == BC_MODE_PLAIN_SCAN && !ext) return run_scan(g, r, tg, groups, ws, st, slots[0], ex, out);
  if (r.mode == BC_MODE_PER_WORKGROUP) return run_wg(g, r, ext, tg, groups, ws, st, slots, nslots, ex, out);
  if (r.mode == BC_MODE_PLAIN || r.mode == BC_MODE_PLAIN_SCAN) {  // (wrapped scan sources: extended plain form)
    s = run_plain(g, r, ext, tg, groups, ws, st, slots[0], nullptr, ex, out);
    if (s == BC_OK && out->err) return fail(BC_E_CAPACITY, "level-list capacity exceeded");
    return s;
  }
  s = run_batched(g, r, ext, tg, groups, triples, ws, r.cap_factor, st, slots, nslots, nullptr, ex, out, nullptr);
  if (s != BC_OK || out->fail.empty()) return s;
  if (user_ws) return fail(BC_E_CAPACITY, "level-list capacity exceeded; some batches added nothing");
  // rerun the failed batches' sources without derivation, with lists sized
  // for the worst case (n * B entries); if that would not fit 32-bit list
  // indices, with narrower batches
  std::vector<Group> again = groups_at(g->n, groups, out->fail);
  Resolved r2 = r;
  while (r2.B > 64 && (int64_t)g->n * r2.B + 1024 > (int64_t)INT32_MAX / 2) {
    r2.B = std::max(64, r2.B / 128 * 64);
    r2.K = r2.B / 64;
  }
  if ((int64_t)g->n * r2.B + 1024 > (int64_t)INT32_MAX / 2)
    return fail(BC_E_CAPACITY, "graph too large for worst-case level lists");
  s = get_ws(g, ws_bytes_for(g, r2, r2.B), nullptr, 0, &ws);
  if (s != BC_OK) return s;
  CallOut o2;
  s = run_batched(g, r2, ext, tg, again, {}, ws, r2.B, st, slots, nslots, nullptr, ex, &o2, nullptr);
  if (s != BC_OK) return s;
  if (!o2.fail.empty()) return fail(BC_E_CAPACITY, "level-list capacity exceeded at worst-case size");
  out->merge(o2);
  out->ovf.insert(out->ovf.end(), o2.ovf.begin(), o2.ovf.end());
  out->fail.clear();
  return BC_OK;
}

// The full compute path shared by bc_compute and the server: `slots[i]` is
// the device score array of result slot i (Group::slot).
bc_status compute_groups(bc_graph* g, const Resolved& r, std::vector<Group>& groups, int64_t credited,
                         void* workspace, size_t ws_bytes, hipStream_t st, double* const* slots, int nslots,
                         Exec* ex, bc_run_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  HIPCHK(hipSetDevice(g->ctx->device));
  const TravGraph tg = trav(g, r.deg1);
  std::vector<Triple> triples;
  if (r.mode == BC_MODE_BATCHED) {
    // sources close in the graph share words: denser level masks and rows
    std::call_once(g->rank_once, [g] { g->rank = locality_rank(g->n, g->h_rp.data(), g->h_ci.data()); });
    order_groups(g->rank, groups);
  }
  // AUTO counts probe one word of sources first (below); 2-degree
  // derivation is chosen among the other sources
  // (once a probe on this graph has found most counts wrapping, later calls
  // go to the extended form directly)
  const bool auto_counts =
      (r.mode == BC_MODE_BATCHED || r.mode == BC_MODE_PER_WORKGROUP) && r.sigma_mode == BC_SIGMA_AUTO;
  const bool hinted = auto_counts && g->ext_hint.load();
  const bool probe = auto_counts && !hinted &&
                     groups.size() > (size_t)(r.mode == BC_MODE_PER_WORKGROUP ? 64 : r.B);
  std::vector<Group> rest;
  if (probe) rest.assign(groups.begin() + 64, groups.end());
  if (r.deg2) choose_deg2(g->n, tg.h_rp, tg.h_ci, probe ? rest : groups, &triples);
  bc_run_stats rs{};
  for (int i = 0; i < 8; ++i) rs.first_overflow[i] = -1;
  rs.sources = credited;
  rs.traversed = (int64_t)groups.size() - (int64_t)triples.size();
  rs.derived = (int64_t)triples.size();
  rs.te = (double)credited * (double)(g->nnz / 2);
  bool ext0 = r.sigma_mode == BC_SIGMA_EXTENDED || hinted;
  // extended batches on such graphs: worst-case lists, batches narrow enough
  // for them (when the library owns the workspace)
  auto worst_case = [&](Resolved* q) {
    if (workspace || q->mode != BC_MODE_BATCHED) return;
    q->cap_factor = 64;
    while (q->B > 64 && (int64_t)g->n * q->B + 1024 > (int64_t)INT32_MAX / 2) {
      q->B /= 2;
      q->K = q->B / 64;
    }
  };
  CallOut co;
  bc_status s = BC_OK;
  if (probe) {
    // probe: one word of sources in exact form (lists at their worst-case
    // size); if most of them wrap (long diameters), the other batches go
    // straight to the extended form, and - when the library owns the
    // workspace - with worst-case lists and batches narrow enough for them,
    // since on such graphs a vertex sits on a different level for nearly
    // every source
    Resolved rp = r, rr = r;
    rp.B = 64;
    rp.K = 1;
    rp.cap_factor = 64;
    std::vector<Group> head(groups.begin(), groups.begin() + 64);
    s = run_groups(g, workspace ? r : rp, false, tg, head, {}, workspace, ws_bytes, st, slots, nslots, ex, &co);
    if (s != BC_OK) return s;
    if (2 * co.ovf.size() > head.size()) {
      ext0 = true;
      g->ext_hint.store(true);
      worst_case(&rr);
    }
    CallOut c2;
    s = run_groups(g, rr, ext0, tg, rest, triples, workspace, ws_bytes, st, slots, nslots, ex, &c2);
    if (s != BC_OK) return s;
    co.merge(c2);
    co.ovf.insert(co.ovf.end(), c2.ovf.begin(), c2.ovf.end());
  } else {
    Resolved rh = r;
    if (hinted) worst_case(&rh);
    s = run_groups(g, rh, ext0, tg, groups, triples, workspace, ws_bytes, st, slots, nslots, ex, &co);
    if (s != BC_OK) return s;
  }
  add_stats(&rs, co);
  std::vector<int32_t> ov = co.ovf;
  std::sort(ov.begin(), ov.end());
  ov.erase(std::unique(ov.begin(), ov.end()), ov.end());
  rs.overflowed = (int64_t)ov.size();
  for (size_t i = 0; i < ov.size() && i < 8; ++i) rs.first_overflow[i] = ov[i];
  if (!ov.empty() && r.sigma_mode == BC_SIGMA_AUTO) {
    std::vector<Group> again = groups_at(g->n, groups, ov);
    CallOut c2;
    s = run_groups(g, r, true, tg, again, {}, workspace, ws_bytes, st, slots, nslots, ex, &c2);
    if (s != BC_OK) return s;
    add_stats(&rs, c2);
    rs.rerun_extended = (int64_t)again.size();
  }
  rs.raw_te = (double)rs.traversed * (double)(tg.nnz / 2);
  rs.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  rs.mode = r.mode;
  if (stats) *stats = rs;
  return BC_OK;
}

bc_status resolve_opts(const bc_graph* g, const bc_compute_opts* o, Resolved* r) { return resolve(g, o, r); }

bc_status compute_noalloc(bc_graph* g, const int32_t* sources, int64_t k, const bc_compute_opts* opts, void* scratch,
                          size_t scratch_bytes, hipStream_t st, bc_run_stats* stats) {
  std::lock_guard<std::mutex> lk(g->mu);
  Resolved r;
  bc_status s = resolve(g, opts, &r);
  if (s != BC_OK) return s;
  if (r.mode != BC_MODE_PLAIN) return fail(BC_E_INVALID_ARG, "bc_compute_noalloc runs the plain form only");
  if (r.graph_launches) return fail(BC_E_INVALID_ARG, "bc_compute_noalloc takes no graph_launches (a graph allocates)");
  r.no_alloc = true;
  const size_t need = ws_bytes_for(g, r, r.cap_factor);
  if (need > scratch_bytes)
    return fail(BC_E_CAPACITY, "graph needs " + std::to_string(need) + " bytes of workspace; bc_compute_noalloc holds " +
                                   std::to_string(scratch_bytes));
  if (k < 0 || (!sources && k != 0 && k != g->n)) return fail(BC_E_INVALID_ARG, "bad source count");
  if (!sources) k = g->n;
  for (int64_t i = 0; sources && i < k; ++i)
    if (sources[i] < 0 || sources[i] >= g->n) return fail(BC_E_INVALID_ARG, "source id out of range");
  std::vector<int32_t> isrc;
  if (sources) isrc = to_internal(g, sources, k);
  std::vector<Group> groups;
  int64_t credited = 0;
  map_sources(g->n, g->h_rp.data(), r.deg1 ? &g->pr : nullptr, sources ? isrc.data() : nullptr, k, &groups,
              &credited);
  double* slots[1] = {g->d_bc};
  bc_status s2 = compute_groups(g, r, groups, credited, scratch, scratch_bytes, st, slots, 1, nullptr, stats);
  if (s2 == BC_OK) add_tree_scores(g, r, sources ? isrc.data() : nullptr, k);
  return s2;
}

void graph_groups(const bc_graph* g, const Resolved& r, const int32_t* sources, int64_t k, std::vector<Group>* groups,
                  int64_t* credited) {
  const std::vector<int32_t> isrc = to_internal(g, sources, k);
  map_sources(g->n, g->h_rp.data(), r.deg1 ? &g->pr : nullptr, isrc.data(), k, groups, credited);
}

int64_t graph_n(const bc_graph* g) { return g->n; }
int context_device(const bc_context* c) { return c->device; }
int context_cus(const bc_context* c) { return c->cus; }
bool graph_pruned(const bc_graph* g) { return g->pruned; }
int batch_occupancy(int K) {
  int e = 0, x = 0;
  (void)K;
  if (batch_max_grid(false, kBatchBlock, &e) != hipSuccess || batch_max_grid(true, kBatchBlock, &x) != hipSuccess)
    return 0;
  return std::min(e, x);
}
int64_t graph_nnz(const bc_graph* g) { return g->nnz; }
int graph_device(const bc_graph* g) { return g->ctx->device; }
size_t graph_ws_bytes(const bc_graph* g, const Resolved& r) { return ws_bytes_for(g, r, r.cap_factor); }

}  // namespace bcx

extern "C" {

bc_status bc_workspace_size(const bc_graph* g, const bc_compute_opts* opts, size_t* bytes) {
  if (!g || !bytes) return fail(BC_E_INVALID_ARG, "null argument");
  Resolved r;
  bc_status s = resolve(g, opts, &r);
  if (s != BC_OK) return s;
  *bytes = ws_bytes_for(g, r, 32);
  return BC_OK;
}

bc_status bc_compute(bc_graph* g, const int32_t* sources, int64_t k, const bc_compute_opts* opts, void* workspace,
                     size_t ws_bytes, void* stream, bc_run_stats* stats) {
  if (!g) return fail(BC_E_INVALID_ARG, "null graph");
  std::lock_guard<std::mutex> lk(g->mu);
  Resolved r;
  bc_status s = resolve(g, opts, &r);
  if (s != BC_OK) return s;
  if (k < 0 || (!sources && k != 0 && k != g->n)) return fail(BC_E_INVALID_ARG, "bad source count");
  if (!sources) k = g->n;
  for (int64_t i = 0; sources && i < k; ++i)
    if (sources[i] < 0 || sources[i] >= g->n) return fail(BC_E_INVALID_ARG, "source id out of range");
  std::vector<int32_t> isrc;
  if (sources) isrc = to_internal(g, sources, k);
  std::vector<Group> groups;
  int64_t credited = 0;
  map_sources(g->n, g->h_rp.data(), r.deg1 ? &g->pr : nullptr, sources ? isrc.data() : nullptr, k, &groups,
              &credited);
  double* slots[1] = {g->d_bc};
  bc_status s2 = compute_groups(g, r, groups, credited, workspace, ws_bytes, (hipStream_t)stream, slots, 1, &g->exec,
                                stats);
  if (s2 == BC_OK) add_tree_scores(g, r, sources ? isrc.data() : nullptr, k);
  return s2;
}

bc_status bc_scores(const bc_graph* g, double* out, int32_t norm, int32_t out_on_device) {
  if (!g || !out) return fail(BC_E_INVALID_ARG, "null argument");
  if (norm != BC_RAW && norm != BC_UNDIRECTED) return fail(BC_E_INVALID_ARG, "unknown normalisation");
  HIPCHK(hipSetDevice(g->ctx->device));
  std::vector<double> h((size_t)g->n);
  HIPCHK(hipMemcpy(h.data(), g->d_bc, sizeof(double) * g->n, hipMemcpyDeviceToHost));
  if (!g->h_tree.empty())
    for (int64_t v = 0; v < g->n; ++v) h[v] += g->h_tree[v];
  scores_to_caller(g, h.data());
  if (norm == BC_UNDIRECTED) for (auto& x : h) x *= 0.5;
  if (out_on_device) HIPCHK(hipMemcpy(out, h.data(), sizeof(double) * g->n, hipMemcpyHostToDevice));
  else memcpy(out, h.data(), sizeof(double) * g->n);
  return BC_OK;
}

bc_status bc_scores_reset(bc_graph* g) {
  if (!g) return fail(BC_E_INVALID_ARG, "null graph");
  HIPCHK(hipSetDevice(g->ctx->device));
  HIPCHK(hipMemset(g->d_bc, 0, sizeof(double) * g->n));
  std::fill(g->h_tree.begin(), g->h_tree.end(), 0.0);
  return BC_OK;
}

bc_status bc_autotune(bc_graph* g, const int32_t* sample, int64_t k, bc_compute_opts* opts, double budget_ms,
                      double* gteps) {
  if (!g || !sample || k <= 0 || !opts) return fail(BC_E_INVALID_ARG, "bad arguments");
  for (int64_t i = 0; i < k; ++i)
    if (sample[i] < 0 || sample[i] >= g->n) return fail(BC_E_INVALID_ARG, "source id out of range");
  std::lock_guard<std::mutex> lk(g->mu);
  HIPCHK(hipSetDevice(g->ctx->device));
  bc_compute_opts base = *opts;
  base.mode = BC_MODE_BATCHED;
  Resolved r0;
  bc_status s = resolve(g, &base, &r0);
  if (s != BC_OK) return s;
  std::vector<Group> groups;
  int64_t credited = 0;
  const std::vector<int32_t> isample = to_internal(g, sample, k);
  map_sources(g->n, g->h_rp.data(), r0.deg1 ? &g->pr : nullptr, isample.data(), k, &groups, &credited);
  if (groups.empty()) return fail(BC_E_INVALID_ARG, "sample has no non-isolated source");
  double* scratch = nullptr;
  HIPCHK(hipMalloc((void**)&scratch, sizeof(double) * g->n));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const auto t_start = std::chrono::steady_clock::now();
  auto elapsed = [&] {
    return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start).count();
  };
  auto trial = [&](const bc_compute_opts& o, double* ms) -> bc_status {
    Resolved r;
    bc_status st = resolve(g, &o, &r);
    if (st != BC_OK) return st;
    std::vector<Group> gr = groups;
    double* slots[1] = {scratch};
    HIPCHK(hipEventRecord(e0, nullptr));
    st = compute_groups(g, r, gr, credited, nullptr, 0, nullptr, slots, 1, &g->exec, nullptr);
    HIPCHK(hipEventRecord(e1, nullptr));
    HIPCHK(hipEventSynchronize(e1));
    float f = 0.f;
    HIPCHK(hipEventElapsedTime(&f, e0, e1));
    *ms = f;
    return st;
  };
  bc_compute_opts best = base;
  if (!best.batch) best.batch = 256;
  best.grid_per_cu = 0;
  double best_ms = 0.0;
  s = trial(best, &best_ms);             // warms allocations
  if (s == BC_OK) s = trial(best, &best_ms);
  auto consider = [&](bc_compute_opts o) {
    if (s != BC_OK || (budget_ms > 0 && elapsed() > budget_ms)) return;
    double ms = 0.0;
    bc_status st = trial(o, &ms);
    if (st == BC_OK && ms < best_ms) { best = o; best_ms = ms; }
    if (st != BC_OK && st != BC_E_CAPACITY) s = st;
  };
  for (int B : {64, 128, 256, 512, 1024}) { bc_compute_opts o = best; o.batch = B; if (B != best.batch) consider(o); }
  for (double al : {-1.0, 0.5, 1.0, 2.0, 4.0, 8.0}) { bc_compute_opts o = best; o.alpha = al; consider(o); }
  if (best.alpha >= 0)  // bottom-up in play: its switch-back threshold
    for (double be : {2.0, 8.0, 24.0, 64.0}) { bc_compute_opts o = best; o.beta = be; consider(o); }
  {
    int occ = 0;
    if (batch_max_grid(false, kBatchBlock, &occ) == hipSuccess && occ > 1) {
      bc_compute_opts o = best;
      o.grid_per_cu = occ / 2;
      consider(o);
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipFree(scratch);
  if (s != BC_OK) return s;
  g->tuned = true;
  g->tuned_batch = best.batch;
  g->tuned_alpha = best.alpha > 0 ? best.alpha : 0.0;  // 0: never bottom-up
  g->tuned_grid = best.grid_per_cu;
  g->tuned_beta = best.beta;
  {  // graphs of the same shape loaded later in this context start from it
    std::lock_guard<std::mutex> tl(g->ctx->tune_mu);
    g->ctx->tune_cache[shape_key(g, r0.deg1)] =
        TunedSet{g->tuned_batch, g->tuned_grid, g->tuned_alpha, g->tuned_beta};
  }
  *opts = best;
  if (gteps) *gteps = (double)credited * (double)(g->nnz / 2) / (best_ms * 1e-3) / 1e9;
  return BC_OK;
}

static bc_status trace_internal(bc_graph* g, const int32_t* sources, int64_t k, const bc_compute_opts* opts,
                                int32_t* d, uint64_t* sigma, double* sigma_mant, int32_t* sigma_exp, double* delta,
                                int32_t* overflow);

bc_status bc_trace(bc_graph* g, const int32_t* sources, int64_t k, const bc_compute_opts* opts, int32_t* d,
                   uint64_t* sigma, double* sigma_mant, int32_t* sigma_exp, double* delta, int32_t* overflow) {
  if (!g || !sources || k <= 0) return fail(BC_E_INVALID_ARG, "bad arguments");
  for (int64_t i = 0; i < k; ++i)
    if (sources[i] < 0 || sources[i] >= g->n) return fail(BC_E_INVALID_ARG, "source id out of range");
  std::lock_guard<std::mutex> lk(g->mu);
  const std::vector<int32_t> isrc = to_internal(g, sources, k);
  bc_status s = trace_internal(g, isrc.data(), k, opts, d, sigma, sigma_mant, sigma_exp, delta, overflow);
  if (s != BC_OK) return s;
  rows_to_caller(g, d, k);
  rows_to_caller(g, sigma, k);
  rows_to_caller(g, sigma_mant, k);
  rows_to_caller(g, sigma_exp, k);
  rows_to_caller(g, delta, k);
  return BC_OK;
}

static bc_status trace_internal(bc_graph* g, const int32_t* sources, int64_t k, const bc_compute_opts* opts,
                                int32_t* d, uint64_t* sigma, double* sigma_mant, int32_t* sigma_exp, double* delta,
                                int32_t* overflow) {
  Resolved r;
  bc_status s = resolve(g, opts, &r);
  if (s != BC_OK) return s;
  if (r.deg1 || (r.deg2 && r.mode != BC_MODE_BATCHED))
    return fail(BC_E_INVALID_ARG, "traces run on the unpruned graph (2-degree derivation: batched only)");
  if (r.mode == BC_MODE_PLAIN_SCAN || r.mode == BC_MODE_PER_WORKGROUP)
    return fail(BC_E_INVALID_ARG, "traces run in the plain or batched mode");
  r.trace = true;
  r.graph_launches = 0;
  for (int64_t i = 0; i < k; ++i)
    if (sources[i] < 0 || sources[i] >= g->n) return fail(BC_E_INVALID_ARG, "source id out of range");
  HIPCHK(hipSetDevice(g->ctx->device));
  const int64_t n = g->n;
  const TravGraph tg = trav(g, false);
  hipStream_t st = nullptr;
  const bool ext_only = r.sigma_mode == BC_SIGMA_EXTENDED;
  const bool rerun = r.sigma_mode == BC_SIGMA_AUTO;
  char* ws = nullptr;
  s = get_ws(g, ws_bytes_for(g, r, r.B), nullptr, 0, &ws);
  if (s != BC_OK) return s;
  std::vector<int32_t> ovf_row((size_t)k, 0);

  if (r.mode == BC_MODE_PLAIN) {
    PlainWs w;
    plain_layout(n, g->nnz, ws, &w);
    for (int64_t i = 0; i < k; ++i) {
      const std::vector<Group> one{Group{sources[i], 1.0, 0, 0}};
      for (int pass = 0; pass < 2; ++pass) {
        const bool ext = ext_only || pass == 1;
        HIPCHK(hipMemset(w.delta, 0, sizeof(double) * n));
        HIPCHK(hipMemset(w.bc_tmp, 0, sizeof(double) * n));
        CallOut co;
        s = run_plain(g, r, ext, tg, one, ws, st, w.bc_tmp, w.delta, &g->exec, &co);
        if (s != BC_OK) return s;
        if (co.err) return fail(BC_E_CAPACITY, "capacity exceeded");
        if (pass == 0 && !ext) ovf_row[i] = co.ovf.empty() ? 0 : 1;
        if (d) HIPCHK(hipMemcpy(d + i * n, w.d, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
        if (!ext) {
          std::vector<uint64_t> sg((size_t)n);
          HIPCHK(hipMemcpy(sg.data(), w.sig, sizeof(uint64_t) * n, hipMemcpyDeviceToHost));
          if (sigma) memcpy(sigma + i * n, sg.data(), sizeof(uint64_t) * n);
          if (sigma_mant) for (int64_t v = 0; v < n; ++v) sigma_mant[i * n + v] = (double)sg[v];
          if (sigma_exp) memset(sigma_exp + i * n, 0, sizeof(int32_t) * n);
        } else {
          if (sigma) memset(sigma + i * n, 0, sizeof(uint64_t) * n);
          if (sigma_mant) HIPCHK(hipMemcpy(sigma_mant + i * n, w.sm, sizeof(double) * n, hipMemcpyDeviceToHost));
          if (sigma_exp) HIPCHK(hipMemcpy(sigma_exp + i * n, w.se, sizeof(int32_t) * n, hipMemcpyDeviceToHost));
        }
        if (delta) HIPCHK(hipMemcpy(delta + i * n, w.delta, sizeof(double) * n, hipMemcpyDeviceToHost));
        if (ext || !ovf_row[i] || !rerun) break;
      }
    }
    if (overflow) memcpy(overflow, ovf_row.data(), sizeof(int32_t) * k);
    return BC_OK;
  }

  // batched traces: every source its own lane, all in result slot 0 (scratch)
  const int B = r.B;
  BatchWs w;
  batch_layout(n, g->nnz, B, B, r.max_slots, true, ws, &w);
  const size_t cells = (size_t)B * n;
  double *dd = nullptr, *dbc = nullptr;
  uint64_t* dsg = nullptr;
  int32_t* dse = nullptr;
  bc_status res = BC_OK;
  if (hipMalloc((void**)&dd, sizeof(double) * cells) != hipSuccess ||
      hipMalloc((void**)&dsg, sizeof(uint64_t) * cells) != hipSuccess ||
      hipMalloc((void**)&dse, sizeof(int32_t) * cells) != hipSuccess ||
      hipMalloc((void**)&dbc, sizeof(double) * n) != hipSuccess)
    res = fail(BC_E_OUT_OF_MEMORY, "trace buffers");
  std::vector<int32_t> lv((size_t)n * B);
  std::vector<uint64_t> vis((size_t)n * r.K), dla((size_t)n * r.K), dlb((size_t)n * r.K);
  std::vector<double> hd(cells), hm;
  std::vector<uint64_t> hs;
  std::vector<int32_t> he;
  double* slots[1] = {dbc};
  for (int64_t b0 = 0, nb = 0; b0 < k && res == BC_OK; b0 += nb) {
    nb = std::min<int64_t>(B, k - b0);
    if (r.deg2) {
      // triples share a word, so padding can push B sources past one launch:
      // take fewer sources until their lanes pack into one
      while (nb > 1) {
        std::vector<Group> probe;
        for (int64_t i = 0; i < nb; ++i) probe.push_back(Group{sources[b0 + i], 1.0, 0, 0});
        std::vector<Triple> tp;
        choose_deg2(g->n, tg.h_rp, tg.h_ci, probe, &tp);
        Packing pk;
        pack_lanes(probe, tp, B, &pk);
        if (pk.nbatches <= 1) break;
        nb -= 8;
        if (nb < 1) nb = 1;
      }
    }
    for (int pass = 0; pass < 2 && res == BC_OK; ++pass) {
      const bool ext = ext_only || pass == 1;
      std::vector<Group> run;
      std::vector<int64_t> row;  // trace row of each group
      for (int64_t i = 0; i < nb; ++i) {
        if (pass == 1 && !ovf_row[b0 + i]) continue;
        run.push_back(Group{sources[b0 + i], 1.0, 0, 0});
        row.push_back(b0 + i);
      }
      if (run.empty()) break;
      if (hipMemset(dd, 0, sizeof(double) * cells) != hipSuccess) { res = fail(BC_E_DEVICE, "memset"); break; }
      // 2-degree derivation on the first pass (reruns of wrapped sources traverse)
      std::vector<Triple> triples;
      if (r.deg2 && pass == 0) choose_deg2(g->n, tg.h_rp, tg.h_ci, run, &triples);
      std::vector<char> derived(run.size(), 0);
      std::vector<std::pair<int32_t, int32_t>> partners(run.size(), {-1, -1});
      for (const auto& t : triples) {
        derived[t.c] = 1;
        partners[t.c] = {t.a, t.b};
      }
      TraceDev tdv{dd, dsg, (double*)dsg, dse, dbc};
      CallOut co;
      std::vector<int32_t> lanes;
      res = run_batched(g, r, ext, tg, run, triples, ws, B, st, slots, 1, &tdv, &g->exec, &co, &lanes);
      if (res != BC_OK) break;
      if (!co.fail.empty()) { res = fail(BC_E_CAPACITY, "capacity exceeded"); break; }
      if (hipMemcpy(lv.data(), w.lv, sizeof(int32_t) * lv.size(), hipMemcpyDeviceToHost) != hipSuccess ||
          hipMemcpy(vis.data(), w.vis, sizeof(uint64_t) * vis.size(), hipMemcpyDeviceToHost) != hipSuccess ||
          (!triples.empty() &&
           (hipMemcpy(dla.data(), w.dla, sizeof(uint64_t) * dla.size(), hipMemcpyDeviceToHost) != hipSuccess ||
            hipMemcpy(dlb.data(), w.dlb, sizeof(uint64_t) * dlb.size(), hipMemcpyDeviceToHost) != hipSuccess)) ||
          hipMemcpy(hd.data(), dd, sizeof(double) * cells, hipMemcpyDeviceToHost) != hipSuccess) {
        res = fail(BC_E_DEVICE, "trace copy");
        break;
      }
      if (ext) {
        hm.resize(cells);
        he.resize(cells);
        (void)hipMemcpy(hm.data(), dsg, sizeof(double) * cells, hipMemcpyDeviceToHost);
        (void)hipMemcpy(he.data(), dse, sizeof(int32_t) * cells, hipMemcpyDeviceToHost);
      } else {
        hs.resize(cells);
        (void)hipMemcpy(hs.data(), dsg, sizeof(uint64_t) * cells, hipMemcpyDeviceToHost);
      }
      std::vector<char> wrapped(run.size(), 0);
      for (int32_t v : co.ovf)
        for (size_t gi = 0; gi < run.size(); ++gi)
          if (run[gi].v == v) wrapped[gi] = 1;
      std::vector<int32_t> lane_of(run.size(), -1);
      for (int j = 0; j < B; ++j)
        if (lanes[j] >= 0) lane_of[lanes[j]] = j;
      for (int j = 0; j < B; ++j) {
        const int32_t gi = lanes[j];
        if (gi < 0) continue;
        const int64_t rw = row[gi];
        if (pass == 0 && !ext) ovf_row[rw] = wrapped[gi];
        // a derived source keeps no levels of its own: it reaches v where the
        // kernel recorded a partner's arrival (dla / dlb), at 1 + the smaller
        // of the partners' levels; its own vertex is level 0 with one path
        const int ja = derived[gi] ? lane_of[partners[gi].first] : -1;
        const int jb = derived[gi] ? lane_of[partners[gi].second] : -1;
        for (int64_t v = 0; v < n; ++v) {
          const size_t vk = (size_t)v * r.K + (j >> 6);
          bool reached = (vis[vk] >> (j & 63)) & 1ull;
          int32_t lvl = reached ? lv[(size_t)v * B + j] : -1;
          const bool self = derived[gi] && v == run[gi].v;
          if (derived[gi]) {
            reached = self || (((dla[vk] | dlb[vk]) >> (j & 63)) & 1ull);
            lvl = -1;
            if (self) {
              lvl = 0;
            } else if (reached) {
              const bool ra = (vis[(size_t)v * r.K + (ja >> 6)] >> (ja & 63)) & 1ull;
              const bool rb = (vis[(size_t)v * r.K + (jb >> 6)] >> (jb & 63)) & 1ull;
              const int32_t la = ra ? lv[(size_t)v * B + ja] : INT32_MAX, lb = rb ? lv[(size_t)v * B + jb] : INT32_MAX;
              lvl = 1 + std::min(la, lb);
            }
          }
          const size_t c = (size_t)j * n + v;
          if (d) d[rw * n + v] = lvl;
          if (self) {
            if (sigma) sigma[rw * n + v] = ext ? 0 : 1;
            if (sigma_mant) sigma_mant[rw * n + v] = 1.0;
            if (sigma_exp) sigma_exp[rw * n + v] = 0;
          } else if (ext) {
            if (sigma) sigma[rw * n + v] = 0;
            if (sigma_mant) sigma_mant[rw * n + v] = hm[c];
            if (sigma_exp) sigma_exp[rw * n + v] = he[c];
          } else {
            if (sigma) sigma[rw * n + v] = hs[c];
            if (sigma_mant) sigma_mant[rw * n + v] = (double)hs[c];
            if (sigma_exp) sigma_exp[rw * n + v] = 0;
          }
          if (delta) delta[rw * n + v] = hd[c];
        }
      }
      if (ext || !rerun) break;
    }
  }
  if (dd) (void)hipFree(dd);
  if (dsg) (void)hipFree(dsg);
  if (dse) (void)hipFree(dse);
  if (dbc) (void)hipFree(dbc);
  if (res == BC_OK && overflow) memcpy(overflow, ovf_row.data(), sizeof(int32_t) * k);
  return res;
}

}  // extern "C"
