// Continuous-batching server for betweenness queries (graph, source subset).
//
// Queries wait in a FIFO.  A query is admitted when its result array fits
// the HBM budget next to the other admitted queries' results and one
// workspace for the largest graph among them (so some batch can always run);
// a query that could never fit alone is rejected.  Worker threads (one HIP
// stream and one cached workspace each) repeatedly form a batch: the sources
// of the oldest admitted query that is not running, topped up with sources
// of other admitted queries on the same graph, each query's sweeps writing
// into its own result array (one result slot per query in the batch).  A
// query takes part in at most one running batch at a time, so its result
// array has a single writer.
//
// Batches of different queries and graphs run at the same time on their
// workers' streams.  The workgroups the device keeps resident are cut into
// max_inflight shares and a batch's persistent grid holds whole shares, never
// more than are free, so all running grids fit on the device together (their
// grid barriers never wait for a workgroup that another grid keeps out).  A
// batch takes one share while other queries wait for a batch; a query that
// is alone takes every free share but one, the one left for the next query
// to arrive, so a large query on an otherwise idle server is not held to a
// quarter of the device.
//
// Device memory is never allocated or freed while the server lock is held:
// admission and batch formation only do the accounting, the worker (or the
// submitting thread) allocates, zeroes and frees afterwards on its own.
// Result arrays of finished queries go to a pool and are reused; pooled
// arrays and idle workers' workspaces are given back only when the head of
// the queue, or a worker's next batch, cannot otherwise fit the budget.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "../../include/bc.h"
#include "bc_api_internal.h"

using namespace bcx;

namespace {

using Clock = std::chrono::steady_clock;

struct Buf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct Query {
  uint64_t ticket = 0;
  bc_graph* g = nullptr;
  std::vector<Group> groups;  // traversal sources, weights = multiplicity
  size_t next = 0;            // first group not yet dispatched
  int64_t credited = 0;
  double* out = nullptr;      // host result (caller-owned)
  size_t d_bytes = 0;         // result bytes (n doubles)
  int64_t ws_bytes = 0;       // workspace a batch of this query's graph needs
  bool wide = false;          // its batches may take several shares (the batched form: a
                              // workspace that does not grow with the grid)
  Buf res;                    // device result array (from the pool, or to be allocated)
  bool need_alloc = false;    // res is reserved in the budget but not allocated yet
  bool zeroed = false;
  bool admitted = false, running = false, done = false;
  bc_status status = BC_OK;
  double submit_ms = 0, start_ms = -1, end_ms = 0;
  int64_t n = 0, m = 0;
  std::vector<double> tree;   // closed-form scores of tree vertices (iterated reduction), caller order
};

struct Worker {
  std::thread th;
  int shares = 0;  // shares of the device the current batch's grid holds
  hipStream_t st = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  size_t grow_to = 0;  // reserved growth of the workspace, allocated outside the lock
  bool busy = false;
  Exec exec;
};

}  // namespace

struct bc_server {
  int device = 0;
  int grid_share = 0;  // workgroups of one share of the device
  int free_shares = 0;
  bc_server_config cfg{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Query>> queue;       // submitted, not finished
  std::map<uint64_t, std::shared_ptr<Query>> all;  // ticket -> query (until waited)
  std::vector<std::unique_ptr<Worker>> workers;
  uint64_t next_ticket = 1;
  // device bytes: results of admitted unfinished queries, pooled result
  // arrays, worker workspaces (held = all three, including reservations)
  int64_t res_bytes = 0, pool_bytes = 0, ws_bytes = 0;
  std::vector<Buf> pool;     // free result arrays
  std::vector<Buf> to_free;  // given back, freed outside the lock
  bool stop = false;
  // in-flight accounting
  int running = 0, max_running = 0;
  int64_t batches = 0, reclaims = 0, allocations = 0, wide_batches = 0, share_sum = 0;
  double area_ms = 0.0, busy_ms = 0.0, last_change_ms = 0.0;
  Clock::time_point t0 = Clock::now();
  double now_ms() const { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }
  int64_t held() const { return res_bytes + pool_bytes + ws_bytes; }
  void note_running(int delta) {
    const double t = now_ms();
    if (running > 0) {
      area_ms += running * (t - last_change_ms);
      busy_ms += t - last_change_ms;
    }
    last_change_ms = t;
    running += delta;
    max_running = std::max(max_running, running);
  }
};

namespace {

bc_compute_opts serve_opts(const bc_server* s, const bc_graph* g) {
  bc_compute_opts o{};
  o.mode = BC_MODE_AUTO;  // long-diameter graphs run one source per workgroup
  o.batch = s->cfg.batch;
  o.sigma_mode = BC_SIGMA_AUTO;
  o.heuristics = ((s->cfg.heuristics & BC_H_DEG1) && graph_pruned(g)) ? BC_H_DEG1 : 0u;
  return o;
}

bc_status serve_resolved(const bc_server* s, const bc_graph* g, int shares, Resolved* r) {
  bc_compute_opts o = serve_opts(s, g);
  bc_status st = resolve_opts(g, &o, r);
  r->cap_factor = r->B;  // worst-case level lists: a batch never runs out of them
  r->max_slots = 64;
  r->grid_total = s->grid_share * shares;
  return st;
}

// Gives back pooled result arrays and the workspaces of idle workers other
// than `self` (their memory is freed outside the lock).  Lock held.
void reclaim(bc_server* s, const Worker* self) {
  for (auto& b : s->pool) {
    s->pool_bytes -= (int64_t)b.bytes;
    s->to_free.push_back(b);
  }
  s->pool.clear();
  for (auto& w : s->workers) {
    if (w.get() == self || w->busy || !w->ws) continue;
    s->ws_bytes -= (int64_t)w->ws_bytes;
    s->to_free.push_back(Buf{w->ws, w->ws_bytes});
    w->ws = nullptr;
    w->ws_bytes = 0;
  }
  ++s->reclaims;
}

// Frees what was given back.  Called without the lock.
void drain(std::vector<Buf>& bufs) {
  for (auto& b : bufs) (void)hipFree(b.p);
  bufs.clear();
}

// Admission in FIFO order; lock held.  Only accounting: result arrays
// still to be allocated are marked need_alloc.
void admit(bc_server* s) {
  const int64_t budget = s->cfg.hbm_budget_bytes;
  int64_t max_ws = 0;
  for (auto& q : s->queue)
    if (q->admitted && !q->done) max_ws = std::max(max_ws, q->ws_bytes);
  for (auto& q : s->queue) {
    if (q->admitted || q->done) continue;
    if ((int64_t)q->d_bytes + q->ws_bytes > budget) {
      q->status = BC_E_REJECTED;
      q->done = true;
      q->end_ms = s->now_ms();
      continue;
    }
    // room for every admitted result plus one workspace for the largest graph
    const int64_t mw = std::max(max_ws, q->ws_bytes);
    // a pooled array that is large enough (the smallest such), else a new one
    size_t best = s->pool.size();
    for (size_t i = 0; i < s->pool.size(); ++i)
      if (s->pool[i].bytes >= q->d_bytes && (best == s->pool.size() || s->pool[i].bytes < s->pool[best].bytes))
        best = i;
    if (best < s->pool.size() && s->res_bytes + (int64_t)s->pool[best].bytes + mw <= budget) {
      q->res = s->pool[best];
      s->pool.erase(s->pool.begin() + (ptrdiff_t)best);
      s->pool_bytes -= (int64_t)q->res.bytes;
      s->res_bytes += (int64_t)q->res.bytes;
    } else {
      if (s->res_bytes + (int64_t)q->d_bytes + mw > budget) break;  // FIFO: wait
      if (s->held() + (int64_t)q->d_bytes > budget) reclaim(s, nullptr);
      if (s->held() + (int64_t)q->d_bytes > budget) break;  // busy workspaces: wait for them
      q->res = Buf{nullptr, q->d_bytes};
      q->need_alloc = true;
      s->res_bytes += (int64_t)q->d_bytes;
    }
    q->admitted = true;
    max_ws = mw;
  }
  s->cv_done.notify_all();
}

struct Job {
  bc_graph* g = nullptr;
  std::vector<std::shared_ptr<Query>> qs;
  std::vector<Group> lanes;
  std::vector<double*> slots;
};

// Forms the next batch; lock held.  Returns false if none can run now.
bool take_job(bc_server* s, Worker* w, Job* job) {
  const int B = s->cfg.batch;
  if (s->free_shares < 1) return false;
  auto ready = [](const std::shared_ptr<Query>& q) {
    return q->admitted && !q->running && !q->done && q->next < q->groups.size();
  };
  std::shared_ptr<Query> lead;
  for (auto& q : s->queue)
    if (ready(q)) { lead = q; break; }
  if (!lead) return false;
  const size_t need = (size_t)lead->ws_bytes;
  w->grow_to = 0;
  if (w->ws_bytes < need) {
    const int64_t grow = (int64_t)need - (int64_t)w->ws_bytes;
    if (s->held() + grow > s->cfg.hbm_budget_bytes) reclaim(s, w);
    if (s->held() + grow > s->cfg.hbm_budget_bytes) return false;  // wait for running batches
    s->ws_bytes += grow;  // reserved; the worker reallocates outside the lock
    w->grow_to = need;
  }
  job->g = lead->g;
  job->qs.clear();
  job->lanes.clear();
  job->slots.clear();
  for (auto& q : s->queue) {
    if ((int)job->lanes.size() >= B || (int)job->slots.size() >= 64) break;
    if (q->g != lead->g || !ready(q)) continue;
    job->qs.push_back(q);
    q->running = true;
    if (q->start_ms < 0) q->start_ms = s->now_ms();
    const int slot = (int)job->slots.size();
    job->slots.push_back(nullptr);  // filled once the result array exists
    while ((int)job->lanes.size() < B && q->next < q->groups.size()) {
      Group gr = q->groups[q->next++];
      gr.slot = slot;
      job->lanes.push_back(gr);
    }
  }
  // one share while another query waits for a batch, else all free but one
  bool others = false;
  for (auto& q : s->queue)
    if (ready(q)) { others = true; break; }
  w->shares = (others || !lead->wide) ? 1 : std::max(1, s->free_shares - 1);
  s->free_shares -= w->shares;
  s->share_sum += w->shares;
  if (w->shares > 1) ++s->wide_batches;
  w->busy = true;
  s->note_running(+1);
  ++s->batches;
  return true;
}

// Device work of a job that needs no lock: the workspace growth, result
// arrays of first-time queries (allocated and zeroed on the worker's
// stream), the batch itself and the download of finished results.
bc_status run_job(bc_server* s, Worker* w, Job& job, std::vector<std::shared_ptr<Query>>* complete,
                  int64_t* allocs) {
  if (w->grow_to) {
    if (w->ws) (void)hipFree(w->ws);
    w->ws = nullptr;
    if (hipMalloc(&w->ws, w->grow_to) != hipSuccess) {
      w->ws = nullptr;
      return BC_E_OUT_OF_MEMORY;
    }
    ++*allocs;
  }
  for (size_t i = 0; i < job.qs.size(); ++i) {
    Query& q = *job.qs[i];
    if (q.need_alloc) {
      if (hipMalloc(&q.res.p, q.res.bytes) != hipSuccess) { q.res.p = nullptr; return BC_E_OUT_OF_MEMORY; }
      q.need_alloc = false;
      ++*allocs;
    }
    if (!q.zeroed) {
      if (hipMemsetAsync(q.res.p, 0, q.d_bytes, w->st) != hipSuccess) return BC_E_DEVICE;
      q.zeroed = true;
    }
    job.slots[i] = (double*)q.res.p;
  }
  Resolved r;
  bc_status st = serve_resolved(s, job.g, w->shares, &r);
  const size_t cap = w->grow_to ? w->grow_to : w->ws_bytes;
  if (st == BC_OK)
    st = compute_groups(job.g, r, job.lanes, (int64_t)job.lanes.size(), w->ws, cap, w->st, job.slots.data(),
                        (int)job.slots.size(), &w->exec, nullptr);
  for (auto& q : job.qs) if (q->next >= q->groups.size() || st != BC_OK) complete->push_back(q);
  for (auto& q : *complete) {
    if (st == BC_OK && q->out &&
        hipMemcpyAsync(q->out, q->res.p, q->d_bytes, hipMemcpyDeviceToHost, w->st) != hipSuccess)
      st = BC_E_DEVICE;
  }
  if (!complete->empty() && hipStreamSynchronize(w->st) != hipSuccess) st = BC_E_DEVICE;
  if (st == BC_OK)
    for (auto& q : *complete) {
      if (!q->out) continue;
      scores_to_caller(q->g, q->out);  // the library's vertex order to the caller's
      for (size_t v = 0; v < q->tree.size(); ++v) q->out[v] += q->tree[v];
    }
  return st;
}

// A finished query's result array goes to the pool; lock held.
void finish(bc_server* s, const std::shared_ptr<Query>& q) {
  q->done = true;
  q->end_ms = s->now_ms();
  s->res_bytes -= (int64_t)q->res.bytes;
  if (q->res.p) {
    s->pool.push_back(q->res);
    s->pool_bytes += (int64_t)q->res.bytes;
  }
  q->res = Buf{};
  s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), q), s->queue.end());
}

void worker_loop(bc_server* s, Worker* w) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  std::vector<Buf> frees;
  while (true) {
    Job job;
    while (!s->stop && !take_job(s, w, &job)) {
      if (!s->to_free.empty()) {
        frees.swap(s->to_free);
        lk.unlock();
        drain(frees);
        lk.lock();
        continue;
      }
      s->cv_work.wait(lk);
    }
    if (s->stop) break;
    frees.swap(s->to_free);
    const size_t grown = w->grow_to;
    lk.unlock();
    drain(frees);
    std::vector<std::shared_ptr<Query>> complete;
    int64_t allocs = 0;
    bc_status st = run_job(s, w, job, &complete, &allocs);
    if (st != BC_OK) complete = job.qs;  // a failed batch ends its queries
    lk.lock();
    if (grown) {
      // the reservation already counts the new size for this worker
      if (w->ws) {
        w->ws_bytes = grown;
      } else {
        s->ws_bytes -= (int64_t)grown;  // growth failed: nothing is held
        w->ws_bytes = 0;
      }
      w->grow_to = 0;
    }
    s->allocations += allocs;
    for (auto& q : job.qs) {
      q->running = false;
      if (st != BC_OK) q->status = st;
    }
    for (auto& q : complete) finish(s, q);
    s->free_shares += w->shares;
    w->shares = 0;
    w->busy = false;
    s->note_running(-1);
    admit(s);
    s->cv_work.notify_all();
    s->cv_done.notify_all();
  }
}

}  // namespace

extern "C" {

bc_status bc_server_create(bc_context* ctx, const bc_server_config* cfg, bc_server** out) {
  if (!ctx || !out) return fail(BC_E_INVALID_ARG, "null argument");
  auto* s = new bc_server;
  s->device = context_device(ctx);
  if (hipSetDevice(s->device) != hipSuccess) { delete s; return fail(BC_E_DEVICE, "hipSetDevice"); }
  if (cfg) s->cfg = *cfg;
  if (s->cfg.hbm_budget_bytes <= 0) s->cfg.hbm_budget_bytes = 64ll << 30;
  if (s->cfg.max_inflight <= 0) s->cfg.max_inflight = 4;
  if (s->cfg.batch <= 0) s->cfg.batch = 256;
  if (s->cfg.queue_capacity <= 0) s->cfg.queue_capacity = 4096;
  if (s->cfg.batch % 64 || s->cfg.batch > 256) { delete s; return fail(BC_E_INVALID_ARG, "batch must be 64..256, multiple of 64"); }
  if (s->cfg.heuristics & ~(uint32_t)BC_H_DEG1) { delete s; return fail(BC_E_INVALID_ARG, "the server takes BC_H_DEG1 only"); }
  // Persistent kernels wait at grid barriers for all their workgroups, so
  // kernels running side by side must all fit on the device at once: the
  // resident workgroups are cut into max_inflight shares, and the grids
  // running together never hold more shares than there are.
  const int occ = batch_occupancy(s->cfg.batch / 64);
  if (occ < 1) { delete s; return fail(BC_E_DEVICE, "occupancy query failed"); }
  const int resident = context_cus(ctx) * occ;
  if (s->cfg.max_inflight > resident / 8) s->cfg.max_inflight = std::max(1, resident / 8);
  s->grid_share = resident / s->cfg.max_inflight;
  s->free_shares = s->cfg.max_inflight;
  for (int i = 0; i < s->cfg.max_inflight; ++i) {
    auto w = std::make_unique<Worker>();
    if (hipStreamCreateWithFlags(&w->st, hipStreamNonBlocking) != hipSuccess) {
      bc_server_destroy(s);
      return fail(BC_E_DEVICE, "stream creation failed");
    }
    s->workers.push_back(std::move(w));
  }
  for (auto& w : s->workers) w->th = std::thread(worker_loop, s, w.get());
  *out = s;
  return BC_OK;
}

bc_status bc_server_destroy(bc_server* s) {
  if (!s) return BC_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  for (auto& w : s->workers)
    if (w->th.joinable()) w->th.join();
  for (auto& w : s->workers) {
    if (w->ws) (void)hipFree(w->ws);
    if (w->st) (void)hipStreamDestroy(w->st);
    w->exec.release();
  }
  for (auto& q : s->queue)
    if (q->res.p) (void)hipFree(q->res.p);
  for (auto& b : s->pool) (void)hipFree(b.p);
  drain(s->to_free);
  delete s;
  return BC_OK;
}

bc_status bc_submit(bc_server* s, bc_graph* g, const int32_t* sources, int64_t k, double* out, uint64_t* ticket) {
  if (!s || !g || !ticket || k < 0 || (k > 0 && !sources)) return fail(BC_E_INVALID_ARG, "bad arguments");
  const int64_t n = graph_n(g);
  for (int64_t i = 0; i < k; ++i)
    if (sources[i] < 0 || sources[i] >= n) return fail(BC_E_INVALID_ARG, "source id out of range");
  auto q = std::make_shared<Query>();
  q->g = g;
  q->out = out;
  q->n = n;
  q->m = graph_nnz(g) / 2;
  q->d_bytes = sizeof(double) * (size_t)n;
  Resolved r;
  bc_status st = serve_resolved(s, g, 1, &r);
  if (st != BC_OK) return st;
  q->ws_bytes = (int64_t)graph_ws_bytes(g, r);
  q->wide = r.mode == BC_MODE_BATCHED;
  graph_groups(g, r, sources, k, &q->groups, &q->credited);
  if (r.deg1) tree_scores_caller(g, sources, k, &q->tree);
  std::vector<Buf> frees;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if ((int)s->queue.size() >= s->cfg.queue_capacity) return fail(BC_E_BUSY, "server queue full");
    q->ticket = s->next_ticket++;
    q->submit_ms = s->now_ms();
    *ticket = q->ticket;
    s->all[q->ticket] = q;
    if (q->groups.empty()) {
      // nothing to traverse: only closed-form scores (tree vertices), else zeros
      if (out) std::fill(out, out + n, 0.0);
      if (out) for (size_t v = 0; v < q->tree.size(); ++v) out[v] = q->tree[v];
      q->done = true;
      q->end_ms = q->submit_ms;
      return BC_OK;
    }
    s->queue.push_back(q);
    admit(s);
    frees.swap(s->to_free);
  }
  drain(frees);
  s->cv_work.notify_all();
  return BC_OK;
}

bc_status bc_wait(bc_server* s, uint64_t ticket, int64_t timeout_us, bc_query_stats* stats) {
  if (!s) return fail(BC_E_INVALID_ARG, "null server");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->all.find(ticket);
  if (it == s->all.end()) return fail(BC_E_NOT_FOUND, "unknown ticket");
  auto q = it->second;
  auto pred = [&] { return q->done; };
  if (timeout_us < 0) s->cv_done.wait(lk, pred);
  else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), pred)) return fail(BC_E_TIMEOUT, "query still running");
  s->all.erase(it);
  if (stats) {
    stats->submit_ms = q->submit_ms;
    stats->start_ms = q->start_ms;
    stats->end_ms = q->end_ms;
    stats->latency_ms = q->end_ms - q->submit_ms;
    stats->sources = q->credited;
    stats->te = (double)q->credited * (double)q->m;
    stats->status = q->status;
  }
  if (q->status != BC_OK) return fail((bc_status)q->status, "query failed");
  return BC_OK;
}

bc_status bc_server_stats_get(bc_server* s, bc_server_stats* out) {
  if (!s || !out) return fail(BC_E_INVALID_ARG, "null argument");
  std::lock_guard<std::mutex> lk(s->mu);
  s->note_running(0);
  out->workers = (int32_t)s->workers.size();
  out->grid_workgroups = s->grid_share;
  out->max_inflight_seen = s->max_running;
  out->batches = s->batches;
  out->mean_inflight = s->busy_ms > 0 ? s->area_ms / s->busy_ms : 0.0;
  out->busy_ms = s->busy_ms;
  out->held_bytes = s->held();
  out->reclaims = s->reclaims;
  out->allocations = s->allocations;
  out->wide_batches = s->wide_batches;
  out->mean_shares = s->batches ? (double)s->share_sum / (double)s->batches : 0.0;
  return BC_OK;
}

}  // extern "C"
