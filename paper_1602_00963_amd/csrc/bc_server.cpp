// Continuous-batching server for betweenness queries (graph, source subset).
//
// Queries wait in a FIFO.  A query is admitted when its result array fits
// the HBM budget next to the workspaces already held; one that could never
// fit is rejected.  Worker threads (one HIP stream and one workspace each)
// repeatedly form a batch: the sources of the oldest admitted query that is
// not running, topped up with sources of other waiting queries on the same
// graph, each query's sweeps writing into its own result array (one result
// slot per query in the batch).  A query takes part in at most one running
// batch at a time, so its result array has a single writer; batches of
// different queries and graphs run concurrently on their own streams.
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

struct Query {
  uint64_t ticket = 0;
  bc_graph* g = nullptr;
  std::vector<Group> groups;  // traversal sources, weights = multiplicity
  size_t next = 0;            // first group not yet dispatched
  int64_t credited = 0;
  double* out = nullptr;      // host result (caller-owned)
  double* d_out = nullptr;    // device result
  size_t d_bytes = 0;
  bool admitted = false, running = false, done = false;
  bc_status status = BC_OK;
  double submit_ms = 0, start_ms = -1, end_ms = 0;
  int64_t n = 0, m = 0;
};

struct Worker {
  std::thread th;
  hipStream_t st = nullptr;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  Exec exec;
};

}  // namespace

struct bc_server {
  int device = 0;
  int grid_per_cu = 1;  // per batch kernel, so that all in-flight kernels are co-resident
  bc_server_config cfg{};
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<std::shared_ptr<Query>> queue;       // submitted, not finished
  std::map<uint64_t, std::shared_ptr<Query>> all;  // ticket -> query (until waited)
  std::vector<std::unique_ptr<Worker>> workers;
  uint64_t next_ticket = 1;
  int64_t reserved = 0;  // bytes: worker workspaces + admitted result arrays
  bool stop = false;
  Clock::time_point t0 = Clock::now();
  double now_ms() const { return std::chrono::duration<double, std::milli>(Clock::now() - t0).count(); }
};

namespace {

bc_compute_opts serve_opts(const bc_server* s) {
  bc_compute_opts o{};
  o.mode = BC_MODE_BATCHED;
  o.batch = s->cfg.batch;
  o.sigma_mode = BC_SIGMA_AUTO;
  o.grid_per_cu = s->grid_per_cu;
  return o;
}

// Admission in FIFO order; called with the lock held.
void admit(bc_server* s) {
  for (auto& q : s->queue) {
    if (q->admitted || q->done) continue;
    bc_compute_opts o = serve_opts(s);
    Resolved r;
    if (resolve_opts(q->g, &o, &r) != BC_OK) { q->status = BC_E_INVALID_ARG; q->done = true; continue; }
    r.cap_factor = r.B;
    r.max_slots = 64;
    const int64_t ws = (int64_t)graph_ws_bytes(q->g, r);
    if ((int64_t)q->d_bytes + ws > s->cfg.hbm_budget_bytes) {
      q->status = BC_E_REJECTED;
      q->done = true;
      q->end_ms = s->now_ms();
      continue;
    }
    if (s->reserved + (int64_t)q->d_bytes > s->cfg.hbm_budget_bytes) break;  // FIFO: wait
    if (hipMalloc((void**)&q->d_out, q->d_bytes) != hipSuccess ||
        hipMemset(q->d_out, 0, q->d_bytes) != hipSuccess) {
      q->status = BC_E_OUT_OF_MEMORY;
      q->done = true;
      continue;
    }
    s->reserved += (int64_t)q->d_bytes;
    q->admitted = true;
  }
  s->cv_done.notify_all();
}

struct Job {
  bc_graph* g = nullptr;
  std::vector<std::shared_ptr<Query>> qs;
  std::vector<Group> lanes;
  std::vector<double*> slots;
};

// Forms the next batch; called with the lock held.  Returns false if none.
bool take_job(bc_server* s, Worker* w, Job* job) {
  const int B = s->cfg.batch;
  std::shared_ptr<Query> lead;
  for (auto& q : s->queue)
    if (q->admitted && !q->running && !q->done && q->next < q->groups.size()) { lead = q; break; }
  if (!lead) return false;
  bc_compute_opts o = serve_opts(s);
  Resolved r;
  resolve_opts(lead->g, &o, &r);
  r.cap_factor = r.B;  // worst-case level lists: a batch can never run out of them
  r.max_slots = 64;
  const size_t need = graph_ws_bytes(lead->g, r);
  if (w->ws_bytes < need) {
    const int64_t grow = (int64_t)need - (int64_t)w->ws_bytes;
    if (s->reserved + grow > s->cfg.hbm_budget_bytes) {
      // an idle worker's smaller workspace may be what blocks the growth:
      // give it back so a worker can grow once the running batches end
      if (w->ws) {
        (void)hipFree(w->ws);
        w->ws = nullptr;
        s->reserved -= (int64_t)w->ws_bytes;
        w->ws_bytes = 0;
        s->cv_work.notify_all();
      }
      return false;
    }
    if (w->ws) (void)hipFree(w->ws);
    w->ws = nullptr;
    s->reserved -= (int64_t)w->ws_bytes;
    w->ws_bytes = 0;
    if (hipMalloc(&w->ws, need) != hipSuccess) return false;
    w->ws_bytes = need;
    s->reserved += (int64_t)need;
  }
  job->g = lead->g;
  job->qs.clear();
  job->lanes.clear();
  job->slots.clear();
  for (auto& q : s->queue) {
    if ((int)job->lanes.size() >= B || (int)job->slots.size() >= 64) break;
    if (q->g != lead->g || !q->admitted || q->running || q->done || q->next >= q->groups.size()) continue;
    const int slot = (int)job->slots.size();
    job->slots.push_back(q->d_out);
    job->qs.push_back(q);
    q->running = true;
    if (q->start_ms < 0) q->start_ms = s->now_ms();
    while ((int)job->lanes.size() < B && q->next < q->groups.size()) {
      Group gr = q->groups[q->next++];
      gr.slot = slot;
      job->lanes.push_back(gr);
    }
  }
  return true;
}

void finish(bc_server* s, const std::shared_ptr<Query>& q) {
  q->done = true;
  q->end_ms = s->now_ms();
  if (q->d_out) {
    (void)hipFree(q->d_out);
    q->d_out = nullptr;
    s->reserved -= (int64_t)q->d_bytes;
  }
  s->queue.erase(std::remove(s->queue.begin(), s->queue.end(), q), s->queue.end());
}

void worker_loop(bc_server* s, Worker* w) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    Job job;
    while (!s->stop && !take_job(s, w, &job)) s->cv_work.wait(lk);
    if (s->stop) break;
    lk.unlock();
    bc_compute_opts o = serve_opts(s);
    Resolved r;
    bc_status st = resolve_opts(job.g, &o, &r);
    r.cap_factor = r.B;
    r.max_slots = 64;
    if (st == BC_OK)
      st = compute_groups(job.g, r, job.lanes, (int64_t)job.lanes.size(), w->ws, w->ws_bytes, w->st,
                          job.slots.data(), (int)job.slots.size(), &w->exec, nullptr);
    // queries whose sources are all done download their results
    std::vector<std::shared_ptr<Query>> complete;
    for (auto& q : job.qs) if (q->next >= q->groups.size() || st != BC_OK) complete.push_back(q);
    for (auto& q : complete) {
      if (st == BC_OK && q->out &&
          hipMemcpyAsync(q->out, q->d_out, q->d_bytes, hipMemcpyDeviceToHost, w->st) != hipSuccess)
        st = BC_E_DEVICE;
    }
    if (!complete.empty() && hipStreamSynchronize(w->st) != hipSuccess) st = BC_E_DEVICE;
    lk.lock();
    for (auto& q : job.qs) {
      q->running = false;
      if (st != BC_OK) q->status = st;
    }
    for (auto& q : complete) finish(s, q);
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
  // Persistent kernels wait at grid barriers for all their workgroups, so
  // kernels running side by side must all fit on the device at once: give
  // each a 1/max_inflight share of the workgroup slots.
  const int occ = batch_occupancy(s->cfg.batch / 64);
  if (occ < 1) { delete s; return fail(BC_E_DEVICE, "occupancy query failed"); }
  if (s->cfg.max_inflight > occ) s->cfg.max_inflight = occ;
  s->grid_per_cu = occ / s->cfg.max_inflight;
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
    if (q->d_out) (void)hipFree(q->d_out);
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
  bc_compute_opts o = serve_opts(s);
  Resolved r;
  bc_status st = resolve_opts(g, &o, &r);
  if (st != BC_OK) return st;
  graph_groups(g, r, sources, k, &q->groups, &q->credited);
  std::lock_guard<std::mutex> lk(s->mu);
  if ((int)s->queue.size() >= s->cfg.queue_capacity) return fail(BC_E_BUSY, "server queue full");
  q->ticket = s->next_ticket++;
  q->submit_ms = s->now_ms();
  *ticket = q->ticket;
  s->all[q->ticket] = q;
  if (q->groups.empty()) {
    // nothing to traverse: the result is all zeros
    if (out) std::fill(out, out + n, 0.0);
    q->done = true;
    q->end_ms = q->submit_ms;
    return BC_OK;
  }
  s->queue.push_back(q);
  admit(s);
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

}  // extern "C"
