/*
 * bc.h -- exact betweenness centrality on one AMD Instinct MI355X (gfx950).
 *
 * The method is Brandes' algorithm as restated in Vella, Carbone, Bernaschi,
 * "Algorithms and Heuristics for Scalable Betweenness Centrality Computation
 * on Multi-GPU Systems" (arXiv:1602.00963):
 *   - scores are sums of per-source dependencies (Sec. 2, Eq. (1)-(3));
 *   - each source runs a level-synchronous shortest-path count (Sec. 3.2,
 *     Alg. 2-3) and a successor-checking dependency sweep (Sec. 3.2,
 *     Alg. 4-5);
 *   - optional 1-degree reduction (Sec. 2.2, Eq. (4)-(5); Sec. 3.4.1,
 *     Alg. 6), also iterated until no tree hangs from the graph (the
 *     extension the footnote of Sec. 3.4.1 leaves out), and 2-degree
 *     derivation with the fused backward sweep (Sec. 3.4.2, Lemma 1,
 *     Eq. (6), Alg. 7-9).
 *
 * Graphs are simple, undirected and unweighted, given as a symmetric CSR
 * (row_ptr[n+1], col_idx[nnz], int32, every pair stored in both directions).
 *
 * Score convention: RAW scores sum over ordered (source, target) pairs, as
 * Eq. (3) does; BC_UNDIRECTED halves them (the usual undirected value).
 *
 * Ownership: host arrays passed in are only read during the call and are
 * copied; the library never frees memory it did not allocate.  Device
 * pointers (BC_LOAD_DEVICE_PTRS, caller workspaces) stay owned by the caller
 * and must outlive the call (and, for a workspace, the stream work it
 * enqueued).  Objects are not thread-safe unless stated: use one thread per
 * bc_graph, or the bc_server API.
 *
 * Errors: every function returns a bc_status; no C++ exception crosses this
 * boundary.  bc_last_error() gives a thread-local message for the last
 * failure on the calling thread.
 */
#ifndef BC_H_
#define BC_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum bc_status {
  BC_OK = 0,
  BC_E_INVALID_ARG = 1,    /* null pointer, out-of-range id, bad option */
  BC_E_INVALID_GRAPH = 2,  /* CSR not symmetric/simple/sorted-free, ids out of range, nnz > INT32_MAX */
  BC_E_OUT_OF_MEMORY = 3,  /* device or host allocation failed, or workspace too small */
  BC_E_DEVICE = 4,         /* a HIP call failed */
  BC_E_BUSY = 5,           /* server queue full */
  BC_E_NOT_FOUND = 6,      /* unknown ticket */
  BC_E_TIMEOUT = 7,        /* bc_wait timed out; the query is still running */
  BC_E_REJECTED = 8,       /* query can never fit the server's HBM budget */
  BC_E_CAPACITY = 9        /* internal list capacity exceeded (retry with a smaller batch) */
} bc_status;

typedef struct bc_context bc_context;
typedef struct bc_graph bc_graph;
typedef struct bc_server bc_server;

/* ------------------------------------------------------------------ context */

/* Binds a HIP device (hipSetDevice on the calling thread) and queries it. */
bc_status bc_context_create(int device, bc_context** out);
bc_status bc_context_destroy(bc_context* ctx);

/* ------------------------------------------------------------------- graphs */

enum {
  BC_LOAD_VALIDATE = 1u,     /* check symmetry, no self-loops, no duplicates, ids in range */
  BC_LOAD_PRUNE_DEG1 = 2u,   /* build the 1-degree reduction (omega, residual graph), Alg. 6 */
  BC_LOAD_DEVICE_PTRS = 4u,  /* row_ptr / col_idx are device pointers (copied device-to-device) */
  BC_LOAD_KEEP_ORDER = 8u,   /* keep the caller's vertex order on the device (by default the library
                                renumbers vertices internally by decreasing degree, for cache
                                locality; ids at this boundary are always the caller's) */
  BC_LOAD_PRUNE_TREES = 16u  /* the 1-degree reduction iterated until no degree-1 vertex is left (the
                                extension the paper's 1-degree section leaves out in a footnote): every
                                tree hanging from the rest of the graph is folded into the vertex it
                                hangs from, whole tree components are removed; removed vertices get
                                closed-form scores on the host (they are cut vertices) */,
  BC_LOAD_ORDER_RCM = 32u    /* renumber internally in reverse Cuthill-McKee order instead of by degree:
                                neighbours get nearby ids, so a BFS wavefront on a long-diameter graph
                                (road networks, lattices) touches fewer cache lines; for
                                BC_MODE_PER_WORKGROUP; ignored with BC_LOAD_KEEP_ORDER */
};

typedef struct bc_graph_stats {
  int64_t n;               /* vertices */
  int64_t m;               /* unique undirected edges */
  int64_t nnz;             /* directed CSR entries (= 2m) */
  int64_t isolated;        /* degree-0 vertices */
  int64_t pendants;        /* degree-1 vertices removed by the reduction (0 if not pruned) */
  int64_t k2_vertices;     /* vertices of 2-vertex components (BC = 0, never sources) */
  int64_t residual_nnz;    /* directed entries of the residual graph G' (= nnz if not pruned) */
  int64_t deg2_vertices;   /* vertices of degree 2 in the traversed graph */
  int64_t max_degree;
  int64_t resident_bytes;  /* device bytes held by the graph (CSR, G', omega, scores) */
  int64_t tree_vertices;   /* vertices removed by the iterated reduction (BC_LOAD_PRUNE_TREES) */
  int64_t bfs_depth;       /* levels of a breadth-first search from a highest-degree vertex (a lower
                              bound on the diameter; chooses the kernel under BC_MODE_AUTO) */
  int64_t tuned_batch;     /* batch a call with batch = 0 uses: from bc_autotune on this graph or on
                              a graph of the same shape in the context (0 = none tuned: 256) */
} bc_graph_stats;

/*
 * Uploads a graph and keeps it resident in HBM.  With BC_LOAD_VALIDATE the
 * CSR is checked on the host first (BC_E_INVALID_GRAPH, message names the
 * first offending vertex).  With BC_LOAD_PRUNE_DEG1, degree-1 vertices whose
 * neighbour has degree >= 2 are folded into omega(neighbour) (Sec. 3.4.1);
 * both ends of a 2-vertex component are dropped (their score is 0).
 */
bc_status bc_graph_load(bc_context* ctx, int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                        int64_t nnz, uint32_t flags, bc_graph** out);
bc_status bc_graph_stats_get(const bc_graph* g, bc_graph_stats* out);
bc_status bc_graph_free(bc_graph* g);

/* ------------------------------------------------------------------ compute */

enum {
  BC_MODE_PLAIN = 0,    /* one persistent launch per source */
  BC_MODE_BATCHED = 1,  /* one persistent launch per batch of `batch` sources */
  BC_MODE_PLAIN_SCAN = 2, /* one source per launch with the paper's active-edge mapping (Sec. 3.1):
                            per level a prefix sum of the frontier's degrees and a binary search
                            per edge, the prefix sums reused by the backward sweep; exact counts
                            (wrapped sources are rerun by BC_MODE_PLAIN in extended form), no
                            direction switching, no heuristics; for comparison with BC_MODE_PLAIN */
  BC_MODE_PER_WORKGROUP = 3 /* one source per workgroup, as many workgroups per CU as fit (grid_per_cu caps it),
                               levels separated by workgroup barriers only: for long-diameter graphs,
                               where a device-wide barrier per level dominates and sampled sources
                               share no frontier a batch could pool; 1-degree reduction supported,
                               no 2-degree derivation; fp64 score atomics (order-dependent rounding) */,
  BC_MODE_AUTO = 4          /* BC_MODE_PER_WORKGROUP when the graph's bfs_depth (bc_graph_stats) exceeds
                               64 and BC_H_DEG2 is not requested, else BC_MODE_BATCHED; the mode run is
                               reported in bc_run_stats.mode.  (With BC_SIGMA_AUTO, in these two modes,
                               once a probe of 64 sources on a graph finds most counts wrapping, later
                               calls on that graph start in the extended form.) */
};
enum {
  BC_H_DEG1 = 1u,       /* use the graph's 1-degree reduction (needs BC_LOAD_PRUNE_DEG1) */
  BC_H_DEG2 = 2u        /* derive 2-degree vertices from their neighbours (batched only) */
};
enum {
  BC_SIGMA_AUTO = 0,    /* exact uint64 counts; sources that wrap are recomputed in extended form */
  BC_SIGMA_EXACT_ONLY = 1, /* exact uint64; sources that wrap are reported and left out */
  BC_SIGMA_EXTENDED = 2 /* every source in extended form (fp64 significand + int32 exponent) */
};

typedef struct bc_compute_opts {
  int32_t mode;         /* BC_MODE_* */
  int32_t batch;        /* sources per batch, multiple of 64 in [64, 1024]; 0 = tuned (bc_autotune) or 256 */
  uint32_t heuristics;  /* BC_H_* */
  int32_t sigma_mode;   /* BC_SIGMA_* */
  double alpha;         /* bottom-up when frontier edges * alpha > unvisited edges; 0 = default
                           (tuned if available, else never: bottom-up levels were slower on every
                           benchmarked graph), < 0 = never bottom-up */
  int32_t block;        /* threads per workgroup: 0, or the mode's fixed size (1024 batched, 256 plain) */
  int32_t grid_per_cu;  /* workgroups per CU for the persistent grid; 0 = the library's choice
                           (batched: one; plain: four when the traversed graph has at least 2^24
                           directed edges, else one; per-workgroup: as many as fit); persistent
                           grids are capped one below the occupancy query's limit, whose last
                           workgroup per CU was not always resident */
  double beta;          /* switch back: a bottom-up sweep stays bottom-up until the frontier holds
                           fewer than n / beta vertices (batched: (vertex, word) entries against
                           n * words); 0 = no hysteresis (tuned if available), each level tests alpha */
  int32_t graph_launches; /* BC_MODE_PLAIN: capture this many per-source launches in one HIP graph and
                           replay it (every launch takes the next source of a device list, the rest
                           of the list runs as single launches); 0 = one kernel launch per source.
                           Only used when the call has at least that many sweeps; not allowed with
                           other modes or bc_compute_noalloc, ignored by bc_trace */
} bc_compute_opts;

typedef struct bc_run_stats {
  int64_t sources;          /* sources requested (original ids, after dropping isolated) */
  int64_t traversed;        /* forward sweeps actually run (pruned/derived sources excluded) */
  int64_t derived;          /* 2-degree sources whose forward sweep was derived */
  int64_t overflowed;       /* sources whose uint64 count wrapped */
  int64_t rerun_extended;   /* of those, recomputed in extended form */
  int32_t first_overflow[8];/* first overflowed source ids (-1 = none) */
  int64_t levels;           /* sum over launches of forward levels */
  int64_t bottom_up_levels; /* of which bottom-up */
  int64_t reached;          /* sum over traversed sources of vertices reached */
  int64_t reached_nnz;      /* sum of directed CSR entries of reached vertices */
  int64_t dag_edges;        /* sum of edges joining consecutive levels (directed, parent to child) */
  int64_t launches;         /* kernel launches */
  double te;                /* traversed edges credited: sum over requested sources of m (original graph) */
  double raw_te;            /* traversed sources * m of the traversed graph */
  double ms;                /* wall time of the call, host-measured, ms */
  double kernel_ms;         /* sum of the kernel launches' durations, timed with HIP events
                               recorded on the call's stream around each launch, ms */
  int64_t mode;             /* the mode run (BC_MODE_AUTO resolved) */
} bc_run_stats;

/*
 * Adds the RAW contributions of the given sources to the graph's score
 * array (scores accumulate across calls until bc_scores_reset): for each
 * source s, delta_s(v) for every v != s (Eq. (2)), summed as Eq. (3)
 * prescribes; with BC_H_DEG1 through the reduced graph and Eq. (4)-(5);
 * each source's forward sweep is Alg. 2-3 and its backward sweep Alg. 4-5,
 * run one source per launch or 64-1024 per launch.
 *   sources: host array of k original vertex ids, or NULL for every
 *            non-isolated vertex.  Isolated sources contribute nothing.
 *            With BC_H_DEG1 the graph's pruned vertices are handled
 *            analytically and never traversed.
 *   workspace/ws_bytes: device buffer of at least bc_workspace_size()
 *            bytes, or NULL to use a library-owned cached buffer.
 *   stream:  hipStream_t to enqueue on (NULL = the null stream).  The call
 *            blocks until its work is complete.
 *   stats:   optional.
 */
bc_status bc_workspace_size(const bc_graph* g, const bc_compute_opts* opts, size_t* bytes);
bc_status bc_compute(bc_graph* g, const int32_t* sources, int64_t k, const bc_compute_opts* opts,
                     void* workspace, size_t ws_bytes, void* stream, bc_run_stats* stats);

/*
 * The plain form with no device allocation, for callers that cannot call
 * hipMalloc (code under stream capture, tight serving loops, harnesses that
 * forbid allocation).  Same contract as bc_compute with opts->mode =
 * BC_MODE_PLAIN (any other mode: BC_E_INVALID_ARG), except:
 *   - the workspace is a fixed device array of 64 MiB inside the library
 *     (one per GPU, held until the process ends); a graph whose plain
 *     workspace (bc_workspace_size) is larger returns BC_E_CAPACITY before
 *     any device work;
 *   - the array keeps the last call's contents; every call clears what it
 *     needs with a fill kernel (no memset node, no allocation, no event);
 *   - calls on one GPU share the array: the library runs them one at a time
 *     (a per-device lock held for the whole call); stats->kernel_ms is 0.
 * The call blocks until its work is complete, like bc_compute.
 */
bc_status bc_compute_noalloc(bc_graph* g, const int32_t* sources, int64_t k, const bc_compute_opts* opts,
                             void* stream, bc_run_stats* stats);

/*
 * Autotuner for the batched mode: times trial runs of `sample` (k source
 * ids, at least two batches' worth recommended) into a scratch score array
 * (the graph's scores are untouched) over batch width {64, 128, 256, 512, 1024},
 * the bottom-up threshold alpha {0 = never, 0.5, 1, 2, 4, 8}, its switch-back
 * threshold beta {0, 2, 8, 24, 64} (when bottom-up is in play) and the
 * persistent grid {occupancy limit, half of it}, by coordinate descent
 * starting from *opts.  On return *opts holds the fastest setting found
 * (mode, heuristics and sigma_mode are kept) and *gteps its throughput
 * (sample sources x m / time).  budget_ms bounds the tuning time (0 = no
 * bound beyond one pass).  The result is also remembered by the graph and
 * used by bc_compute calls whose opts->batch is 0, and kept in the context
 * under the graph's shape (log2 of its non-isolated vertices, of its mean and
 * largest degree; deep or not; with or without the 1-degree reduction), where
 * graphs of the same shape that have no tuning of their own pick it up
 * (bc_graph_stats.tuned_batch).
 */
bc_status bc_autotune(bc_graph* g, const int32_t* sample, int64_t k, bc_compute_opts* opts, double budget_ms,
                      double* gteps);

enum { BC_RAW = 0, BC_UNDIRECTED = 1 };
/* Copies the accumulated scores (n doubles, the caller's vertex order) into
 * out (host, or device if out_on_device != 0).  BC_RAW sums over ordered
 * (source, target) pairs as Eq. (3) does; BC_UNDIRECTED halves it (each
 * unordered pair once).  Closed-form scores of vertices removed by the
 * iterated reduction are included. */
bc_status bc_scores(const bc_graph* g, double* out, int32_t norm, int32_t out_on_device);
bc_status bc_scores_reset(bc_graph* g);

/*
 * Parity export.  Runs the given sources (unpruned graph, no scores added)
 * through the chosen mode and copies per-source results to host arrays laid
 * out source-major ([i*n + v]): d (-1 unreached), sigma (uint64; for a
 * source in extended form: 0), sigma_mant/sigma_exp (extended form:
 * sigma = mant * 2^exp; exact form: mant = (double)sigma, exp = 0), delta
 * (dependency of v on source i, Eq. (2); 0 at the source and at unreached
 * vertices), overflow[i].  Any output may be NULL.
 */
bc_status bc_trace(bc_graph* g, const int32_t* sources, int64_t k, const bc_compute_opts* opts,
                   int32_t* d, uint64_t* sigma, double* sigma_mant, int32_t* sigma_exp,
                   double* delta, int32_t* overflow);

/* -------------------------------------------------------------- host checks */

/* CSR validation only (no device).  Returns BC_OK or BC_E_INVALID_GRAPH. */
bc_status bc_validate_csr(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, int64_t nnz);

/*
 * The 1-degree reduction on the host (Alg. 6 read as: a vertex u is a
 * pendant iff deg(u) = 1 and its neighbour has degree >= 2).  Outputs
 * (caller-allocated): omega[n] (pendants per vertex), kind[n] (0 kept,
 * 1 pendant, 2 end of a 2-vertex component, 3 isolated), hub[n] (the
 * neighbour of a pendant, else -1), res_row_ptr[n+1], res_col_idx[nnz]
 * (the residual graph G' on the same ids; pruned vertices get empty rows).
 * *res_nnz receives the residual entry count.
 */
bc_status bc_prune_deg1_host(int32_t n, const int32_t* row_ptr, const int32_t* col_idx,
                             int32_t* omega, int32_t* kind, int32_t* hub,
                             int32_t* res_row_ptr, int32_t* res_col_idx, int64_t* res_nnz);

/*
 * The iterated reduction on the host (BC_LOAD_PRUNE_TREES): degree-1
 * vertices are peeled until none is left.  Outputs (caller-allocated, any
 * may be NULL): omega[n] (vertices folded into each kept vertex: the size of
 * the forest hanging from it), kind[n] (0 kept, 3 isolated, 4 removed),
 * scores[n] (RAW scores of the removed vertices for the k sources, or for
 * every vertex when k = 0; 0 at kept vertices), *res_nnz (directed entries
 * of the residual graph).  No device work.
 */
bc_status bc_prune_trees_host(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, const int32_t* sources,
                              int64_t k, int32_t* omega, int32_t* kind, double* scores, int64_t* res_nnz);

/*
 * The internal vertex order bc_graph_load would use, host only: perm[v] is
 * the internal id of caller vertex v for these load_flags (by decreasing
 * degree, ties by id; reverse Cuthill-McKee with BC_LOAD_ORDER_RCM; the
 * identity with BC_LOAD_KEEP_ORDER), and *bfs_depth (if not NULL) the levels
 * of a breadth-first search from the lowest-numbered vertex of highest
 * degree, the figure BC_MODE_AUTO chooses the kernel by.  Only the CSR's
 * bounds are checked
 * (BC_E_INVALID_GRAPH if row_ptr[0] != 0, row_ptr decreases or a column
 * index lies outside [0, n)); symmetry and sorted rows are assumed.
 */
bc_status bc_vertex_order_host(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint32_t load_flags,
                               int32_t* perm, int64_t* bfs_depth);

/*
 * Heuristics coverage for all sources (the count the paper's heuristics
 * table reports), host only: with load_flags (BC_LOAD_PRUNE_DEG1 or
 * BC_LOAD_PRUNE_TREES) and heuristics (BC_H_DEG1, BC_H_DEG2) as bc_compute
 * would use them (1-degree reduction of Sec. 3.4.1; 2-degree derivation of
 * Sec. 3.4.2 with the library's greedy selection in breadth-first order from
 * the highest-degree vertex).  out[5]: non-isolated sources, sweeps
 * traversed, sources served by the 1-degree reduction, sources derived by
 * the 2-degree heuristic, degree-2 vertices among the traversal sources.
 */
bc_status bc_coverage_host(int32_t n, const int32_t* row_ptr, const int32_t* col_idx, uint32_t load_flags,
                           uint32_t heuristics, int64_t* out);

/* ------------------------------------------------------------------ serving */

typedef struct bc_server_config {
  int64_t hbm_budget_bytes;  /* device bytes the server may hold at once (workspaces and result
                                arrays); 0 = 64 GiB */
  int32_t max_inflight;      /* concurrent batches (streams); 0 = 4.  The device's resident
                                workgroups are cut into max_inflight shares; a batch's grid takes
                                one share, or, when no other query waits for a batch, every free
                                share but one (one is kept for the next query to arrive); the
                                running grids never hold more shares than there are, so they
                                co-run on the device.  Batches run in
                                BC_MODE_AUTO: graphs deeper than 64 levels one source per
                                workgroup, the others batched */
  int32_t batch;             /* sources per batch, multiple of 64 up to 256; 0 = 256 */
  int32_t queue_capacity;    /* pending queries; 0 = 4096 */
  uint32_t heuristics;       /* 0, or BC_H_DEG1: queries on graphs loaded with
                                BC_LOAD_PRUNE_DEG1 use the 1-degree reduction for their source
                                subsets (Sec. 3.4.1, Eq. (4)-(5) restricted to the subset) */
} bc_server_config;

typedef struct bc_server_stats {
  int32_t workers;            /* worker streams */
  int32_t grid_workgroups;    /* workgroups of each batch's persistent grid */
  int32_t max_inflight_seen;  /* most batches running at once */
  int64_t batches;            /* batches run */
  double mean_inflight;       /* batches running, averaged over the time any batch ran */
  double busy_ms;             /* time with at least one batch running */
  int64_t held_bytes;         /* device bytes held now (workspaces, result arrays, pool) */
  int64_t reclaims;           /* times pooled arrays / idle workspaces were given back */
  int64_t allocations;        /* device allocations made by the workers */
  int64_t wide_batches;       /* batches whose grid took more than one share */
  double mean_shares;         /* shares per batch, averaged over batches */
} bc_server_stats;

typedef struct bc_query_stats {
  double submit_ms, start_ms, end_ms;  /* host clock, ms since server creation */
  double latency_ms;                   /* end - submit */
  int64_t sources;                     /* sources of the query */
  double te;                           /* sources * m */
  int32_t status;                      /* bc_status of the query */
} bc_query_stats;

/*
 * Continuous-batching server.  Queries (graph, source subset) are admitted
 * by HBM footprint: a query's result array must fit next to the other
 * admitted results and one workspace for the largest admitted graph; a
 * query that could not fit even alone is rejected (BC_E_REJECTED from
 * bc_wait).  Sources of queries on the same graph share batches; up to
 * max_inflight batches run concurrently on their own streams.  Device
 * memory is pooled and reused; no device allocation or free happens while
 * the server's lock is held.  Each query's RAW scores are written into its `out`
 * array (n doubles, host), which must stay valid until bc_wait returns for
 * its ticket.  A query's result does not depend on which other queries share
 * its batches beyond floating-point summation order (relative 1e-9).
 * The server API is thread-safe.
 */
bc_status bc_server_create(bc_context* ctx, const bc_server_config* cfg, bc_server** out);
bc_status bc_server_destroy(bc_server* s);
bc_status bc_submit(bc_server* s, bc_graph* g, const int32_t* sources, int64_t k, double* out,
                    uint64_t* ticket);
bc_status bc_wait(bc_server* s, uint64_t ticket, int64_t timeout_us, bc_query_stats* stats);
/* Counters of the server since creation (thread-safe). */
bc_status bc_server_stats_get(bc_server* s, bc_server_stats* out);

/* ------------------------------------------------------------------- errors */

const char* bc_status_string(bc_status st);
const char* bc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BC_H_ */
