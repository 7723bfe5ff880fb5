/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, sequential, deliberately unoptimised implementations of exact
 * betweenness centrality on simple undirected unweighted graphs.  Only the
 * test suite, the smoke check and the benchmark's CPU-baseline leg may load
 * this library; the GPU product path never links or calls it, and the two
 * share no source.
 *
 * Conventions (the same in every function here):
 *   - Input graph: symmetric CSR, int32 row_ptr[n+1] and col_idx[nnz].
 *   - Scores are RAW: summed over ordered (source, target) pairs, as in the
 *     paper's Eq. (3) (BC(v) = sum over s != v of delta_s(v)).  Halving RAW
 *     gives the usual undirected value.  Pairs with no path add nothing.
 *   - Path counts sigma are exact uint64 with a checked add; a source whose
 *     count would wrap is flagged "overflowed" and recomputed with sigma in
 *     x87 long double (64-bit significand, 15-bit exponent), which holds
 *     counts far beyond 2^64.
 *
 * Contents:
 *   orc_source        Brandes' algorithm for one source (Sec. 2, Alg. 1 with
 *                     its backward loop read as "pop w, then for v in
 *                     Pred[w] accumulate"), returning d, sigma, delta.
 *   orc_bc            The same over a list of sources, optionally threaded
 *                     (static contiguous split, per-thread score arrays
 *                     summed in thread order).
 *   orc_bellman       The pre-Brandes O(n^3) method the paper recalls in
 *                     Sec. 2: Floyd-Warshall distances, path counts, then the
 *                     explicit pair dependencies selected by the Bellman
 *                     criterion (Lemma 2).  A second, independent oracle.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
  int32_t n;
  int32_t* order;   /* BFS visiting order; read backwards it is Brandes' stack S */
  int32_t* pred;    /* predecessor lists: Pred[w] at pred[row_ptr[w] .. + npred[w]) */
  int32_t* npred;
  uint64_t* sig;
  long double* sigl;
  long double* dell;
  double* del;
} orc_ws;

static void ws_free(orc_ws* w) {
  free(w->order); free(w->pred); free(w->npred); free(w->sig); free(w->sigl); free(w->dell); free(w->del);
  memset(w, 0, sizeof(*w));
}

static int ws_init(orc_ws* w, int32_t n, int64_t nnz) {
  memset(w, 0, sizeof(*w));
  w->n = n;
  size_t nn = (size_t)(n > 0 ? n : 1);
  w->order = (int32_t*)malloc(sizeof(int32_t) * nn);
  w->pred = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
  w->npred = (int32_t*)malloc(sizeof(int32_t) * nn);
  w->sig = (uint64_t*)malloc(sizeof(uint64_t) * nn);
  w->sigl = (long double*)malloc(sizeof(long double) * nn);
  w->dell = (long double*)malloc(sizeof(long double) * nn);
  w->del = (double*)malloc(sizeof(double) * nn);
  if (!w->order || !w->pred || !w->npred || !w->sig || !w->sigl || !w->dell || !w->del) { ws_free(w); return -1; }
  return 0;
}

/*
 * Forward phase of Alg. 1: BFS from s with a FIFO queue; every edge (v, w)
 * with d[w] = d[v] + 1 adds sigma[v] into sigma[w] and records v in Pred[w].
 * Returns the number of vertices reached; *ovf is set if a uint64 add wrapped.
 */
static int32_t forward_u64(const int32_t* rp, const int32_t* ci, int32_t n, int32_t s,
                           int32_t* d, orc_ws* w, int* ovf) {
  for (int32_t i = 0; i < n; ++i) { d[i] = -1; w->sig[i] = 0; w->npred[i] = 0; }
  *ovf = 0;
  int32_t head = 0, tail = 0;
  d[s] = 0; w->sig[s] = 1; w->order[tail++] = s;
  while (head < tail) {
    int32_t v = w->order[head++];
    for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
      int32_t x = ci[e];
      if (d[x] < 0) { d[x] = d[v] + 1; w->order[tail++] = x; }
      if (d[x] == d[v] + 1) {
        uint64_t before = w->sig[x];
        w->sig[x] = before + w->sig[v];
        if (w->sig[x] < before) *ovf = 1;
        w->pred[rp[x] + w->npred[x]++] = v;
      }
    }
  }
  return tail;
}

/* The same BFS with sigma held in long double (used only after a wrap). */
static void forward_ld(const int32_t* rp, const int32_t* ci, int32_t n, int32_t s,
                       int32_t* d, orc_ws* w) {
  for (int32_t i = 0; i < n; ++i) { d[i] = -1; w->sigl[i] = 0.0L; w->npred[i] = 0; }
  int32_t head = 0, tail = 0;
  d[s] = 0; w->sigl[s] = 1.0L; w->order[tail++] = s;
  while (head < tail) {
    int32_t v = w->order[head++];
    for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
      int32_t x = ci[e];
      if (d[x] < 0) { d[x] = d[v] + 1; w->order[tail++] = x; }
      if (d[x] == d[v] + 1) {
        w->sigl[x] += w->sigl[v];
        w->pred[rp[x] + w->npred[x]++] = v;
      }
    }
  }
}

/*
 * One source.  Outputs (any may be NULL): d[n] (-1 = unreached), sigma[n]
 * (uint64; meaningless if overflowed), sigma_ld[n] (long double counts,
 * always filled), delta[n].  If bc is non-NULL, delta[w] is added
 * into bc[w] for every w != s, in reverse BFS order.  stats (if non-NULL)
 * receives {vertices reached, directed CSR entries of reached vertices,
 * DAG edges (predecessor relations)}.  Returns 1 if uint64 sigma wrapped,
 * 0 if not, -1 on allocation failure.
 */
static int source_ws(const int32_t* rp, const int32_t* ci, int32_t n, int32_t s, orc_ws* w,
                     int32_t* d_out, uint64_t* sigma_out, long double* sigma_ld_out,
                     double* delta_out, double* bc, int64_t* stats) {
  int32_t* d = d_out;
  int32_t* dtmp = NULL;
  if (!d) { dtmp = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1)); if (!dtmp) return -1; d = dtmp; }
  int ovf = 0;
  int32_t reached = forward_u64(rp, ci, n, s, d, w, &ovf);
  if (sigma_out) memcpy(sigma_out, w->sig, sizeof(uint64_t) * (size_t)n);
  if (ovf) forward_ld(rp, ci, n, s, d, w);
  /* Backward phase: pop w from the stack; every v in Pred[w] receives
   * sigma[v]/sigma[w] * (1 + delta[w])  (Eq. 2). */
  if (!ovf) {
    double* del = w->del;
    for (int32_t i = 0; i < n; ++i) del[i] = 0.0;
    for (int32_t i = reached - 1; i >= 0; --i) {
      int32_t x = w->order[i];
      for (int32_t p = 0; p < w->npred[x]; ++p) {
        int32_t v = w->pred[rp[x] + p];
        del[v] += (double)w->sig[v] / (double)w->sig[x] * (1.0 + del[x]);
      }
      if (x != s && bc) bc[x] += del[x];
    }
    if (delta_out) for (int32_t i = 0; i < n; ++i) delta_out[i] = del[i];
    if (sigma_ld_out) for (int32_t i = 0; i < n; ++i) sigma_ld_out[i] = (long double)w->sig[i];
  } else {
    for (int32_t i = 0; i < n; ++i) w->dell[i] = 0.0L;
    for (int32_t i = reached - 1; i >= 0; --i) {
      int32_t x = w->order[i];
      for (int32_t p = 0; p < w->npred[x]; ++p) {
        int32_t v = w->pred[rp[x] + p];
        w->dell[v] += w->sigl[v] / w->sigl[x] * (1.0L + w->dell[x]);
      }
      if (x != s && bc) bc[x] += (double)w->dell[x];
    }
    if (delta_out) for (int32_t i = 0; i < n; ++i) delta_out[i] = (double)w->dell[i];
    if (sigma_ld_out) for (int32_t i = 0; i < n; ++i) sigma_ld_out[i] = w->sigl[i];
  }
  if (stats) {
    int64_t nnz_r = 0, dag = 0;
    for (int32_t i = 0; i < reached; ++i) {
      int32_t x = w->order[i];
      nnz_r += rp[x + 1] - rp[x];
      dag += w->npred[x];
    }
    stats[0] = reached; stats[1] = nnz_r; stats[2] = dag;
  }
  free(dtmp);
  return ovf;
}

int orc_source(int32_t n, const int32_t* rp, const int32_t* ci, int32_t s,
               int32_t* d, uint64_t* sigma, long double* sigma_ld, double* delta, int64_t* stats) {
  if (n <= 0 || s < 0 || s >= n) return -2;
  orc_ws w;
  if (ws_init(&w, n, rp[n]) != 0) return -1;
  int r = source_ws(rp, ci, n, s, &w, d, sigma, sigma_ld, delta, NULL, stats);
  ws_free(&w);
  return r;
}

typedef struct {
  const int32_t* rp; const int32_t* ci; int32_t n;
  const int32_t* src; int64_t lo, hi;
  double* bc; uint8_t* ovf; int64_t* stats; int err;
} orc_job;

static void* run_job(void* arg) {
  orc_job* j = (orc_job*)arg;
  orc_ws w;
  if (ws_init(&w, j->n, j->rp[j->n]) != 0) { j->err = -1; return NULL; }
  for (int64_t i = j->lo; i < j->hi; ++i) {
    int r = source_ws(j->rp, j->ci, j->n, j->src[i], &w, NULL, NULL, NULL, NULL, j->bc,
                      j->stats ? j->stats + 3 * i : NULL);
    if (r < 0) { j->err = -1; break; }
    if (j->ovf) j->ovf[i] = (uint8_t)r;
  }
  ws_free(&w);
  return NULL;
}

/*
 * RAW scores over sources src[0..k) (repeats count repeatedly) written to
 * bc[n].  ovf[k] and stats[3k] are optional.  nthreads <= 1 runs inline.
 * Returns 0, or -1 on allocation failure, -2 on a bad source id.
 */
int orc_bc(int32_t n, const int32_t* rp, const int32_t* ci, const int32_t* src, int64_t k,
           int nthreads, double* bc, uint8_t* ovf, int64_t* stats) {
  for (int64_t i = 0; i < k; ++i) if (src[i] < 0 || src[i] >= n) return -2;
  for (int32_t i = 0; i < n; ++i) bc[i] = 0.0;
  if (nthreads < 1) nthreads = 1;
  if (nthreads > k) nthreads = (int)(k > 0 ? k : 1);
  orc_job* jobs = (orc_job*)calloc((size_t)nthreads, sizeof(orc_job));
  pthread_t* th = (pthread_t*)calloc((size_t)nthreads, sizeof(pthread_t));
  if (!jobs || !th) { free(jobs); free(th); return -1; }
  int err = 0;
  for (int t = 0; t < nthreads; ++t) {
    orc_job* j = &jobs[t];
    j->rp = rp; j->ci = ci; j->n = n; j->src = src;
    j->lo = k * t / nthreads; j->hi = k * (t + 1) / nthreads;
    j->ovf = ovf; j->stats = stats;
    j->bc = (t == 0) ? bc : (double*)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (!j->bc) { err = -1; nthreads = t; break; }
  }
  if (nthreads == 1 && !err) run_job(&jobs[0]);
  else {
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, run_job, &jobs[t]);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  }
  for (int t = 0; t < nthreads; ++t) if (jobs[t].err) err = jobs[t].err;
  for (int t = 1; t < nthreads; ++t) {
    for (int32_t i = 0; i < n; ++i) bc[i] += jobs[t].bc[i];
    free(jobs[t].bc);
  }
  free(jobs); free(th);
  return err;
}

/*
 * O(n^3) reference (Sec. 2's pre-Brandes method).  Distances by
 * Floyd-Warshall on an n x n matrix; sigma_st by counting, for every s, over
 * vertices t in increasing distance, sigma_st = sum of sigma_su over the
 * neighbours u of t one step closer to s; then
 *   RAW(v) = sum over ordered pairs (s, t), s != v != t, s != t, with
 *            d(s,v) + d(v,t) = d(s,t)  of  sigma_sv * sigma_vt / sigma_st.
 * Counts are long double.  Memory is O(n^2): meant for n up to a few
 * thousand.  Returns 0, -1 on allocation failure.
 */
int orc_bellman(int32_t n, const int32_t* rp, const int32_t* ci, double* bc) {
  const int32_t INF = 0x3fffffff;
  size_t nn = (size_t)n * (size_t)n;
  int32_t* D = (int32_t*)malloc(sizeof(int32_t) * (nn ? nn : 1));
  long double* S = (long double*)malloc(sizeof(long double) * (nn ? nn : 1));
  int32_t* byd = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
  int32_t* cnt = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n + 2));
  if (!D || !S || !byd || !cnt) { free(D); free(S); free(byd); free(cnt); return -1; }
  for (size_t i = 0; i < nn; ++i) D[i] = INF;
  for (int32_t i = 0; i < n; ++i) {
    D[(size_t)i * n + i] = 0;
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) D[(size_t)i * n + ci[e]] = 1;
  }
  for (int32_t k = 0; k < n; ++k)
    for (int32_t i = 0; i < n; ++i) {
      int32_t dik = D[(size_t)i * n + k];
      if (dik >= INF) continue;
      for (int32_t j = 0; j < n; ++j) {
        int32_t t = dik + D[(size_t)k * n + j];
        if (t < D[(size_t)i * n + j]) D[(size_t)i * n + j] = t;
      }
    }
  for (int32_t s = 0; s < n; ++s) {
    int32_t* Ds = D + (size_t)s * n;
    long double* Ss = S + (size_t)s * n;
    /* bucket vertices by distance from s (counting sort) */
    for (int32_t i = 0; i <= n + 1; ++i) cnt[i] = 0;
    for (int32_t t = 0; t < n; ++t) if (Ds[t] < INF) cnt[Ds[t] + 1]++;
    for (int32_t i = 0; i <= n; ++i) cnt[i + 1] += cnt[i];
    int32_t reach = cnt[n + 1];
    for (int32_t t = 0; t < n; ++t) if (Ds[t] < INF) byd[cnt[Ds[t]]++] = t;
    for (int32_t t = 0; t < n; ++t) Ss[t] = 0.0L;
    for (int32_t i = 0; i < reach; ++i) {
      int32_t t = byd[i];
      if (t == s) { Ss[t] = 1.0L; continue; }
      long double acc = 0.0L;
      for (int32_t e = rp[t]; e < rp[t + 1]; ++e) {
        int32_t u = ci[e];
        if (Ds[u] < INF && Ds[u] == Ds[t] - 1) acc += Ss[u];
      }
      Ss[t] = acc;
    }
  }
  for (int32_t v = 0; v < n; ++v) {
    long double acc = 0.0L;
    for (int32_t s = 0; s < n; ++s) {
      if (s == v) continue;
      int32_t dsv = D[(size_t)s * n + v];
      if (dsv >= INF) continue;
      for (int32_t t = 0; t < n; ++t) {
        if (t == v || t == s) continue;
        int32_t dvt = D[(size_t)v * n + t];
        if (dvt >= INF) continue;
        if (dsv + dvt == D[(size_t)s * n + t])
          acc += S[(size_t)s * n + v] * S[(size_t)v * n + t] / S[(size_t)s * n + t];
      }
    }
    bc[v] = (double)acc;
  }
  free(D); free(S); free(byd); free(cnt);
  return 0;
}
