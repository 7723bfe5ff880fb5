/*
 * Seeded synthetic graph generators shared by the tests, the benchmark and
 * the smoke check.  This module only produces inputs: it holds none of the
 * betweenness arithmetic.  Both the CPU oracle and the GPU library consume
 * its output, and neither links against the other.
 *
 * Random numbers come from a counter-based form of splitmix64 (Steele, Lea
 * and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014):
 * the k-th draw of stream `seed` is mix64(mix64(seed) + (k+1)*gamma), so any
 * draw can be recomputed from its (seed, counter) pair alone.
 *
 * Graphs are returned as lists of unordered pairs; gg_build_csr turns such a
 * list into a symmetric CSR with self-loops and duplicate pairs removed and
 * each adjacency list sorted ascending (the input form of the library).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GG_GAMMA 0x9e3779b97f4a7c15ULL

static inline uint64_t gg_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

uint64_t gg_u64(uint64_t seed, uint64_t ctr) {
  return gg_mix64(gg_mix64(seed) + (ctr + 1) * GG_GAMMA);
}

static inline double gg_u01(uint64_t seed, uint64_t ctr) {
  return (double)(gg_u64(seed, ctr) >> 11) * 0x1.0p-53;
}

/* uniform integer in [0, bound) by the multiply-high method */
static inline uint64_t gg_below(uint64_t seed, uint64_t ctr, uint64_t bound) {
  return (uint64_t)(((unsigned __int128)gg_u64(seed, ctr) * bound) >> 64);
}

/* Sub-stream keys so that the pair draws, the relabelling permutation and the
 * sampling steps of one seed never share counters. */
static uint64_t gg_stream(uint64_t seed, uint64_t tag) { return gg_mix64(seed ^ gg_mix64(tag)); }

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos 2004) with quadrant probabilities
 * (a, b, c, 1-a-b-c) and no noise.  Pair e draws `scale` uniforms, one per
 * recursion level, from counters e*scale + level; the first level picks the
 * most significant bit.  The result is then relabelled by a seeded
 * Fisher-Yates permutation so that vertex ids carry no degree order.
 */
void gg_rmat_pairs(int scale, int64_t npairs, double a, double b, double c,
                   uint64_t seed, int32_t* src, int32_t* dst) {
  uint64_t ks = gg_stream(seed, 1);
  double ab = a + b, abc = a + b + c;
  for (int64_t e = 0; e < npairs; ++e) {
    uint32_t u = 0, v = 0;
    for (int l = 0; l < scale; ++l) {
      double r = gg_u01(ks, (uint64_t)e * (uint64_t)scale + (uint64_t)l);
      uint32_t rb, cb;
      if (r < a) { rb = 0; cb = 0; }
      else if (r < ab) { rb = 0; cb = 1; }
      else if (r < abc) { rb = 1; cb = 0; }
      else { rb = 1; cb = 1; }
      u = (u << 1) | rb;
      v = (v << 1) | cb;
    }
    src[e] = (int32_t)u;
    dst[e] = (int32_t)v;
  }
  int64_t n = (int64_t)1 << scale;
  int32_t* perm = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
  if (!perm) return;
  uint64_t kp = gg_stream(seed, 2);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)gg_below(kp, (uint64_t)i, (uint64_t)(i + 1));
    int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
  for (int64_t e = 0; e < npairs; ++e) { src[e] = perm[src[e]]; dst[e] = perm[dst[e]]; }
  free(perm);
}

/* Seeded Fisher-Yates permutation of [0, n) (exported for relabelling tests). */
void gg_permutation(int64_t n, uint64_t seed, int32_t* perm) {
  uint64_t kp = gg_stream(seed, 3);
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)gg_below(kp, (uint64_t)i, (uint64_t)(i + 1));
    int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
}

/* k distinct values from [0, total) by a partial Fisher-Yates over an index
 * array; the chosen values land in out[0..k). */
static int gg_sample_distinct(int64_t total, int64_t k, uint64_t key, int64_t* out) {
  int64_t* idx = (int64_t*)malloc(sizeof(int64_t) * (size_t)total);
  if (!idx) return -1;
  for (int64_t i = 0; i < total; ++i) idx[i] = i;
  for (int64_t i = 0; i < k; ++i) {
    int64_t j = i + (int64_t)gg_below(key, (uint64_t)i, (uint64_t)(total - i));
    int64_t t = idx[i]; idx[i] = idx[j]; idx[j] = t;
    out[i] = idx[i];
  }
  free(idx);
  return 0;
}

/*
 * Pendant attachment: P new vertices n0 .. n0+P-1, vertex n0+i joined to a
 * hub drawn uniformly from [0, n0).
 */
void gg_pendant_pairs(int64_t n0, int64_t P, uint64_t seed, int32_t* src, int32_t* dst) {
  uint64_t kh = gg_stream(seed, 4);
  for (int64_t i = 0; i < P; ++i) {
    src[i] = (int32_t)(n0 + i);
    dst[i] = (int32_t)gg_below(kh, (uint64_t)i, (uint64_t)n0);
  }
}

/*
 * Road-like lattice: an R x C grid (vertex r*C + c) whose 4-neighbour lattice
 * edges lose exactly `drop` of their number, chosen uniformly, and which gains
 * exactly `diag` distinct local diagonals (r,c)-(r+1,c+1) or (r,c)-(r+1,c-1),
 * chosen uniformly among all 2(R-1)(C-1) of them.  Returns the pair count
 * written (R(C-1) + (R-1)C - drop + diag), or -1 on bad arguments.
 */
int64_t gg_grid_pairs(int64_t R, int64_t C, int64_t drop, int64_t diag, uint64_t seed,
                      int32_t* src, int32_t* dst) {
  int64_t nh = R * (C - 1), nv = (R - 1) * C, nl = nh + nv;
  int64_t nd = 2 * (R - 1) * (C - 1);
  if (R < 1 || C < 1 || drop < 0 || drop > nl || diag < 0 || diag > nd) return -1;
  uint8_t* gone = (uint8_t*)calloc((size_t)(nl > 0 ? nl : 1), 1);
  if (!gone) return -1;
  if (drop > 0) {
    int64_t* pick = (int64_t*)malloc(sizeof(int64_t) * (size_t)drop);
    if (!pick || gg_sample_distinct(nl, drop, gg_stream(seed, 5), pick) != 0) {
      free(pick); free(gone); return -1;
    }
    for (int64_t i = 0; i < drop; ++i) gone[pick[i]] = 1;
    free(pick);
  }
  int64_t w = 0;
  for (int64_t e = 0; e < nl; ++e) {
    if (gone[e]) continue;
    int64_t u, v;
    if (e < nh) { int64_t r = e / (C - 1), c = e % (C - 1); u = r * C + c; v = u + 1; }
    else { int64_t f = e - nh; int64_t r = f / C, c = f % C; u = r * C + c; v = u + C; }
    src[w] = (int32_t)u; dst[w] = (int32_t)v; ++w;
  }
  free(gone);
  if (diag > 0) {
    int64_t* pick = (int64_t*)malloc(sizeof(int64_t) * (size_t)diag);
    if (!pick || gg_sample_distinct(nd, diag, gg_stream(seed, 6), pick) != 0) { free(pick); return -1; }
    for (int64_t i = 0; i < diag; ++i) {
      int64_t f = pick[i];
      int64_t kind = f / ((R - 1) * (C - 1));           /* 0: down-right, 1: down-left */
      int64_t g = f % ((R - 1) * (C - 1));
      int64_t r = g / (C - 1), c = g % (C - 1);
      int64_t u, v;
      if (kind == 0) { u = r * C + c; v = (r + 1) * C + c + 1; }
      else { u = r * C + c + 1; v = (r + 1) * C + c; }
      src[w] = (int32_t)u; dst[w] = (int32_t)v; ++w;
    }
    free(pick);
  }
  return w;
}

/* Uniform sample of k distinct values from cand[0..ncand) (seeded), in draw order. */
int gg_sample(const int32_t* cand, int64_t ncand, int64_t k, uint64_t seed, int32_t* out) {
  if (k < 0 || k > ncand) return -1;
  int64_t* pick = (int64_t*)malloc(sizeof(int64_t) * (size_t)(k > 0 ? k : 1));
  if (!pick) return -1;
  if (gg_sample_distinct(ncand, k, gg_stream(seed, 7), pick) != 0) { free(pick); return -1; }
  for (int64_t i = 0; i < k; ++i) out[i] = cand[pick[i]];
  free(pick);
  return 0;
}

/* Stable counting sort of (key, other) pairs by key in [0, n). */
static int gg_counting_sort(int64_t n, int64_t len, const int32_t* key, const int32_t* other,
                            int32_t* key_out, int32_t* other_out) {
  int64_t* cnt = (int64_t*)calloc((size_t)n + 1, sizeof(int64_t));
  if (!cnt) return -1;
  for (int64_t i = 0; i < len; ++i) cnt[key[i] + 1]++;
  for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
  for (int64_t i = 0; i < len; ++i) {
    int64_t p = cnt[key[i]]++;
    key_out[p] = key[i];
    other_out[p] = other[i];
  }
  free(cnt);
  return 0;
}

/*
 * Symmetric, simple CSR from a pair list over vertices [0, n).  Pairs with an
 * id outside [0, n) make the call fail (-2).  col_out must hold 2*npairs
 * entries; returns nnz (directed entries written) or a negative error.
 */
int64_t gg_build_csr(int64_t n, int64_t npairs, const int32_t* src, const int32_t* dst,
                     int64_t* row_ptr, int32_t* col_out) {
  int64_t cap = 2 * npairs;
  int32_t *a = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
  int32_t *b = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
  int32_t *ta = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
  int32_t *tb = (int32_t*)malloc(sizeof(int32_t) * (size_t)(cap > 0 ? cap : 1));
  if (!a || !b || !ta || !tb) { free(a); free(b); free(ta); free(tb); return -1; }
  int64_t len = 0;
  for (int64_t i = 0; i < npairs; ++i) {
    int32_t u = src[i], v = dst[i];
    if (u < 0 || v < 0 || u >= n || v >= n) { free(a); free(b); free(ta); free(tb); return -2; }
    if (u == v) continue;
    a[len] = u; b[len] = v; ++len;
    a[len] = v; b[len] = u; ++len;
  }
  /* sort by (a, b): first by b, then stably by a */
  if (gg_counting_sort(n, len, b, a, tb, ta) != 0 || gg_counting_sort(n, len, ta, tb, a, b) != 0) {
    free(a); free(b); free(ta); free(tb); return -1;
  }
  for (int64_t i = 0; i <= n; ++i) row_ptr[i] = 0;
  int64_t w = 0;
  for (int64_t i = 0; i < len; ++i) {
    if (i > 0 && a[i] == a[i - 1] && b[i] == b[i - 1]) continue;
    col_out[w++] = b[i];
    row_ptr[a[i] + 1]++;
  }
  for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
  free(a); free(b); free(ta); free(tb);
  return w;
}
