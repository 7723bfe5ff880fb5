// Many sources per launch.  A batch of B = 64 K sources advances level by
// level together inside one cooperative persistent kernel.  Lane j of the
// 64-lane word k is source 64 k + j; per-(vertex, source) state is stored
// source-minor ([vertex][lane]) so a wave touching one vertex reads or
// writes one contiguous row per word.  Per vertex, 64-bit lane masks record
// which sources have reached it (vis) and which sit on a given level (F_l,
// four rotating arrays).
//
// Level lists hold (vertex, word) entries, cut into work units of <= 256
// edges that waves take one at a time.  An entry (v, k) joins level
// l+1's list when the first lane of word k reaches v there: the atomic OR
// that turns F_{l+1}(v, k) from zero to non-zero appends it.  Appends are
// staged in the workgroup's LDS and flushed with one reservation per
// workgroup and phase, so the level counters see a few hundred atomics per
// level rather than one per discovering wave.
//
// Forward sweep (shortest-path counting, Alg. 2-3 generalised to B
// sources).  Phase l, one grid barrier each, walks the level-l units once
// and does two jobs per edge (w -> x):
//   counting of level l -- sigma(w) gains sigma(x) on the lanes where x sits
//     on level l-1 (rows gathered several at a time).  2-degree derived
//     lanes (Lemma 1) take Eq. (6) instead: the sum of the two partner
//     lanes' counts at w over the partners sitting on level l-1 at w.
//   top-down discovery of level l+1 -- F_{l+1}(x) |= F_l(w) & ~(F_{l-1}(x)
//     | F_l(x)): in an undirected graph a neighbour of a level-l vertex is
//     at distance l-1, l or l+1, so the two level masks the phase reads
//     anyway tell which lanes have not reached x.  Bottom-up levels instead OR, for every (vertex, word) not
//     yet reached by all the word's sources, its neighbours' level-l masks.
//     Derived lanes are not propagated along edges: lane c reaches v at
//     level l+1 exactly when a partner sits on v at level l and c has not
//     reached v.
// Backward sweep (dependency accumulation, Alg. 4-5, successor checking):
//   per unit of the level-l entries, each lane sums psi over the neighbours
//   whose level-(l+1) mask has the lane's bit, then delta = sigma * sum and
//   psi = (1 + delta + omega) / sigma overwrite the count in place.  The
//   lanes' weight * (delta + omega) are summed (lane order) per result slot
//   into a per-(word, slot) array; after the sweep one pass folds those
//   arrays into the slots' scores in word order.
// Entries spanning several units combine per-unit partial sums in unit
// order (the last arriving wave does it, reading the others' partials
// through device-scope accesses rather than behind cache-wide fences), so
// results do not depend on scheduling.  Units of dense levels are dealt to
// workgroups by stride and claimed inside each workgroup from an LDS
// counter, so a workgroup's waves share its heavy and light units.
// Sparse levels (fewer than two lanes per entry on average, the long tail
// of a deep graph): a unit whose entry has one edge lane and at most 32
// edges is walked by a single lane, 64 such units per wave, both sweeps;
// the others keep the wave-per-unit form.  The forward sweep records each
// entry's lane mask, which the backward sweep reads instead of per-lane
// levels.
#include "bc_common.h"
#include "bc_kernels.h"

namespace bcx {

constexpr int CHB = kBatchChunk;
constexpr int kSlots = 4;                          // rotating level-mask arrays
constexpr int kStageCap = 8192;                    // staged appends per workgroup and phase
constexpr int kWavesPB = kBatchBlock / kWave;
constexpr int kStagePerThread = kStageCap / kBatchBlock;
constexpr int kLaneMaxDeg = 32;                    // longest adjacency a single lane walks

__device__ __forceinline__ int32_t ldr32(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t ldr64(const unsigned long long* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t rl32(int32_t v, int src) { return __builtin_amdgcn_readlane(v, src); }
__device__ __forceinline__ uint64_t rl64(uint64_t v, int src) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, src);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
  return ((uint64_t)hi << 32) | lo;
}

// Workgroup-shared state.
struct Stage {
  uint64_t e[kStageCap];  // staged entries of the level being discovered
  int32_t n;              // entries staged (may pass kStageCap: the rest went straight to the list)
  int32_t base_e, base_u, base_p;
  unsigned long long full;
  unsigned long long newl;  // lanes discovered by the workgroup in this phase
  uint64_t wu[kWavesPB], wp[kWavesPB], wd[kWavesPB];
  uint64_t sX[kMaxWords];
  unsigned long long ctr[3];
  int32_t fclaim[2], bclaim[2];  // unit claims of the forward phases and backward levels, by parity
};

__device__ __forceinline__ void raise_b(const BatchArgs& a, int lvl, int32_t code) {
  atomicOr(&a.lc[lvl].err, code);
  atomicOr(a.err, code);
}

// Writes entry `ent` (its vertex's edges start at rb, deg of them) at list
// position e with its units at u (partial-sum slots at pb when it spans
// several units).
__device__ __forceinline__ void write_entry(const BatchArgs& a, int lvl, int64_t e, int64_t u, int64_t pb,
                                            uint64_t ent, int32_t rb, int32_t deg) {
  const int32_t v = (int32_t)(uint32_t)ent;
  const int32_t k = (int32_t)(ent >> 32);
  const int32_t nun = units_of<CHB>(deg);
  if (e >= a.cap_entries) {
    raise_b(a, lvl, kErrCapEntries);
  } else if (u + nun > a.cap_units) {
    raise_b(a, lvl, kErrCapUnits);
  } else if (nun > 1 && pb + nun > a.cap_parts) {
    raise_b(a, lvl, kErrCapPartials);
  } else {
    a.Q[e] = ent;
    if (nun == 1) {
      a.U[u] = BUnit{v, rb, rb + deg, deg, k, 0, (int32_t)e, 0};
    } else {
      a.arrive[e] = 0;
      for (int32_t c = 0; c < nun; ++c)
        a.U[u + c] = BUnit{v, rb + c * CHB, min(rb + deg, rb + (c + 1) * CHB), deg, k, c, (int32_t)e, (int32_t)pb};
    }
  }
}

// Direct append of one wave's lanes (staging buffer full).
__device__ __forceinline__ void global_append(const BatchArgs& a, int lvl, int32_t ebase, int32_t ubase, bool want,
                                           uint64_t ent) {
  if (ballot(want) == 0) return;
  int32_t deg = 0, nun = 0, rb = 0;
  if (want) {
    const int32_t v = (int32_t)(uint32_t)ent;
    rb = a.rp[v];
    deg = a.rp[v + 1] - rb;
    nun = units_of<CHB>(deg);
  }
  const uint64_t contrib = want ? ((1ull << 32) | (uint64_t)(uint32_t)nun) : 0ull;
  const uint64_t incl = wave_incl_scan_u64(contrib);
  const uint64_t total = shfl(incl, kWave - 1);
  const uint64_t dsum = wave_sum_u64(want ? (uint64_t)deg : 0ull);
  unsigned long long base = 0;
  if (lane_id() == kWave - 1) {
    base = atomicAdd(&a.lc[lvl].packed, (unsigned long long)total);
    atomicAdd(&a.lc[lvl].fedges, (unsigned long long)dsum);
  }
  base = shfl((uint64_t)base, kWave - 1);
  if (want) {
    const uint64_t my = base + incl - contrib;
    int64_t pb = 0;
    if (nun > 1) pb = atomicAdd(&a.lc[lvl].pslots, nun);
    write_entry(a, lvl, (int64_t)ebase + (int64_t)(my >> 32), (int64_t)ubase + (int64_t)(my & 0xffffffffull), pb,
                ent, rb, deg);
  }
}

// Appends the lanes with `want` (one wave, all lanes calling).
__device__ __forceinline__ void stage_append(const BatchArgs& a, Stage& st, int lvl, int32_t ebase, int32_t ubase,
                                             bool want, uint64_t ent) {
  const uint64_t wm = ballot(want);
  if (wm == 0) return;
  int pos = 0;
  if (lane_id() == 0) pos = atomicAdd(&st.n, __popcll(wm));
  pos = __shfl(pos, 0, kWave);
  const int r = pos + lanes_below(wm);
  const bool in = want && r < kStageCap;
  if (in) st.e[r] = ent;
  if (pos + __popcll(wm) > kStageCap) global_append(a, lvl, ebase, ubase, want && !in, ent);
}

// Flushes the staged entries of level `lvl` (whole workgroup): one
// reservation of entries, units, partial-sum slots and frontier edges.
__device__ __forceinline__ void stage_flush(const BatchArgs& a, Stage& st, int lvl, int32_t ebase, int32_t ubase) {
  __syncthreads();
  const int cnt = min(st.n, kStageCap);
  const int t = (int)threadIdx.x, lane = lane_id(), wv = t >> 6;
  if (cnt > 0) {
    int32_t nun[kStagePerThread];
    uint64_t su = 0, sp = 0, sd = 0;
#pragma unroll 1
    for (int r = 0; r < kStagePerThread; ++r) {
      const int i = t * kStagePerThread + r;
      nun[r] = 0;
      if (i < cnt) {
        const int32_t v = (int32_t)(uint32_t)st.e[i];
        const int32_t deg = a.rp[v + 1] - a.rp[v];
        nun[r] = units_of<CHB>(deg);
        su += (uint64_t)nun[r];
        sd += (uint64_t)deg;
        if (nun[r] > 1) sp += (uint64_t)nun[r];
      }
    }
    const uint64_t iu = wave_incl_scan_u64(su), ip = wave_incl_scan_u64(sp);
    const uint64_t ds = wave_sum_u64(sd);
    if (lane == kWave - 1) { st.wu[wv] = iu; st.wp[wv] = ip; st.wd[wv] = ds; }
    __syncthreads();
    if (t == 0) {
      uint64_t tu = 0, tp = 0, td = 0;
      for (int w = 0; w < kWavesPB; ++w) {
        const uint64_t u = st.wu[w], p = st.wp[w];
        st.wu[w] = tu;
        st.wp[w] = tp;
        tu += u;
        tp += p;
        td += st.wd[w];
      }
      const unsigned long long b =
          atomicAdd(&a.lc[lvl].packed, ((unsigned long long)cnt << 32) | (unsigned long long)tu);
      if (td) atomicAdd(&a.lc[lvl].fedges, (unsigned long long)td);
      st.base_e = (int32_t)(b >> 32);
      st.base_u = (int32_t)(b & 0xffffffffull);
      st.base_p = tp ? atomicAdd(&a.lc[lvl].pslots, (int32_t)tp) : 0;
    }
    __syncthreads();
    int64_t uo = (int64_t)ubase + st.base_u + (int64_t)(st.wu[wv] + iu - su);
    int64_t po = (int64_t)st.base_p + (int64_t)(st.wp[wv] + ip - sp);
#pragma unroll 1
    for (int r = 0; r < kStagePerThread; ++r) {
      const int i = t * kStagePerThread + r;
      if (i < cnt) {
        const int32_t v = (int32_t)(uint32_t)st.e[i];
        const int32_t rb = a.rp[v];
        write_entry(a, lvl, (int64_t)ebase + st.base_e + i, uo, po, st.e[i], rb, a.rp[v + 1] - rb);
        uo += nun[r];
        if (nun[r] > 1) po += nun[r];
      }
    }
  }
  __syncthreads();
  if (t == 0) {
    st.n = 0;
    if (st.full) atomicAdd(a.fulledges, st.full);
    if (st.newl) atomicAdd(&a.lc[lvl].lanes, st.newl);
    st.full = 0;
    st.newl = 0;
  }
}

// Appends one entry from a single lane (divergent code): a slot of the
// workgroup's stage, or straight to the list when the stage is full.
__device__ __forceinline__ void lane_append(const BatchArgs& a, Stage& st, int lvl, int32_t ebase, int32_t ubase,
                                            uint64_t ent) {
  const int pos = atomicAdd(&st.n, 1);
  if (pos < kStageCap) {
    st.e[pos] = ent;
    return;
  }
  const int32_t v = (int32_t)(uint32_t)ent;
  const int32_t rb = a.rp[v], deg = a.rp[v + 1] - rb;
  const int32_t nun = units_of<CHB>(deg);
  const unsigned long long b = atomicAdd(&a.lc[lvl].packed, (1ull << 32) | (unsigned long long)(uint32_t)nun);
  atomicAdd(&a.lc[lvl].fedges, (unsigned long long)deg);
  const int64_t pb = nun > 1 ? atomicAdd(&a.lc[lvl].pslots, nun) : 0;
  write_entry(a, lvl, (int64_t)ebase + (int64_t)(b >> 32), (int64_t)ubase + (int64_t)(b & 0xffffffffull), pb, ent,
              rb, deg);
}

// Units of a phase are dealt to workgroups by a fixed stride (workgroup b
// gets units b, b + G, b + 2 G, ... for a grid of G) and claimed inside the
// workgroup one at a time from an LDS counter, so heavy and light units
// spread over the workgroup's waves as they finish.
__device__ __forceinline__ int64_t wg_claim(int32_t* ctr) {
  int32_t v = 0;
  if (lane_id() == 0) v = atomicAdd(ctr, 1);
  return (int64_t)blockIdx.x + (int64_t)gridDim.x * (int64_t)__builtin_amdgcn_readfirstlane(v);
}

// Run counters, per lane (summed over the wave when published).
struct Ctr {
  uint64_t reached = 0, rnnz = 0, dag = 0, full = 0, newl = 0;
};

// ------------------------------------------------------------ forward unit

// A unit of level kl: counting of level kl (when `count`) and top-down
// discovery of level kl+1 (when `td`).
template <bool EXT>
__device__ __forceinline__ void forward_unit(const BatchArgs& a, Stage& st, const BUnit& un, const uint64_t* par,
                                             const uint64_t* cur, uint64_t* nxt, int kl, bool count, bool td,
                                             int32_t ebn, int32_t ubn, Ctr& C) {
  constexpr int G = 8;  // neighbour rows loaded before any is consumed
  const int K = a.K;
  const size_t B = (size_t)64 * K;
  const int lane = lane_id();
  const int32_t* __restrict__ rp = a.rp;
  const int32_t* __restrict__ ci = a.ci;
  const int32_t w = un.v, k = un.k, c = un.c, deg = un.deg;
  const int32_t beg = un.beg, end = un.end;
  // the first chunk's neighbours are fetched with the unit's own masks
  const int32_t vl0 = beg + lane < end ? ci[beg + lane] : 0;
  const size_t wk = (size_t)w * K + k;
  const uint64_t EL = a.edge_lanes[k];
  const uint64_t nbm = cur[wk];  // lanes of word k on level kl at w
  const uint64_t em = nbm & EL;  // of them, lanes that count and propagate along edges
  const bool cnt = count && em != 0;
  const bool disc = td && em != 0;
  uint64_t s = 0;
  Ext x = ext_zero();
  bool wrap = false;
  if (cnt || disc) {
    for (int32_t off0 = beg; off0 < end; off0 += kWave) {
      const int32_t off = off0 + lane;
      int32_t vl = 0;
      uint64_t ml = 0;
      bool claimed = false;
      if (off < end) {
        vl = off0 == beg ? vl0 : ci[off];
        const size_t xk = (size_t)vl * K + k;
        const uint64_t px = par[xk];
        if (cnt) ml = px & em;
        if (disc) {
          // a neighbour of a level-kl vertex is at distance kl-1, kl or kl+1
          // from the lane's source, so "not yet reached" is "on neither level"
          // lanes already set at the neighbour (bits only get set within a
          // level, and the barrier's acquire drops stale lines) need no
          // atomic: hubs would otherwise take one per frontier edge
          const uint64_t nb = em & ~(px | cur[xk]);
          if (nb && (nxt[xk] & nb) != nb) {
            const uint64_t old = atomicOr((unsigned long long*)&nxt[xk], (unsigned long long)nb);
            claimed = old == 0ull;
            C.newl += (uint64_t)__popcll(nb & ~old);
          }
        }
      }
      if (cnt) {
        C.dag += (uint64_t)__popcll(ml);
        uint64_t act = ballot(ml != 0);
        while (act) {
          int ti[G];
#pragma unroll
          for (int i = 0; i < G; ++i) {
            ti[i] = act ? __builtin_ctzll(act) : -1;
            act &= act ? act - 1 : 0ull;
          }
          if (EXT) {
            Ext xs[G];
#pragma unroll
            for (int i = 0; i < G; ++i) {
              xs[i] = ext_zero();
              if (ti[i] >= 0) {
                const int32_t v = rl32(vl, ti[i]);
                const uint64_t mv = rl64(ml, ti[i]);
                const size_t row = (size_t)v * B + 64 * k;  // uniform base, lane offset
                if ((mv >> lane) & 1ull) xs[i] = Ext{(a.sm + row)[lane], (a.se + row)[lane]};
              }
            }
#pragma unroll
            for (int i = 0; i < G; ++i) x = ext_add(x, xs[i]);
          } else {
            uint64_t ys[G];
#pragma unroll
            for (int i = 0; i < G; ++i) {
              ys[i] = 0;
              if (ti[i] >= 0) {
                const int32_t v = rl32(vl, ti[i]);
                const uint64_t mv = rl64(ml, ti[i]);
                const uint64_t* row = a.sig + (size_t)v * B + 64 * k;  // uniform base, lane offset
                if ((mv >> lane) & 1ull) ys[i] = row[lane];
              }
            }
#pragma unroll
            for (int i = 0; i < G; ++i) {
              if (s + ys[i] < s) wrap = true;
              s += ys[i];
            }
          }
        }
      }
      if (disc) stage_append(a, st, kl + 1, ebn, ubn, claimed, bentry(vl, k));
    }
  }
  if (!count) return;
  // combine the units of a split entry in unit order (the last arriving wave)
  if (deg > CHB) {
    const int32_t nunits = units_of<CHB>(deg);
    const size_t pi = (size_t)(un.pb + c) * 64 + lane;
    if (EXT) { part_store(&a.part_m[pi], x.m); part_store(&a.part_e[pi], x.e); }
    else { part_store(&a.part_m[pi], __longlong_as_double((long long)s)); part_store(&a.part_e[pi], wrap ? 1 : 0); }
    part_stores_done();
    int32_t prev = 0;
    if (lane == 0) prev = atomicAdd(&a.arrive[un.e], 1);
    prev = __shfl(prev, 0, kWave);
    if (prev != nunits - 1) return;
    part_loads_after();
    s = 0;
    x = ext_zero();
    wrap = false;
    for (int32_t cc = 0; cc < nunits; ++cc) {
      const size_t pc = (size_t)(un.pb + cc) * 64 + lane;
      const double pm = part_load(&a.part_m[pc]);
      const int32_t pe = part_load(&a.part_e[pc]);
      if (EXT) {
        x = ext_add(x, Ext{pm, pe});
      } else {
        const uint64_t y = (uint64_t)__double_as_longlong(pm);
        if (s + y < s || pe) wrap = true;
        s += y;
      }
    }
  }
  // derived lanes (2-degree vertex c with partner lanes a, b; Lemma 1,
  // Eq. (6)): the first partner to reach w fixes d_c(w) = 1 + min(d_a, d_b)
  // and sigma_c(w) = the partners' counts on that level; dla / dlb record
  // whether d_a(w) <= d_b(w) / d_b(w) <= d_a(w) (both at a tie), which the
  // fused backward sweep uses to merge the two partners' frontiers
  if (a.derived_lanes[k] != 0) {
    const int pa = a.lane_pa[64 * k + lane], pb = a.lane_pb[64 * k + lane];
    const uint64_t before = a.vis[wk];  // lanes of the word that reached w on earlier levels
    bool la = false, lb = false;
    if (pa >= 0 && a.lane_src[64 * k + lane] != w) {
      la = ((nbm >> pa) & 1ull) && !((before >> pb) & 1ull);
      lb = ((nbm >> pb) & 1ull) && !((before >> pa) & 1ull);
    }
    const int qa = pa >= 0 ? pa : lane, qb = pb >= 0 ? pb : lane;
    const size_t idc = (size_t)w * B + 64 * k + lane;
    if (EXT) {
      const Ext xa{__shfl(x.m, qa, kWave), __shfl(x.e, qa, kWave)};
      const Ext xb{__shfl(x.m, qb, kWave), __shfl(x.e, qb, kWave)};
      Ext t = ext_zero();
      if (la) t = ext_add(t, xa);
      if (lb) t = ext_add(t, xb);
      if (la || lb) {
        const Ext z = ext_norm(t);
        a.sm[idc] = z.m;
        a.se[idc] = z.e;
      }
    } else {
      const uint64_t sa = __shfl(s, qa, kWave), sb = __shfl(s, qb, kWave);
      const bool wa = __shfl((int)wrap, qa, kWave) != 0, wb = __shfl((int)wrap, qb, kWave) != 0;
      uint64_t t = la ? sa : 0ull;
      bool wc = (la && wa) || (lb && wb);
      if (lb) {
        if (t + sb < t) wc = true;
        t += sb;
      }
      if (la || lb) {
        a.sig[idc] = t;
        if (wc) atomicOr(&a.lane_ovf[64 * k + lane], 1u);
      }
    }
    const uint64_t LA = ballot(la), LB = ballot(lb);
    if (lane == 0 && LA) atomicOr((unsigned long long*)&a.dla[wk], (unsigned long long)LA);
    if (lane == 0 && LB) atomicOr((unsigned long long*)&a.dlb[wk], (unsigned long long)LB);
  }
  // finalise word k at w: counts, levels, visited mask
  if ((nbm >> lane) & 1ull) {
    const size_t idx = (size_t)w * B + 64 * k + lane;
    if (EXT) {
      const Ext z = ext_norm(x);
      a.sm[idx] = z.m;
      a.se[idx] = z.e;
    } else {
      a.sig[idx] = s;
      if (wrap) atomicOr(&a.lane_ovf[64 * k + lane], 1u);
    }
    if (a.keep_lv) a.lv[idx] = kl;
  }
  if (lane == 0) {
    a.emask[un.e] = nbm;
    if (a.alpha > 0.0) {
      const uint64_t ov = a.vis[wk];
      const uint64_t nv = ov | nbm;
      a.vis[wk] = nv;
      // edges of word k no source of the word can still discover (bottom-up test)
      if ((nv & EL) == EL && (ov & EL) != EL) C.full += (uint64_t)deg;
    } else {
      atomicOr((unsigned long long*)&a.vis[wk], (unsigned long long)nbm);  // no round trip
    }
  }
  if (lane == 0) {
    const uint64_t pc = (uint64_t)__popcll(nbm);
    C.reached += pc;
    C.rnnz += pc * (uint64_t)deg;
  }
}

// The same unit worked by one lane: an entry of <= 32 edges whose word has
// a single lane l on level kl, and that lane propagates along edges.  Sparse
// levels (a lane or so per entry, as on long-diameter graphs) put 64 such
// units in a wave instead of one.  Sums run in edge order, as in the wave
// form, so results are identical.
template <bool EXT>
__device__ __forceinline__ void lane_forward_unit(const BatchArgs& a, Stage& st, const BUnit& un, uint64_t bit,
                                                  const uint64_t* par, const uint64_t* cur, uint64_t* nxt, int kl,
                                                  bool count, bool td, int32_t ebn, int32_t ubn, Ctr& C) {
  const int K = a.K;
  const size_t B = (size_t)64 * K;
  const int32_t* __restrict__ ci = a.ci;
  const int32_t w = un.v, k = un.k, deg = un.deg;
  const int l = __builtin_ctzll(bit);
  const size_t col = 64 * (size_t)k + l;
  uint64_t s = 0;
  Ext x = ext_zero();
  bool wrap = false;
  // four edges at a time: their neighbours, masks and counts are in flight together
  constexpr int Q4 = 4;
  for (int32_t e0 = un.beg; e0 < un.end; e0 += Q4) {
    int32_t xv[Q4];
    uint64_t px[Q4], cx[Q4];
#pragma unroll
    for (int j = 0; j < Q4; ++j) xv[j] = e0 + j < un.end ? ci[e0 + j] : -1;
#pragma unroll
    for (int j = 0; j < Q4; ++j) {
      px[j] = 0;
      cx[j] = 0;
      if (xv[j] >= 0) {
        const size_t xk = (size_t)xv[j] * K + k;
        px[j] = par[xk];
        if (td) cx[j] = cur[xk];
      }
    }
    if (count) {
      if (EXT) {
        Ext ys[Q4];
#pragma unroll
        for (int j = 0; j < Q4; ++j) {
          ys[j] = ext_zero();
          if (px[j] & bit) ys[j] = Ext{a.sm[(size_t)xv[j] * B + col], a.se[(size_t)xv[j] * B + col]};
        }
#pragma unroll
        for (int j = 0; j < Q4; ++j)
          if (px[j] & bit) { x = ext_add(x, ys[j]); C.dag += 1; }
      } else {
        uint64_t ys[Q4];
#pragma unroll
        for (int j = 0; j < Q4; ++j) ys[j] = (px[j] & bit) ? a.sig[(size_t)xv[j] * B + col] : 0ull;
#pragma unroll
        for (int j = 0; j < Q4; ++j) {
          if (px[j] & bit) {
            if (s + ys[j] < s) wrap = true;
            s += ys[j];
            C.dag += 1;
          }
        }
      }
    }
    if (td) {
#pragma unroll
      for (int j = 0; j < Q4; ++j) {
        if (xv[j] >= 0 && !((px[j] | cx[j]) & bit) && !(nxt[(size_t)xv[j] * K + k] & bit)) {
          const size_t xk = (size_t)xv[j] * K + k;
          const uint64_t old = atomicOr((unsigned long long*)&nxt[xk], (unsigned long long)bit);
          if (!(old & bit)) C.newl += 1;
          if (old == 0ull) lane_append(a, st, kl + 1, ebn, ubn, bentry(xv[j], k));
        }
      }
    }
  }
  if (!count) return;
  const size_t idx = (size_t)w * B + col;
  if (EXT) {
    const Ext z = ext_norm(x);
    a.sm[idx] = z.m;
    a.se[idx] = z.e;
  } else {
    a.sig[idx] = s;
    if (wrap) atomicOr(&a.lane_ovf[col], 1u);
  }
  if (a.keep_lv) a.lv[idx] = kl;
  a.emask[un.e] = bit;
  const size_t wk = (size_t)w * K + k;
  const uint64_t EL = a.edge_lanes[k];
  if (a.alpha > 0.0) {
    const uint64_t ov = a.vis[wk];
    const uint64_t nv = ov | bit;
    a.vis[wk] = nv;
    if ((nv & EL) == EL && (ov & EL) != EL) C.full += (uint64_t)deg;
  } else {
    atomicOr((unsigned long long*)&a.vis[wk], (unsigned long long)bit);
  }
  C.reached += 1;
  C.rnnz += (uint64_t)deg;
}

// ----------------------------------------------------------- backward unit

template <bool EXT>
__device__ __forceinline__ void backward_unit(const BatchArgs& a, const BUnit& un, const uint64_t* cmv, uint64_t* own,
                                              int lb, int depth, const Stage& st) {
  constexpr int G = EXT ? 8 : 16;
  const int K = a.K;
  const size_t B = (size_t)64 * K;
  const int lane = lane_id();
  const int32_t* __restrict__ rp = a.rp;
  const int32_t* __restrict__ ci = a.ci;
  double* psi = EXT ? a.sm : (double*)a.sig;
  const int32_t w = un.v, k = un.k, c = un.c;
  const int32_t beg = un.beg, end = un.end;
  const size_t wk = (size_t)w * K + k;
  const size_t idx = (size_t)w * B + 64 * k + lane;
  // issued together: the first chunk's neighbours, the unit's lanes and
  // levels, and what the lanes' dependencies will need
  const int32_t vl0 = beg + lane < end ? ci[beg + lane] : 0;
  // the word's edge lanes on level lb at w (level 0: the lanes whose source is w)
  const uint64_t at = lb > 0 ? a.emask[un.e]
                             : ballot(a.lane_src[64 * k + lane] == w && a.lane_pa[64 * k + lane] < 0);
  const uint64_t om = lb > 0 ? at & ~st.sX[k] : 0ull;  // edge lanes accumulating here (none at a source)
  const double sw = EXT ? a.sm[idx] : (double)a.sig[idx];
  const double lw = a.lane_w[64 * k + lane];
  const int pr = a.lane_pair[64 * k + lane];
  // Dynamic merging of frontiers (fused 2-degree backward): a derived lane c
  // accumulates delta_c(w) here, at level lb = d_c(w) - 1, when its partner
  // lane a sits on w at this level and d_a(w) <= d_b(w) (a-pass), or b does
  // and d_b(w) < d_a(w) (b-pass).  Its successors v are those of that
  // partner (d_x(v) = lb + 1) with d_x(v) <= d_y(v) (the dla / dlb masks);
  // c's own vertex is never one (dla, dlb stay clear there).
  const uint64_t DL = a.derived_lanes[k] & ~st.sX[k];
  uint64_t dm = 0, dA = 0, PL = 0;
  int pa = 0, pb = 0;
  if (DL) {
    const uint64_t LAw = a.dla[wk], LBw = a.dlb[wk];
    pa = a.lane_pa[64 * k + lane];
    pb = a.lane_pb[64 * k + lane];
    bool ia = false, ib = false;
    if ((DL >> lane) & 1ull) {
      ia = ((at >> pa) & 1ull) && ((LAw >> lane) & 1ull);
      ib = ((at >> pb) & 1ull) && ((LBw >> lane) & 1ull) && !((LAw >> lane) & 1ull);
    }
    dm = ballot(ia || ib);
    dA = ballot(ia);
    PL = wave_or_u64((ia || ib) ? ((1ull << pa) | (1ull << pb)) : 0ull);
  }
  const uint64_t om2 = om | dm;
  const bool mine = (dm >> lane) & 1ull, apass = (dA >> lane) & 1ull;
  if (c == 0 && lane == 0 && lb > 0) own[wk] = om;
  double acc = 0.0;
  if (om2 && lb < depth) {
    const int32_t ew = (EXT && ((om2 >> lane) & 1ull)) ? a.se[idx] : 0;
    for (int32_t off0 = beg; off0 < end; off0 += kWave) {
      const int32_t off = off0 + lane;
      int32_t vl = 0;
      uint64_t ml = 0, cm = 0, lav = 0, lbv = 0;
      bool dc = false;
      if (off < end) {
        vl = off0 == beg ? vl0 : ci[off];
        cm = cmv[(size_t)vl * K + k];
        ml = cm & om;
        if (dm && (cm & PL)) {
          lav = a.dla[(size_t)vl * K + k];
          lbv = a.dlb[(size_t)vl * K + k];
          dc = ((lav | lbv) & dm) != 0;
        }
      }
      uint64_t act = ballot(ml != 0 || dc);
      while (act) {
        int ti[G];
#pragma unroll
        for (int i = 0; i < G; ++i) {
          ti[i] = act ? __builtin_ctzll(act) : -1;
          act &= act ? act - 1 : 0ull;
        }
        double ys[G];
#pragma unroll
        for (int i = 0; i < G; ++i) {
          ys[i] = 0.0;
          if (ti[i] >= 0) {
            const int32_t v = rl32(vl, ti[i]);
            const uint64_t mv = rl64(ml, ti[i]);
            const size_t row = (size_t)v * B + 64 * k;  // uniform base, lane offset
            bool take = (mv >> lane) & 1ull;
            if (dm) {
              const uint64_t cv = rl64(cm, ti[i]), av = rl64(lav, ti[i]), bv = rl64(lbv, ti[i]);
              if (mine)
                take = apass ? (((cv >> pa) & 1ull) && ((av >> lane) & 1ull))
                             : (((cv >> pb) & 1ull) && ((bv >> lane) & 1ull));
            }
            if (take) {
              ys[i] = (psi + row)[lane];
              if (EXT) ys[i] = ldexp(ys[i], ew - (a.se + row)[lane]);
            }
          }
        }
#pragma unroll
        for (int i = 0; i < G; ++i) acc += ys[i];
      }
    }
  }
  if (un.deg > CHB) {
    const int32_t nunits = units_of<CHB>(un.deg);
    part_store(&a.part_m[(size_t)(un.pb + c) * 64 + lane], acc);
    part_stores_done();
    int32_t prev = 0;
    if (lane == 0) prev = atomicAdd(&a.arrive[un.e], 1);
    prev = __shfl(prev, 0, kWave);
    // the forward counting phase took the first nunits arrivals (none at level 0)
    if (prev != (lb > 0 ? 2 : 1) * nunits - 1) return;
    part_loads_after();
    acc = 0.0;
    for (int32_t cc = 0; cc < nunits; ++cc) acc += part_load(&a.part_m[(size_t)(un.pb + cc) * 64 + lane]);
  }
  if (!om2) return;
  const double omw = a.omega ? (double)a.omega[w] : 0.0;
  double cs = 0.0;
  if ((om2 >> lane) & 1ull) {
    const double delta = sw * acc;
    psi[idx] = (1.0 + delta + omw) / sw;
    cs = lw * (delta + omw);
    if (a.delta_out) a.delta_out[(size_t)(64 * k + lane) * a.n + w] = delta;
  }
  // per (word, slot) sums in lane order
  uint64_t rem = om2;
  while (rem) {
    const int pv = __builtin_amdgcn_readlane(pr, __builtin_ctzll(rem));
    const uint64_t same = ballot(pr == pv) & rem;
    const double part = wave_sum(((same >> lane) & 1ull) ? cs : 0.0);
    // one unit per (pair, vertex) and level: the adds land in level order;
    // an atomic add needs no round trip before the wave moves on
    if (lane == 0) atomicAdd(&a.pair_bc[(size_t)pv * a.n + w], part);
    rem &= ~same;
  }
}

// The backward unit worked by one lane (entries of <= 32 edges with at most
// one lane on level lb).
template <bool EXT>
__device__ __forceinline__ void lane_backward_unit(const BatchArgs& a, const BUnit& un, uint64_t om,
                                                   const uint64_t* cmv, uint64_t* own, int lb, int depth) {
  const int K = a.K;
  const size_t B = (size_t)64 * K;
  const int32_t* __restrict__ ci = a.ci;
  double* psi = EXT ? a.sm : (double*)a.sig;
  const int32_t w = un.v, k = un.k;
  const size_t wk = (size_t)w * K + k;
  own[wk] = om;
  if (!om) return;
  const int l = __builtin_ctzll(om);
  const size_t col = 64 * (size_t)k + l;
  const size_t idx = (size_t)w * B + col;
  const int32_t ew = EXT ? a.se[idx] : 0;
  double acc = 0.0;
  if (lb < depth) {
    constexpr int Q4 = 4;
    for (int32_t e0 = un.beg; e0 < un.end; e0 += Q4) {
      int32_t xv[Q4];
      bool on[Q4];
      double ys[Q4];
#pragma unroll
      for (int j = 0; j < Q4; ++j) xv[j] = e0 + j < un.end ? ci[e0 + j] : -1;
#pragma unroll
      for (int j = 0; j < Q4; ++j) on[j] = xv[j] >= 0 && (cmv[(size_t)xv[j] * K + k] & om) != 0;
#pragma unroll
      for (int j = 0; j < Q4; ++j) {
        ys[j] = 0.0;
        if (on[j]) {
          ys[j] = psi[(size_t)xv[j] * B + col];
          if (EXT) ys[j] = ldexp(ys[j], ew - a.se[(size_t)xv[j] * B + col]);
        }
      }
#pragma unroll
      for (int j = 0; j < Q4; ++j)
        if (on[j]) acc += ys[j];
    }
  }
  const double omw = a.omega ? (double)a.omega[w] : 0.0;
  const double sw = EXT ? a.sm[idx] : (double)a.sig[idx];
  const double delta = sw * acc;
  psi[idx] = (1.0 + delta + omw) / sw;
  if (a.delta_out) a.delta_out[col * a.n + w] = delta;
  atomicAdd(&a.pair_bc[(size_t)a.lane_pair[col] * a.n + w], a.lane_w[col] * (delta + omw));
}

// ------------------------------------------------------------- kernel

template <bool EXT>
__global__ void __launch_bounds__(kBatchBlock) __attribute__((amdgpu_waves_per_eu(4))) batch_kernel(BatchArgs a) {
  __shared__ Stage st;
  const int K = a.K;
  const size_t B = (size_t)64 * K;
  const int lane = lane_id();
  const int wib = (int)(threadIdx.x >> 6);
  const int64_t gw = (int64_t)blockIdx.x * kWavesPB + wib;
  const int64_t nw = (int64_t)gridDim.x * kWavesPB;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  const int32_t n = a.n;
  const int32_t* __restrict__ rp = a.rp;
  const int32_t* __restrict__ ci = a.ci;
  const size_t fms = (size_t)n * K;
  auto F = [&](int level) { return a.fm + (size_t)(level % kSlots) * fms; };
  int kact = 0;  // words with lanes that propagate along edges
  for (int k = 0; k < K; ++k) kact += a.edge_lanes[k] != 0;
  Ctr C;
  if (threadIdx.x == 0) {
    st.n = 0;
    st.full = 0;
    st.newl = 0;
    st.ctr[0] = st.ctr[1] = st.ctr[2] = 0;
    st.fclaim[0] = st.fclaim[1] = st.bclaim[0] = st.bclaim[1] = 0;
  }
  __syncthreads();

  // ---- seed the sources at level 0 (masks are clear on entry)
  {
    bool claimed = false;
    uint64_t ent = 0;
    if (tid < (int64_t)B && a.lane_pa[tid] >= 0) {
      // a derived lane c (Lemma 1): its partners a and b sit at distance 1
      // from c, each reached first by its own partner lane at level 0
      const int j = (int)tid, w0 = j & ~63;
      const uint64_t bit = 1ull << (j & 63);
      const int32_t va = a.lane_src[w0 + a.lane_pa[j]], vb = a.lane_src[w0 + a.lane_pb[j]];
      if (EXT) {
        a.sm[(size_t)va * B + j] = 1.0; a.se[(size_t)va * B + j] = 0;
        a.sm[(size_t)vb * B + j] = 1.0; a.se[(size_t)vb * B + j] = 0;
      } else {
        a.sig[(size_t)va * B + j] = 1ull;
        a.sig[(size_t)vb * B + j] = 1ull;
      }
      atomicOr((unsigned long long*)&a.dla[(size_t)va * K + (j >> 6)], (unsigned long long)bit);
      atomicOr((unsigned long long*)&a.dlb[(size_t)vb * K + (j >> 6)], (unsigned long long)bit);
    } else if (tid < (int64_t)B) {
      const int32_t s = a.lane_src[tid];
      if (s >= 0) {
        const int j = (int)tid;
        const uint64_t bit = 1ull << (j & 63);
        if (a.keep_lv) a.lv[(size_t)s * B + j] = 0;
        if (EXT) { a.sm[(size_t)s * B + j] = 1.0; a.se[(size_t)s * B + j] = 0; }
        else a.sig[(size_t)s * B + j] = 1ull;
        atomicOr((unsigned long long*)&a.vis[(size_t)s * K + (j >> 6)], (unsigned long long)bit);
        claimed = atomicOr((unsigned long long*)&a.fm[(size_t)s * K + (j >> 6)], (unsigned long long)bit) == 0ull;
        C.newl += 1;
        ent = bentry(s, j >> 6);
        atomicAdd(&st.ctr[0], 1ull);
        atomicAdd(&st.ctr[1], (unsigned long long)(rp[s + 1] - rp[s]));
      }
    }
    stage_append(a, st, 0, 0, 0, claimed, ent);
    const uint64_t nl0 = wave_sum_u64(C.newl);
    if (lane == 0 && nl0) atomicAdd(&st.newl, (unsigned long long)nl0);
    C.newl = 0;
    stage_flush(a, st, 0, 0, 0);
  }
  if (tid == 0) { a.qoff[0] = 0; a.uoff[0] = 0; }
  if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;

  // ---- forward sweep: phase kl counts level kl and discovers level kl+1
  int kl = 0;
  int32_t ebase = 0, ubase = 0;   // level kl's list
  int32_t eprev = 0, eprev2 = 0;  // starts of levels kl-1 and kl-2
  int levels = 0, bu_levels = 0;
  bool failed = false, was_bu = false;
  while (true) {
    if (ldr32(&a.lc[kl].err) != 0) { failed = true; break; }
    const uint64_t pk = ldr64(&a.lc[kl].packed);
    const int32_t ne = (int32_t)(pk >> 32), nu = (int32_t)(pk & 0xffffffffull);
    if (ne == 0) break;  // level kl is empty: the deepest level is kl - 1
    const int32_t ebn = ebase + ne, ubn = ubase + nu;
    const int32_t nl = kl + 1;
    const uint64_t* par = F(kl + kSlots - 1);  // level kl-1
    const uint64_t* cur = F(kl);
    uint64_t* nxt = F(nl);
    uint64_t* clr = F(kl + 2);                 // level kl-2
    // direction: bottom-up once the frontier's edges outweigh alpha times
    // the edges still undiscovered (both counted once per word); with beta,
    // a bottom-up sweep stays bottom-up until the frontier holds fewer than
    // n / beta (vertex, word) entries
    const double fe = (double)ldr64(&a.lc[kl].fedges);
    const double unvisited = (double)a.nnz * kact - (double)ldr64(a.fulledges);
    bool bu = kl > 0 && a.alpha > 0.0 && fe * a.alpha > unvisited;
    if (was_bu && a.beta > 0.0) bu = (double)ne * a.beta >= (double)n * kact;
    was_bu = bu;
    if (threadIdx.x == 0) st.fclaim[nl & 1] = 0;  // phase kl+1's counter; kl-1 used it before the barrier
    if (tid == 0) {
      a.qoff[nl] = ebn;
      a.uoff[nl] = ubn;
      if (kl + 2 < a.cap_levels) a.lc[kl + 2] = LevelCtr{0ull, 0, 0, 0ull, 0, 0};
    }
    ++levels;
    // sparse levels (fewer than two lanes per entry): one unit per lane for
    // the entries with a single edge lane, a wave per unit for the others
    const bool sparse = ldr64(&a.lc[kl].lanes) < 2ull * (uint64_t)ne;
    if ((kl >= 1 || !bu) && sparse) {
      for (int64_t first = gw; first < nu; first += nw * kWave) {
        const int64_t i = first + nw * lane;  // the wave's units: first, first + nw, ...
        bool dense = false;
        if (i < nu) {
          const BUnit un = a.U[ubase + i];
          const uint64_t nbm = cur[(size_t)un.v * K + un.k];
          if (un.deg <= kLaneMaxDeg && __popcll(nbm) == 1 && (nbm & a.edge_lanes[un.k]) != 0 &&
              a.derived_lanes[un.k] == 0)
            lane_forward_unit<EXT>(a, st, un, nbm, par, cur, nxt, kl, kl >= 1, !bu, ebn, ubn, C);
          else
            dense = true;
        }
        uint64_t dm = ballot(dense);
        while (dm) {
          const int j = __builtin_ctzll(dm);
          dm &= dm - 1;
          forward_unit<EXT>(a, st, a.U[ubase + first + nw * j], par, cur, nxt, kl, kl >= 1, !bu, ebn, ubn, C);
        }
      }
    } else if (kl >= 1 || !bu) {
      for (int64_t i = wg_claim(&st.fclaim[kl & 1]); i < nu; i = wg_claim(&st.fclaim[kl & 1]))
        forward_unit<EXT>(a, st, a.U[ubase + i], par, cur, nxt, kl, kl >= 1, !bu, ebn, ubn, C);
    }
    if (bu) {
      ++bu_levels;
      const int64_t ni = (int64_t)a.ngu * K;
      for (int64_t i = gw; i < ni; i += nw) {
        const int32_t q = (int32_t)(i / K);
        const int k = (int)(i - (int64_t)q * K);
        const int2 gu = a.gu[q];
        const int32_t w = gu.x;
        const size_t wk = (size_t)w * K + k;
        const uint64_t EL = a.edge_lanes[k];
        const uint64_t vk = a.vis[wk] | cur[wk];
        if ((vk & EL) == EL) continue;  // every edge lane of the word already reached w (uniform)
        const int32_t re = rp[w + 1];
        const int32_t beg = rp[w] + gu.y * CHB;
        const int32_t end = min(re, beg + CHB);
        // pull the neighbours' level-kl masks; stop once every edge lane of
        // the word not yet at w has been found on a neighbour
        const uint64_t want = EL & ~vk;
        uint64_t orr = 0;
        for (int32_t base = beg; base < end; base += kWave) {
          const int32_t off = base + lane;
          if (off < end) orr |= cur[(size_t)ci[off] * K + k];
          if (base + kWave < end && (wave_or_u64(orr) & want) == want) break;
        }
        const uint64_t nb = wave_or_u64(orr) & want;
        bool claimed = false;
        if (nb && lane == 0) {
          const uint64_t old = atomicOr((unsigned long long*)&nxt[wk], (unsigned long long)nb);
          claimed = old == 0ull;
          C.newl += (uint64_t)__popcll(nb & ~old);
        }
        stage_append(a, st, nl, ebn, ubn, claimed, bentry(w, k));
      }
    }
    // level kl-2 masks are no longer read: clear them for reuse as level kl+2
    if (kl >= 2) {
      for (int64_t i = tid; i < (int64_t)(eprev - eprev2); i += nth) {
        const uint64_t ent = a.Q[eprev2 + i];
        clr[(size_t)(uint32_t)ent * K + (ent >> 32)] = 0;
      }
    }
    {
      const uint64_t fs = wave_sum_u64(C.full), ls = wave_sum_u64(C.newl);
      if (lane == 0 && fs) atomicAdd(&st.full, (unsigned long long)fs);
      if (lane == 0 && ls) atomicAdd(&st.newl, (unsigned long long)ls);
      C.full = 0;
      C.newl = 0;
    }
    stage_flush(a, st, nl, ebn, ubn);
    if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;
    eprev2 = eprev;
    eprev = ebase;
    ebase = ebn;
    ubase = ubn;
    kl = nl;
  }
  const int depth = kl - 1;

  // ---- forward counters (workgroup first) and component sizes
  {
    const uint64_t reached = wave_sum_u64(C.reached), rnnz = wave_sum_u64(C.rnnz), dag = wave_sum_u64(C.dag);
    if (lane == 0) {
      if (reached) atomicAdd(&st.ctr[0], (unsigned long long)reached);
      if (rnnz) atomicAdd(&st.ctr[1], (unsigned long long)rnnz);
      if (dag) atomicAdd(&st.ctr[2], (unsigned long long)dag);
    }
  }
  if (a.has_own && !failed) {
    // n_s of each lane: 1 + omega summed over the vertices the lane reached.
    // The workgroup's vertex range is cut into 64-vertex chunks shared by its
    // waves; each lane loads one vertex's mask, then every lane adds the
    // weights of the chunk's vertices whose mask has its bit.  Totals meet in
    // LDS (the append stage is free here), one global add per lane.
    unsigned long long* acc_l = (unsigned long long*)st.e;
    for (int j = (int)threadIdx.x; j < (int)B; j += (int)blockDim.x) acc_l[j] = 0;
    __syncthreads();
    const int64_t per = ((int64_t)n + gridDim.x - 1) / gridDim.x;
    const int64_t v0 = (int64_t)blockIdx.x * per;
    const int64_t v1 = min((int64_t)n, v0 + per);
    for (int k = 0; k < K; ++k) {
      unsigned long long acc = 0;
      for (int64_t c = v0 + 64 * wib; c < v1; c += 64 * kWavesPB) {
        const int64_t v = c + lane;
        uint64_t m = 0;
        int32_t wt = 0;
        if (v < v1) {
          m = a.vis[(size_t)v * K + k];
          wt = 1 + (a.omega ? a.omega[v] : 0);
        }
        uint64_t nz = ballot(m != 0);
        while (nz) {
          const int i = __builtin_ctzll(nz);
          nz &= nz - 1;
          const uint64_t mv = rl64(m, i);
          const int32_t wv = rl32(wt, i);
          if ((mv >> lane) & 1ull) acc += (unsigned long long)wv;
        }
      }
      if (acc) atomicAdd(&acc_l[64 * k + lane], acc);
    }
    __syncthreads();
    for (int j = (int)threadIdx.x; j < (int)B; j += (int)blockDim.x)
      if (acc_l[j]) atomicAdd(&a.lane_ns[j], acc_l[j]);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    if (st.ctr[0]) atomicAdd(&a.stats[kStReached], st.ctr[0]);
    if (st.ctr[1]) atomicAdd(&a.stats[kStReachedNnz], st.ctr[1]);
    if (st.ctr[2]) atomicAdd(&a.stats[kStDag], st.ctr[2]);
  }
  if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;

  // lanes whose count wrapped (and lanes derived from them) take no part in
  // the backward sweep; the host reruns them in extended form
  for (int k = wib; k < K; k += kWavesPB) {
    uint64_t X = ballot(__hip_atomic_load(&a.lane_ovf[64 * k + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0);
    const int pa = a.lane_pa[64 * k + lane], pb = a.lane_pb[64 * k + lane];
    X |= ballot(pa >= 0 && ((((X >> pa) | (X >> pb)) & 1ull) != 0));
    if (lane == 0) st.sX[k] = X;
  }
  __syncthreads();

  if (!failed && (a.sig_out || a.sm_out)) {
    // trace: keep the counts before psi overwrites them
    for (int64_t i = tid; i < (int64_t)n * (int64_t)B; i += nth) {
      const int32_t v = (int32_t)(i / (int64_t)B), j = (int32_t)(i % (int64_t)B);
      const size_t vk = (size_t)v * K + (j >> 6);
      bool r = (a.vis[vk] >> (j & 63)) & 1ull;
      if (a.has_derived && ((a.derived_lanes[j >> 6] >> (j & 63)) & 1ull))  // reached through a partner
        r = ((a.dla[vk] | a.dlb[vk]) >> (j & 63)) & 1ull;
      if (EXT) { a.sm_out[(size_t)j * n + v] = r ? a.sm[i] : 0.0; a.se_out[(size_t)j * n + v] = r ? a.se[i] : 0; }
      else a.sig_out[(size_t)j * n + v] = r ? a.sig[i] : 0ull;
    }
    if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;
  }

  // ---- backward sweep
  if (!failed) {
    // level 0 only for derived lanes: their dependency at the partners'
    // vertices (d_c = 1) is accumulated at the partners' sources
    for (int lb = depth; lb >= (a.has_derived ? 0 : 1); --lb) {
      const uint64_t* cmv = F(lb + 1);
      uint64_t* own = F(lb);
      uint64_t* clr = F(lb + 2);
      const int32_t ub = a.uoff[lb], ue = a.uoff[lb + 1];
      const int64_t nub = ue - ub;
      if (threadIdx.x == 0) st.bclaim[(lb - 1) & 1] = 0;  // the next level's counter
      if (lb == 0) {
        for (int64_t i = wg_claim(&st.bclaim[0]); i < nub; i = wg_claim(&st.bclaim[0])) {
          const BUnit un = a.U[ub + i];
          if (a.derived_lanes[un.k] != 0) backward_unit<EXT>(a, un, cmv, own, 0, depth, st);
        }
      } else if (ldr64(&a.lc[lb].lanes) < 2ull * (uint64_t)(a.qoff[lb + 1] - a.qoff[lb])) {
        // sparse level: one unit per lane where the word has at most one lane here
        for (int64_t first = gw; first < nub; first += nw * kWave) {
          const int64_t i = first + nw * lane;
          bool dense = false;
          if (i < nub) {
            const BUnit un = a.U[ub + i];
            const uint64_t om = a.emask[un.e] & ~st.sX[un.k];
            if (un.deg <= kLaneMaxDeg && __popcll(om) <= 1 && a.derived_lanes[un.k] == 0)
              lane_backward_unit<EXT>(a, un, om, cmv, own, lb, depth);
            else
              dense = true;
          }
          uint64_t dm = ballot(dense);
          while (dm) {
            const int j = __builtin_ctzll(dm);
            dm &= dm - 1;
            backward_unit<EXT>(a, a.U[ub + first + nw * j], cmv, own, lb, depth, st);
          }
        }
      } else {
        for (int64_t i = wg_claim(&st.bclaim[lb & 1]); i < nub; i = wg_claim(&st.bclaim[lb & 1]))
          backward_unit<EXT>(a, a.U[ub + i], cmv, own, lb, depth, st);
      }
      // level lb+2 masks are no longer read
      if (lb + 2 <= depth) {
        const int32_t e0 = a.qoff[lb + 2], e1 = a.qoff[lb + 3];
        for (int64_t i = tid; i < (int64_t)(e1 - e0); i += nth) {
          const uint64_t ent = a.Q[e0 + i];
          clr[(size_t)(uint32_t)ent * K + (ent >> 32)] = 0;
        }
      }
      if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;
    }
  }

  // ---- epilogue: own terms of the 1-degree reduction, overflow and failure lists
  if (tid == 0) {
    for (int j = 0; j < (int)B; ++j) {
      const int32_t s = a.lane_src[j];
      if (s < 0) continue;
      if (failed) {
        const int32_t q = atomicAdd(a.fail_count, 1);
        a.fail_list[q] = s;
      } else if ((st.sX[j >> 6] >> (j & 63)) & 1ull) {
        const int32_t q = atomicAdd(a.ovf_count, 1);
        a.ovf_list[q] = s;
      } else if (a.has_own && a.lane_own[j] != 0) {
        // each folded source reaches its component through s, except s and
        // its own subtree (Eq. (4) for pendants: own * (n_s - 2))
        // (a derived lane's component is its partners')
        const int jn = a.lane_pa[j] >= 0 ? (j & ~63) + a.lane_pa[j] : j;
        a.pair_bc[(size_t)a.lane_pair[j] * n + s] +=
            (double)a.lane_own[j] * ((double)a.lane_ns[jn] - 1.0) - a.lane_tsub[j];
      }
    }
    atomicAdd(&a.stats[kStLevels], (unsigned long long)levels);
    atomicAdd(&a.stats[kStBuLevels], (unsigned long long)bu_levels);
    atomicAdd(&a.stats[kStLaunches], 1ull);
  }
  if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;  // everything above has read the lane arrays, the level counters and the sums
  // fold the per-(word, slot) sums into the slots' scores, in word order
  for (int64_t v = tid; v < n; v += nth) {
    for (int p = 0; p < a.npairs; ++p) {
      double* src = a.pair_bc + (size_t)p * n + v;
      const double t = *src;
      if (t != 0.0) {
        a.slot_bc[a.pair_slot[p]][v] += t;
        *src = 0.0;
      }
    }
  }
  // leave the control state and (unless a trace wants them) the masks clear for the next launch
  if (tid == 0) {
    for (int i = 0; i < 3 && i < a.cap_levels; ++i) a.lc[i] = LevelCtr{0ull, 0, 0, 0ull, 0, 0};
    *a.fulledges = 0;
  }
  for (int64_t j = tid; j < (int64_t)B; j += nth) { a.lane_ns[j] = 0; a.lane_ovf[j] = 0; }
  if (a.clear_at_end) {
    for (int64_t i = tid; i < (int64_t)fms; i += nth) {
      a.vis[i] = 0;
#pragma unroll
      for (int s = 0; s < kSlots; ++s) a.fm[(size_t)s * fms + i] = 0;
      if (a.has_derived) { a.dla[i] = 0; a.dlb[i] = 0; }
    }
  }
}

hipError_t launch_batch(const BatchArgs& a, bool ext, int grid, int block, hipStream_t st) {
  if (a.K < 1 || a.K > kMaxWords || block != kBatchBlock || a.npairs < 0 || a.npairs > a.cap_pairs)
    return hipErrorInvalidValue;
  void* args[] = {(void*)&a};
  const void* fn = ext ? (const void*)batch_kernel<true> : (const void*)batch_kernel<false>;
  return hipLaunchKernel(fn, dim3(grid), dim3(block), args, 0, st);
}

hipError_t batch_max_grid(bool ext, int block, int* blocks_per_cu) {
  const void* fn = ext ? (const void*)batch_kernel<true> : (const void*)batch_kernel<false>;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, block, 0);
}

}  // namespace bcx
