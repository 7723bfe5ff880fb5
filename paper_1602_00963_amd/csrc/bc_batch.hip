// Many sources per launch.  A batch of B = 64 K sources advances level by
// level together inside one cooperative persistent kernel.  Lane j of a
// 64-lane word k is source 64 k + j; per-(vertex, source) state is stored
// source-minor ([vertex][lane]) so a wave touching one vertex reads or
// writes one contiguous row per word.  Per vertex, 64-bit lane masks record
// which sources have reached it (vis) and which sit on a given level (F_l,
// four rotating arrays).
//
// Forward sweep (shortest-path counting, Alg. 2-3 generalised to B sources).
// Phase k, one grid barrier each, does two independent jobs:
//   counting of level k -- one wave per unit (<= 256 edges) of the level-k
//     entries, lanes = sources: sigma(w) = sum of sigma(v) over neighbours v
//     whose level-(k-1) mask has the lane's bit.  2-degree derived lanes
//     (Lemma 1) take Eq. (6) instead: the sum of the two partner lanes'
//     counts at w over the partners sitting on level k-1 at w.
//   discovery of level k+1 -- top-down: one wave per unit of the level-k
//     entries, lanes = edges; each edge ORs mask_k(v) & ~reached(w) into
//     F_{k+1}(w); bottom-up: one wave per static unit of every vertex some
//     source has not reached, OR-ing its neighbours' level-k masks.  A
//     vertex entering level k+1 is appended once (per-level stamp).  Derived
//     lanes are not propagated along edges: lane c reaches v at level k+1
//     exactly when a partner sits on v at level k and c has not reached v.
//   "reached(w)" is vis(w) | F_k(w): vis is being updated with F_k by the
//   counting job of the same phase, and either value gives the same result.
// Backward sweep (dependency accumulation, Alg. 4-5, successor checking):
//   one wave per unit of the level-l entries; per lane, sum psi over the
//   neighbours whose level-(l+1) mask has the lane's bit, then
//   delta = sigma * sum and psi = (1 + delta + omega) / sigma overwrite the
//   count in place.  The vertex's score gains sum over its lanes of
//   weight * (delta + omega), summed in lane order into each lane's result
//   slot.
// Entries spanning several units combine per-unit partial sums in unit
// order (the last arrival does it), so results do not depend on scheduling.
#include "bc_common.h"
#include "bc_kernels.h"

namespace bcx {

constexpr int CHB = kBatchChunk;
constexpr int kGather = 8;  // neighbour rows loaded before any is consumed
constexpr int kSlots = 4;   // rotating level-mask arrays

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

// Stamp-protected append: a vertex joins level `lvl`'s list once.
template <int CH>
__device__ __forceinline__ void claim_and_append(const BatchArgs& a, const Lists& L, int lvl, int32_t ebase,
                                                 int32_t ubase, bool want, int32_t w) {
  bool claimed = false;
  if (want && ldr32(&a.stamp[w]) != lvl) claimed = atomicExch(&a.stamp[w], lvl) != lvl;
  append_entries<CH>(L, lvl, ebase, ubase, claimed, w);
}

// Per-wave run counters.
template <int K>
struct Counters {
  uint64_t reached = 0, rnnz = 0, dag = 0, full = 0;
  uint64_t ns[K];
};

// ------------------------------------------------------------ counting

// Counts of the new lanes of one level-k unit.  `par` = level-(k-1) masks,
// `now` = level-k masks.
template <bool EXT, int K>
__device__ __forceinline__ void count_unit(const BatchArgs& a, const Unit& un, const uint64_t* par,
                                           const uint64_t* now, int k_level, const uint64_t (&EL)[K],
                                           Counters<K>& C) {
  constexpr int B = 64 * K;
  const int lane = lane_id();
  const int32_t* __restrict__ rp = a.rp;
  const int32_t* __restrict__ ci = a.ci;
  const int32_t w = un.v;
  const int32_t rb = rp[w], re = rp[w + 1];
  const int32_t beg = rb + un.c * CHB;
  const int32_t end = min(re, beg + CHB);
  uint64_t nbm[K], em[K];
  bool anye = false;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    nbm[k] = now[(size_t)w * K + k];
    em[k] = nbm[k] & EL[k];
    anye |= em[k] != 0;
  }
  uint64_t s[K];
  Ext x[K];
  bool wrap[K];
#pragma unroll
  for (int k = 0; k < K; ++k) { s[k] = 0; x[k] = ext_zero(); wrap[k] = false; }
  if (anye) {
    for (int32_t off0 = beg; off0 < end; off0 += kWave) {
      const int32_t off = off0 + lane;
      int32_t vl = 0;
      uint64_t ml[K];
      if (off < end) {
        vl = ci[off];
#pragma unroll
        for (int k = 0; k < K; ++k) ml[k] = par[(size_t)vl * K + k] & em[k];
      } else {
#pragma unroll
        for (int k = 0; k < K; ++k) ml[k] = 0;
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        C.dag += (uint64_t)__popcll(ml[k]);
        // only the neighbours with a wanted lane; 8 rows in flight per word
        uint64_t act = ballot(ml[k] != 0);
        while (act) {
          int ti[kGather];
#pragma unroll
          for (int i = 0; i < kGather; ++i) {
            ti[i] = act ? __builtin_ctzll(act) : -1;
            act &= act ? act - 1 : 0ull;
          }
          if (EXT) {
            Ext xs[kGather];
#pragma unroll
            for (int i = 0; i < kGather; ++i) {
              xs[i] = ext_zero();
              if (ti[i] >= 0) {
                const int32_t v = rl32(vl, ti[i]);
                const uint64_t mv = rl64(ml[k], ti[i]);
                const size_t row = (size_t)v * B + 64 * k;  // uniform: scalar base + lane offset
                if ((mv >> lane) & 1ull) xs[i] = Ext{(a.sm + row)[lane], (a.se + row)[lane]};
              }
            }
#pragma unroll
            for (int i = 0; i < kGather; ++i) x[k] = ext_add(x[k], xs[i]);
          } else {
            uint64_t ys[kGather];
#pragma unroll
            for (int i = 0; i < kGather; ++i) {
              ys[i] = 0;
              if (ti[i] >= 0) {
                const int32_t v = rl32(vl, ti[i]);
                const uint64_t mv = rl64(ml[k], ti[i]);
                const uint64_t* row = a.sig + (size_t)v * B + 64 * k;  // uniform base, lane offset
                if ((mv >> lane) & 1ull) ys[i] = row[lane];
              }
            }
#pragma unroll
            for (int i = 0; i < kGather; ++i) {
              if (s[k] + ys[i] < s[k]) wrap[k] = true;
              s[k] += ys[i];
            }
          }
        }
      }
    }
  }
  // combine the units of a split entry in unit order
  if (un.mi >= 0) {
    const int32_t nunits = units_of<CHB>(re - rb);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const size_t pi = ((size_t)(un.pb + un.c) * K + k) * 64 + lane;
      if (EXT) { a.part_m[pi] = x[k].m; a.part_e[pi] = x[k].e; }
      else { a.part_m[pi] = __longlong_as_double((long long)s[k]); a.part_e[pi] = wrap[k] ? 1 : 0; }
    }
    fence_release();
    int32_t prev = 0;
    if (lane == 0) prev = atomicAdd(&a.arrive[un.mi], 1);
    prev = __shfl(prev, 0, kWave);
    if (prev != nunits - 1) return;
    fence_acquire();
#pragma unroll
    for (int k = 0; k < K; ++k) { s[k] = 0; x[k] = ext_zero(); wrap[k] = false; }
    for (int32_t c = 0; c < nunits; ++c) {
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const size_t pi = ((size_t)(un.pb + c) * K + k) * 64 + lane;
        const double pm = __hip_atomic_load(&a.part_m[pi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int32_t pe = __hip_atomic_load(&a.part_e[pi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (EXT) {
          x[k] = ext_add(x[k], Ext{pm, pe});
        } else {
          const uint64_t y = (uint64_t)__double_as_longlong(pm);
          if (s[k] + y < s[k] || pe) wrap[k] = true;
          s[k] += y;
        }
      }
    }
  }
  // finalise: counts, levels, visited masks; derived lanes by Eq. (6)
  const uint64_t* parw = par + (size_t)w * K;
  bool fullnow = true;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const size_t idx = (size_t)w * B + 64 * k + lane;
    if ((nbm[k] >> lane) & 1ull) {
      if (!((em[k] >> lane) & 1ull)) {
        const int pa = a.lane_pa[64 * k + lane], pb = a.lane_pb[64 * k + lane];
        const uint64_t cw = parw[k];
        const size_t ia = (size_t)w * B + 64 * k + pa, ib = (size_t)w * B + 64 * k + pb;
        if (EXT) {
          Ext t = ext_zero();
          if ((cw >> pa) & 1ull) t = ext_add(t, Ext{a.sm[ia], a.se[ia]});
          if ((cw >> pb) & 1ull) t = ext_add(t, Ext{a.sm[ib], a.se[ib]});
          x[k] = t;
        } else {
          uint64_t t = 0;
          if ((cw >> pa) & 1ull) t += a.sig[ia];
          if ((cw >> pb) & 1ull) {
            const uint64_t y = a.sig[ib];
            if (t + y < t) wrap[k] = true;
            t += y;
          }
          s[k] = t;
        }
      }
      if (EXT) {
        const Ext z = ext_norm(x[k]);
        a.sm[idx] = z.m;
        a.se[idx] = z.e;
      } else {
        a.sig[idx] = s[k];
        if (wrap[k]) atomicOr(&a.lane_ovf[64 * k + lane], 1u);
      }
      a.lv[idx] = k_level;
      if (a.has_own) C.ns[k] += 1 + (a.omega ? (uint64_t)a.omega[w] : 0);
    }
    const uint64_t nv = a.vis[(size_t)w * K + k] | nbm[k];
    if (lane == 0) a.vis[(size_t)w * K + k] = nv;
    fullnow &= (nv & EL[k]) == EL[k];
    if (lane == 0) {
      const uint64_t pc = (uint64_t)__popcll(nbm[k]);
      C.reached += pc;
      C.rnnz += pc * (uint64_t)(re - rb);
    }
  }
  if (fullnow && lane == 0) C.full += (uint64_t)(re - rb);
}

// ----------------------------------------------------------- backward

template <bool EXT, int K>
__device__ __forceinline__ void backward_unit(const BatchArgs& a, const Unit& un, const uint64_t* cmv, uint64_t* own,
                                              int lb, int depth, const uint64_t (&X)[K]) {
  constexpr int B = 64 * K;
  const int lane = lane_id();
  const int32_t* __restrict__ rp = a.rp;
  const int32_t* __restrict__ ci = a.ci;
  double* psi = EXT ? a.sm : (double*)a.sig;
  const int32_t w = un.v;
  const int32_t rb = rp[w], re = rp[w + 1];
  uint64_t om[K];
  bool anyo = false;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const size_t idx = (size_t)w * B + 64 * k + lane;
    const bool r = (a.vis[(size_t)w * K + k] >> lane) & 1ull;
    om[k] = ballot(r && a.lv[idx] == lb) & ~X[k];
    anyo |= om[k] != 0;
    if (un.c == 0 && lane == 0) own[(size_t)w * K + k] = om[k];
  }
  double acc[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc[k] = 0.0;
  int32_t ew[K];
  if (EXT) {
#pragma unroll
    for (int k = 0; k < K; ++k) ew[k] = ((om[k] >> lane) & 1ull) ? a.se[(size_t)w * B + 64 * k + lane] : 0;
  }
  if (anyo && lb < depth) {
    const int32_t beg = rb + un.c * CHB;
    const int32_t end = min(re, beg + CHB);
    for (int32_t off0 = beg; off0 < end; off0 += kWave) {
      const int32_t off = off0 + lane;
      int32_t vl = 0;
      uint64_t ml[K];
      if (off < end) {
        vl = ci[off];
#pragma unroll
        for (int k = 0; k < K; ++k) ml[k] = cmv[(size_t)vl * K + k] & om[k];
      } else {
#pragma unroll
        for (int k = 0; k < K; ++k) ml[k] = 0;
      }
#pragma unroll
      for (int k = 0; k < K; ++k) {
        uint64_t act = ballot(ml[k] != 0);
        while (act) {
          int ti[kGather];
#pragma unroll
          for (int i = 0; i < kGather; ++i) {
            ti[i] = act ? __builtin_ctzll(act) : -1;
            act &= act ? act - 1 : 0ull;
          }
          double ys[kGather];
#pragma unroll
          for (int i = 0; i < kGather; ++i) {
            ys[i] = 0.0;
            if (ti[i] >= 0) {
              const int32_t v = rl32(vl, ti[i]);
              const uint64_t mv = rl64(ml[k], ti[i]);
              const size_t row = (size_t)v * B + 64 * k;  // uniform base, lane offset
              if ((mv >> lane) & 1ull) {
                ys[i] = (psi + row)[lane];
                if (EXT) ys[i] = ldexp(ys[i], ew[k] - (a.se + row)[lane]);
              }
            }
          }
#pragma unroll
          for (int i = 0; i < kGather; ++i) acc[k] += ys[i];
        }
      }
    }
  }
  if (un.mi >= 0) {
    const int32_t nunits = units_of<CHB>(re - rb);
#pragma unroll
    for (int k = 0; k < K; ++k) a.part_m[((size_t)(un.pb + un.c) * K + k) * 64 + lane] = acc[k];
    fence_release();
    int32_t prev = 0;
    if (lane == 0) prev = atomicAdd(&a.arrive[un.mi], 1);
    prev = __shfl(prev, 0, kWave);
    if (prev != 2 * nunits - 1) return;  // the forward counting phase took the first nunits arrivals
    fence_acquire();
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.0;
    for (int32_t c = 0; c < nunits; ++c) {
#pragma unroll
      for (int k = 0; k < K; ++k)
        acc[k] += __hip_atomic_load(&a.part_m[((size_t)(un.pb + c) * K + k) * 64 + lane], __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  if (!anyo) return;
  const double omw = a.omega ? (double)a.omega[w] : 0.0;
  // contributions go to each lane's result slot; lanes of one slot are
  // summed in lane order, words in order, slots in order of first lane
  double cs[K];
  int sl[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    cs[k] = 0.0;
    sl[k] = a.lane_slot[64 * k + lane];
    if ((om[k] >> lane) & 1ull) {
      const size_t idx = (size_t)w * B + 64 * k + lane;
      const double sw = EXT ? a.sm[idx] : (double)a.sig[idx];
      const double delta = sw * acc[k];
      psi[idx] = (1.0 + delta + omw) / sw;
      cs[k] = a.lane_w[64 * k + lane] * (delta + omw);
      if (a.delta_out) a.delta_out[(size_t)(64 * k + lane) * a.n + w] = delta;
    }
  }
  int slot = -1;
  double tot = 0.0;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    uint64_t rem = om[k];
    while (rem) {
      const int first = __builtin_ctzll(rem);
      const int sv = __builtin_amdgcn_readlane(sl[k], first);
      const uint64_t same = ballot(sl[k] == sv) & rem;
      const double part = wave_sum(((same >> lane) & 1ull) ? cs[k] : 0.0);
      if (sv != slot) {
        if (slot >= 0 && lane == 0) a.slot_bc[slot][w] += tot;
        slot = sv;
        tot = 0.0;
      }
      tot += part;
      rem &= ~same;
    }
  }
  if (slot >= 0 && lane == 0) a.slot_bc[slot][w] += tot;
}

// ------------------------------------------------------------- kernel

template <bool EXT, int K>
__global__ void __launch_bounds__(256) batch_kernel(BatchArgs a) {
  constexpr int B = 64 * K;
  const int lane = lane_id();
  const int wpb = blockDim.x / kWave;
  const int gw = blockIdx.x * wpb + (int)(threadIdx.x / kWave);
  const int nw = gridDim.x * wpb;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  const int32_t n = a.n;
  const int32_t* __restrict__ rp = a.rp;
  const int32_t* __restrict__ ci = a.ci;
  const Lists L{a.Q, a.U, a.lc, a.arrive, a.gmulti, a.err, a.rp,
                a.cap_entries, a.cap_units, a.cap_parts, a.cap_multi};
  uint64_t EL[K];
#pragma unroll
  for (int k = 0; k < K; ++k) EL[k] = a.edge_lanes[k];
  const size_t fms = (size_t)n * K;
  auto F = [&](int level) { return a.fm + (size_t)(level % kSlots) * fms; };
  Counters<K> C;
#pragma unroll
  for (int k = 0; k < K; ++k) C.ns[k] = 0;

  // ---- seed the sources at level 0 (masks and stamps are clear on entry)
  for (int64_t j = tid; j < B; j += nth) {
    const int32_t s = a.lane_src[j];
    if (s >= 0) {
      const uint64_t bit = 1ull << (j & 63);
      a.lv[(size_t)s * B + j] = 0;
      if (EXT) { a.sm[(size_t)s * B + j] = 1.0; a.se[(size_t)s * B + j] = 0; }
      else a.sig[(size_t)s * B + j] = 1ull;
      atomicOr((unsigned long long*)&a.vis[(size_t)s * K + (j >> 6)], (unsigned long long)bit);
      atomicOr((unsigned long long*)&a.fm[(size_t)s * K + (j >> 6)], (unsigned long long)bit);
      a.lane_ns[j] = 1 + (a.omega ? (uint64_t)a.omega[s] : 0);
      C.reached += 1;
      C.rnnz += (uint64_t)(rp[s + 1] - rp[s]);
    }
  }
  if (gw == 0) {
    for (int32_t base = 0; base < a.nl0; base += kWave) {
      const bool want = base + lane < a.nl0;
      const int32_t s = want ? a.l0[base + lane] : 0;
      if (want) a.stamp[s] = 0;
      append_entries<CHB>(L, 0, 0, 0, want, s);
    }
  }
  if (tid == 0) { a.qoff[0] = 0; a.uoff[0] = 0; }
  grid_barrier(a.bar);

  // ---- forward sweep: phase kl counts level kl and discovers level kl+1
  int kl = 0;
  int32_t ebase = 0, ubase = 0;   // level kl's list
  int32_t eprev = 0, eprev2 = 0;  // starts of levels kl-1 and kl-2
  int levels = 0, bu_levels = 0;
  bool failed = false;
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
    const uint64_t fe = ldr64(&a.lc[kl].fedges);
    const uint64_t full = ldr64(a.fulledges);
    const double unvisited = (double)a.nnz - (double)full;
    const bool bu = kl > 0 && a.alpha > 0.0 && (double)fe * a.alpha > unvisited;
    if (tid == 0) {
      a.qoff[nl] = ebn;
      a.uoff[nl] = ubn;
      if (kl + 2 < a.cap_levels) a.lc[kl + 2] = LevelCtr{0ull, 0, 0, 0ull, 0, 0};
    }
    ++levels;
    // counting of level kl
    if (kl >= 1) {
      for (int32_t u = ubase + gw; u < ubn; u += nw) count_unit<EXT, K>(a, a.U[u], par, cur, kl, EL, C);
    }
    // discovery of level kl+1
    if (!bu) {
      for (int32_t u = ubase + gw; u < ubn; u += nw) {
        const Unit un = a.U[u];
        const int32_t v = un.v;
        uint64_t cm[K];
        bool any = false;
#pragma unroll
        for (int k = 0; k < K; ++k) { cm[k] = cur[(size_t)v * K + k] & EL[k]; any |= cm[k] != 0; }
        if (!any) continue;  // only derived lanes on v (uniform)
        const int32_t beg = rp[v] + un.c * CHB;
        const int32_t end = min(rp[v + 1], beg + CHB);
        for (int32_t off0 = beg; off0 < end; off0 += kWave) {
          const int32_t off = off0 + lane;
          bool want = false;
          int32_t w = 0;
          if (off < end) {
            w = ci[off];
#pragma unroll
            for (int k = 0; k < K; ++k) {
              const uint64_t reached = a.vis[(size_t)w * K + k] | cur[(size_t)w * K + k];
              const uint64_t nb = cm[k] & ~reached;
              if (nb) {
                atomicOr((unsigned long long*)&nxt[(size_t)w * K + k], (unsigned long long)nb);
                want = true;
              }
            }
          }
          claim_and_append<CHB>(a, L, nl, ebn, ubn, want, w);
        }
      }
    } else {
      ++bu_levels;
      for (int32_t g = gw; g < a.ngu; g += nw) {
        const int2 gu = a.gu[g];
        const int32_t w = gu.x;
        uint64_t vk[K];
        bool done = true;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          vk[k] = a.vis[(size_t)w * K + k] | cur[(size_t)w * K + k];
          done &= (vk[k] & EL[k]) == EL[k];
        }
        if (done) continue;  // every edge lane already reached w (uniform)
        const int32_t re = rp[w + 1];
        const int32_t beg = rp[w] + gu.y * CHB;
        const int32_t end = min(re, beg + CHB);
        uint64_t orr[K];
#pragma unroll
        for (int k = 0; k < K; ++k) orr[k] = 0;
        for (int32_t off = beg + lane; off < end; off += kWave) {
          const int32_t v = ci[off];
#pragma unroll
          for (int k = 0; k < K; ++k) orr[k] |= cur[(size_t)v * K + k];
        }
        bool want = false;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const uint64_t nb = wave_or_u64(orr[k]) & EL[k] & ~vk[k];
          if (nb) {
            if (lane == 0) atomicOr((unsigned long long*)&nxt[(size_t)w * K + k], (unsigned long long)nb);
            want = true;
          }
        }
        claim_and_append<CHB>(a, L, nl, ebn, ubn, want && lane == 0, w);
      }
    }
    if (a.has_derived) {
      // 2-degree derived lanes: elementwise over the level-kl entries (Lemma 1)
      for (int32_t e = ebase + gw; e < ebn; e += nw) {
        const int32_t v = a.Q[e];
        bool want = false;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const uint64_t ck = cur[(size_t)v * K + k];
          const uint64_t reached = a.vis[(size_t)v * K + k] | ck;
          const int pa = a.lane_pa[64 * k + lane], pb = a.lane_pb[64 * k + lane];
          bool mine = false;
          if (pa >= 0) mine = ((((ck >> pa) | (ck >> pb)) & 1ull) != 0) && (((reached >> lane) & 1ull) == 0);
          const uint64_t nb = ballot(mine);
          if (nb) {
            if (lane == 0) atomicOr((unsigned long long*)&nxt[(size_t)v * K + k], (unsigned long long)nb);
            want = true;
          }
        }
        claim_and_append<CHB>(a, L, nl, ebn, ubn, want && lane == 0, v);
      }
    }
    // level kl-2 masks are no longer read: clear them for reuse as level kl+2
    if (kl >= 2) {
      for (int64_t i = tid; i < (int64_t)(eprev - eprev2) * K; i += nth) {
        const int32_t v = a.Q[eprev2 + (int32_t)(i / K)];
        clr[(size_t)v * K + (i % K)] = 0;
      }
    }
    const uint64_t fsum = wave_sum_u64(C.full);
    if (lane == 0 && fsum) atomicAdd(a.fulledges, (unsigned long long)fsum);
    C.full = 0;
    grid_barrier(a.bar);
    eprev2 = eprev;
    eprev = ebase;
    ebase = ebn;
    ubase = ubn;
    kl = nl;
  }
  const int depth = kl - 1;

  // publish forward counters and component sizes
  {
    const uint64_t r0 = wave_sum_u64(C.reached), r1 = wave_sum_u64(C.rnnz), r2 = wave_sum_u64(C.dag);
    if (lane == 0) {
      if (r0) atomicAdd(&a.stats[kStReached], (unsigned long long)r0);
      if (r1) atomicAdd(&a.stats[kStReachedNnz], (unsigned long long)r1);
      if (r2) atomicAdd(&a.stats[kStDag], (unsigned long long)r2);
    }
    if (a.has_own) {
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (C.ns[k]) atomicAdd(&a.lane_ns[64 * k + lane], (unsigned long long)C.ns[k]);
    }
  }
  grid_barrier(a.bar);

  // lanes whose count wrapped (and lanes derived from them) take no part in
  // the backward sweep; the host reruns them in extended form
  uint64_t X[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    X[k] = ballot(__hip_atomic_load(&a.lane_ovf[64 * k + lane], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0);
    const int pa = a.lane_pa[64 * k + lane], pb = a.lane_pb[64 * k + lane];
    X[k] |= ballot(pa >= 0 && ((((X[k] >> pa) | (X[k] >> pb)) & 1ull) != 0));
  }

  if (!failed && (a.sig_out || a.sm_out)) {
    // trace: keep the counts before psi overwrites them
    for (int64_t i = tid; i < (int64_t)n * B; i += nth) {
      const int32_t v = (int32_t)(i / B), j = (int32_t)(i % B);
      const bool r = (a.vis[(size_t)v * K + (j >> 6)] >> (j & 63)) & 1ull;
      if (EXT) { a.sm_out[(size_t)j * n + v] = r ? a.sm[i] : 0.0; a.se_out[(size_t)j * n + v] = r ? a.se[i] : 0; }
      else a.sig_out[(size_t)j * n + v] = r ? a.sig[i] : 0ull;
    }
    grid_barrier(a.bar);
  }

  // ---- backward sweep
  if (!failed) {
    for (int lb = depth; lb >= 1; --lb) {
      const uint64_t* cmv = F(lb + 1);
      uint64_t* own = F(lb);
      uint64_t* clr = F(lb + 2);
      const int32_t ub = a.uoff[lb], ue = a.uoff[lb + 1];
      for (int32_t u = ub + gw; u < ue; u += nw) backward_unit<EXT, K>(a, a.U[u], cmv, own, lb, depth, X);
      // level lb+2 masks are no longer read
      if (lb + 2 <= depth) {
        const int32_t e0 = a.qoff[lb + 2], e1 = a.qoff[lb + 3];
        for (int64_t i = tid; i < (int64_t)(e1 - e0) * K; i += nth) {
          const int32_t v = a.Q[e0 + (int32_t)(i / K)];
          clr[(size_t)v * K + (i % K)] = 0;
        }
      }
      grid_barrier(a.bar);
    }
  }

  // ---- epilogue: own terms of the 1-degree reduction, overflow and failure lists
  if (tid == 0) {
    if (!failed && a.has_own) {
      for (int j = 0; j < B; ++j) {
        const int32_t s = a.lane_src[j];
        if (s < 0 || a.lane_own[j] == 0 || ((X[j >> 6] >> (j & 63)) & 1ull)) continue;
        a.slot_bc[a.lane_slot[j]][s] += (double)a.lane_own[j] * ((double)a.lane_ns[j] - 2.0);
      }
    }
    for (int j = 0; j < B; ++j) {
      if (a.lane_src[j] < 0) continue;
      if (failed) {
        const int32_t k = atomicAdd(a.fail_count, 1);
        a.fail_list[k] = a.lane_src[j];
      } else if ((X[j >> 6] >> (j & 63)) & 1ull) {
        const int32_t k = atomicAdd(a.ovf_count, 1);
        a.ovf_list[k] = a.lane_src[j];
      }
    }
    atomicAdd(&a.stats[kStLevels], (unsigned long long)levels);
    atomicAdd(&a.stats[kStBuLevels], (unsigned long long)bu_levels);
    atomicAdd(&a.stats[kStLaunches], 1ull);
  }
  grid_barrier(a.bar);  // everything above has read the lane arrays and the level counters
  // leave the control state and (unless a trace wants them) the masks clear for the next launch
  if (tid == 0) {
    for (int i = 0; i < 3 && i < a.cap_levels; ++i) a.lc[i] = LevelCtr{0ull, 0, 0, 0ull, 0, 0};
    *a.gmulti = 0;
    *a.fulledges = 0;
  }
  for (int64_t j = tid; j < B; j += nth) { a.lane_ns[j] = 0; a.lane_ovf[j] = 0; }
  if (a.clear_at_end) {
    for (int64_t i = tid; i < (int64_t)fms; i += nth) {
      a.vis[i] = 0;
#pragma unroll
      for (int s = 0; s < kSlots; ++s) a.fm[(size_t)s * fms + i] = 0;
    }
    for (int64_t i = tid; i < n; i += nth) a.stamp[i] = -1;
  }
}

template <bool EXT>
static const void* batch_fn(int K) {
  switch (K) {
    case 1: return (const void*)batch_kernel<EXT, 1>;
    case 2: return (const void*)batch_kernel<EXT, 2>;
    case 3: return (const void*)batch_kernel<EXT, 3>;
    default: return (const void*)batch_kernel<EXT, 4>;
  }
}

hipError_t launch_batch(const BatchArgs& a, bool ext, int grid, int block, hipStream_t st) {
  if (a.K < 1 || a.K > 4) return hipErrorInvalidValue;
  void* args[] = {(void*)&a};
  const void* fn = ext ? batch_fn<true>(a.K) : batch_fn<false>(a.K);
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(block), args, 0, st);
}

hipError_t batch_max_grid(bool ext, int K, int block, int* blocks_per_cu) {
  const void* fn = ext ? batch_fn<true>(K) : batch_fn<false>(K);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, block, 0);
}

}  // namespace bcx
