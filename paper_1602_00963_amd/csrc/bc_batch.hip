// Many sources per launch.  A batch of B = 64 K sources advances level by
// level together inside one cooperative persistent kernel.  Lane j of a
// 64-lane word k is source 64 k + j; per-(vertex, source) state is stored
// source-minor ([vertex][lane]) so a wave touching one vertex reads or
// writes one contiguous row per word.  Per vertex, 64-bit lane masks record
// which sources have reached it (vis) and which sit on a given level (fm,
// three rotating arrays).
//
// Forward level l (shortest-path counting, Alg. 2-3 generalised to B
// sources):
//   discovering phase -- top-down: one wave per unit (<= 256 edges) of the
//     level-l entries; every edge ORs (mask(v) & ~vis(w)) into the next
//     mask of w; bottom-up: one wave per static unit of every vertex some
//     source has not reached, OR-ing its neighbours' level-l masks.  A
//     vertex entering level l+1 is appended once (per-level stamp) to the
//     level list.
//     2-degree derived lanes (Lemma 1) take no part in edge propagation: a
//     derived lane c with partner lanes a, b reaches vertex v at level l+1
//     exactly when a or b sits on v at level l and c has not reached v yet.
//   counting phase -- one wave per unit of the level-(l+1) entries, lanes =
//     sources: sigma(w) = sum of sigma(v) over neighbours v with the lane's
//     bit in mask_l(v).  Derived lanes instead take Eq. (6): the sum of the
//     partners' counts at w over the partners on level l.
// Backward level l (dependency accumulation, Alg. 4-5, successor checking):
//   one wave per unit of the level-l entries; per lane, sum psi over the
//   neighbours whose mask for level l+1 has the lane's bit, then
//   delta = sigma * sum and psi = (1 + delta + omega) / sigma overwrite the
//   count in place.  The vertex's score gains sum over its lanes of
//   weight * (delta + omega), summed in lane order.
// Entries spanning several units combine per-unit partial sums in unit
// order (the last arrival does it), so results do not depend on scheduling.
#include <hip/hip_cooperative_groups.h>

#include "bc_common.h"
#include "bc_kernels.h"

namespace cg = cooperative_groups;

namespace bcx {

constexpr int CHB = kBatchChunk;

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

template <bool EXT, int K>
__global__ void __launch_bounds__(256) batch_kernel(BatchArgs a) {
  cg::grid_group grid = cg::this_grid();
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
  const size_t fmstride = (size_t)n * K;

  // per-lane run counters
  uint64_t c_reached = 0, c_rnnz = 0, c_dag = 0, c_full = 0;
  uint64_t c_ns[K];
#pragma unroll
  for (int k = 0; k < K; ++k) c_ns[k] = 0;

  // ---- phase 0: clear masks and stamps
  for (int64_t i = tid; i < (int64_t)n * K; i += nth) {
    a.vis[i] = 0;
    a.fm[i] = 0;
    a.fm[fmstride + i] = 0;
    a.fm[2 * fmstride + i] = 0;
  }
  for (int64_t i = tid; i < n; i += nth) a.stamp[i] = -1;
  grid.sync();

  // ---- phase 1: seed the sources at level 0
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
      c_reached += 1;
      c_rnnz += (uint64_t)(rp[s + 1] - rp[s]);
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
  grid.sync();

  // ---- forward sweep
  int l = 0;
  int32_t ebase = 0, ubase = 0, eprev = 0;
  int levels = 0, bu_levels = 0;
  bool failed = false;
  while (true) {
    if (ldr32(&a.lc[l].err) != 0) { failed = true; break; }
    const uint64_t pk = ldr64(&a.lc[l].packed);
    const int32_t ne = (int32_t)(pk >> 32), nu = (int32_t)(pk & 0xffffffffull);
    if (ne == 0) break;
    const uint64_t fe = ldr64(&a.lc[l].fedges);
    const uint64_t full = ldr64(a.fulledges);
    const double unvisited = (double)a.nnz - (double)full;
    const bool bu = l > 0 && a.alpha > 0.0 && (double)fe * a.alpha > unvisited;
    const int32_t ebn = ebase + ne, ubn = ubase + nu;
    const int32_t nl = l + 1;
    const uint64_t* cur = a.fm + (size_t)(l % 3) * fmstride;
    uint64_t* nxt = a.fm + (size_t)(nl % 3) * fmstride;
    uint64_t* old = a.fm + (size_t)((l + 2) % 3) * fmstride;
    if (tid == 0) {
      a.qoff[nl] = ebn;
      a.uoff[nl] = ubn;
      if (l + 2 < a.cap_levels) a.lc[l + 2] = LevelCtr{0ull, 0, 0, 0ull, 0, 0};
    }
    ++levels;

    // ---- discovering phase
    if (!bu) {
      for (int32_t u = ubase + gw; u < ubase + nu; u += nw) {
        const Unit un = a.U[u];
        const int32_t v = a.Q[un.e];
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
              const uint64_t nb = cm[k] & ~a.vis[(size_t)w * K + k];
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
        for (int k = 0; k < K; ++k) { vk[k] = a.vis[(size_t)w * K + k]; done &= (vk[k] & EL[k]) == EL[k]; }
        if (done) continue;  // every edge lane already reached w (uniform)
        const int32_t rb = rp[w], re = rp[w + 1];
        const int32_t beg = rb + gu.y * CHB;
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
      // 2-degree derived lanes: elementwise over the level-l entries (Lemma 1)
      for (int32_t e = ebase + gw; e < ebn; e += nw) {
        const int32_t v = a.Q[e];
        bool want = false;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          const uint64_t ck = cur[(size_t)v * K + k];
          const uint64_t vkk = a.vis[(size_t)v * K + k];
          const int pa = a.lane_pa[64 * k + lane], pb = a.lane_pb[64 * k + lane];
          bool mine = false;
          if (pa >= 0) mine = ((((ck >> pa) | (ck >> pb)) & 1ull) != 0) && (((vkk >> lane) & 1ull) == 0);
          const uint64_t nb = ballot(mine);
          if (nb) {
            if (lane == 0) atomicOr((unsigned long long*)&nxt[(size_t)v * K + k], (unsigned long long)nb);
            want = true;
          }
        }
        claim_and_append<CHB>(a, L, nl, ebn, ubn, want && lane == 0, v);
      }
    }
    grid.sync();
    if (ldr32(&a.lc[nl].err) != 0) { failed = true; break; }

    // ---- counting phase over the level-(l+1) entries
    {
      const uint64_t pk2 = ldr64(&a.lc[nl].packed);
      const int32_t nu2 = (int32_t)(pk2 & 0xffffffffull);
      for (int32_t u = ubn + gw; u < ubn + nu2; u += nw) {
        const Unit un = a.U[u];
        const int32_t w = a.Q[un.e];
        const int32_t rb = rp[w], re = rp[w + 1];
        const int32_t beg = rb + un.c * CHB;
        const int32_t end = min(re, beg + CHB);
        uint64_t nbm[K], em[K];
        bool anye = false;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          nbm[k] = nxt[(size_t)w * K + k];
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
            const int32_t cnt = min(kWave, end - off0);
            int32_t vl = 0;
            uint64_t ml[K];
            if (off < end) {
              vl = ci[off];
#pragma unroll
              for (int k = 0; k < K; ++k) ml[k] = cur[(size_t)vl * K + k] & em[k];
            } else {
#pragma unroll
              for (int k = 0; k < K; ++k) ml[k] = 0;
            }
#pragma unroll
            for (int k = 0; k < K; ++k) c_dag += (uint64_t)__popcll(ml[k]);
            for (int t = 0; t < cnt; ++t) {
              const int32_t v = rl32(vl, t);
#pragma unroll
              for (int k = 0; k < K; ++k) {
                const uint64_t mv = rl64(ml[k], t);
                if (mv == 0) continue;
                if ((mv >> lane) & 1ull) {
                  const size_t idx = (size_t)v * B + 64 * k + lane;
                  if (EXT) {
                    x[k] = ext_add(x[k], Ext{a.sm[idx], a.se[idx]});
                  } else {
                    const uint64_t y = a.sig[idx];
                    if (s[k] + y < s[k]) wrap[k] = true;
                    s[k] += y;
                  }
                }
              }
            }
          }
        }
        // combine the units of a split entry in unit order
        bool fin = true;
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
          fin = prev == nunits - 1;
          if (fin) {
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
        }
        if (fin) {
          // finalise: counts, levels, visited masks; derived lanes by Eq. (6)
          const uint64_t* curw = cur + (size_t)w * K;
          bool fullnow = true;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            const size_t idx = (size_t)w * B + 64 * k + lane;
            if ((nbm[k] >> lane) & 1ull) {
              if (!((em[k] >> lane) & 1ull)) {
                // derived lane: partners' counts at w over the partners on level l
                const int pa = a.lane_pa[64 * k + lane], pb = a.lane_pb[64 * k + lane];
                const uint64_t cw = curw[k];
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
              a.lv[idx] = nl;
              if (a.has_own) c_ns[k] += 1 + (a.omega ? (uint64_t)a.omega[w] : 0);
            }
            const uint64_t nv = a.vis[(size_t)w * K + k] | nbm[k];
            if (lane == 0) a.vis[(size_t)w * K + k] = nv;
            fullnow &= (nv & EL[k]) == EL[k];
            if (lane == 0) {
              const uint64_t pc = (uint64_t)__popcll(nbm[k]);
              c_reached += pc;
              c_rnnz += pc * (uint64_t)(re - rb);
            }
          }
          if (fullnow && lane == 0) c_full += (uint64_t)(re - rb);
        }
      }
      // clear the level-(l-1) masks so this array can take level l+2
      if (l >= 1) {
        for (int64_t i = tid; i < (int64_t)(ebase - eprev) * K; i += nth) {
          const int32_t v = a.Q[eprev + (int32_t)(i / K)];
          old[(size_t)v * K + (i % K)] = 0;
        }
      }
      {
        const uint64_t fsum = wave_sum_u64(c_full);
        if (lane == 0 && fsum) atomicAdd(a.fulledges, (unsigned long long)fsum);
        c_full = 0;
      }
    }
    grid.sync();
    eprev = ebase;
    l = nl;
    ebase = ebn;
    ubase = ubn;
  }
  const int depth = l - 1;

  // publish forward counters and component sizes
  {
    const uint64_t r0 = wave_sum_u64(c_reached), r1 = wave_sum_u64(c_rnnz), r2 = wave_sum_u64(c_dag);
    if (lane == 0) {
      if (r0) atomicAdd(&a.stats[kStReached], (unsigned long long)r0);
      if (r1) atomicAdd(&a.stats[kStReachedNnz], (unsigned long long)r1);
      if (r2) atomicAdd(&a.stats[kStDag], (unsigned long long)r2);
    }
    if (a.has_own) {
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (c_ns[k]) atomicAdd(&a.lane_ns[64 * k + lane], (unsigned long long)c_ns[k]);
    }
  }
  grid.sync();

  // lanes whose count wrapped take no part in the backward sweep
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
    grid.sync();
  }

  // ---- backward sweep
  if (!failed) {
    double* psi = EXT ? a.sm : (double*)a.sig;
    for (int lb = depth; lb >= 1; --lb) {
      const uint64_t* cmv = a.fm + (size_t)((lb + 1) % 3) * fmstride;
      uint64_t* own = a.fm + (size_t)(lb % 3) * fmstride;
      uint64_t* clr = a.fm + (size_t)((lb + 2) % 3) * fmstride;
      const int32_t ub = a.uoff[lb], ue = a.uoff[lb + 1];
      for (int32_t u = ub + gw; u < ue; u += nw) {
        const Unit un = a.U[u];
        const int32_t w = a.Q[un.e];
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
            const int32_t cnt = min(kWave, end - off0);
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
            for (int t = 0; t < cnt; ++t) {
              const int32_t v = rl32(vl, t);
#pragma unroll
              for (int k = 0; k < K; ++k) {
                const uint64_t mv = rl64(ml[k], t);
                if (mv == 0) continue;
                if ((mv >> lane) & 1ull) {
                  const size_t idx = (size_t)v * B + 64 * k + lane;
                  double y = psi[idx];
                  if (EXT) y = ldexp(y, ew[k] - a.se[idx]);
                  acc[k] += y;
                }
              }
            }
          }
        }
        bool fin = true;
        if (un.mi >= 0) {
          const int32_t nunits = units_of<CHB>(re - rb);
#pragma unroll
          for (int k = 0; k < K; ++k) a.part_m[((size_t)(un.pb + un.c) * K + k) * 64 + lane] = acc[k];
          fence_release();
          int32_t prev = 0;
          if (lane == 0) prev = atomicAdd(&a.arrive[un.mi], 1);
          prev = __shfl(prev, 0, kWave);
          fin = prev == 2 * nunits - 1;
          if (fin) {
            fence_acquire();
#pragma unroll
            for (int k = 0; k < K; ++k) acc[k] = 0.0;
            for (int32_t c = 0; c < nunits; ++c) {
#pragma unroll
              for (int k = 0; k < K; ++k)
                acc[k] += __hip_atomic_load(&a.part_m[((size_t)(un.pb + c) * K + k) * 64 + lane],
                                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
          }
        }
        if (fin && anyo) {
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
              if (a.delta_out) a.delta_out[(size_t)(64 * k + lane) * n + w] = delta;
            }
          }
          int slot = -1;
          double tot = 0.0;
#pragma unroll
          for (int k = 0; k < K; ++k) {
            uint64_t rem = om[k];
            while (rem) {
              const int first = __builtin_ctzll(rem);
              const int s = __builtin_amdgcn_readlane(sl[k], first);
              const uint64_t same = ballot(sl[k] == s) & rem;
              const double part = wave_sum(((same >> lane) & 1ull) ? cs[k] : 0.0);
              if (s != slot) {
                if (slot >= 0 && lane == 0) a.slot_bc[slot][w] += tot;
                slot = s;
                tot = 0.0;
              }
              tot += part;
              rem &= ~same;
            }
          }
          if (slot >= 0 && lane == 0) a.slot_bc[slot][w] += tot;
        }
      }
      // the level-(lb+2) masks are no longer needed
      if (lb + 2 <= depth) {
        const int32_t e0 = a.qoff[lb + 2], e1 = a.qoff[lb + 3];
        for (int64_t i = tid; i < (int64_t)(e1 - e0) * K; i += nth) {
          const int32_t v = a.Q[e0 + (int32_t)(i / K)];
          clr[(size_t)v * K + (i % K)] = 0;
        }
      }
      grid.sync();
    }
  }

  // ---- epilogue: own terms of the 1-degree reduction, reset control state
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
  grid.sync();  // the epilogue above has read lane_ns and lane_ovf
  if (tid == 0) {
    for (int i = 0; i < 3 && i < a.cap_levels; ++i) a.lc[i] = LevelCtr{0ull, 0, 0, 0ull, 0, 0};
    *a.gmulti = 0;
    *a.fulledges = 0;
  }
  for (int64_t j = tid; j < B; j += nth) { a.lane_ns[j] = 0; a.lane_ovf[j] = 0; }
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
