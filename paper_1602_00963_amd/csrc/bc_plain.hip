// One source per launch: a cooperative persistent kernel runs the whole
// forward sweep (level-synchronous shortest-path counting, Alg. 2-3) and
// the whole backward sweep (successor-checking dependency accumulation,
// Alg. 4-5) of one source, with a grid barrier between phases.
//
// Forward, exact counts (uint64):
//   top-down level: one wave per work unit (<= 64 edges of one frontier
//     vertex); each edge claims its far end with an atomic compare-and-swap
//     on d (the paper's bmap test-and-set, made atomic) and adds sigma by a
//     64-bit atomic add whose returned value exposes wrap-around;
//   bottom-up level: one wave per static unit of every vertex still
//     unreached; it sums sigma over neighbours on the frontier (no atomics
//     unless the vertex spans several units).
// Forward, extended counts: discovery as above but without sigma, then a
//   counting phase pulls sigma over the new frontier in (m, e) form.
// Backward: one wave per unit of the level's entries; a vertex w at level
//   l sums psi(v) = (1 + delta(v) + omega(v)) / sigma(v) over successors v
//   (d(v) = l + 1), then delta(w) = sigma(w) * sum (Eq. (2), with the
//   1-degree weights of Eq. (5)).  Split vertices combine their per-unit
//   partial sums in unit order (the last arrival does it), so scores do not
//   depend on scheduling.
#include "bc_common.h"
#include "bc_kernels.h"
#include "bc_plain.h"

namespace bcx {

constexpr int CHP = kPlainChunkHost;

__device__ __forceinline__ bool add_wraps(uint64_t a, uint64_t b) { return a + b < a; }

// Exact wave sum with wrap detection at every butterfly step.
__device__ __forceinline__ uint64_t wave_sum_checked(uint64_t v, bool& wrapped) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    uint64_t t = __shfl_xor(v, o, kWave);
    if (v + t < v) wrapped = true;
    v += t;
  }
  return v;
}

// Extended-form wave sum; ext_add is commutative, so all lanes agree.
__device__ __forceinline__ Ext wave_sum_ext(Ext x) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    Ext t{__shfl_xor(x.m, o, kWave), __shfl_xor(x.e, o, kWave)};
    x = ext_add(x, t);
  }
  return x;
}

__device__ __forceinline__ int32_t ld_relaxed(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <bool EXT>
__device__ __forceinline__ void plain_finalize(const PlainArgs& a, int32_t w, double acc) {
  const double sw = EXT ? a.sm[w] : (double)a.sig[w];
  const double delta = sw * acc;
  const double om = a.omega ? (double)a.omega[w] : 0.0;
  a.psi[w] = (1.0 + delta + om) / sw;
  a.bc[w] += a.weight * (delta + om);
  if (a.delta_out) a.delta_out[w] = delta;
}

template <bool EXT>
__global__ void __launch_bounds__(256) plain_kernel(PlainArgs a, PlainFeed f) {
  if (f.srcs) {  // replayed launch: the next source of the device list
    const int32_t k = *f.cursor;  // advanced by the previous launch on the stream
    if (k >= f.nsrc) return;
    const PlainSrc s = f.srcs[k];
    a.src = s.v;
    a.own = s.own;
    a.tsub = s.tsub;
    a.weight = s.weight;
  }
  const int lane = lane_id();
  const int wpb = blockDim.x / kWave;
  const int gw = blockIdx.x * wpb + (int)(threadIdx.x / kWave);
  const int nw = gridDim.x * wpb;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  const int32_t n = a.n;
  const int32_t* __restrict__ rp = a.rp;
  const int32_t* __restrict__ ci = a.ci;
  int32_t* __restrict__ d = a.d;
  const Lists L{a.Q, a.U, a.lc, a.arrive, a.gmulti, a.err, a.rp,
                a.cap_entries, a.cap_units, a.cap_parts, a.cap_multi, 1};

  // per-lane counters, reduced once at the end of the forward sweep
  uint64_t c_reached = 0, c_rnnz = 0, c_dag = 0, c_ns = 0;
  bool wrapped = false;

  // ---- phase 0: initialise d and sigma, enqueue the source at level 0
  for (int64_t i = tid; i < n; i += nth) {
    const bool s = (i == a.src);
    d[i] = s ? 0 : -1;
    if (EXT) { a.sm[i] = s ? 1.0 : 0.0; a.se[i] = 0; }
    else a.sig[i] = s ? 1ull : 0ull;
  }
  if (gw == 0) {
    append_entries<CHP>(L, 0, 0, 0, lane == 0, a.src);
    if (lane == 0) {
      c_reached += 1;
      c_rnnz += (uint64_t)(rp[a.src + 1] - rp[a.src]);
      c_ns += 1 + (a.omega ? (uint64_t)a.omega[a.src] : 0);
    }
  }
  if (tid == 0) { a.qoff[0] = 0; a.uoff[0] = 0; }
  if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;

  // ---- forward sweep
  int l = 0;
  int32_t ebase = 0, ubase = 0;
  int64_t visited_edges = 0;
  int levels = 0, bu_levels = 0;
  bool failed = false, was_bu = false;
  while (true) {
    if (ld_relaxed(&a.lc[l].err) != 0) { failed = true; break; }
    const unsigned long long pk = __hip_atomic_load(&a.lc[l].packed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int32_t ne = (int32_t)(pk >> 32), nu = (int32_t)(pk & 0xffffffffull);
    if (ne == 0) break;
    const unsigned long long fe = __hip_atomic_load(&a.lc[l].fedges, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    visited_edges += (int64_t)fe;
    const int64_t unvisited = a.nnz - visited_edges;
    // direction: bottom-up once the frontier's edges outweigh alpha times
    // the edges still unvisited; with beta, a bottom-up sweep stays
    // bottom-up until the frontier holds fewer than n / beta vertices
    bool bu = l > 0 && a.alpha > 0.0 && (double)fe * a.alpha > (double)unvisited;
    if (was_bu && a.beta > 0.0) bu = (double)ne * a.beta >= (double)n;
    was_bu = bu;
    const int32_t ebn = ebase + ne, ubn = ubase + nu;
    const int32_t nl = l + 1;
    if (tid == 0) {
      a.qoff[nl] = ebn;
      a.uoff[nl] = ubn;
      if (l + 2 < a.cap_levels) a.lc[l + 2] = LevelCtr{0ull, 0, 0, 0ull, 0, 0};
    }
    ++levels;
    if (!bu) {
      // top-down: one wave per unit of the frontier
      for (int32_t u = ubase + gw; u < ubase + nu; u += nw) {
        const Unit un = a.U[u];
        const int32_t v = un.v;
        const int32_t beg = rp[v] + un.c * CHP;
        const int32_t end = min(rp[v + 1], beg + CHP);
        const int32_t off = beg + lane;
        bool claimed = false, dag = false;
        int32_t w = 0;
        if (off < end) {
          w = ci[off];
          int32_t dw = d[w];
          if (dw == -1) {
            int32_t expect = -1;
            claimed = __hip_atomic_compare_exchange_strong(&d[w], &expect, nl, __ATOMIC_RELAXED,
                                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            dw = claimed ? nl : expect;
          }
          if (dw == nl) {
            dag = true;
            if (!EXT) {
              const uint64_t sv = a.sig[v];
              const uint64_t old = atomicAdd((unsigned long long*)&a.sig[w], (unsigned long long)sv);
              if (add_wraps(old, sv)) wrapped = true;
            }
          }
        }
        c_dag += dag ? 1 : 0;
        append_entries<CHP>(L, nl, ebn, ubn, claimed, w);
        if (claimed) {
          c_reached += 1;
          c_rnnz += (uint64_t)(rp[w + 1] - rp[w]);
          c_ns += 1 + (a.omega ? (uint64_t)a.omega[w] : 0);
        }
      }
    } else {
      ++bu_levels;
      // bottom-up: one wave per static unit of every vertex
      for (int32_t g = gw; g < a.ngu; g += nw) {
        const int2 gu = a.gu[g];
        const int32_t w = gu.x;
        const int32_t dw0 = ld_relaxed(&d[w]);
        if (dw0 != -1 && dw0 != nl) continue;  // reached at an earlier level (uniform)
        const int32_t rb = rp[w], re = rp[w + 1];
        const bool split = (re - rb) > CHP;
        const int32_t off = rb + gu.y * CHP + lane;
        bool match = false;
        uint64_t term = 0;
        Ext eterm = ext_zero();
        if (off < re) {
          const int32_t v = ci[off];
          match = d[v] == l;
          if (match && !EXT) term = a.sig[v];
        }
        const uint64_t mm = ballot(match);
        c_dag += match ? 1 : 0;
        (void)eterm;
        uint64_t sum = 0;
        if (!EXT) sum = wave_sum_checked(term, wrapped);
        bool claimed = false;
        if (mm != 0 && lane == 0) {
          if (!split) {
            d[w] = nl;
            if (!EXT) a.sig[w] = sum;
            claimed = true;
          } else {
            int32_t expect = -1;
            claimed = __hip_atomic_compare_exchange_strong(&d[w], &expect, nl, __ATOMIC_RELAXED,
                                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!EXT) {
              const uint64_t old = atomicAdd((unsigned long long*)&a.sig[w], (unsigned long long)sum);
              if (add_wraps(old, sum)) wrapped = true;
            }
          }
        }
        append_entries<CHP>(L, nl, ebn, ubn, claimed, w);
        if (claimed) {
          c_reached += 1;
          c_rnnz += (uint64_t)(re - rb);
          c_ns += 1 + (a.omega ? (uint64_t)a.omega[w] : 0);
        }
      }
    }
    if (ballot(wrapped) != 0 && lane == 0) atomicOr(a.ovf_now, 1);
    if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;
    if (EXT) {
      // counting phase: sigma of the new frontier, pulled from level l
      if (ld_relaxed(&a.lc[nl].err) != 0) { failed = true; break; }
      const unsigned long long pk2 = __hip_atomic_load(&a.lc[nl].packed, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const int32_t nu2 = (int32_t)(pk2 & 0xffffffffull);
      for (int32_t u = ubn + gw; u < ubn + nu2; u += nw) {
        const Unit un = a.U[u];
        const int32_t w = un.v;
        const int32_t beg = a.rp[w] + un.c * CHP;
        const int32_t end = min(rp[w + 1], beg + CHP);
        const int32_t off = beg + lane;
        Ext t = ext_zero();
        if (off < end) {
          const int32_t v = ci[off];
          if (d[v] == l) t = Ext{a.sm[v], a.se[v]};
        }
        const Ext s = wave_sum_ext(t);
        if (lane == 0) {
          if (un.mi < 0) {
            const Ext z = ext_norm(s);
            a.sm[w] = z.m; a.se[w] = z.e;
          } else {
            const int32_t nunits = units_of<CHP>(rp[w + 1] - rp[w]);
            part_store(&a.part_m[un.pb + un.c], s.m);
            part_store(&a.part_e[un.pb + un.c], s.e);
            part_stores_done();
            const int32_t old = atomicAdd(&a.arrive[un.mi], 1);
            if (old == nunits - 1) {
              part_loads_after();
              Ext tot = ext_zero();
              for (int32_t c = 0; c < nunits; ++c) {
                const double pm = part_load(&a.part_m[un.pb + c]);
                const int32_t pe = part_load(&a.part_e[un.pb + c]);
                tot = ext_add(tot, Ext{pm, pe});
              }
              const Ext z = ext_norm(tot);
              a.sm[w] = z.m; a.se[w] = z.e;
            }
          }
        }
      }
      if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;
    }
    l = nl;
    ebase = ebn;
    ubase = ubn;
  }
  const int depth = l - 1;

  // publish the forward counters; the barrier makes them (and ns) visible
  {
    const uint64_t r0 = wave_sum_u64(c_reached), r1 = wave_sum_u64(c_rnnz);
    const uint64_t r2 = wave_sum_u64(c_dag), r3 = wave_sum_u64(c_ns);
    if (lane == 0) {
      if (r0) atomicAdd(&a.stats[kStReached], (unsigned long long)r0);
      if (r1) atomicAdd(&a.stats[kStReachedNnz], (unsigned long long)r1);
      if (r2) atomicAdd(&a.stats[kStDag], (unsigned long long)r2);
      if (r3) atomicAdd((unsigned long long*)a.ns, (unsigned long long)r3);
    }
  }
  if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;
  const bool overflowed = ld_relaxed(a.ovf_now) != 0;

  // ---- backward sweep (skipped when counts wrapped: the host reruns the source)
  if (!failed && !overflowed) {
    for (int lb = depth; lb >= 1; --lb) {
      const int32_t ub = a.uoff[lb], ue = a.uoff[lb + 1];
      for (int32_t u = ub + gw; u < ue; u += nw) {
        const Unit un = a.U[u];
        const int32_t w = un.v;
        double t = 0.0;
        if (lb < depth) {
          const int32_t beg = rp[w] + un.c * CHP;
          const int32_t end = min(rp[w + 1], beg + CHP);
          const int32_t off = beg + lane;
          if (off < end) {
            const int32_t v = ci[off];
            if (d[v] == lb + 1) {
              t = a.psi[v];
              if (EXT) t = ldexp(t, a.se[w] - a.se[v]);
            }
          }
        }
        const double s = wave_sum(t);
        if (lane == 0) {
          if (un.mi < 0) {
            plain_finalize<EXT>(a, w, s);
          } else {
            const int32_t nunits = units_of<CHP>(rp[w + 1] - rp[w]);
            const int32_t target = (EXT ? 2 : 1) * nunits - 1;
            part_store(&a.part_m[un.pb + un.c], s);
            part_stores_done();
            const int32_t old = atomicAdd(&a.arrive[un.mi], 1);
            if (old == target) {
              part_loads_after();
              double tot = 0.0;
              for (int32_t c = 0; c < nunits; ++c) tot += part_load(&a.part_m[un.pb + c]);
              plain_finalize<EXT>(a, w, tot);
            }
          }
        }
      }
      if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;
    }
  }

  // ---- epilogue: own term of the 1-degree reduction, reset the control block
  if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;  // nobody reads ovf_now, ns or the level counters past this point
  if (tid == 0) {
    if (!failed && !overflowed && a.own > 0) {
      const double ns = (double)*a.ns;
      a.bc[a.src] += (double)a.own * (ns - 1.0) - a.tsub;  // pendants alone: own * (n_s - 2)
    }
    if (overflowed && !failed) {
      const int32_t k = atomicAdd(a.ovf_count, 1);
      a.ovf_list[k] = a.src;
    }
    atomicAdd(&a.stats[kStLevels], (unsigned long long)levels);
    atomicAdd(&a.stats[kStBuLevels], (unsigned long long)bu_levels);
    atomicAdd(&a.stats[kStLaunches], 1ull);
    for (int i = 0; i < 3 && i < a.cap_levels; ++i) a.lc[i] = LevelCtr{0ull, 0, 0, 0ull, 0, 0};
    *a.gmulti = 0;
    *a.ns = 0;
    *a.ovf_now = 0;
    if (f.srcs) atomicAdd(f.cursor, 1);  // every wave read it before the first barrier
  }
}

hipError_t launch_plain_fed(const PlainArgs& a, const PlainFeed& f, bool ext, int grid, int block, hipStream_t st) {
  void* args[] = {(void*)&a, (void*)&f};
  const void* fn = ext ? (const void*)plain_kernel<true> : (const void*)plain_kernel<false>;
  return hipLaunchKernel(fn, dim3(grid), dim3(block), args, 0, st);
}

hipError_t launch_plain(const PlainArgs& a, bool ext, int grid, int block, hipStream_t st) {
  return launch_plain_fed(a, PlainFeed{nullptr, nullptr, 0}, ext, grid, block, st);
}

hipError_t plain_max_grid(bool ext, int block, int* blocks_per_cu) {
  const void* fn = ext ? (const void*)plain_kernel<true> : (const void*)plain_kernel<false>;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, block, 0);
}

}  // namespace bcx
