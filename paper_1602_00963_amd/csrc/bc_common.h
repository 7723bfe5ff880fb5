// Internal declarations shared by the HIP kernels and the host runtime.
// Wave64 primitives for gfx950 and the device-side bookkeeping structures
// of the forward (shortest-path counting) and backward (dependency) sweeps.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/bc.h"

namespace bcx {

constexpr int kWave = 64;

// ------------------------------------------------------------ wave helpers

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0)); }

// Number of set bits of `mask` strictly below the calling lane.
__device__ __forceinline__ int lanes_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

template <typename T>
__device__ __forceinline__ T shfl(T v, int src) { return __shfl(v, src, kWave); }

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// Butterfly sum in a fixed order: every lane ends with the same total.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
  return v;
}
__device__ __forceinline__ uint64_t wave_or_u64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o, kWave);
  return v;
}

// Inclusive prefix sum of a 64-bit value over the wave (Hillis-Steele).
__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    uint64_t t = __shfl_up(v, o, kWave);
    if (l >= o) v += t;
  }
  return v;
}

// ----------------------------------------------------- extended-range counts
// A path count too large for uint64 is held as (m, e) = m * 2^e with m in
// [1, 2) (or 0).  Sums align to the larger exponent; terms smaller by more
// than 2^-1074 relative vanish, far below the 1e-9 tolerance.

struct Ext {
  double m;
  int32_t e;
};

__device__ __forceinline__ Ext ext_zero() { return Ext{0.0, INT32_MIN / 2}; }

__device__ __forceinline__ Ext ext_add(Ext a, Ext b) {
  if (a.m == 0.0) return b;
  if (b.m == 0.0) return a;
  if (a.e >= b.e) {
    int d = b.e - a.e;
    return Ext{a.m + (d < -1100 ? 0.0 : ldexp(b.m, d)), a.e};
  }
  int d = a.e - b.e;
  return Ext{b.m + (d < -1100 ? 0.0 : ldexp(a.m, d)), b.e};
}

__device__ __forceinline__ Ext ext_norm(Ext a) {
  if (a.m == 0.0) return ext_zero();
  int k;
  double f = frexp(a.m, &k);  // f in [0.5, 1)
  return Ext{f * 2.0, a.e + k - 1};
}

// ------------------------------------------------------------ work records

// One unit of edge work: chunk `c` (edges [c*CH, (c+1)*CH) of the
// adjacency) of the level-list entry for vertex `v`.  Entries whose
// adjacency spans several chunks ("split" entries) also carry `mi`, a
// run-unique index of their arrival counter, and `pb`, the level-relative
// base of their partial-sum slots; single-chunk entries have mi = -1.
struct Unit {
  int32_t v;
  int32_t c;
  int32_t mi;
  int32_t pb;
};

// Per-level counters of a level list, written by atomic appends during the
// discovering phase of the previous level.  `packed` = entries << 32 | units.
struct LevelCtr {
  unsigned long long packed;
  int32_t multi;      // split entries appended (run-unique indices taken from a global counter)
  int32_t pslots;     // partial-sum slots reserved (level-relative)
  unsigned long long fedges;  // sum of degrees of the appended entries
  int32_t err;        // capacity errors raised while this level's list was built
  int32_t pad;
  unsigned long long lanes;  // (vertex, source) pairs discovered on this level (batched kernel)
};
// Every workgroup reads a level's counters only after the barrier that ends
// the phase building that level, so all of them take the same decisions.

// Grid-wide barrier of a persistent launch (every workgroup resident at
// once), two-level: the workgroups of one residue class of blockIdx mod 8
// (the round-robin order in which workgroups are spread over the eight
// XCDs) meet on their own counter, the last of each class on a top counter,
// and the very last bumps a generation word the others poll.  Counters
// return to 0 by themselves; the generation only grows.  Every wave first
// waits until its own stores and atomics are performed at the L2 of its
// XCD; the workgroup's first thread then publishes them to the other XCDs
// with one agent-scope release fence (an L2 write-back) before arriving,
// and takes one agent-scope acquire fence (an L1/L2 invalidation, which
// serves all the workgroup's waves: they run on one CU) after leaving.  A
// fence in every wave costs a write-back per wave, which dominated the
// barrier at a thousand workgroups.
//
// The wait is bounded: a workgroup that has polled for longer than `limit`
// ticks of the constant-rate wall clock (workgroups of the grid that never
// became resident, e.g. because other persistent work holds the CUs) raises
// the abort word and gives up; every later arrival sees the word and gives
// up at once.  grid_barrier returns false after a give-up, and the kernel
// then returns, so every workgroup ends normally; the host reports the
// launch as failed.
struct alignas(128) BarSlot {
  unsigned v;
  unsigned pad[31];
};
struct GridBar {
  BarSlot xcd[8];
  BarSlot top;
  BarSlot gen;
  BarSlot abort;
};

constexpr int32_t kErrBarrier = 16;  // a grid-barrier wait gave up (DevErr bit)

__device__ __forceinline__ bool grid_barrier(GridBar* b, uint64_t limit, int32_t* err) {
  __shared__ int s_go;
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    int go = 1;
    if (__hip_atomic_load(&b->abort.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
      go = 0;
    } else {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      const unsigned nb = gridDim.x;
      const unsigned g = __hip_atomic_load(&b->gen.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned x = blockIdx.x & 7u;
      const unsigned nx = (nb + 7u - x) / 8u;
      const unsigned ntop = nb < 8u ? nb : 8u;
      bool last = false;
      // Arrivals are relaxed: each workgroup's writes were released by the
      // fence above.  Only the workgroups that pass an arrival on (the last
      // of an XCD, the last overall) acquire and release again, so that the
      // others' writes reach the waiters through them.
      if (__hip_atomic_fetch_add(&b->xcd[x].v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == nx - 1u) {
        __hip_atomic_store(&b->xcd[x].v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        if (__hip_atomic_fetch_add(&b->top.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == ntop - 1u) {
          __hip_atomic_store(&b->top.v, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          last = true;
        }
      }
      if (last) {
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __hip_atomic_store(&b->gen.v, g + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        const uint64_t t0 = wall_clock64();
        while (__hip_atomic_load(&b->gen.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == g) {
          if (__hip_atomic_load(&b->abort.v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) { go = 0; break; }
          if (wall_clock64() - t0 > limit) {
            __hip_atomic_store(&b->abort.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            atomicOr(err, kErrBarrier);
            go = 0;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    s_go = go;
  }
  __syncthreads();
  return s_go != 0;
}

// Errors raised inside a persistent kernel; the host maps them to bc_status.
enum DevErr : int32_t { kErrNone = 0, kErrCapEntries = 1, kErrCapUnits = 2, kErrCapPartials = 4, kErrCapMulti = 8 };
// (kErrBarrier = 16 above: a grid-barrier wait gave up.)

}  // namespace bcx

namespace bcx {

// Level lists: the stacked queue Q of the paper's Alg. 2 (Q with offsets
// Q_off), extended with a work-unit list so that long adjacency lists are
// split across waves.  Entries of level l occupy Q[ebase(l) .. ebase(l+1)),
// their units U[ubase(l) .. ubase(l+1)).
struct Lists {
  int32_t* Q;
  Unit* U;
  LevelCtr* lc;
  int32_t* arrive;   // arrival counters of split entries (run-unique index)
  int32_t* gmulti;   // next split-entry index
  int32_t* err;
  const int32_t* rp;
  int32_t cap_entries, cap_units, cap_parts, cap_multi;
  int32_t words;     // arrival counters per split entry (one per 64-lane word)
};

__device__ __forceinline__ void raise_err(const Lists& L, int lvl, int32_t code) {
  atomicOr(&L.lc[lvl].err, code);
  atomicOr(L.err, code);
}

// Partial sums of a split entry pass from the waves that work its units to
// the last one to arrive, possibly on another XCD.  They are written and
// read with device-scope accesses, which go through each XCD's L2 to the
// device's coherence point, and a wave waits for its partial stores to
// complete before it counts its arrival.  No agent-scope fence is needed:
// on this chip a release fence writes back the XCD's whole L2 and an
// acquire fence invalidates it, which once per split unit cost about half
// of the batched kernel's time.
template <typename T>
__device__ __forceinline__ void part_store(T* p, T v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __forceinline__ T part_load(const T* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// The wave's partial stores have completed (before its arrival is counted).
__device__ __forceinline__ void part_stores_done() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
// Keeps the compiler from moving partial loads above the arrival count.
__device__ __forceinline__ void part_loads_after() { asm volatile("" ::: "memory"); }

// Wave-aggregated append of the lanes with `want` to level `lvl`'s list:
// one 64-bit atomic per wave reserves both the entry positions and the
// unit positions (entries << 32 | units), lanes take their slots by an
// inclusive scan.  Adds the appended degrees to the level's frontier-edge
// counter.  Returns the number of lanes appended (uniform).
template <int CH>
__device__ __forceinline__ int append_entries(const Lists& L, int lvl, int32_t ebase, int32_t ubase,
                                              bool want, int32_t vtx) {
  const uint64_t wmask = ballot(want);
  if (wmask == 0) return 0;
  int32_t deg = 0, nunits = 0;
  if (want) {
    deg = L.rp[vtx + 1] - L.rp[vtx];
    nunits = deg <= CH ? 1 : (deg + CH - 1) / CH;
  }
  const uint64_t contrib = want ? ((1ull << 32) | (uint64_t)(uint32_t)nunits) : 0ull;
  const uint64_t incl = wave_incl_scan_u64(contrib);
  const uint64_t total = shfl(incl, kWave - 1);
  const uint64_t dsum = wave_sum_u64(want ? (uint64_t)deg : 0ull);
  unsigned long long base = 0;
  if (lane_id() == kWave - 1) {
    base = atomicAdd(&L.lc[lvl].packed, (unsigned long long)total);
    atomicAdd(&L.lc[lvl].fedges, (unsigned long long)dsum);
  }
  base = shfl((uint64_t)base, kWave - 1);
  if (want) {
    const uint64_t my = base + incl - contrib;
    const int64_t e = (int64_t)ebase + (int64_t)(my >> 32);
    const int64_t u = (int64_t)ubase + (int64_t)(my & 0xffffffffull);
    if (e >= L.cap_entries) {
      raise_err(L, lvl, kErrCapEntries);
    } else if (u + nunits > L.cap_units) {
      raise_err(L, lvl, kErrCapUnits);
    } else {
      L.Q[e] = vtx;
      if (nunits == 1) {
        L.U[u] = Unit{vtx, 0, -1, 0};
      } else {
        const int32_t mi = atomicAdd(L.gmulti, 1);
        const int32_t pb = atomicAdd(&L.lc[lvl].pslots, nunits);
        atomicAdd(&L.lc[lvl].multi, 1);
        if (mi >= L.cap_multi) {
          raise_err(L, lvl, kErrCapMulti);
        } else if (pb + nunits > L.cap_parts) {
          raise_err(L, lvl, kErrCapPartials);
        } else {
          for (int32_t k = 0; k < L.words; ++k) L.arrive[(size_t)mi * L.words + k] = 0;
          for (int32_t c = 0; c < nunits; ++c) L.U[u + c] = Unit{vtx, c, mi, pb};
        }
      }
    }
  }
  return __popcll(wmask);
}

// Units of a split entry with degree deg.
template <int CH>
__device__ __forceinline__ int32_t units_of(int32_t deg) { return deg <= CH ? 1 : (deg + CH - 1) / CH; }

}  // namespace bcx
