// One source per workgroup, many workgroups at once (BC_MODE_PER_WORKGROUP).
// Every workgroup owns a private copy of the per-source state (one 16-byte
// record per vertex, the stacked level queue) and walks its sources one
// after the other; the levels of one source are separated by workgroup
// barriers only.  On long-diameter graphs (thousands of levels, a few
// thousand frontier vertices each) a grid-wide barrier per level is what a
// whole-device launch pays for, and sources spread over the graph share no
// frontier vertices a batch could pool; here each level costs one workgroup
// barrier and the device is filled by running hundreds of sources side by
// side.
//
// Forward (Alg. 2-3), one pass per level: threads take frontier vertices;
// each neighbour still unreached is claimed by an atomic compare-and-swap on
// its level and appended to the next level, and the frontier entry keeps a
// mask of which of its neighbours are successors.  Exact counts are pushed by
// atomic 64-bit adds whose returned value exposes a wrap; an extended count
// (significand, exponent) is pulled by the thread that claimed the vertex,
// from its neighbours on the current level, whose counts are final; the pull
// also notes those predecessors in the new vertex's queue entry, so that its
// own claim pass skips them.  Backward (Alg. 4-5, successor checking):
// threads take the level's vertices and sum psi = (1 + delta + omega) /
// sigma over the successors the mask names; psi replaces the count in the
// record, which no later step reads.  Adjacency comes from a packed slot per
// vertex (degree and up to seven neighbours in one 32-byte block), the CSR
// only for longer rows.  Each source's contributions go to its own result
// array with fp64 atomics (order-dependent rounding, within the 1e-9
// tolerance).  Between sources the exact form clears the records it touched;
// the extended form tags level words with a generation instead (below).
#include "bc_common.h"
#include "bc_kernels.h"
#include "bc_wg.h"

namespace bcx {

constexpr int kWgBlock = 1024;
constexpr int kEllIn = kEllWidth - 1;  // neighbours held in a slot

__device__ __forceinline__ double as_f64(uint64_t x) { return __longlong_as_double((long long)x); }
__device__ __forceinline__ uint64_t as_u64(double x) { return (uint64_t)__double_as_longlong(x); }

// A vertex's packed adjacency slot (two 16-byte loads from one 32-byte block).
struct Adj {
  int32_t deg;
  int32_t nb[kEllIn];  // nb[0] is the CSR row start when deg > kEllIn
};

__device__ __forceinline__ Adj load_adj(const int32_t* __restrict__ ell, int32_t v) {
  const int4* p = reinterpret_cast<const int4*>(ell) + 2 * (size_t)v;
  const int4 a = p[0], b = p[1];
  return Adj{a.x, {a.y, a.z, a.w, b.x, b.y, b.z, b.w}};
}

// f(j, x) for the neighbours x of a vertex in row order (j = position).
template <class F>
__device__ __forceinline__ void for_adj(const Adj& A, const int32_t* __restrict__ ci, F&& f) {
  if (A.deg <= kEllIn) {
#pragma unroll
    for (int j = 0; j < kEllIn; ++j)
      if (j < A.deg) f(j, A.nb[j]);
  } else {
    const int32_t b = A.nb[0];
    for (int32_t j = 0; j < A.deg; ++j) f(j, ci[b + j]);
  }
}

__device__ __forceinline__ uint32_t succ_bit(int32_t j) { return 1u << (j < 31 ? j : 31); }

// Generation tags (extended counts): a record's level word is
// (generation << kGenShift) | (level + 1), the generation counting the
// workgroup's sources in the launch; a record of an older generation reads
// as not reached, so the records need no clearing between sources.  After
// kGenMax sources the workgroup clears its slice and starts again.  Exact
// counts are pushed by atomic adds into a record that must start at zero,
// so that form clears the touched records instead.
constexpr int kGenShift = 24;
constexpr int32_t kGenMax = 127;
constexpr int32_t kLevelMask = (1 << kGenShift) - 1;

template <bool EXT>
__global__ void __launch_bounds__(kWgBlock) wg_kernel(WgArgs a) {
  // appends of a level go to counter slot l % 3: the slot of level l + 1 is
  // cleared at the start of level l, two barriers after its last reader
  __shared__ int32_t s_cnt[3], s_wrap;
  __shared__ unsigned long long s_ns, s_rnnz, s_dag;
  const int32_t n = a.n;
  const int t = (int)threadIdx.x, nt = (int)blockDim.x;
  WgVert* __restrict__ V = a.vs + (size_t)blockIdx.x * (size_t)n;
  int2* __restrict__ Q = a.Q + (size_t)blockIdx.x * (size_t)n;
  int32_t* __restrict__ qoff = a.qoff + (size_t)blockIdx.x * (size_t)(n + 2);
  const int32_t* __restrict__ ell = a.ell;
  const int32_t* __restrict__ ci = a.ci;
  int levels = 0;
  // generations need level + 1 to fit below the tag (no BFS is deeper than n - 1)
  const bool gens = EXT && n < kLevelMask - 1;
  int32_t gen = 0;

  for (int64_t si = blockIdx.x; si < a.nsrc; si += gridDim.x) {
    const int32_t src = a.src[si];
    if (gens) {
      if (gen == kGenMax) {
        for (int32_t v = t; v < n; v += nt) V[v] = WgVert{0, 0, 0ull};
        __syncthreads();
        gen = 0;
      }
      ++gen;
    }
    const int32_t tag = gens ? gen << kGenShift : 0;  // records with other tags are not reached
    if (t == 0) {
      V[src].lvl = tag | 1;
      V[src].e = 0;
      V[src].val = EXT ? as_u64(1.0) : 1ull;
      Q[0] = make_int2(src, 0);
      qoff[0] = 0;
      qoff[1] = 1;
      s_cnt[0] = 0;
      s_wrap = 0;
      s_ns = 1 + (a.omega ? (unsigned long long)a.omega[src] : 0ull);
      s_rnnz = (unsigned long long)ell[(size_t)src * kEllWidth];
      s_dag = 0;
    }
    __syncthreads();
    // ---- forward: level l holds records with lvl == l + 1
    int32_t l = 0, e0 = 0, e1 = 1;
    while (e1 > e0) {
      if (t == 0) s_cnt[(l + 1) % 3] = 0;
      int32_t* cnt = &s_cnt[l % 3];
      const int32_t here = tag | (l + 1), next = tag | (l + 2);
      unsigned long long ns = 0, rnnz = 0, dag = 0;
      bool wrap = false;
      for (int32_t i = e0 + t; i < e1; i += nt) {
        const int2 qv = Q[i];
        const int32_t v = qv.x;
        const uint32_t pmask = (uint32_t)qv.y;  // predecessors found when v's count was pulled
        const uint64_t sv = EXT ? 0ull : V[v].val;
        const Adj A = load_adj(ell, v);
        uint32_t smask = 0;
        for_adj(A, ci, [&](int32_t j, int32_t x) {
          if (j < 31 && ((pmask >> j) & 1u)) return;  // on level l - 1: neither claimable nor a successor
          int32_t dx = V[x].lvl;
          bool mine = false;
          // not reached from this source: claim it; a failed swap returns the
          // current word, either this level's claim (stop) or an older one
          // the first read did not see (try again with it)
          while (gens ? (dx & ~kLevelMask) != tag : dx == 0) {
            int32_t expect = dx;
            if (__hip_atomic_compare_exchange_strong(&V[x].lvl, &expect, next, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                     __HIP_MEMORY_SCOPE_WORKGROUP)) {
              mine = true;
              dx = next;
              break;
            }
            dx = expect;
          }
          if (mine) {
            const int32_t pos = atomicAdd(cnt, 1);
            const Adj X = load_adj(ell, x);
            ns += 1 + (a.omega ? (unsigned long long)a.omega[x] : 0ull);
            rnnz += (unsigned long long)X.deg;
            uint32_t pm = 0;
            if (EXT) {
              // the new vertex's count, pulled from its neighbours on level l
              // (its predecessors, remembered for its own claim pass)
              Ext acc = ext_zero();
              for_adj(X, ci, [&](int32_t jx, int32_t u) {
                const WgVert ru = V[u];
                if (ru.lvl == here) {
                  acc = ext_add(acc, Ext{as_f64(ru.val), ru.e});
                  if (jx < 31) pm |= 1u << jx;
                }
              });
              const Ext z = ext_norm(acc);
              V[x].val = as_u64(z.m);
              V[x].e = z.e;
            }
            Q[e1 + pos] = make_int2(x, (int32_t)pm);
          }
          if (dx == next) {
            dag += 1;
            smask |= succ_bit(j);
            if (!EXT) {
              const uint64_t old = atomicAdd((unsigned long long*)&V[x].val, (unsigned long long)sv);
              if (old + sv < old) wrap = true;
            }
          }
        });
        reinterpret_cast<int32_t*>(Q)[2 * (size_t)i + 1] = (int32_t)smask;  // now the successors
      }
      if (ns) atomicAdd(&s_ns, ns);
      if (rnnz) atomicAdd(&s_rnnz, rnnz);
      if (dag) atomicAdd(&s_dag, dag);
      if (wrap) s_wrap = 1;
      __syncthreads();
      const int32_t e2 = e1 + *cnt;
      if (t == 0) qoff[l + 2] = e2;
      ++l;
      e0 = e1;
      e1 = e2;
    }
    __syncthreads();  // qoff of the last level
    const int32_t depth = l - 1;
    levels += l;
    const bool wrapped = s_wrap != 0;
    // ---- backward (skipped when a count wrapped: the host reruns the source
    // extended); only the neighbours the forward pass marked as successors
    double* __restrict__ bc = a.sbc[si];  // the result array of the source's query
    if (!wrapped) {
      const double wt = a.w[si];
      for (int32_t lb = depth; lb >= 1; --lb) {
        const int32_t b0 = qoff[lb], b1 = qoff[lb + 1];
        const int32_t succ = tag | (lb + 2);
        for (int32_t i = b0 + t; i < b1; i += nt) {
          const int2 qw = Q[i];
          const int32_t w = qw.x;
          const uint32_t mask = (uint32_t)qw.y;
          const WgVert me = V[w];
          double acc = 0.0;
          if (mask) {
            const Adj A = load_adj(ell, w);
            for_adj(A, ci, [&](int32_t j, int32_t u) {
              if (!(mask & succ_bit(j))) return;
              const WgVert ru = V[u];
              if (ru.lvl == succ) acc += EXT ? ldexp(as_f64(ru.val), me.e - ru.e) : as_f64(ru.val);
            });
          }
          const double sw = EXT ? as_f64(me.val) : (double)me.val;
          const double delta = sw * acc;
          const double om = a.omega ? (double)a.omega[w] : 0.0;
          V[w].val = as_u64((1.0 + delta + om) / sw);
          const double add = wt * (delta + om);
          if (add != 0.0) atomicAdd(&bc[w], add);
        }
        __syncthreads();
      }
    }
    if (t == 0) {
      if (wrapped) {
        const int32_t k = atomicAdd(a.ovf_count, 1);
        a.ovf_list[k] = src;
      } else if (a.own[si] != 0) {
        atomicAdd(&bc[src], (double)a.own[si] * ((double)s_ns - 1.0) - a.tsub[si]);
      }
      atomicAdd(&a.stats[kStReached], (unsigned long long)qoff[depth + 1]);
      atomicAdd(&a.stats[kStReachedNnz], s_rnnz);
      atomicAdd(&a.stats[kStDag], s_dag);
    }
    // clear what this source touched (generations: the next tag does it)
    if (!gens) {
      const int32_t touched = qoff[depth + 1];
      for (int32_t i = t; i < touched; i += nt) V[Q[i].x] = WgVert{0, 0, 0ull};
    }
    __syncthreads();
  }
  if (t == 0) {
    atomicAdd(&a.stats[kStLevels], (unsigned long long)levels);
    if (blockIdx.x == 0) atomicAdd(&a.stats[kStLaunches], 1ull);
  }
}

hipError_t launch_wg(const WgArgs& a, bool ext, int grid, hipStream_t st) {
  void* args[] = {(void*)&a};
  const void* fn = ext ? (const void*)wg_kernel<true> : (const void*)wg_kernel<false>;
  return hipLaunchKernel(fn, dim3(grid), dim3(kWgBlock), args, 0, st);
}

hipError_t wg_max_grid(int* blocks_per_cu) {
  int a = 0, b = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, (const void*)wg_kernel<false>, kWgBlock, 0);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, (const void*)wg_kernel<true>, kWgBlock, 0);
  *blocks_per_cu = a < b ? a : b;
  return e;
}

}  // namespace bcx
