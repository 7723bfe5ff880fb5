// One source per launch with the paper's active-edge mapping (Sec. 3.1,
// Alg. 2-5): every level's frontier Q[Q_off[l] .. Q_off[l+1]) gets the
// prefix sum CD of its vertices' degrees; then one thread per frontier edge
// finds the vertex owning its edge by binary search in CD.  The forward
// sweep pushes path counts along the edges (atomic test-and-set claims, as
// Alg. 3 made atomic, and atomic 64-bit count adds whose returned value
// exposes a wrap); the backward sweep reuses each level's CD (the paper's
// prefix-sum reuse) with one thread per edge adding psi(v) = (1 + delta(v)) /
// sigma(v) of every successor into an fp64 accumulator of its owner, then a
// pass over the level's vertices turns the accumulator into delta (Eq. (2)).
//
// This is the mapping the paper uses, kept for comparison with the
// wave-aggregated work units of the plain kernel: exact counts only (a
// source whose count wraps is reported and rerun by the plain kernel in
// extended form), no direction switching, no 1-degree weights.  The fp64
// accumulation order depends on scheduling (within the 1e-9 tolerance).
#include "bc_common.h"
#include "bc_kernels.h"

namespace bcx {

constexpr int kScanBlock = 256;

__device__ __forceinline__ int32_t ld32(const int32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Index i in [0, ne) of the last entry with cd[i] <= t (cd non-decreasing, cd[0] = 0).
__device__ __forceinline__ int32_t owner(const int64_t* cd, int32_t ne, int64_t t) {
  int32_t lo = 0, hi = ne;  // first index with cd > t lies in (lo, hi]
  while (hi - lo > 1) {
    const int32_t mid = (lo + hi) >> 1;
    if (cd[mid] <= t) lo = mid;
    else hi = mid;
  }
  return lo;
}

__global__ void __launch_bounds__(kScanBlock) scan_kernel(ScanArgs a) {
  __shared__ int64_t s_scan[kScanBlock];
  __shared__ int64_t s_off;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nth = (int64_t)gridDim.x * blockDim.x;
  const int lane = lane_id();
  const int32_t n = a.n;
  const int32_t* __restrict__ rp = a.rp;
  const int32_t* __restrict__ ci = a.ci;
  int32_t* __restrict__ d = a.d;
  uint64_t c_reached = 0, c_rnnz = 0, c_dag = 0;
  bool wrapped = false;

  for (int64_t i = tid; i < n; i += nth) {
    const bool s = i == a.src;
    d[i] = s ? 0 : -1;
    a.sig[i] = s ? 1ull : 0ull;
    a.acc[i] = 0.0;
  }
  if (tid == 0) {
    // the launch's control words start clear: they are written here, before
    // the first barrier, because every workgroup reads the overflow flag
    // after the forward sweep with no barrier before the epilogue
    *a.ovf_now = 0;
    a.Q[0] = a.src;
    a.qoff[0] = 0;
    a.qoff[1] = 1;
    a.qoff[2] = 0;  // append counter of level 1
    c_reached = 1;
    c_rnnz = (uint64_t)(rp[a.src + 1] - rp[a.src]);
  }
  if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;

  // ---- forward: per level, CD over the frontier, then one thread per edge
  int32_t l = 0;
  while (true) {
    const int32_t e0 = ld32(&a.qoff[l]), e1 = ld32(&a.qoff[l + 1]);
    const int32_t ne = e1 - e0;
    if (ne == 0) break;
    // CD, step 1: each workgroup scans its contiguous chunk of the frontier
    const int32_t per = (ne + (int32_t)gridDim.x - 1) / (int32_t)gridDim.x;
    const int32_t c0 = e0 + min(ne, (int32_t)blockIdx.x * per), c1 = e0 + min(ne, ((int32_t)blockIdx.x + 1) * per);
    int64_t running = 0;
    for (int32_t base = c0; base < c1; base += kScanBlock) {
      const int32_t i = base + (int32_t)threadIdx.x;
      const int64_t x = i < c1 ? (int64_t)(rp[a.Q[i] + 1] - rp[a.Q[i]]) : 0;
      s_scan[threadIdx.x] = x;
      __syncthreads();
      for (int o = 1; o < kScanBlock; o <<= 1) {  // inclusive Hillis-Steele scan
        const int64_t y = threadIdx.x >= (unsigned)o ? s_scan[threadIdx.x - o] : 0;
        __syncthreads();
        s_scan[threadIdx.x] += y;
        __syncthreads();
      }
      if (i < c1) a.cd[i] = running + s_scan[threadIdx.x] - x;
      running += s_scan[kScanBlock - 1];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.bsum[blockIdx.x] = running;
    if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;
    // CD, step 2: add the totals of the chunks before this one
    {
      int64_t part = 0;
      for (unsigned b = threadIdx.x; b < blockIdx.x; b += kScanBlock) part += a.bsum[b];
      s_scan[threadIdx.x] = part;
      __syncthreads();
      for (int o = kScanBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s_scan[threadIdx.x] += s_scan[threadIdx.x + o];
        __syncthreads();
      }
      if (threadIdx.x == 0) {
        s_off = s_scan[0];
        if (blockIdx.x == gridDim.x - 1) a.tot[l] = s_scan[0] + a.bsum[blockIdx.x];
      }
      __syncthreads();
    }
    for (int32_t i = c0 + (int32_t)threadIdx.x; i < c1; i += kScanBlock) a.cd[i] += s_off;
    if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;
    // expand: one thread per frontier edge
    const int64_t T = a.tot[l];
    const int32_t nl = l + 1;
    for (int64_t base = tid - lane; base < T; base += nth) {
      const int64_t t = base + lane;
      bool claimed = false;
      int32_t w = 0;
      if (t < T) {
        const int32_t i = owner(a.cd + e0, ne, t);
        const int32_t v = a.Q[e0 + i];
        w = ci[rp[v] + (int32_t)(t - a.cd[e0 + i])];
        int32_t dw = d[w];
        if (dw == -1) {
          int32_t expect = -1;
          claimed = __hip_atomic_compare_exchange_strong(&d[w], &expect, nl, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
          dw = claimed ? nl : expect;
        }
        if (dw == nl) {
          const uint64_t sv = a.sig[v];
          const uint64_t old = atomicAdd((unsigned long long*)&a.sig[w], (unsigned long long)sv);
          if (old + sv < old) wrapped = true;
          c_dag += 1;
        }
      }
      // the wave's claimed vertices join the next frontier (one reservation per wave)
      const uint64_t cm = ballot(claimed);
      if (cm) {
        int32_t pos = 0;
        if (lane == 0) pos = atomicAdd(&a.qoff[nl + 1], __popcll(cm));
        pos = __shfl(pos, 0, kWave);
        if (claimed) {
          a.Q[e1 + pos + lanes_below(cm)] = w;
          c_reached += 1;
          c_rnnz += (uint64_t)(rp[w + 1] - rp[w]);
        }
      }
    }
    if (ballot(wrapped) != 0 && lane == 0) atomicOr(a.ovf_now, 1);
    if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;
    // qoff[nl + 1] counted the appends: turn it into the next level's end
    if (tid == 0) {
      a.qoff[nl + 1] += e1;
      if (nl + 2 <= n + 2) a.qoff[nl + 2] = 0;
    }
    if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;
    l = nl;
  }
  const int32_t depth = l - 1;
  {
    const uint64_t r0 = wave_sum_u64(c_reached), r1 = wave_sum_u64(c_rnnz), r2 = wave_sum_u64(c_dag);
    if (lane == 0) {
      if (r0) atomicAdd(&a.stats[kStReached], (unsigned long long)r0);
      if (r1) atomicAdd(&a.stats[kStReachedNnz], (unsigned long long)r1);
      if (r2) atomicAdd(&a.stats[kStDag], (unsigned long long)r2);
    }
  }
  if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;
  const bool overflowed = ld32(a.ovf_now) != 0;

  // ---- backward: the deepest level's psi, then level by level with CD reused
  if (!overflowed) {
    for (int32_t lb = depth; lb >= 1; --lb) {
      const int32_t e0 = a.qoff[lb], e1 = a.qoff[lb + 1];
      const int32_t ne = e1 - e0;
      if (lb < depth) {
        const int64_t T = a.tot[lb];
        for (int64_t t = tid; t < T; t += nth) {
          const int32_t i = owner(a.cd + e0, ne, t);
          const int32_t w = a.Q[e0 + i];
          const int32_t v = ci[rp[w] + (int32_t)(t - a.cd[e0 + i])];
          if (d[v] == lb + 1) atomicAdd(&a.acc[w], a.psi[v]);
        }
        if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;
      }
      for (int64_t i = tid; i < ne; i += nth) {
        const int32_t w = a.Q[e0 + i];
        const double sw = (double)a.sig[w];
        const double delta = sw * a.acc[w];
        a.psi[w] = (1.0 + delta) / sw;
        a.bc[w] += a.weight * delta;
        if (a.delta_out) a.delta_out[w] = delta;
      }
      if (!grid_barrier(a.bar, a.bar_limit, a.err)) return;
    }
  }

  // ---- epilogue: report a wrapped source (the next launch clears the
  // control words itself: a workgroup may still be about to read them here)
  if (tid == 0) {
    if (overflowed) {
      const int32_t k = atomicAdd(a.ovf_count, 1);
      a.ovf_list[k] = a.src;
    }
    atomicAdd(&a.stats[kStLevels], (unsigned long long)(depth + 1));
    atomicAdd(&a.stats[kStLaunches], 1ull);
  }
}

hipError_t launch_scan(const ScanArgs& a, int grid, hipStream_t st) {
  void* args[] = {(void*)&a};
  return hipLaunchKernel((const void*)scan_kernel, dim3(grid), dim3(kScanBlock), args, 0, st);
}

hipError_t scan_max_grid(int* blocks_per_cu) {
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, (const void*)scan_kernel, kScanBlock, 0);
}

}  // namespace bcx
