// The entry point that allocates nothing: bc_compute_noalloc runs the
// one-source-per-launch form with its workspace in a fixed device array
// (`scratch`) that the code object brings with it, so the call makes no
// device allocation at all.  The array's device address is looked up once
// per device (hipGetSymbolAddress) when a context is created there, or on
// the first call on that device, and only that address is ever handed to
// kernels, fills or copies: in host code the array's name is not a device
// address.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bc.h"
#include "bc_api_internal.h"

namespace bcx {

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

struct DevScratch {
  void* ptr = nullptr;  // device address of `scratch` on this device
  std::mutex call;      // calls on one device run one at a time
};
std::mutex g_init_mu;
DevScratch g_dev[kMaxDevices];

__global__ void zero_words(uint64_t* p, size_t words) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride) p[i] = 0;
}

}  // namespace

hipError_t noalloc_scratch_init(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_init_mu);
  if (g_dev[device].ptr) return hipSuccess;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));  // the calling thread's current device
  if (e != hipSuccess) return e;
  g_dev[device].ptr = p;
  return hipSuccess;
}

// Clears `bytes` (a multiple of 8, 8-aligned) with a fill kernel rather than
// a memset node, so that the call stays usable under stream capture.
hipError_t zero_async(void* p, size_t bytes, hipStream_t st) {
  const size_t words = bytes / 8;
  if (words == 0) return hipSuccess;
  const int block = 256;
  const int grid = (int)std::min<size_t>((words + block - 1) / block, 1024);
  zero_words<<<grid, block, 0, st>>>((uint64_t*)p, words);
  return hipGetLastError();
}

}  // namespace bcx

using namespace bcx;

extern "C" {

bc_status bc_compute_noalloc(bc_graph* g, const int32_t* sources, int64_t k, const bc_compute_opts* opts,
                             void* stream, bc_run_stats* stats) {
  if (!g) return fail(BC_E_INVALID_ARG, "null graph");
  const int dev = graph_device(g);
  if (dev < 0 || dev >= kMaxDevices) return fail(BC_E_INVALID_ARG, "device id beyond the library's table");
  if (hipSetDevice(dev) != hipSuccess) return fail(BC_E_DEVICE, "hipSetDevice failed");
  hipError_t e = noalloc_scratch_init(dev);
  if (e != hipSuccess) return fail(BC_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  std::lock_guard<std::mutex> lk(g_dev[dev].call);
  return compute_noalloc(g, sources, k, opts, g_dev[dev].ptr, kNoAllocScratchBytes, (hipStream_t)stream, stats);
}

}  // extern "C"
