// Static device scratch of the entry points that allocate nothing (for
// callers that cannot allocate: code under graph capture, tight serving loops).
// The array lives in the code object of every GPU the library runs on and is
// held until the process ends.  Host code never passes the array's name to a
// kernel (that is a host-side stand-in, not a device address): at context
// creation the device address of the current device's copy is looked up once
// with hipGetSymbolAddress and kept per device, and only that address is used.
#include <mutex>

#include "common.hpp"
#include "grid.hpp"
#include "kernels.hpp"

namespace mlmc {
namespace {

constexpr size_t kScratchBytes = (size_t)16 << 20;   // 16 MiB per GPU
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

size_t noalloc_scratch_bytes() { return kScratchBytes; }

hipError_t noalloc_scratch_init(int* device, void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  if (device) *device = dev;
  if (out) *out = g_scratch_ptr[dev];
  return hipSuccess;
}

size_t qoi_scratch_bytes(int n, int B) { return (size_t)B * sgeom<double>(n).chunks * sizeof(double); }

hipError_t launch_qoi_scratch(int n, int B, int qoi, const double* u, double* q, void* scratch_dev, hipStream_t st) {
  if (!scratch_dev || B < 1 || qoi_scratch_bytes(n, B) > kScratchBytes) return hipErrorInvalidValue;
  // the partial sums of each sample in the scratch (every entry the reduction
  // reads is written first, so nothing has to start at zero)
  SolveState s{};
  s.partial = static_cast<double*>(scratch_dev);
  s.pstride = sgeom<double>(n).chunks;
  uint32_t np = 0;
  const hipError_t e = launch_qoi_partial(n, B, qoi, u, s, &np, st, false);
  if (e != hipSuccess) return e;
  return launch_reduce(B, RED_STORE, 0.0, np, s, q, st);
}

}  // namespace mlmc
