// Pause model (Sec. 5.1, "A benchmarking example"): the device side of a
// model evaluation that only waits.  One 64-thread workgroup per occupied
// workgroup slot waits a given number of ticks of the device wall clock
// (constant rate, independent of the shader clock), sleeping between reads.
#include "common.hpp"
#include "kernels.hpp"

namespace mlmc {
namespace {

__global__ void __launch_bounds__(64) k_pause_spin(const uint32_t* __restrict__ spin, uint64_t* __restrict__ meas,
                                                   int nwg) {
  const int w = (int)blockIdx.x;
  if (w >= nwg) return;
  const uint64_t t = spin[w];
  const uint64_t t0 = wall_clock64();
  uint64_t now = t0;
  // a read-sleep round takes far more than one tick, so the cap only bounds
  // the loop should the clock not advance
  const uint64_t cap = 2 * t + 1024;
  for (uint64_t it = 0; now - t0 < t && it < cap; ++it) {
    __builtin_amdgcn_s_sleep(1);
    now = wall_clock64();
  }
  if (threadIdx.x == 0) meas[w] += now - t0;
}

}  // namespace

hipError_t launch_pause_spin(const uint32_t* spin, uint64_t* meas, int nwg, hipStream_t st) {
  if (nwg <= 0) return hipSuccess;
  k_pause_spin<<<dim3((unsigned)nwg), dim3(64), 0, st>>>(spin, meas, nwg);
  return hipGetLastError();
}

}  // namespace mlmc
