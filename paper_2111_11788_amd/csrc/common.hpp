// Internal definitions shared by the HIP kernels and the host engine.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace mlmc {

// Entries per sample of the grid layout: (n+1) planes of n*n nodes (plane
// k = n and the i = 0 / j = 0 positions hold the zero boundary), plus n+1
// trailing zeros so that every 27-point neighbourhood of an interior node
// stays inside the sample's block, rounded up to 64 entries (256/512 B).
inline size_t grid_stride(int n) {
  size_t s = (size_t)(n + 1) * n * n + n + 1;
  return (s + 63) / 64 * 64;
}
inline size_t elem_count(int n) { return (size_t)n * n * n; }

// Workgroups are dispatched round-robin over the 8 XCDs by linear id; this
// maps the dispatch id to a logical id so that each XCD receives a contiguous
// range of logical blocks (neighbouring tiles then share that XCD's L2).
__device__ __forceinline__ uint32_t xcd_remap(uint32_t lin, uint32_t total) {
  const uint32_t per = total >> 3, rem = total & 7u;
  const uint32_t xcd = lin & 7u, idx = lin >> 3;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

constexpr int kBlock = 256;          // threads per workgroup of the grid kernels

}  // namespace mlmc
