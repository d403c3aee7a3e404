// Device-side helpers for the grid-layout kernels: vector types and the
// thread geometry of the z-marching stencil engine and of the streaming
// kernels.  Host code uses the same geometry to size partial-sum buffers.
#pragma once

#include "common.hpp"

namespace mlmc {

// Values per thread along x in the z-marching stencil kernels: one 16-byte
// vector of the row segment (4 floats or 2 doubles).
template <class T>
struct ZV { static constexpr int V = 16 / (int)sizeof(T); };

// Geometry of a z-marching launch on an n^3 grid for B samples.
// A thread owns V consecutive nodes i0 .. i0+V-1 of row j and marches over a
// chunk of planes; a workgroup holds `rows` rows of one sample and one plane
// chunk.  Workgroups of a sample are numbered rb + row_blocks * zb.
struct ZGeom {
  int n = 0;
  int G = 0;            // vector groups per row (n / V)
  int rows = 0;         // rows per workgroup
  int row_blocks = 0;   // workgroups per plane chunk
  int zc = 1;           // plane chunks
  int zlen = 0;         // planes per chunk
  int threads = 256;    // threads per workgroup
  __host__ __device__ uint32_t parts() const { return (uint32_t)row_blocks * zc; }
};

// waves of a launch from which the samples' planes are no longer split
constexpr long kFillWaves = 8192;

template <class T>
inline ZGeom zgeom(int n, int B) {
  ZGeom g;
  constexpr int V = ZV<T>::V;
  g.n = n;
  g.G = n / V;
  if (g.G < 1) {   // a row narrower than one vector: no z-march geometry (callers check G)
    g.rows = 0;
    g.row_blocks = 0;
    g.zlen = 0;
    return g;
  }
  const int rowthreads = (n - 1) * g.G;
  g.threads = rowthreads >= 256 ? 256 : ((rowthreads + 63) / 64) * 64;
  g.rows = g.threads / g.G;
  if (g.rows < 1) g.rows = 1;
  g.row_blocks = (n - 1 + g.rows - 1) / g.rows;
  // split the planes when there are few samples, so the chip has >= ~8 waves per SIMD
  const long waves = (long)B * g.row_blocks * (g.threads / 64);
  int zc = 1;
  while (waves * zc < kFillWaves && (n - 1) / (zc * 2) >= 8) zc *= 2;
  g.zc = zc;
  g.zlen = (n - 1 + zc - 1) / zc;
  return g;
}

// The geometry of zgeom with `rows` rows per workgroup instead of the most
// that fit (rows >= 1, same thread count).
template <class T>
inline ZGeom zgeom_rows(int n, int B, int rows) {
  ZGeom g = zgeom<T>(n, B);
  if (g.G < 1 || rows < 1) return g;
  g.rows = rows;
  g.row_blocks = (n - 1 + rows - 1) / rows;
  const long waves = (long)B * g.row_blocks * (g.threads / 64);
  int zc = 1;
  while (waves * zc < kFillWaves && (n - 1) / (zc * 2) >= 8) zc *= 2;
  g.zc = zc;
  g.zlen = (n - 1 + zc - 1) / zc;
  return g;
}

// Tiles of the corrected smoothing step with its operand formed on the fly,
// which stages two rows more than it computes: with rows of 16 lanes (G = 16)
// a 16-row tile stages 18 rows with 16 rows of threads, and the wave that
// takes the extra rows (each formed from the kappa ring and the coarse
// correction) runs a second pass per plane while the others wait at the
// plane's barrier.  14-row tiles stage 16 rows in one pass at about the same
// total work (5 tiles of 63 rows instead of 4): 9.7 -> 9.4 ms per 64^3 x 1024
// step.
template <class T>
inline ZGeom zgeom_tall(int n, int B) {
  const ZGeom g = zgeom<T>(n, B);
  // only where the shorter tiles add at most a quarter more tiles (63 rows:
  // 5 instead of 4; not 31 rows: 3 instead of 2)
  const bool fits = 4 * ((n - 1 + 13) / 14) <= 5 * ((n - 1 + 15) / 16);
  return g.G == 16 && g.threads == 256 && g.rows == 16 && fits ? zgeom_rows<T>(n, B, 14) : g;
}

// Streaming kernels cover the flat range [n^2, n^3) of every sample (planes
// 1..n-1, boundary positions included: they hold zero in every vector) in
// 16-byte vectors; `chunks` workgroups per sample.
struct SGeom {
  int n = 0;
  uint32_t vecs = 0;    // 16-byte vectors per sample in the range
  uint32_t chunks = 0;  // workgroups per sample
};

template <class T>
inline SGeom sgeom(int n) {
  SGeom g;
  g.n = n;
  const size_t elems = (size_t)(n - 1) * n * n;
  g.vecs = (uint32_t)(elems * sizeof(T) / 16);
  uint32_t c = (uint32_t)((g.vecs + 256 * 8 - 1) / (256 * 8));   // ~8 vectors per thread
  if (c > 64) c = 64;
  if (c < 1) c = 1;
  g.chunks = c;
  return g;
}

// Largest number of per-sample partial sums any kernel writes for a mesh.
inline uint32_t max_parts(int n, int B) {
  uint32_t m = sgeom<float>(n).chunks;
  if (sgeom<double>(n).chunks > m) m = sgeom<double>(n).chunks;
  if (n >= 4 && zgeom<float>(n, B).parts() > m) m = zgeom<float>(n, B).parts();
  if (zgeom<double>(n, B).parts() > m) m = zgeom<double>(n, B).parts();
  if (n >= 4 && zgeom_tall<float>(n, B).parts() > m) m = zgeom_tall<float>(n, B).parts();
  if (zgeom_tall<double>(n, B).parts() > m) m = zgeom_tall<double>(n, B).parts();
  return m;
}

}  // namespace mlmc
