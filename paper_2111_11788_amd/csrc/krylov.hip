// Batched preconditioned conjugate gradients: vector updates, dot products
// and the per-sample scalar recurrences (alpha, beta, convergence), plus the
// QoI reduction.  Vectors may be fp32 or fp64; every dot product and every
// scalar is accumulated in fp64.
//
// The streaming kernels walk the flat range of planes 1..n-1 of each sample
// (boundary positions included: they hold zero in every vector, so updates
// keep them zero) in 16-byte vectors, several per thread.
//
// Reductions are deterministic and per sample: each workgroup (one chunk of
// one sample) reduces its values in a fixed tree and writes one partial sum;
// k_reduce then sums a sample's partials in a fixed order.  A sample's scalars
// therefore never depend on which other samples share the batch.
#include "common.hpp"
#include "grid.hpp"
#include "kernels.hpp"

namespace mlmc {
namespace {

__device__ __forceinline__ double block_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __shared__ double wsum[kBlock / 64];
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) t += wsum[w];
  }
  return t;
}

template <class T, int V>
struct Vec {
  typedef T type __attribute__((ext_vector_type(V)));
};

// Range of 16-byte vectors [lo, hi) of workgroup chunk c, and the sample.
struct Span {
  uint32_t b, c;
  size_t lo, hi;
};

__device__ __forceinline__ Span span_of(const SGeom& g) {
  const uint32_t logical = xcd_remap(blockIdx.x, gridDim.x);
  Span s;
  s.b = logical / g.chunks;
  s.c = logical - s.b * g.chunks;
  const uint32_t per = (g.vecs + g.chunks - 1) / g.chunks;
  s.lo = (size_t)s.c * per;
  s.hi = s.lo + per;
  if (s.hi > g.vecs) s.hi = g.vecs;
  return s;
}

// x += alpha p, r -= alpha q, partial sums of r . r
template <class T>
__global__ void __launch_bounds__(kBlock) k_pcg_update(SGeom g, size_t stride, T* __restrict__ x,
                                                       const T* __restrict__ p, T* __restrict__ r,
                                                       const T* __restrict__ q, SolveState st) {
  constexpr int V = 16 / sizeof(T);
  typedef typename Vec<T, V>::type vt;
  const Span sp = span_of(g);
  if (!st.active[sp.b]) return;
  const size_t base = (size_t)sp.b * stride + (size_t)g.n * g.n;
  vt* xv = reinterpret_cast<vt*>(x + base);
  const vt* pv = reinterpret_cast<const vt*>(p + base);
  vt* rv = reinterpret_cast<vt*>(r + base);
  const vt* qv = reinterpret_cast<const vt*>(q + base);
  const T a = (T)st.alpha[sp.b];
  double acc = 0.0;
  for (size_t t = sp.lo + threadIdx.x; t < sp.hi; t += kBlock) {
    xv[t] = xv[t] + a * pv[t];
    const vt rn = rv[t] - a * qv[t];
    rv[t] = rn;
#pragma unroll
    for (int c = 0; c < V; ++c) acc += (double)rn[c] * (double)rn[c];
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) st.partial[(size_t)sp.b * st.pstride + sp.c] = acc;
}

// r -= alpha q, partial sums of r . r (the iterate is updated by the fused
// direction step one iteration later)
template <class T>
__global__ void __launch_bounds__(kBlock) k_pcg_rupdate(SGeom g, size_t stride, T* __restrict__ r,
                                                        const T* __restrict__ q, SolveState st) {
  constexpr int V = 16 / sizeof(T);
  typedef typename Vec<T, V>::type vt;
  const Span sp = span_of(g);
  if (!st.active[sp.b]) return;
  const size_t base = (size_t)sp.b * stride + (size_t)g.n * g.n;
  vt* rv = reinterpret_cast<vt*>(r + base);
  const vt* qv = reinterpret_cast<const vt*>(q + base);
  const T a = (T)st.alpha[sp.b];
  double acc = 0.0;
  for (size_t t = sp.lo + threadIdx.x; t < sp.hi; t += kBlock) {
    const vt rn = rv[t] - a * qv[t];
    rv[t] = rn;
#pragma unroll
    for (int c = 0; c < V; ++c) acc += (double)rn[c] * (double)rn[c];
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) st.partial[(size_t)sp.b * st.pstride + sp.c] = acc;
}

// the update a fused-direction solve still owes its iterate: x += alpha p
// with p the sample's current direction (buffer pstate & 1), on samples with
// mask[b] that took at least one step (pstate bit 1 clear); x = alpha p when
// the iterate was never written (pstate bit 2: a fresh correction)
template <class T>
__global__ void __launch_bounds__(kBlock) k_pcg_finish(SGeom g, size_t stride, T* __restrict__ x,
                                                       const T* __restrict__ p0, const T* __restrict__ p1,
                                                       const int* __restrict__ mask, SolveState st) {
  constexpr int V = 16 / sizeof(T);
  typedef typename Vec<T, V>::type vt;
  const Span sp = span_of(g);
  if (!mask[sp.b]) return;
  const int ps = st.pstate[sp.b];
  if (ps & 2) return;
  const size_t base = (size_t)sp.b * stride + (size_t)g.n * g.n;
  vt* xv = reinterpret_cast<vt*>(x + base);
  const vt* pv = reinterpret_cast<const vt*>(((ps & 1) ? p1 : p0) + base);
  const T a = (T)st.alpha[sp.b];
  if (ps & 4) {
    for (size_t t = sp.lo + threadIdx.x; t < sp.hi; t += kBlock) xv[t] = a * pv[t];
  } else {
    for (size_t t = sp.lo + threadIdx.x; t < sp.hi; t += kBlock) xv[t] = xv[t] + a * pv[t];
  }
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_dot(SGeom g, size_t stride, const T* __restrict__ a,
                                                const T* __restrict__ b, SolveState st) {
  constexpr int V = 16 / sizeof(T);
  typedef typename Vec<T, V>::type vt;
  const Span sp = span_of(g);
  if (!st.active[sp.b]) return;
  const size_t base = (size_t)sp.b * stride + (size_t)g.n * g.n;
  const vt* av = reinterpret_cast<const vt*>(a + base);
  const vt* bv = reinterpret_cast<const vt*>(b + base);
  double acc = 0.0;
  for (size_t t = sp.lo + threadIdx.x; t < sp.hi; t += kBlock) {
    const vt x = av[t], y = bv[t];
#pragma unroll
    for (int c = 0; c < V; ++c) acc += (double)x[c] * (double)y[c];
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) st.partial[(size_t)sp.b * st.pstride + sp.c] = acc;
}

// p = z + beta p
template <class T>
__global__ void __launch_bounds__(kBlock) k_pcg_direction(SGeom g, size_t stride, const T* __restrict__ z,
                                                          T* __restrict__ p, SolveState st) {
  constexpr int V = 16 / sizeof(T);
  typedef typename Vec<T, V>::type vt;
  const Span sp = span_of(g);
  if (!st.active[sp.b]) return;
  const size_t base = (size_t)sp.b * stride + (size_t)g.n * g.n;
  const vt* zv = reinterpret_cast<const vt*>(z + base);
  vt* pv = reinterpret_cast<vt*>(p + base);
  const T be = (T)st.beta[sp.b];
  for (size_t t = sp.lo + threadIdx.x; t < sp.hi; t += kBlock) pv[t] = zv[t] + be * pv[t];
}

// p = z
template <class T>
__global__ void __launch_bounds__(kBlock) k_copy(SGeom g, size_t stride, const T* __restrict__ z, T* __restrict__ p,
                                                 SolveState st) {
  constexpr int V = 16 / sizeof(T);
  typedef typename Vec<T, V>::type vt;
  const Span sp = span_of(g);
  if (!st.active[sp.b]) return;
  const size_t base = (size_t)sp.b * stride + (size_t)g.n * g.n;
  const vt* zv = reinterpret_cast<const vt*>(z + base);
  vt* pv = reinterpret_cast<vt*>(p + base);
  for (size_t t = sp.lo + threadIdx.x; t < sp.hi; t += kBlock) pv[t] = zv[t];
}

// x64 += d32 (4 values per step)
__global__ void __launch_bounds__(kBlock) k_add_correction(SGeom g, size_t stride, double* __restrict__ x,
                                                           const float* __restrict__ d, SolveState st) {
  typedef Vec<double, 2>::type d2;
  typedef Vec<float, 4>::type f4;
  const Span sp = span_of(g);
  if (!st.active[sp.b]) return;
  const size_t base = (size_t)sp.b * stride + (size_t)g.n * g.n;
  d2* xv = reinterpret_cast<d2*>(x + base);
  const f4* dv = reinterpret_cast<const f4*>(d + base);
  for (size_t t = sp.lo + threadIdx.x; t < sp.hi; t += kBlock) {
    const f4 dd = dv[t];
    d2 a = xv[2 * t], b = xv[2 * t + 1];
    a.x += (double)dd.x; a.y += (double)dd.y;
    b.x += (double)dd.z; b.y += (double)dd.w;
    xv[2 * t] = a;
    xv[2 * t + 1] = b;
  }
}

// r32 = (float) r64 (4 values per step)
__global__ void __launch_bounds__(kBlock) k_demote(SGeom g, size_t stride, const double* __restrict__ r,
                                                   float* __restrict__ r32, SolveState st) {
  typedef Vec<double, 2>::type d2;
  typedef Vec<float, 4>::type f4;
  const Span sp = span_of(g);
  if (!st.active[sp.b]) return;
  const size_t base = (size_t)sp.b * stride + (size_t)g.n * g.n;
  const d2* rv = reinterpret_cast<const d2*>(r + base);
  f4* ov = reinterpret_cast<f4*>(r32 + base);
  for (size_t t = sp.lo + threadIdx.x; t < sp.hi; t += kBlock) {
    const d2 a = rv[2 * t], b = rv[2 * t + 1];
    f4 o;
    o.x = (float)a.x; o.y = (float)a.y; o.z = (float)b.x; o.w = (float)b.y;
    ov[t] = o;
  }
}

// interior positions := value (boundary positions of the range stay 0)
template <class T>
__global__ void __launch_bounds__(kBlock) k_fill_interior(SGeom g, size_t stride, T* __restrict__ v, T value,
                                                          const int* __restrict__ active) {
  constexpr int V = 16 / sizeof(T);
  typedef typename Vec<T, V>::type vt;
  const Span sp = span_of(g);
  if (active && !active[sp.b]) return;
  const int n = g.n;
  const size_t n2 = (size_t)n * n;
  vt* out = reinterpret_cast<vt*>(v + (size_t)sp.b * stride + n2);
  const int lg = __builtin_ctz((unsigned)n);   // n is a power of two
  for (size_t t = sp.lo + threadIdx.x; t < sp.hi; t += kBlock) {
    vt o;
#pragma unroll
    for (int c = 0; c < V; ++c) {
      const size_t pos = t * V + c;      // offset from plane 1
      const int i = (int)(pos & (n - 1)), j = (int)((pos >> lg) & (n - 1));
      o[c] = (i != 0 && j != 0) ? value : T(0);
    }
    out[t] = o;
  }
}

// QoI weights: domain average h^3 at every node (k_qoi_partial); subcube
// [1/4,3/4]^3 average h^3 prod_d c(i_d) with c = 2 strictly inside, 1 on the
// faces, 0 outside (the number of subcube elements touching the node along
// each axis; k_qoi_subcube).
__global__ void __launch_bounds__(kBlock) k_qoi_partial(SGeom g, size_t stride, const double* __restrict__ u,
                                                        SolveState st, bool masked) {
  const Span sp = span_of(g);
  if (masked && !st.active[sp.b]) return;
  const size_t n2 = (size_t)g.n * g.n;
  const double* ub = u + (size_t)sp.b * stride + n2;
  const double h = 1.0 / g.n, h3 = h * h * h;
  typedef Vec<double, 2>::type d2;
  const d2* uv = reinterpret_cast<const d2*>(ub);
  double acc = 0.0;
  for (size_t t = sp.lo + threadIdx.x; t < sp.hi; t += kBlock) {
    const d2 u2 = uv[t];
    acc += h3 * u2.x;   // boundary positions hold 0
    acc += h3 * u2.y;
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) st.partial[(size_t)sp.b * st.pstride + sp.c] = acc;
}

// The subcube QoI reads only the nodes its weights cover: the box
// [n/4, 3n/4]^3 of m^3 nodes (m = n/2 + 1), in `chunks` workgroups per sample,
// x fastest; the weights as above.
__global__ void __launch_bounds__(kBlock) k_qoi_subcube(int n, uint32_t chunks, size_t stride,
                                                        const double* __restrict__ u, SolveState st, bool masked) {
  const uint32_t logical = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t b = logical / chunks, c = logical - b * chunks;
  if (masked && !st.active[b]) return;
  const int lo = n / 4, hi = 3 * n / 4;
  const uint32_t m = (uint32_t)(hi - lo + 1), total = m * m * m;
  const uint32_t per = (total + chunks - 1) / chunks;
  const uint32_t t0 = c * per, t1 = t0 + per < total ? t0 + per : total;
  const double* ub = u + (size_t)b * stride;
  const double h = 1.0 / n, h3 = h * h * h;
  auto cw = [&](int x) { return (x == lo || x == hi) ? 1.0 : 2.0; };
  double acc = 0.0;
  for (uint32_t t = t0 + threadIdx.x; t < t1; t += kBlock) {
    const uint32_t a = t / m, i = t - a * m;
    const uint32_t k = a / m, j = a - k * m;
    const int x = lo + (int)i, y = lo + (int)j, z = lo + (int)k;
    acc += h3 * cw(x) * cw(y) * cw(z) * ub[(size_t)z * n * n + (size_t)y * n + x];
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) st.partial[(size_t)b * st.pstride + c] = acc;
}

// one workgroup per sample: fixed-order sum of its partials, then the scalar op
__global__ void __launch_bounds__(kBlock) k_reduce(int op, double tol2, uint32_t nparts, SolveState st, double* out) {
  const int b = blockIdx.x;
  if (op != RED_STORE && st.active && !st.active[b]) return;
  const double* p = st.partial + (size_t)b * st.pstride;
  double v = 0.0;
  for (uint32_t c = threadIdx.x; c < nparts; c += kBlock) v += p[c];
  v = block_sum(v);
  if (threadIdx.x != 0) return;
  switch (op) {
    case RED_BB: st.bb[b] = v; break;
    case RED_ALPHA: st.alpha[b] = st.rz[b] / v; st.iters[b] += 1; break;
    case RED_RR:
      st.rr[b] = v;
      if (v <= tol2 * st.bb[b] || !isfinite(v)) st.active[b] = 0;
      break;
    case RED_RZ_INIT: st.rz[b] = v; break;
    case RED_BETA: st.beta[b] = v / st.rz[b]; st.rz[b] = v; break;
    case RED_BETA_DIR:
      if (!(st.pstate[b] & 2)) st.beta[b] = v / st.rz[b];
      st.rz[b] = v;
      break;
    case RED_ALPHA_DIR: {
      // next direction buffer; first cleared; the fresh bit survives the first
      // step (which does not touch x) and is cleared by the one that writes x
      const int ps = st.pstate[b];
      st.alpha[b] = st.rz[b] / v;
      st.iters[b] += 1;
      st.pstate[b] = ((ps & 1) ^ 1) | ((ps & 2) ? (ps & 4) : 0) | (ps & 8);
      break;
    }
    case RED_RR_INNER:
      st.rr[b] = v;
      if (v <= tol2 * st.bb[b] || !isfinite(v)) st.phase[b] = PHASE_TRANSITION;
      break;
    case RED_RR_UPD:
    case RED_RR_INNER_UPD: {
      // the residual just written by the fused update is in the other buffer
      const int ps = st.pstate[b];
      if (!(ps & 2)) st.pstate[b] = ps ^ 8;
      st.rr[b] = v;
      if (v <= tol2 * st.bb[b] || !isfinite(v)) {
        st.active[b] = 0;
        if (op == RED_RR_INNER_UPD) st.phase[b] = PHASE_TRANSITION;
      }
      break;
    }
    case RED_RR_OUTER:
      st.rr[b] = v;
      st.phase[b] = (v <= tol2 * st.bb[b] || !isfinite(v)) ? PHASE_DONE : PHASE_RESTART;
      break;
    default: out[b] = v; break;
  }
}

// One Welford push of y into (n, mean, m2)
__device__ __forceinline__ void welford_push(double& n, double& mean, double& m2, double y) {
#pragma clang fp contract(off)
  n += 1.0;
  const double d = y - mean;
  mean += d / n;
  m2 += d * (y - mean);
}

// Level statistics fold, one workgroup per job (see launch_level_stats).  A
// tile of up to kTile values is compacted to its finite values (in order) in
// LDS; thread 0 continues the incomplete block with the first of them, one
// thread per complete block reduces it, thread 0 merges the blocks in order
// and starts the next incomplete block with the rest.
constexpr int kStatsTile = 16 * kBlock;
__global__ void __launch_bounds__(kBlock) k_level_stats(StatsJobs jobs) {
  const StatsJob J = jobs.j[blockIdx.x];
  __shared__ double buf[kStatsTile];
  __shared__ int cnt[kBlock];
  __shared__ double bmean[kStatsTile / kStatsBlock], bm2[kStatsTile / kStatsBlock];
  __shared__ double rec[6];
  __shared__ unsigned long long nonfin;
  __shared__ int k0s;
  const int tid = threadIdx.x;
  if (tid < 6) rec[tid] = J.rec[tid];
  if (tid == 0) nonfin = reinterpret_cast<const unsigned long long*>(J.rec)[6];
  __syncthreads();
  for (uint64_t base = 0; base < J.count; base += kStatsTile) {
    const int m = (int)(J.count - base < (uint64_t)kStatsTile ? J.count - base : (uint64_t)kStatsTile);
    // pass 1: finite values among this thread's 16 consecutive ones
    int c = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const int idx = tid * 16 + k;
      if (idx < m && isfinite(J.qf[base + idx] - (J.qc ? J.qc[base + idx] : 0.0))) ++c;
    }
    cnt[tid] = c;
    __syncthreads();
    for (int off = 1; off < kBlock; off <<= 1) {
      const int t = tid >= off ? cnt[tid - off] : 0;
      __syncthreads();
      cnt[tid] += t;
      __syncthreads();
    }
    const int total = cnt[kBlock - 1];
    // pass 2: the finite values, compacted in sample order
    int pos = cnt[tid] - c;
    for (int k = 0; k < 16; ++k) {
      const int idx = tid * 16 + k;
      if (idx < m) {
        const double y = J.qf[base + idx] - (J.qc ? J.qc[base + idx] : 0.0);
        if (isfinite(y)) buf[pos++] = y;
      }
    }
    __syncthreads();
    if (tid == 0) {
      int k0 = 0;
      if (rec[3] > 0.0) {   // continue the incomplete block
        k0 = kStatsBlock - (int)rec[3];
        if (k0 > total) k0 = total;
        for (int k = 0; k < k0; ++k) welford_push(rec[3], rec[4], rec[5], buf[k]);
        if (rec[3] == (double)kStatsBlock) {
          chan_merge(rec[0], rec[1], rec[2], rec[3], rec[4], rec[5]);
          rec[3] = rec[4] = rec[5] = 0.0;
        }
      }
      k0s = k0;
      nonfin += (unsigned long long)(m - total);
    }
    __syncthreads();
    const int k0 = k0s;
    const int nb = (total - k0) / kStatsBlock;
    if (tid < nb) {
      double n = 0.0, mean = 0.0, m2 = 0.0;
      for (int k = 0; k < kStatsBlock; ++k) welford_push(n, mean, m2, buf[k0 + tid * kStatsBlock + k]);
      bmean[tid] = mean;
      bm2[tid] = m2;
    }
    __syncthreads();
    if (tid == 0) {
      for (int q = 0; q < nb; ++q) chan_merge(rec[0], rec[1], rec[2], (double)kStatsBlock, bmean[q], bm2[q]);
      for (int k = k0 + nb * kStatsBlock; k < total; ++k) welford_push(rec[3], rec[4], rec[5], buf[k]);
    }
    __syncthreads();
  }
  if (tid < 6) J.rec[tid] = rec[tid];
  if (tid == 0) reinterpret_cast<unsigned long long*>(J.rec)[6] = nonfin;
}

// out[p] = the interior unknown at grid position p of a sample, or -1
__global__ void __launch_bounds__(kBlock) k_node_map(int n, size_t stride, int32_t* __restrict__ out) {
  const size_t p = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= stride) return;
  const size_t n2 = (size_t)n * n;
  const int i = (int)(p % n), j = (int)((p / n) % n);
  const size_t k = p / n2;
  const int m = n - 1;
  const bool interior = i >= 1 && j >= 1 && k >= 1 && k <= (size_t)m;
  out[p] = interior ? (int32_t)((i - 1) + (size_t)m * ((j - 1) + (size_t)m * (k - 1))) : -1;
}

// load vector of an elementwise-constant forcing f (n^3 values per sample):
// b = (h^3 / 8) sum of f over the 8 elements around an interior node (the
// integral of its Q1 hat function over each element is h^3 / 8); every other
// position of the grid layout, tail included, gets 0
__global__ void __launch_bounds__(kBlock) k_load(int n, size_t stride, int64_t total, const double* __restrict__ f,
                                                 double* __restrict__ b) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int64_t s = t / (int64_t)stride;
  const size_t p = (size_t)(t - s * (int64_t)stride);
  const int lg = __builtin_ctz((unsigned)n);   // n is a power of two
  const int i = (int)(p & (size_t)(n - 1)), j = (int)((p >> lg) & (size_t)(n - 1));
  const size_t k = p >> (2 * lg);
  double v = 0.0;
  if (i >= 1 && j >= 1 && k >= 1 && k <= (size_t)(n - 1)) {
    const size_t n2 = (size_t)n * n;
    const double* fe = f + (size_t)s * n2 * n + (size_t)(i - 1) + (size_t)n * (j - 1) + n2 * (k - 1);
    const double lo = (fe[0] + fe[1]) + (fe[n] + fe[n + 1]);
    const double hi = (fe[n2] + fe[n2 + 1]) + (fe[n2 + n] + fe[n2 + n + 1]);
    const double h = 1.0 / n;
    v = (h * h * h * 0.125) * (lo + hi);
  }
  b[t] = v;
}

// per-slot masks of the serving phases
__global__ void k_phase_masks(int S, const int* __restrict__ phase, int* __restrict__ inner, int* __restrict__ trans,
                              int* __restrict__ restart, int* __restrict__ done) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= S) return;
  const int ph = phase[b];
  inner[b] = ph == PHASE_INNER;
  trans[b] = ph == PHASE_TRANSITION;
  restart[b] = ph == PHASE_RESTART;
  done[b] = ph == PHASE_DONE;
}

// phase[slots[r]] = value for r < count
__global__ void k_set_phase_list(int count, const int* __restrict__ slots, int* __restrict__ phase, int value) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < count) phase[slots[r]] = value;
}

// phase[b] = value where mask[b]; optionally also zero an int array there
__global__ void k_set_phase_mask(int S, const int* __restrict__ mask, int* __restrict__ phase, int value,
                                 int* __restrict__ zero) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < S && mask[b]) {
    phase[b] = value;
    if (zero) zero[b] = 0;
  }
}

__global__ void k_count_active(int B, SolveState st) {
  int v = 0;
  for (int b = threadIdx.x; b < B; b += blockDim.x) v += st.active[b];
  v = (int)block_sum((double)v);
  if (threadIdx.x == 0) *st.nactive = v;
}

__global__ void k_count_mask(const int* __restrict__ mask, int B, int* __restrict__ out) {
  int v = 0;
  for (int b = threadIdx.x; b < B; b += blockDim.x) v += mask[b] != 0;
  v = (int)block_sum((double)v);
  if (threadIdx.x == 0) *out = v;
}

// a fused-direction solve starts: direction buffer 0, first direction (and
// with `fresh` an iterate that holds no value yet and is written, not updated,
// by the first step that touches it), on active samples; the active set is
// remembered for the final update
__global__ void k_dir_begin(int B, SolveState st, int fresh) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= B) return;
  const int a = st.active[b];
  st.began[b] = a;
  if (a) st.pstate[b] = fresh ? 6 : 2;
}

__global__ void k_set_active(int B, SolveState st, int value) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) st.active[b] = value;
}

template <class T>
inline dim3 sgrid(const SGeom& g, int B) { return dim3(g.chunks * (uint32_t)B); }

}  // namespace

template <class T>
hipError_t launch_pcg_update(int n, int B, T* x, const T* p, T* r, const T* q, SolveState s, uint32_t* nparts,
                             hipStream_t st) {
  const SGeom g = sgeom<T>(n);
  if (nparts) *nparts = g.chunks;
  k_pcg_update<T><<<sgrid<T>(g, B), kBlock, 0, st>>>(g, grid_stride(n), x, p, r, q, s);
  return hipGetLastError();
}

template <class T>
hipError_t launch_pcg_rupdate(int n, int B, T* r, const T* q, SolveState s, uint32_t* nparts, hipStream_t st) {
  const SGeom g = sgeom<T>(n);
  if (nparts) *nparts = g.chunks;
  k_pcg_rupdate<T><<<sgrid<T>(g, B), kBlock, 0, st>>>(g, grid_stride(n), r, q, s);
  return hipGetLastError();
}

template <class T>
hipError_t launch_pcg_finish(int n, int B, T* x, const T* p0, const T* p1, const int* mask, SolveState s,
                             hipStream_t st) {
  const SGeom g = sgeom<T>(n);
  k_pcg_finish<T><<<sgrid<T>(g, B), kBlock, 0, st>>>(g, grid_stride(n), x, p0, p1, mask, s);
  return hipGetLastError();
}

hipError_t launch_dir_begin(int B, SolveState s, bool fresh, hipStream_t st) {
  k_dir_begin<<<dim3((B + kBlock - 1) / kBlock), kBlock, 0, st>>>(B, s, fresh ? 1 : 0);
  return hipGetLastError();
}

template <class T>
hipError_t launch_dot(int n, int B, const T* a, const T* b, SolveState s, uint32_t* nparts, hipStream_t st) {
  const SGeom g = sgeom<T>(n);
  if (nparts) *nparts = g.chunks;
  k_dot<T><<<sgrid<T>(g, B), kBlock, 0, st>>>(g, grid_stride(n), a, b, s);
  return hipGetLastError();
}

template <class T>
hipError_t launch_pcg_direction(int n, int B, const T* z, T* p, SolveState s, hipStream_t st) {
  const SGeom g = sgeom<T>(n);
  k_pcg_direction<T><<<sgrid<T>(g, B), kBlock, 0, st>>>(g, grid_stride(n), z, p, s);
  return hipGetLastError();
}

template <class T>
hipError_t launch_copy(int n, int B, const T* z, T* p, SolveState s, hipStream_t st) {
  const SGeom g = sgeom<T>(n);
  k_copy<T><<<sgrid<T>(g, B), kBlock, 0, st>>>(g, grid_stride(n), z, p, s);
  return hipGetLastError();
}

hipError_t launch_add_correction(int n, int B, double* x, const float* d, SolveState s, hipStream_t st) {
  const SGeom g = sgeom<float>(n);   // units of 4 values
  k_add_correction<<<sgrid<float>(g, B), kBlock, 0, st>>>(g, grid_stride(n), x, d, s);
  return hipGetLastError();
}

hipError_t launch_demote(int n, int B, const double* r, float* r32, SolveState s, hipStream_t st) {
  const SGeom g = sgeom<float>(n);
  k_demote<<<sgrid<float>(g, B), kBlock, 0, st>>>(g, grid_stride(n), r, r32, s);
  return hipGetLastError();
}

template <class T>
hipError_t launch_fill_interior(int n, int B, T* v, double value, const int* active, hipStream_t st) {
  const SGeom g = sgeom<T>(n);
  k_fill_interior<T><<<sgrid<T>(g, B), kBlock, 0, st>>>(g, grid_stride(n), v, T(value), active);
  return hipGetLastError();
}

hipError_t launch_level_stats(int njobs, const StatsJobs& jobs, hipStream_t st) {
  if (njobs < 1 || njobs > kMaxStatsJobs) return hipErrorInvalidValue;
  k_level_stats<<<dim3(njobs), dim3(kBlock), 0, st>>>(jobs);
  return hipGetLastError();
}

hipError_t launch_reduce(int B, int op, double tol2, uint32_t nparts, SolveState s, double* out, hipStream_t st) {
  k_reduce<<<dim3(B), kBlock, 0, st>>>(op, tol2, nparts, s, out);
  return hipGetLastError();
}

hipError_t launch_node_map(int n, int32_t* out, hipStream_t st) {
  const size_t stride = grid_stride(n);
  k_node_map<<<dim3((unsigned)((stride + kBlock - 1) / kBlock)), kBlock, 0, st>>>(n, stride, out);
  return hipGetLastError();
}

hipError_t launch_load(int n, int B, const double* f, double* b, hipStream_t st) {
  const size_t stride = grid_stride(n);
  const int64_t total = (int64_t)B * (int64_t)stride;
  if (total <= 0) return hipSuccess;
  k_load<<<dim3((unsigned)((total + kBlock - 1) / kBlock)), kBlock, 0, st>>>(n, stride, total, f, b);
  return hipGetLastError();
}

hipError_t launch_count_active(int B, SolveState s, hipStream_t st) {
  k_count_active<<<1, kBlock, 0, st>>>(B, s);
  return hipGetLastError();
}

hipError_t launch_count_mask(const int* mask, int B, int* out, hipStream_t st) {
  k_count_mask<<<1, kBlock, 0, st>>>(mask, B, out);
  return hipGetLastError();
}

hipError_t launch_set_active(int B, SolveState s, int value, hipStream_t st) {
  k_set_active<<<dim3((B + kBlock - 1) / kBlock), kBlock, 0, st>>>(B, s, value);
  return hipGetLastError();
}

hipError_t launch_qoi_partial(int n, int B, int qoi, const double* u, SolveState s, uint32_t* nparts,
                              hipStream_t st, bool masked) {
  const SGeom g = sgeom<double>(n);
  if (qoi == 1) {
    // the subcube's nodes only, in at most as many parts as the whole-mesh form
    const uint32_t m = (uint32_t)(3 * n / 4 - n / 4 + 1);
    uint32_t ch = (uint32_t)(((size_t)m * m * m + kBlock * 8 - 1) / (kBlock * 8));
    if (ch > g.chunks) ch = g.chunks;
    if (ch < 1) ch = 1;
    if (nparts) *nparts = ch;
    k_qoi_subcube<<<dim3(ch * (uint32_t)B), kBlock, 0, st>>>(n, ch, grid_stride(n), u, s, masked);
    return hipGetLastError();
  }
  if (nparts) *nparts = g.chunks;
  k_qoi_partial<<<sgrid<double>(g, B), kBlock, 0, st>>>(g, grid_stride(n), u, s, masked);
  return hipGetLastError();
}

hipError_t launch_phase_masks(int S, const int* phase, int* inner, int* trans, int* restart, int* done,
                              hipStream_t st) {
  k_phase_masks<<<dim3((S + kBlock - 1) / kBlock), kBlock, 0, st>>>(S, phase, inner, trans, restart, done);
  return hipGetLastError();
}

hipError_t launch_set_phase_list(int count, const int* slots, int* phase, int value, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  k_set_phase_list<<<dim3((count + kBlock - 1) / kBlock), kBlock, 0, st>>>(count, slots, phase, value);
  return hipGetLastError();
}

hipError_t launch_set_phase_mask(int S, const int* mask, int* phase, int value, int* zero, hipStream_t st) {
  k_set_phase_mask<<<dim3((S + kBlock - 1) / kBlock), kBlock, 0, st>>>(S, mask, phase, value, zero);
  return hipGetLastError();
}

template hipError_t launch_pcg_update<float>(int, int, float*, const float*, float*, const float*, SolveState,
                                             uint32_t*, hipStream_t);
template hipError_t launch_pcg_update<double>(int, int, double*, const double*, double*, const double*, SolveState,
                                              uint32_t*, hipStream_t);
template hipError_t launch_pcg_rupdate<float>(int, int, float*, const float*, SolveState, uint32_t*, hipStream_t);
template hipError_t launch_pcg_rupdate<double>(int, int, double*, const double*, SolveState, uint32_t*, hipStream_t);
template hipError_t launch_pcg_finish<float>(int, int, float*, const float*, const float*, const int*, SolveState,
                                             hipStream_t);
template hipError_t launch_pcg_finish<double>(int, int, double*, const double*, const double*, const int*, SolveState,
                                              hipStream_t);
template hipError_t launch_dot<float>(int, int, const float*, const float*, SolveState, uint32_t*, hipStream_t);
template hipError_t launch_dot<double>(int, int, const double*, const double*, SolveState, uint32_t*, hipStream_t);
template hipError_t launch_pcg_direction<float>(int, int, const float*, float*, SolveState, hipStream_t);
template hipError_t launch_pcg_direction<double>(int, int, const double*, double*, SolveState, hipStream_t);
template hipError_t launch_copy<float>(int, int, const float*, float*, SolveState, hipStream_t);
template hipError_t launch_copy<double>(int, int, const double*, double*, SolveState, hipStream_t);
template hipError_t launch_fill_interior<float>(int, int, float*, double, const int*, hipStream_t);
template hipError_t launch_fill_interior<double>(int, int, double*, double, const int*, hipStream_t);

}  // namespace mlmc
