// Batched preconditioned conjugate gradients: vector updates, dot products
// and the per-sample scalar recurrences (alpha, beta, convergence), plus the
// QoI reduction.  Vectors may be fp32 or fp64; every dot product and every
// scalar is accumulated in fp64.
//
// Reductions are deterministic and per sample: each workgroup (one chunk of
// one sample) reduces its values in a fixed tree and writes one partial sum;
// k_reduce then sums a sample's partials in a fixed order.  A sample's scalars
// therefore never depend on which other samples share the batch.
#include "common.hpp"
#include "kernels.hpp"

namespace mlmc {
namespace {

__device__ __forceinline__ int ilog2(int n) { return 31 - __clz(n); }

struct Node {
  uint32_t b, c, s;
  bool ok;
};

__device__ __forceinline__ Node node_of_thread(int n, uint32_t nchunk) {
  const uint32_t logical = xcd_remap(blockIdx.x, gridDim.x);
  Node nd;
  nd.b = logical / nchunk;
  nd.c = logical - nd.b * nchunk;
  const uint32_t n2 = (uint32_t)n * n;
  const uint32_t p = n2 + nd.c * kBlock + threadIdx.x;
  const uint32_t lg = (uint32_t)ilog2(n);
  const uint32_t i = p & (n - 1), j = (p >> lg) & (n - 1);
  nd.ok = (p < n2 * (uint32_t)n) && i != 0 && j != 0;
  nd.s = p;
  return nd;
}

uint32_t chunks_of(int n) { return (uint32_t)(((size_t)(n - 1) * n * n + kBlock - 1) / kBlock); }

// Sum over the workgroup; result valid in thread 0.
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

template <class T>
__device__ __forceinline__ T q1_apply(const T* __restrict__ u, const T* __restrict__ kap, int n,
                                      uint32_t s, T h) {
  const int n2 = n * n;
  const uint32_t e0 = s - (uint32_t)(1 + n + n2);
  const T u0 = u[s];
  T ks = T(0), far = T(0);
#pragma unroll
  for (int sz = 0; sz < 2; ++sz)
#pragma unroll
    for (int sy = 0; sy < 2; ++sy)
#pragma unroll
      for (int sx = 0; sx < 2; ++sx) {
        const T kv = kap[e0 + sx + n * sy + n2 * sz];
        const int ox = sx ? 1 : -1, oy = sy ? n : -n, oz = sz ? n2 : -n2;
        const T f = (u[s + ox + oy] + u[s + ox + oz]) + (u[s + oy + oz] + u[s + ox + oy + oz]);
        ks += kv;
        far += kv * f;
      }
  return h * (ks * u0 * (T(1) / T(3)) - far * (T(1) / T(12)));
}

// q = A p and the partial sums of p . q
template <class T>
__global__ void __launch_bounds__(kBlock) k_pcg_apply_dot(int n, uint32_t nchunk, size_t stride, T h,
                                                          const T* __restrict__ kap, const T* __restrict__ p,
                                                          T* __restrict__ q, SolveState st) {
  const Node nd = node_of_thread(n, nchunk);
  if (!st.active[nd.b]) return;
  double v = 0.0;
  if (nd.ok) {
    const size_t g = nd.b * stride + nd.s;
    const T aq = q1_apply(p + nd.b * stride, kap + nd.b * (size_t)n * n * n, n, nd.s, h);
    q[g] = aq;
    v = (double)p[g] * (double)aq;
  }
  v = block_sum(v);
  if (threadIdx.x == 0) st.partial[(size_t)nd.b * st.nchunk + nd.c] = v;
}

// x += alpha p, r -= alpha q, partial sums of r . r
template <class T>
__global__ void __launch_bounds__(kBlock) k_pcg_update(int n, uint32_t nchunk, size_t stride,
                                                       T* __restrict__ x, const T* __restrict__ p,
                                                       T* __restrict__ r, const T* __restrict__ q,
                                                       SolveState st) {
  const Node nd = node_of_thread(n, nchunk);
  if (!st.active[nd.b]) return;
  double v = 0.0;
  if (nd.ok) {
    const size_t g = nd.b * stride + nd.s;
    const T a = (T)st.alpha[nd.b];
    x[g] += a * p[g];
    const T rn = r[g] - a * q[g];
    r[g] = rn;
    v = (double)rn * (double)rn;
  }
  v = block_sum(v);
  if (threadIdx.x == 0) st.partial[(size_t)nd.b * st.nchunk + nd.c] = v;
}

template <class Ta, class Tb>
__global__ void __launch_bounds__(kBlock) k_dot(int n, uint32_t nchunk, size_t stride,
                                                const Ta* __restrict__ a, const Tb* __restrict__ b,
                                                SolveState st) {
  const Node nd = node_of_thread(n, nchunk);
  if (!st.active[nd.b]) return;
  double v = 0.0;
  if (nd.ok) {
    const size_t g = nd.b * stride + nd.s;
    v = (double)a[g] * (double)b[g];
  }
  v = block_sum(v);
  if (threadIdx.x == 0) st.partial[(size_t)nd.b * st.nchunk + nd.c] = v;
}

// p = z + beta p
template <class T>
__global__ void __launch_bounds__(kBlock) k_pcg_direction(int n, uint32_t nchunk, size_t stride,
                                                          const T* __restrict__ z, T* __restrict__ p,
                                                          SolveState st) {
  const Node nd = node_of_thread(n, nchunk);
  if (!st.active[nd.b] || !nd.ok) return;
  const size_t g = nd.b * stride + nd.s;
  p[g] = z[g] + (T)st.beta[nd.b] * p[g];
}

__global__ void __launch_bounds__(kBlock) k_true_residual(int n, uint32_t nchunk, size_t stride, double h,
                                                          const double* __restrict__ kap, double bconst,
                                                          const double* __restrict__ x, double* __restrict__ r,
                                                          SolveState st) {
  const Node nd = node_of_thread(n, nchunk);
  if (!st.active[nd.b]) return;
  double v = 0.0;
  if (nd.ok) {
    const size_t g = nd.b * stride + nd.s;
    const double rv = bconst - q1_apply(x + nd.b * stride, kap + nd.b * (size_t)n * n * n, n, nd.s, h);
    r[g] = rv;
    v = rv * rv;
  }
  v = block_sum(v);
  if (threadIdx.x == 0) st.partial[(size_t)nd.b * st.nchunk + nd.c] = v;
}

__global__ void __launch_bounds__(kBlock) k_add_correction(int n, uint32_t nchunk, size_t stride,
                                                           double* __restrict__ x, const float* __restrict__ d,
                                                           SolveState st) {
  const Node nd = node_of_thread(n, nchunk);
  if (!st.active[nd.b] || !nd.ok) return;
  const size_t g = nd.b * stride + nd.s;
  x[g] += (double)d[g];
}

__global__ void __launch_bounds__(kBlock) k_demote(int n, uint32_t nchunk, size_t stride,
                                                   const double* __restrict__ r, float* __restrict__ r32,
                                                   SolveState st) {
  const Node nd = node_of_thread(n, nchunk);
  if (!st.active[nd.b] || !nd.ok) return;
  const size_t g = nd.b * stride + nd.s;
  r32[g] = (float)r[g];
}

// one workgroup per sample: fixed-order sum of its partials, then the scalar op
__global__ void __launch_bounds__(kBlock) k_reduce(int op, double tol2, SolveState st, double* out) {
  const int b = blockIdx.x;
  if (op != RED_STORE && op != RED_BB && !st.active[b]) return;
  const double* p = st.partial + (size_t)b * st.nchunk;
  double v = 0.0;
  for (int c = threadIdx.x; c < st.nchunk; c += kBlock) v += p[c];
  v = block_sum(v);
  if (threadIdx.x != 0) return;
  switch (op) {
    case RED_BB: st.bb[b] = v; break;
    case RED_ALPHA: st.alpha[b] = st.rz[b] / v; st.iters[b] += 1; break;
    case RED_RR:
      st.rr[b] = v;
      if (v <= tol2 * st.bb[b]) st.active[b] = 0;
      break;
    case RED_RZ_INIT: st.rz[b] = v; break;
    case RED_BETA: st.beta[b] = v / st.rz[b]; st.rz[b] = v; break;
    default: out[b] = v; break;
  }
}

__global__ void k_count_active(int B, SolveState st) {
  int v = 0;
  for (int b = threadIdx.x; b < B; b += blockDim.x) v += st.active[b];
  v = (int)block_sum((double)v);
  if (threadIdx.x == 0) *st.nactive = v;
}

__global__ void k_set_active(int B, SolveState st, int value) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b < B) st.active[b] = value;
}

// QoI weights: domain average h^3; subcube [1/4,3/4]^3 average
// h^3 prod_d c(i_d) with c = 2 strictly inside, 1 on the faces, 0 outside
// (the number of subcube elements touching the node along each axis).
__global__ void __launch_bounds__(kBlock) k_qoi_partial(int n, uint32_t nchunk, size_t stride, int qoi,
                                                        const double* __restrict__ u, SolveState st) {
  const Node nd = node_of_thread(n, nchunk);
  double v = 0.0;
  if (nd.ok) {
    const int lg = ilog2(n);
    const int i = nd.s & (n - 1), j = (nd.s >> lg) & (n - 1), k = nd.s >> (2 * lg);
    const double h = 1.0 / n;
    double w = h * h * h;
    if (qoi == 1) {
      const int lo = n / 4, hi = 3 * n / 4;
      auto c = [&](int t) { return (t < lo || t > hi) ? 0.0 : ((t == lo || t == hi) ? 1.0 : 2.0); };
      w *= c(i) * c(j) * c(k);
    }
    v = w * u[nd.b * stride + nd.s];
  }
  v = block_sum(v);
  if (threadIdx.x == 0) st.partial[(size_t)nd.b * st.nchunk + nd.c] = v;
}

inline dim3 grid_of(int n, int B) { return dim3(chunks_of(n) * (uint32_t)B); }

}  // namespace

int krylov_chunks(int n) { return (int)chunks_of(n); }

template <class T>
hipError_t launch_pcg_apply_dot(int n, int B, const T* kap, const T* p, T* q, SolveState s, hipStream_t st) {
  k_pcg_apply_dot<T><<<grid_of(n, B), kBlock, 0, st>>>(n, chunks_of(n), grid_stride(n), T(1) / T(n), kap, p, q, s);
  return hipGetLastError();
}

template <class T>
hipError_t launch_pcg_update(int n, int B, T* x, const T* p, T* r, const T* q, SolveState s, hipStream_t st) {
  k_pcg_update<T><<<grid_of(n, B), kBlock, 0, st>>>(n, chunks_of(n), grid_stride(n), x, p, r, q, s);
  return hipGetLastError();
}

template <class Ta, class Tb>
hipError_t launch_dot(int n, int B, const Ta* a, const Tb* b, SolveState s, hipStream_t st) {
  k_dot<Ta, Tb><<<grid_of(n, B), kBlock, 0, st>>>(n, chunks_of(n), grid_stride(n), a, b, s);
  return hipGetLastError();
}

template <class T>
hipError_t launch_pcg_direction(int n, int B, const T* z, T* p, SolveState s, hipStream_t st) {
  k_pcg_direction<T><<<grid_of(n, B), kBlock, 0, st>>>(n, chunks_of(n), grid_stride(n), z, p, s);
  return hipGetLastError();
}

hipError_t launch_true_residual(int n, int B, const double* kap, double bconst, const double* x, double* r,
                                SolveState s, hipStream_t st) {
  k_true_residual<<<grid_of(n, B), kBlock, 0, st>>>(n, chunks_of(n), grid_stride(n), 1.0 / n, kap, bconst, x, r, s);
  return hipGetLastError();
}

hipError_t launch_add_correction(int n, int B, double* x, const float* d, SolveState s, hipStream_t st) {
  k_add_correction<<<grid_of(n, B), kBlock, 0, st>>>(n, chunks_of(n), grid_stride(n), x, d, s);
  return hipGetLastError();
}

hipError_t launch_demote(int n, int B, const double* r, float* r32, SolveState s, hipStream_t st) {
  k_demote<<<grid_of(n, B), kBlock, 0, st>>>(n, chunks_of(n), grid_stride(n), r, r32, s);
  return hipGetLastError();
}

hipError_t launch_reduce(int B, int op, double tol2, SolveState s, double* out, hipStream_t st) {
  k_reduce<<<dim3(B), kBlock, 0, st>>>(op, tol2, s, out);
  return hipGetLastError();
}

hipError_t launch_count_active(int B, SolveState s, hipStream_t st) {
  k_count_active<<<1, kBlock, 0, st>>>(B, s);
  return hipGetLastError();
}

hipError_t launch_set_active(int B, SolveState s, int value, hipStream_t st) {
  k_set_active<<<dim3((B + kBlock - 1) / kBlock), kBlock, 0, st>>>(B, s, value);
  return hipGetLastError();
}

hipError_t launch_qoi_partial(int n, int B, int qoi, const double* u, SolveState s, hipStream_t st) {
  k_qoi_partial<<<grid_of(n, B), kBlock, 0, st>>>(n, chunks_of(n), grid_stride(n), qoi, u, s);
  return hipGetLastError();
}

template hipError_t launch_pcg_apply_dot<float>(int, int, const float*, const float*, float*, SolveState, hipStream_t);
template hipError_t launch_pcg_apply_dot<double>(int, int, const double*, const double*, double*, SolveState,
                                                 hipStream_t);
template hipError_t launch_pcg_update<float>(int, int, float*, const float*, float*, const float*, SolveState,
                                             hipStream_t);
template hipError_t launch_pcg_update<double>(int, int, double*, const double*, double*, const double*, SolveState,
                                              hipStream_t);
template hipError_t launch_dot<float, float>(int, int, const float*, const float*, SolveState, hipStream_t);
template hipError_t launch_dot<double, double>(int, int, const double*, const double*, SolveState, hipStream_t);
template hipError_t launch_pcg_direction<float>(int, int, const float*, float*, SolveState, hipStream_t);
template hipError_t launch_pcg_direction<double>(int, int, const double*, double*, SolveState, hipStream_t);

}  // namespace mlmc
