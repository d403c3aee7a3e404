// Matrix-free Q1 operator and the geometric-multigrid kernels (grid layout).
//
// Operator (eq. model with per-element kappa, Q1 hexahedra, Sec. 2.1-2.2):
//   (A u)_i = h sum_{e owns i} kappa_e sum_b Khat[a_i(e)][b] u_b
// with Khat the unit-cube Q1 stiffness.  Khat[a][b] is 1/3 for a = b, 0 when
// a and b share an edge, and -1/12 when they differ in two or three
// coordinates, so for element e seen from node i (local corner pointing along
// signs (sx, sy, sz)) the row reduces to
//   kappa_e [ u_i / 3 - (u_(sx,sy,0) + u_(sx,0,sz) + u_(0,sy,sz) + u_(sx,sy,sz)) / 12 ]
// i.e. 20 neighbour values (12 edge, 8 corner) and the 8 element coefficients
// per node; face neighbours never enter.  The Jacobi diagonal is
// D_i = (h/3) sum_{e owns i} kappa_e, computed from the same 8 coefficients.
//
// Multigrid pieces: Chebyshev-Jacobi smoothing step (three-term recurrence),
// full-weighting restriction P^T and trilinear prolongation P between the n
// and n/2 grids, exact solve of the single unknown of the 2^3 mesh, and the
// 8-child mean of kappa for the rediscretised coarse operators.
#include "common.hpp"
#include "kernels.hpp"

namespace mlmc {
namespace {

__device__ __forceinline__ int ilog2(int n) { return 31 - __clz(n); }

struct Node {
  uint32_t b;     // sample
  uint32_t s;     // position inside the sample's grid block
  bool ok;        // interior node
};

// 1D grid of nchunk * B workgroups, each covering 256 consecutive positions of
// the interior planes 1..n-1 of one sample.
__device__ __forceinline__ Node node_of_thread(int n, uint32_t nchunk) {
  const uint32_t logical = xcd_remap(blockIdx.x, gridDim.x);
  Node nd;
  nd.b = logical / nchunk;
  const uint32_t c = logical - nd.b * nchunk;
  const uint32_t n2 = (uint32_t)n * n;
  const uint32_t p = n2 + c * kBlock + threadIdx.x;
  const uint32_t lg = (uint32_t)ilog2(n);
  const uint32_t i = p & (n - 1), j = (p >> lg) & (n - 1);
  nd.ok = (p < n2 * (uint32_t)n) && i != 0 && j != 0;
  nd.s = p;
  return nd;
}

inline uint32_t chunks_of(int n) {
  return (uint32_t)(((size_t)(n - 1) * n * n + kBlock - 1) / kBlock);
}

// (A u)_s and the diagonal at interior position s of an n^3 grid block.
template <class T>
__device__ __forceinline__ void q1_row(const T* __restrict__ u, const T* __restrict__ kap, int n,
                                       uint32_t s, T h, T& au, T& diag) {
  const int n2 = n * n;
  const uint32_t e0 = s - (uint32_t)(1 + n + n2);     // element (i-1, j-1, k-1)
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
  const T third = T(1) / T(3), twelfth = T(1) / T(12);
  au = h * (ks * u0 * third - far * twelfth);
  diag = h * ks * third;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_apply(int n, uint32_t nchunk, size_t stride, T h,
                                                  const T* __restrict__ kap, const T* __restrict__ u,
                                                  T* __restrict__ y, const int* __restrict__ active) {
  const Node nd = node_of_thread(n, nchunk);
  if (active && !active[nd.b]) return;
  if (!nd.ok) return;
  const size_t ne = (size_t)n * n * n;
  T au, dg;
  q1_row(u + nd.b * stride, kap + nd.b * ne, n, nd.s, h, au, dg);
  y[nd.b * stride + nd.s] = au;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_residual(int n, uint32_t nchunk, size_t stride, T h,
                                                     const T* __restrict__ kap, const T* __restrict__ b,
                                                     const T* __restrict__ x, T* __restrict__ r,
                                                     const int* __restrict__ active) {
  const Node nd = node_of_thread(n, nchunk);
  if (active && !active[nd.b]) return;
  if (!nd.ok) return;
  const size_t ne = (size_t)n * n * n;
  T ax, dg;
  q1_row(x + nd.b * stride, kap + nd.b * ne, n, nd.s, h, ax, dg);
  const size_t g = nd.b * stride + nd.s;
  r[g] = b[g] - ax;
}

// D_i from the 8 element coefficients around interior position s
template <class T>
__device__ __forceinline__ T q1_diag(const T* __restrict__ kap, int n, uint32_t s, T h) {
  const int n2 = n * n;
  const uint32_t e0 = s - (uint32_t)(1 + n + n2);
  T ks = T(0);
#pragma unroll
  for (int sz = 0; sz < 2; ++sz)
#pragma unroll
    for (int sy = 0; sy < 2; ++sy)
#pragma unroll
      for (int sx = 0; sx < 2; ++sx) ks += kap[e0 + sx + n * sy + n2 * sz];
  return h * ks * (T(1) / T(3));
}

template <class T, bool ZERO_X, bool USE_XO>
__global__ void __launch_bounds__(kBlock) k_cheb(int n, uint32_t nchunk, size_t stride, T h,
                                                 const T* __restrict__ kap, const T* __restrict__ b,
                                                 const T* __restrict__ x, const T* xo, T* out, T c1, T c2,
                                                 const int* __restrict__ active) {
  const Node nd = node_of_thread(n, nchunk);
  if (active && !active[nd.b]) return;
  if (!nd.ok) return;
  const size_t ne = (size_t)n * n * n;
  const size_t g = nd.b * stride + nd.s;
  const T* kb = kap + nd.b * ne;
  if (ZERO_X) {
    out[g] = c2 * b[g] / q1_diag(kb, n, nd.s, h);
  } else {
    T ax, dg;
    q1_row(x + nd.b * stride, kb, n, nd.s, h, ax, dg);
    const T xv = x[g];
    // without a previous iterate the three-term step takes x_{k-1} = 0
    const T prev = USE_XO ? xv - xo[g] : xv;
    out[g] = xv + c1 * prev + c2 * (b[g] - ax) / dg;
  }
}

// full weighting: coarse node (I,J,K) gathers fine (2I+dx, 2J+dy, 2K+dz) with
// weights prod_d (dx == 0 ? 1 : 1/2)
template <class T>
__global__ void __launch_bounds__(kBlock) k_restrict(int nc, uint32_t nchunk, size_t sc, size_t sf,
                                                     const T* __restrict__ rf, T* __restrict__ bc,
                                                     const int* __restrict__ active) {
  const Node nd = node_of_thread(nc, nchunk);
  if (active && !active[nd.b]) return;
  if (!nd.ok) return;
  const int nf = 2 * nc, lg = ilog2(nc);
  const uint32_t I = nd.s & (nc - 1), J = (nd.s >> lg) & (nc - 1), K = nd.s >> (2 * lg);
  const T* r = rf + nd.b * sf;
  const int f2 = nf * nf;
  const uint32_t c = 2 * I + nf * 2 * J + f2 * 2 * K;
  T acc = T(0);
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz) {
    T az = T(0);
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const uint32_t row = c + nf * dy + f2 * dz;
      const T ay = T(0.5) * (r[row - 1] + r[row + 1]) + r[row];
      az += (dy == 0 ? T(1) : T(0.5)) * ay;
    }
    acc += (dz == 0 ? T(1) : T(0.5)) * az;
  }
  bc[nd.b * sc + nd.s] = acc;
}

// trilinear interpolation from the n/2 grid, added to the fine values
template <class T>
__global__ void __launch_bounds__(kBlock) k_prolong_add(int nf, uint32_t nchunk, size_t sf, size_t sc,
                                                        const T* __restrict__ xc, T* __restrict__ xf,
                                                        const int* __restrict__ active) {
  const Node nd = node_of_thread(nf, nchunk);
  if (active && !active[nd.b]) return;
  if (!nd.ok) return;
  const int nc = nf / 2, lg = ilog2(nf);
  const uint32_t i = nd.s & (nf - 1), j = (nd.s >> lg) & (nf - 1), k = nd.s >> (2 * lg);
  const uint32_t i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1, k1 = (k + 1) >> 1;
  const T wi = (i & 1) ? T(0.5) : T(1), wj = (j & 1) ? T(0.5) : T(1), wk = (k & 1) ? T(0.5) : T(1);
  const T* c = xc + nd.b * sc;
  const int c2 = nc * nc;
  auto row = [&](uint32_t jj, uint32_t kk) -> T {
    const uint32_t base = nc * jj + c2 * kk;
    return (i & 1) ? wi * (c[base + i0] + c[base + i1]) : c[base + i0];
  };
  auto plane = [&](uint32_t kk) -> T {
    return (j & 1) ? wj * (row(j0, kk) + row(j1, kk)) : row(j0, kk);
  };
  const T v = (k & 1) ? wk * (plane(k0) + plane(k1)) : plane(k0);
  xf[nd.b * sf + nd.s] += v;
}

// 2^3 mesh: one unknown at node (1,1,1), A_11 = (h/3) sum of the 8 kappa, h = 1/2
template <class T>
__global__ void k_coarsest(int B, size_t stride, const T* __restrict__ kap, const T* __restrict__ b,
                           T* __restrict__ x, const int* __restrict__ active) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= B) return;
  if (active && !active[s]) return;
  const T* k = kap + 8 * s;
  const T ks = ((k[0] + k[1]) + (k[2] + k[3])) + ((k[4] + k[5]) + (k[6] + k[7]));
  const T a11 = T(0.5) * ks * (T(1) / T(3));
  x[s * stride + 7] = b[s * stride + 7] / a11;
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_coarsen(int nc, int64_t total, const T* __restrict__ kf,
                                                    T* __restrict__ kc) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int64_t nce = (int64_t)nc * nc * nc;
  const int64_t b = t / nce, E = t - b * nce;
  const int nf = 2 * nc;
  const int EX = (int)(E % nc), EY = (int)((E / nc) % nc), EZ = (int)(E / ((int64_t)nc * nc));
  const T* f = kf + b * nce * 8 + 2 * EX + (int64_t)nf * 2 * EY + (int64_t)nf * nf * 2 * EZ;
  const int64_t f2 = (int64_t)nf * nf;
  const T s = ((f[0] + f[1]) + (f[nf] + f[nf + 1])) + ((f[f2] + f[f2 + 1]) + (f[f2 + nf] + f[f2 + nf + 1]));
  kc[t] = s * T(0.125);
}

template <class Ts, class Td>
__global__ void __launch_bounds__(kBlock) k_convert(size_t count, const Ts* __restrict__ src,
                                                    Td* __restrict__ dst) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) dst[t] = (Td)src[t];
}

template <class T>
__global__ void __launch_bounds__(kBlock) k_fill_interior(int n, uint32_t nchunk, size_t stride,
                                                          T* __restrict__ v, T value,
                                                          const int* __restrict__ active) {
  const Node nd = node_of_thread(n, nchunk);
  if (active && !active[nd.b]) return;
  if (!nd.ok) return;
  v[nd.b * stride + nd.s] = value;
}

inline dim3 grid_of(int n, int B) { return dim3(chunks_of(n) * (uint32_t)B); }

}  // namespace

template <class T>
hipError_t launch_apply(int n, int B, const T* kap, const T* u, T* y, const int* active, hipStream_t st) {
  k_apply<T><<<grid_of(n, B), kBlock, 0, st>>>(n, chunks_of(n), grid_stride(n), T(1) / T(n), kap, u, y, active);
  return hipGetLastError();
}

template <class T>
hipError_t launch_residual(int n, int B, const T* kap, const T* b, const T* x, T* r, const int* active,
                           hipStream_t st) {
  k_residual<T><<<grid_of(n, B), kBlock, 0, st>>>(n, chunks_of(n), grid_stride(n), T(1) / T(n), kap, b, x, r,
                                                  active);
  return hipGetLastError();
}

template <class T>
hipError_t launch_cheb(int n, int B, const T* kap, const T* b, const T* x, const T* xo, T* out, double c1,
                       double c2, bool zero_x, bool use_xo, const int* active, hipStream_t st) {
  const dim3 g = grid_of(n, B);
  const uint32_t nc = chunks_of(n);
  const size_t sd = grid_stride(n);
  const T h = T(1) / T(n);
  if (zero_x)
    k_cheb<T, true, false><<<g, kBlock, 0, st>>>(n, nc, sd, h, kap, b, x, xo, out, T(c1), T(c2), active);
  else if (use_xo)
    k_cheb<T, false, true><<<g, kBlock, 0, st>>>(n, nc, sd, h, kap, b, x, xo, out, T(c1), T(c2), active);
  else
    k_cheb<T, false, false><<<g, kBlock, 0, st>>>(n, nc, sd, h, kap, b, x, xo, out, T(c1), T(c2), active);
  return hipGetLastError();
}

template <class T>
hipError_t launch_restrict(int nf, int B, const T* rf, T* bc, const int* active, hipStream_t st) {
  const int nc = nf / 2;
  k_restrict<T><<<grid_of(nc, B), kBlock, 0, st>>>(nc, chunks_of(nc), grid_stride(nc), grid_stride(nf), rf, bc,
                                                   active);
  return hipGetLastError();
}

template <class T>
hipError_t launch_prolong_add(int nf, int B, const T* xc, T* xf, const int* active, hipStream_t st) {
  k_prolong_add<T><<<grid_of(nf, B), kBlock, 0, st>>>(nf, chunks_of(nf), grid_stride(nf), grid_stride(nf / 2),
                                                      xc, xf, active);
  return hipGetLastError();
}

template <class T>
hipError_t launch_coarsest(int B, const T* kap, const T* b, T* x, const int* active, hipStream_t st) {
  k_coarsest<T><<<dim3((B + 63) / 64), 64, 0, st>>>(B, grid_stride(2), kap, b, x, active);
  return hipGetLastError();
}

template <class T>
hipError_t launch_coarsen(int nf, int B, const T* kf, T* kc, hipStream_t st) {
  const int nc = nf / 2;
  const int64_t total = (int64_t)B * nc * nc * nc;
  k_coarsen<T><<<dim3((unsigned)((total + kBlock - 1) / kBlock)), kBlock, 0, st>>>(nc, total, kf, kc);
  return hipGetLastError();
}

template <class Ts, class Td>
hipError_t launch_convert(size_t count, const Ts* src, Td* dst, hipStream_t st) {
  if (!count) return hipSuccess;
  k_convert<Ts, Td><<<dim3((unsigned)((count + kBlock - 1) / kBlock)), kBlock, 0, st>>>(count, src, dst);
  return hipGetLastError();
}

template <class T>
hipError_t launch_fill_interior(int n, int B, T* v, double value, const int* active, hipStream_t st) {
  k_fill_interior<T><<<grid_of(n, B), kBlock, 0, st>>>(n, chunks_of(n), grid_stride(n), v, T(value), active);
  return hipGetLastError();
}

#define MLMC_INST(T)                                                                                    \
  template hipError_t launch_apply<T>(int, int, const T*, const T*, T*, const int*, hipStream_t);      \
  template hipError_t launch_residual<T>(int, int, const T*, const T*, const T*, T*, const int*,       \
                                         hipStream_t);                                                 \
  template hipError_t launch_cheb<T>(int, int, const T*, const T*, const T*, const T*, T*, double,     \
                                     double, bool, bool, const int*, hipStream_t);                     \
  template hipError_t launch_restrict<T>(int, int, const T*, T*, const int*, hipStream_t);             \
  template hipError_t launch_prolong_add<T>(int, int, const T*, T*, const int*, hipStream_t);          \
  template hipError_t launch_coarsest<T>(int, const T*, const T*, T*, const int*, hipStream_t);        \
  template hipError_t launch_coarsen<T>(int, int, const T*, T*, hipStream_t);                          \
  template hipError_t launch_fill_interior<T>(int, int, T*, double, const int*, hipStream_t);
MLMC_INST(float)
MLMC_INST(double)
#undef MLMC_INST
template hipError_t launch_convert<double, float>(size_t, const double*, float*, hipStream_t);
template hipError_t launch_convert<float, double>(size_t, const float*, double*, hipStream_t);

}  // namespace mlmc
