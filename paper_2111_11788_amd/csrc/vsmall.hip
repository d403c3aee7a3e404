// The coarse end of the V-cycle in one kernel: one workgroup per sample runs
// the whole V-cycle from an N0^3 mesh (N0 <= 16) down to the 2^3 mesh and
// back, with every vector of every level and the coarse kappa in LDS.
//
// It computes exactly what the level-by-level kernels compute (Chebyshev-
// Jacobi pre/post smoothing, residual, full-weighting restriction, exact
// solve on 2^3, trilinear prolongation; the same operator rows and the same
// three-term recurrence), but the coarse levels then cost one launch per
// V-cycle instead of ~7 per level, and their data never leaves the CU.
//
// LDS per level n: x and a second iterate/residual buffer in the grid layout
// (grid_stride(n) entries each), the restricted right-hand side, and the n^3
// kappa.  The finest (N0) right-hand side stays in global memory.
#include "common.hpp"
#include "kernels.hpp"

namespace mlmc {
namespace {

constexpr int kMaxLv = 4;   // 16, 8, 4, 2

struct SmallArgs {
  int n0, nlev, degree;
  double c1[16], c2[16];
  size_t gstride;             // grid stride of the N0 level in global memory
  const void* kap[kMaxLv];    // global kappa of each level (element layout, per-sample n^3)
};

__host__ __device__ inline int lds_stride(int n) {
  const int s = (n + 1) * n * n + n + 1;
  return (s + 63) / 64 * 64;
}

template <class T>
__device__ __forceinline__ void q1(const T* u, const T* kap, int n, int s, T h, T& au, T& dg) {
  const int n2 = n * n;
  const int e0 = s - (1 + n + n2);
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
  au = h * (ks * u0 * (T(1) / T(3)) - far * (T(1) / T(12)));
  dg = h * ks * (T(1) / T(3));
}

__device__ __forceinline__ int lg2(int n) { return 31 - __clz(n); }

// loop over the interior nodes of an n^3 grid (positions of planes 1..n-1);
// n is a power of two, so the row/column tests are masks
#define FOR_INTERIOR(n, s)                                                          \
  for (int s = (n) * (n) + (int)threadIdx.x; s < (n) * (n) * (n); s += blockDim.x)   \
    if ((s & ((n) - 1)) != 0 && ((s >> lg2(n)) & ((n) - 1)) != 0)

template <class T>
__global__ void __launch_bounds__(256) k_vsmall(SmallArgs a, const T* __restrict__ bglob, T* __restrict__ xglob,
                                                const int* __restrict__ active) {
  const int smp = blockIdx.x;
  if (active && !active[smp]) return;
  extern __shared__ __align__(16) unsigned char smem[];
  T* X[kMaxLv][2];
  T* Bv[kMaxLv];
  T* Kp[kMaxLv];
  {
    T* p = reinterpret_cast<T*>(smem);
    for (int l = 0; l < a.nlev; ++l) {
      const int n = a.n0 >> l, S = lds_stride(n);
      X[l][0] = p; p += S;
      X[l][1] = p; p += S;
      Bv[l] = l == 0 ? nullptr : p;
      if (l > 0) p += S;
      Kp[l] = p; p += n * n * n;
    }
    // zero everything (boundary positions must read as 0), then load kappa
    const int total = (int)(p - reinterpret_cast<T*>(smem));
    T* base = reinterpret_cast<T*>(smem);
    for (int q = threadIdx.x; q < total; q += blockDim.x) base[q] = T(0);
    __syncthreads();
    for (int l = 0; l < a.nlev; ++l) {
      const int n = a.n0 >> l, ne = n * n * n;
      const T* kg = reinterpret_cast<const T*>(a.kap[l]) + (size_t)smp * ne;
      for (int q = threadIdx.x; q < ne; q += blockDim.x) Kp[l][q] = kg[q];
    }
    __syncthreads();
  }
  const T* b0 = bglob + (size_t)smp * a.gstride;
  int cur[kMaxLv];   // which of X[l][0..1] holds the current iterate

  // ------------------------------------------------ down: smooth, restrict
  for (int l = 0; l < a.nlev - 1; ++l) {
    const int n = a.n0 >> l;
    const T h = T(1) / T(n);
    const T* b = l == 0 ? b0 : Bv[l];
    const T* kap = Kp[l];
    T* x = X[l][0];
    // x1 = c2 D^-1 b
    FOR_INTERIOR(n, s) {
      T au, dg;
      q1(x, kap, n, s, h, au, dg);   // x is zero here: only the diagonal is used
      x[s] = T(a.c2[0]) * b[s] / dg;
    }
    __syncthreads();
    int c = 0;
    for (int st = 1; st < a.degree; ++st) {
      const T* xc = X[l][c];
      T* xo = X[l][c ^ 1];
      const T c1 = T(a.c1[st]), c2 = T(a.c2[st]);
      const bool use_xo = st > 1;
      FOR_INTERIOR(n, s) {
        T au, dg;
        q1(xc, kap, n, s, h, au, dg);
        const T prev = use_xo ? xc[s] - xo[s] : xc[s];
        xo[s] = xc[s] + c1 * prev + c2 * (b[s] - au) / dg;
      }
      __syncthreads();
      c ^= 1;
    }
    cur[l] = c;
    // residual into the free buffer, then restrict to the next level's rhs
    {
      const T* xc = X[l][c];
      T* t = X[l][c ^ 1];
      FOR_INTERIOR(n, s) {
        T au, dg;
        q1(xc, kap, n, s, h, au, dg);
        t[s] = b[s] - au;
      }
      __syncthreads();
      const int nc = n / 2, f2 = n * n;
      T* bc = Bv[l + 1];
      const int lc = lg2(nc);
      FOR_INTERIOR(nc, S) {
        const int I = S & (nc - 1), J = (S >> lc) & (nc - 1), K = S >> (2 * lc);
        const int ci = 2 * I + n * 2 * J + f2 * 2 * K;
        T acc = T(0);
        for (int dz = -1; dz <= 1; ++dz) {
          T az = T(0);
          for (int dy = -1; dy <= 1; ++dy) {
            const int row = ci + n * dy + f2 * dz;
            az += (dy == 0 ? T(1) : T(0.5)) * (T(0.5) * (t[row - 1] + t[row + 1]) + t[row]);
          }
          acc += (dz == 0 ? T(1) : T(0.5)) * az;
        }
        bc[S] = acc;
      }
      __syncthreads();
    }
  }
  // ------------------------------------------------- coarsest (2^3): exact
  {
    const int l = a.nlev - 1;
    if (threadIdx.x == 0) {
      const T* k = Kp[l];
      const T ks = ((k[0] + k[1]) + (k[2] + k[3])) + ((k[4] + k[5]) + (k[6] + k[7]));
      const T* b = l == 0 ? b0 : Bv[l];
      X[l][0][7] = b[7] / (T(0.5) * ks * (T(1) / T(3)));
    }
    cur[l] = 0;
    __syncthreads();
  }
  // ------------------------------------------------ up: prolong, smooth
  for (int l = a.nlev - 2; l >= 0; --l) {
    const int n = a.n0 >> l, nc = n / 2, c2n = nc * nc;
    const T h = T(1) / T(n);
    const T* b = l == 0 ? b0 : Bv[l];
    const T* kap = Kp[l];
    int c = cur[l];
    {
      T* x = X[l][c];
      const T* xc = X[l + 1][cur[l + 1]];
      const int ln = lg2(n);
      FOR_INTERIOR(n, s) {
        const int i = s & (n - 1), j = (s >> ln) & (n - 1), k = s >> (2 * ln);
        const int i0 = i >> 1, i1 = (i + 1) >> 1, j0 = j >> 1, j1 = (j + 1) >> 1, k0 = k >> 1, k1 = (k + 1) >> 1;
        auto at = [&](int ii, int jj, int kk) { return xc[ii + nc * jj + c2n * kk]; };
        auto row = [&](int jj, int kk) { return (i & 1) ? T(0.5) * (at(i0, jj, kk) + at(i1, jj, kk)) : at(i0, jj, kk); };
        auto pl = [&](int kk) { return (j & 1) ? T(0.5) * (row(j0, kk) + row(j1, kk)) : row(j0, kk); };
        x[s] += (k & 1) ? T(0.5) * (pl(k0) + pl(k1)) : pl(k0);
      }
      __syncthreads();
    }
    for (int st = 0; st < a.degree; ++st) {
      const T* xc = X[l][c];
      T* xo = X[l][c ^ 1];
      const T c1 = st == 0 ? T(0) : T(a.c1[st]), c2 = T(a.c2[st]);
      const bool use_xo = st > 0;
      FOR_INTERIOR(n, s) {
        T au, dg;
        q1(xc, kap, n, s, h, au, dg);
        const T prev = use_xo ? xc[s] - xo[s] : xc[s];
        xo[s] = xc[s] + c1 * prev + c2 * (b[s] - au) / dg;
      }
      __syncthreads();
      c ^= 1;
    }
    cur[l] = c;
  }
  // write the N0 result
  {
    const int n = a.n0;
    const T* x = X[0][cur[0]];
    T* xg = xglob + (size_t)smp * a.gstride;
    FOR_INTERIOR(n, s) xg[s] = x[s];
  }
}

}  // namespace

template <class T>
size_t vsmall_lds_bytes(int n0) {
  size_t tot = 0;
  for (int n = n0, l = 0; n >= 2; n /= 2, ++l) tot += (size_t)(2 + (l > 0)) * lds_stride(n) + (size_t)n * n * n;
  return tot * sizeof(T);
}

template <class T>
hipError_t launch_vsmall(int n0, int B, int degree, const double* c1, const double* c2, const T* const* kap_levels,
                         const T* b, T* x, const int* active, hipStream_t st) {
  SmallArgs a{};
  a.n0 = n0;
  a.nlev = 0;
  for (int n = n0; n >= 2; n /= 2) a.nlev++;
  if (a.nlev > kMaxLv || degree < 1 || degree > 16) return hipErrorInvalidValue;
  a.degree = degree;
  for (int s = 0; s < degree; ++s) {
    a.c1[s] = c1[s];
    a.c2[s] = c2[s];
  }
  a.gstride = grid_stride(n0);
  for (int l = 0; l < a.nlev; ++l) a.kap[l] = kap_levels[l];
  const size_t lds = vsmall_lds_bytes<T>(n0);
  k_vsmall<T><<<dim3(B), dim3(256), lds, st>>>(a, b, x, active);
  return hipGetLastError();
}

template size_t vsmall_lds_bytes<float>(int);
template size_t vsmall_lds_bytes<double>(int);
template hipError_t launch_vsmall<float>(int, int, int, const double*, const double*, const float* const*,
                                         const float*, float*, const int*, hipStream_t);
template hipError_t launch_vsmall<double>(int, int, int, const double*, const double*, const double* const*,
                                          const double*, double*, const int*, hipStream_t);

}  // namespace mlmc
