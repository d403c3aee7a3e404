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

// one of a level's two iterate buffers, chosen without indexing an array
// (a run-time index would put the pointer arrays in scratch memory)
template <class T>
__device__ __forceinline__ T* pick(T* const (&p)[2], int c) { return c ? p[1] : p[0]; }

// One V-cycle from the n0 = 2^NL mesh with every level in LDS: b0 the n0
// right-hand side (global or LDS), X/Bv/Kp the levels' buffers (boundary
// positions 0); the result is left in pick(X[0], cur[0]).  Called by every
// thread of the workgroup.  The level loops unroll (NL is a constant), so every
// mesh size and index mask is a constant too.
template <class T, int NL>
__device__ void vcycle_lds(const SmallArgs& a, const T* b0, T* (&X)[kMaxLv][2], T* const (&Bv)[kMaxLv],
                           T* const (&Kp)[kMaxLv], int (&cur)[kMaxLv]) {
  constexpr int N0 = 1 << NL;

  // ------------------------------------------------ down: smooth, restrict
#pragma unroll
  for (int l = 0; l < NL - 1; ++l) {
    const int n = N0 >> l;
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
      const T* xc = pick(X[l], c);
      T* xo = pick(X[l], c ^ 1);
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
      const T* xc = pick(X[l], c);
      T* t = pick(X[l], c ^ 1);
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
    constexpr int l = NL - 1;
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
#pragma unroll
  for (int l = NL - 2; l >= 0; --l) {
    const int n = N0 >> l, nc = n / 2, c2n = nc * nc;
    const T h = T(1) / T(n);
    const T* b = l == 0 ? b0 : Bv[l];
    const T* kap = Kp[l];
    int c = cur[l];
    {
      T* x = pick(X[l], c);
      const T* xc = pick(X[l + 1], cur[l + 1]);
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
      const T* xc = pick(X[l], c);
      T* xo = pick(X[l], c ^ 1);
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
}

// carve the V-cycle levels from LDS at p (x, second buffer, restricted
// right-hand side below n0, kappa); returns the end
template <class T, int NL>
__device__ T* carve_levels(T* p, T* (&X)[kMaxLv][2], T* (&Bv)[kMaxLv], T* (&Kp)[kMaxLv]) {
#pragma unroll
  for (int l = 0; l < NL; ++l) {
    const int n = (1 << NL) >> l, S = lds_stride(n);
    X[l][0] = p; p += S;
    X[l][1] = p; p += S;
    Bv[l] = l == 0 ? nullptr : p;
    if (l > 0) p += S;
    Kp[l] = p; p += n * n * n;
  }
  return p;
}

// threads of a k_vsmall workgroup: the 16^3 form holds 64 KB of LDS (two
// workgroups per CU), so it takes 16 waves to keep the SIMDs busy (1024
// threads: 55 us per launch of 1024 samples against 90 us with 256; 512 fell
// in between)
template <int NL>
constexpr int vsmall_threads() { return NL == 4 ? 1024 : 256; }

template <class T, int NL>
__global__ void __launch_bounds__(vsmall_threads<NL>()) k_vsmall(SmallArgs a, const T* __restrict__ bglob, T* __restrict__ xglob,
                                                const int* __restrict__ active) {
  const int smp = blockIdx.x;
  if (active && !active[smp]) return;
  extern __shared__ __align__(16) unsigned char smem[];
  T* X[kMaxLv][2];
  T* Bv[kMaxLv];
  T* Kp[kMaxLv];
  {
    T* p = carve_levels<T, NL>(reinterpret_cast<T*>(smem), X, Bv, Kp);
    // zero everything (boundary positions must read as 0), then load kappa
    const int total = (int)(p - reinterpret_cast<T*>(smem));
    T* base = reinterpret_cast<T*>(smem);
    for (int q = threadIdx.x; q < total; q += blockDim.x) base[q] = T(0);
    __syncthreads();
#pragma unroll
    for (int l = 0; l < NL; ++l) {
      const int n = (1 << NL) >> l, ne = n * n * n;
      const T* kg = reinterpret_cast<const T*>(a.kap[l]) + (size_t)smp * ne;
      for (int q = threadIdx.x; q < ne; q += blockDim.x) Kp[l][q] = kg[q];
    }
    __syncthreads();
  }
  const T* b0 = bglob + (size_t)smp * a.gstride;
  int cur[kMaxLv];   // which of X[l][0..1] holds the current iterate
  vcycle_lds<T, NL>(a, b0, X, Bv, Kp, cur);
  // write the N0 result
  {
    constexpr int n = 1 << NL;
    const T* x = pick(X[0], cur[0]);
    T* xg = xglob + (size_t)smp * a.gstride;
    FOR_INTERIOR(n, s) xg[s] = x[s];
  }
}

// --------------------------------------------- whole solve in one workgroup
// A mesh of at most 8^3 elements fits one workgroup with the whole state of
// the mixed-precision solve: in LDS the fp64 iterate, the fp32 inner residual
// and direction and the fp32 multigrid levels; in registers each node's fp64
// residual, fp32 correction and operator image (a node is owned by the same
// thread in every sweep).  One workgroup per sample then runs the fp64
// iterative refinement around the fp32 GMG-PCG
// (the same method as the level-by-level kernels: V-cycle preconditioner from
// vcycle_lds, inner relative tolerance, fp64 outer residual) with no launch
// per step.  Sums are taken over the workgroup in a fixed order, so a
// sample's result does not depend on its batch.
struct SolveSmallArgs {
  SmallArgs v;                // the V-cycle (n0 = the mesh)
  double rtol2, inner_tol2, bconst;
  int max_iter, max_outer;
};

// sum of v over the workgroup, the same value in every thread (wave sums,
// then the wave partials in order)
__device__ __forceinline__ double wg_allsum(double v, double* ws) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  const int nw = blockDim.x >> 6;
  for (int w = 0; w < nw; ++w) t += ws[w];
  return t;
}

// threads of a k_solve_small workgroup: one wave for 4^3 (27 unknowns), four for 8^3
template <int NL>
constexpr int solve_small_threads() { return NL == 2 ? 64 : 256; }

// 8^3: 20 KB of LDS per workgroup; held to 80 VGPRs (two spilled) so that
// six workgroups share a CU (4, 5, 6 and 7 per CU measured 0.21, 0.194,
// 0.187 and 0.185 us per sample over a 65536-sample batch)
template <int NL>
__global__ void __launch_bounds__(256, (NL == 3 ? 6 : 1)) k_solve_small(SolveSmallArgs a, const double* __restrict__ kap,
                                                     const double* __restrict__ bvec, double* __restrict__ uglob,
                                                     int* __restrict__ active, int* __restrict__ iters,
                                                     double* __restrict__ rr_out) {
  const int smp = blockIdx.x;
  constexpr int n = 1 << NL, n2 = n * n, ne = n2 * n;
  constexpr int TPB = solve_small_threads<NL>();
  constexpr int MAXP = (ne - n2 + TPB - 1) / TPB;   // positions per thread
  const int S = lds_stride(n);
  extern __shared__ __align__(16) unsigned char smem[];
  // LDS: what other threads read (the iterate for the fp64 operator, the
  // V-cycle's right-hand side, the PCG direction and the levels); the rest of
  // a node's state (fp64 residual, fp32 correction, operator image) stays in
  // the registers of the thread that owns the node in every sweep
  double* U = reinterpret_cast<double*>(smem);   // fp64 iterate
  double* ws = U + S;                              // wave partials
  float* Ri = reinterpret_cast<float*>(ws + 8);    // inner residual
  float* P = Ri + S;                               // direction
  float* X[kMaxLv][2];
  float* Bv[kMaxLv];
  float* Kp[kMaxLv];
  float* end = carve_levels<float, NL>(P + S, X, Bv, Kp);
  // the interior nodes this thread owns: position n^2 + tid + t * TPB
  auto own = [&](auto&& f) {
#pragma unroll
    for (int t = 0; t < MAXP; ++t) {
      const int s = n2 + (int)threadIdx.x + t * TPB;
      if (s < ne && (s & (n - 1)) != 0 && ((s >> NL) & (n - 1)) != 0) f(t, s);
    }
  };
  // zero everything (boundary positions must read as 0)
  for (int q = threadIdx.x; q < (int)(reinterpret_cast<double*>(Ri) - U); q += TPB) U[q] = 0.0;
  for (int q = threadIdx.x; q < (int)(end - Ri); q += TPB) Ri[q] = 0.0f;
  __syncthreads();
  const double* kg = kap + (size_t)smp * ne;
  for (int q = threadIdx.x; q < ne; q += TPB) Kp[0][q] = (float)kg[q];
  __syncthreads();
  // coarse kappa: the mean of the 8 children, in the order of k_coarsen
#pragma unroll
  for (int l = 1; l < NL; ++l) {
    const int nc = n >> l, nf = 2 * nc, f2 = nf * nf, nce = nc * nc * nc, lc = lg2(nc);
    for (int E = threadIdx.x; E < nce; E += TPB) {
      const int EX = E & (nc - 1), EY = (E >> lc) & (nc - 1), EZ = E >> (2 * lc);
      const float* f = Kp[l - 1] + 2 * EX + nf * 2 * EY + f2 * 2 * EZ;
      const float sv = ((f[0] + f[1]) + (f[nf] + f[nf + 1])) + ((f[f2] + f[f2 + 1]) + (f[f2 + nf] + f[f2 + nf + 1]));
      Kp[l][E] = sv * 0.125f;
    }
    __syncthreads();
  }
  const double* bg = bvec ? bvec + (size_t)smp * a.v.gstride : nullptr;
  const double h = 1.0 / n;
  const float hf = 1.0f / (float)n;
  double r64[MAXP];
  float xd[MAXP], qv[MAXP];
#pragma unroll
  for (int t = 0; t < MAXP; ++t) {
    r64[t] = 0.0;
    xd[t] = 0.0f;
    qv[t] = 0.0f;
  }
  double acc = 0.0;
  own([&](int t, int s) {
    const double bv = bg ? bg[s] : a.bconst;
    r64[t] = bv;
    acc += bv * bv;
  });
  const double bb = wg_allsum(acc, ws);
  int total = 0;
  bool done = false;
  double rr_last = bb;
  for (int outer = 0; outer < a.max_outer && total < a.max_iter && !done; ++outer) {
    // inner fp32 GMG-PCG on A d = fp32(r), from d = 0, to the inner tolerance
    acc = 0.0;
    own([&](int t, int s) {
      const float r = (float)r64[t];
      Ri[s] = r;
      xd[t] = 0.0f;
      acc += (double)r * (double)r;
    });
    const double tol2 = a.inner_tol2 * wg_allsum(acc, ws);
    int cur[kMaxLv];
    vcycle_lds<float, NL>(a.v, Ri, X, Bv, Kp, cur);
    acc = 0.0;
    own([&](int t, int s) {
      const float z = pick(X[0], cur[0])[s];
      P[s] = z;
      acc += (double)Ri[s] * (double)z;
    });
    double rz = wg_allsum(acc, ws);
    while (total < a.max_iter) {
      acc = 0.0;
      own([&](int t, int s) {
        float au, dg;
        q1<float>(P, Kp[0], n, s, hf, au, dg);
        qv[t] = au;
        acc += (double)P[s] * (double)au;
      });
      const double pq = wg_allsum(acc, ws);
      const float alpha = (float)(rz / pq);
      acc = 0.0;
      own([&](int t, int s) {
        xd[t] += alpha * P[s];
        const float r = Ri[s] - alpha * qv[t];
        Ri[s] = r;
        acc += (double)r * (double)r;
      });
      const double rr = wg_allsum(acc, ws);
      ++total;
      if (rr <= tol2 || !isfinite(rr)) break;   // a NaN or Inf residual ends the sample's solve
      vcycle_lds<float, NL>(a.v, Ri, X, Bv, Kp, cur);
      acc = 0.0;
      own([&](int t, int s) { acc += (double)Ri[s] * (double)pick(X[0], cur[0])[s]; });
      const double rzn = wg_allsum(acc, ws);
      const float beta = (float)(rzn / rz);
      rz = rzn;
      own([&](int t, int s) { P[s] = pick(X[0], cur[0])[s] + beta * P[s]; });
      __syncthreads();
    }
    // fp64 refinement: u += d, r = b - A u (fp64 kappa from global memory)
    own([&](int t, int s) { U[s] += (double)xd[t]; });
    __syncthreads();
    acc = 0.0;
    own([&](int t, int s) {
      double au, dg;
      q1<double>(U, kg, n, s, h, au, dg);
      const double r = (bg ? bg[s] : a.bconst) - au;
      r64[t] = r;
      acc += r * r;
    });
    rr_last = wg_allsum(acc, ws);
    done = rr_last <= a.rtol2 * bb || !isfinite(rr_last);
  }
  double* ug = uglob + (size_t)smp * a.v.gstride;
  for (int q = threadIdx.x; q < S; q += TPB) ug[q] = U[q];
  if (threadIdx.x == 0) {
    active[smp] = done ? 0 : 1;
    iters[smp] = total;
    if (rr_out) rr_out[smp] = rr_last;
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
  switch (a.nlev) {
    case 2: k_vsmall<T, 2><<<dim3(B), dim3(vsmall_threads<2>()), lds, st>>>(a, b, x, active); break;
    case 3: k_vsmall<T, 3><<<dim3(B), dim3(vsmall_threads<3>()), lds, st>>>(a, b, x, active); break;
    case 4: k_vsmall<T, 4><<<dim3(B), dim3(vsmall_threads<4>()), lds, st>>>(a, b, x, active); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

size_t solve_small_lds_bytes(int n) {
  const int S = lds_stride(n);
  return ((size_t)S + 8) * sizeof(double) + (size_t)2 * S * sizeof(float) + vsmall_lds_bytes<float>(n);
}

hipError_t launch_solve_small(int n, int B, int degree, const double* c1, const double* c2, const double* kap,
                              const double* bvec, double bconst, double* u, int* active, int* iters, double rtol,
                              double inner_rtol, int max_iter, int max_outer, hipStream_t st, double* rr_out) {
  if (n < 4 || n > 8 || (n & (n - 1)) || degree < 1 || degree > 16 || B <= 0) return hipErrorInvalidValue;
  SolveSmallArgs a{};
  a.v.n0 = n;
  for (int m = n; m >= 2; m /= 2) a.v.nlev++;
  a.v.degree = degree;
  for (int q = 0; q < degree; ++q) {
    a.v.c1[q] = c1[q];
    a.v.c2[q] = c2[q];
  }
  a.v.gstride = grid_stride(n);
  a.rtol2 = rtol * rtol;
  a.inner_tol2 = inner_rtol * inner_rtol;
  a.bconst = bconst;
  a.max_iter = max_iter;
  a.max_outer = max_outer;
  const size_t lds = solve_small_lds_bytes(n);
  if (n == 4)
    k_solve_small<2><<<dim3(B), dim3(solve_small_threads<2>()), lds, st>>>(a, kap, bvec, u, active, iters, rr_out);
  else
    k_solve_small<3><<<dim3(B), dim3(solve_small_threads<3>()), lds, st>>>(a, kap, bvec, u, active, iters, rr_out);
  return hipGetLastError();
}

template size_t vsmall_lds_bytes<float>(int);
template size_t vsmall_lds_bytes<double>(int);
template hipError_t launch_vsmall<float>(int, int, int, const double*, const double*, const float* const*,
                                         const float*, float*, const int*, hipStream_t);
template hipError_t launch_vsmall<double>(int, int, int, const double*, const double*, const double* const*,
                                          const double*, double*, const int*, hipStream_t);

}  // namespace mlmc
