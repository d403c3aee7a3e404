// Matrix-free Q1 operator and the geometric-multigrid kernels (grid layout).
//
// Operator (eq. model with per-element kappa, Q1 hexahedra, Sec. 2.1-2.2):
//   (A u)_i = h sum_{e owns i} kappa_e sum_b Khat[a_i(e)][b] u_b
// with Khat the unit-cube Q1 stiffness.  Khat[a][b] is 1/3 for a = b, 0 when
// a and b share an edge, and -1/12 when they differ in two or three
// coordinates, so for element e seen from node i (its far corner along signs
// (sx, sy, sz)) the row reduces to
//   kappa_e [ u_i / 3 - (u_(sx,sy,0) + u_(sx,0,sz) + u_(0,sy,sz) + u_(sx,sy,sz)) / 12 ]
// i.e. 20 neighbour values (12 edge, 8 corner) and the 8 element coefficients
// per node; face neighbours never enter.  The Jacobi diagonal is
// D_i = (h/3) sum_{e owns i} kappa_e, from the same 8 coefficients.
//
// z-marching engine: a thread owns V consecutive nodes of one row (one
// 16-byte vector: 4 floats or 2 doubles) and walks up the planes of a chunk,
// keeping the 3 x 3 x (V+2) window of u (planes k-1..k+1, rows j-1..j+1) and
// the 2 x 2 x (V+1) window of kappa in registers.  Each plane step loads one
// new u plane (3 row vectors + 2 halo values per row) and one kappa plane (2
// row vectors + 1 halo value per row): ~3 vector loads per node in fp32
// instead of 29 scalar ones, so the kernel is limited by HBM rather than by
// the L1/TA path.  The epilogue (apply, residual, Chebyshev step, PCG apply
// with its dot product, fp64 outer residual) consumes A u and D per node.
//
// Multigrid pieces: full-weighting restriction P^T and trilinear
// prolongation P between the n and n/2 grids, exact solve of the single
// unknown of the 2^3 mesh, and the 8-child mean of kappa for the
// rediscretised coarse operators.
#include "common.hpp"
#include "grid.hpp"
#include "kernels.hpp"

#include <type_traits>

namespace mlmc {
namespace {

__device__ __forceinline__ int ilog2(int n) { return 31 - __clz(n); }

__device__ __forceinline__ double block_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __shared__ double wsum[kBlock / 64];
  const int nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < nw; ++w) t += wsum[w];
  return t;
}

template <int X>
using Ic = std::integral_constant<int, X>;

template <class T, int V>
struct Vec {
  typedef T type __attribute__((ext_vector_type(V)));
};

template <class T, int V>
__device__ __forceinline__ void vload(const T* p, T* dst) {
  if constexpr (V == 1) {
    dst[0] = *p;
  } else {
    typedef typename Vec<T, V>::type vt;
    const vt v = *reinterpret_cast<const vt*>(p);
#pragma unroll
    for (int q = 0; q < V; ++q) dst[q] = v[q];
  }
}

template <class T, int V>
__device__ __forceinline__ void vstore(T* p, const T* src) {
  if constexpr (V == 1) {
    *p = src[0];
  } else {
    typedef typename Vec<T, V>::type vt;
    vt v;
#pragma unroll
    for (int q = 0; q < V; ++q) v[q] = src[q];
    *reinterpret_cast<vt*>(p) = v;
  }
}

// 1 / D for the Jacobi scaling: the hardware reciprocal in fp32 (1 ulp; the
// smoother only needs a fixed diagonal scaling, and it is the same one in
// every smoothing step, so the V-cycle stays symmetric), a correctly rounded
// division in fp64.
__device__ __forceinline__ float inv_diag(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double inv_diag(double d) { return 1.0 / d; }

// ------------------------------------------------------------ epilogues
// Each epilogue sees, for the V nodes i0 .. i0+V-1 at position `pos` (index
// of node i0 in the batch array), A u, D and the centre values of u; `ok[v]`
// is false for the boundary node i = 0.  Stores write 0 there.  The vectors
// an epilogue reads at its own nodes are loaded by pre(pos) into its members:
// the engines call it one plane step ahead (LDS engine), or before the loads
// of the stencil window (register engine), so those loads are in flight while
// the stencil is computed instead of being waited for right after it.

template <class T, int V>
struct EpiApply {
  static constexpr bool kReduce = false;
  static constexpr bool kBegin = false;
  T* y;
  __device__ void pre(size_t) {}
  __device__ void operator()(size_t pos, const T* au, const T* dg, const T* uc, const bool* ok, double&) const {
    T o[V];
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = ok[v] ? au[v] : T(0);
    vstore<T, V>(y + pos, o);
  }
};

template <class T, int V>
struct EpiResidual {
  static constexpr bool kReduce = false;
  static constexpr bool kBegin = false;
  const T* b;
  T* r;
  T bv[V];
  __device__ void pre(size_t pos) { vload<T, V>(b + pos, bv); }
  __device__ void operator()(size_t pos, const T* au, const T* dg, const T* uc, const bool* ok, double&) const {
    T o[V];
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = ok[v] ? bv[v] - au[v] : T(0);
    vstore<T, V>(r + pos, o);
  }
};

// out = x + c1 (x - xo) + c2 D^-1 (b - A x); without xo the previous iterate is
// 0.  DOT also accumulates b . out (the r . z of the enclosing PCG when this is
// the last smoothing step of the finest level).
// `save` (may be null) receives the iterate the step started from (used when
// that iterate was formed on the fly, see PRO below).
template <class T, int V, bool USE_XO, bool DOT>
struct EpiCheb {
  static constexpr bool kReduce = DOT;
  static constexpr bool kBegin = true;
  const T* b;
  const T* xo;
  T* out;
  T c1, c2;
  T* save = nullptr;
  // per-sample right-hand side: b1 where (bstate[s] & 8) (may be null)
  const T* b1 = nullptr;
  const int* bstate = nullptr;
  T bv[V], xov[V];
  __device__ void begin(uint32_t s) {
    if (bstate && (bstate[s] & 8)) b = b1;
  }
  __device__ void pre(size_t pos) {
    vload<T, V>(b + pos, bv);
    if (USE_XO) vload<T, V>(xo + pos, xov);
  }
  __device__ void operator()(size_t pos, const T* au, const T* dg, const T* uc, const bool* ok, double& acc) const {
    T o[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const T prev = USE_XO ? uc[v] - xov[v] : uc[v];
      o[v] = ok[v] ? uc[v] + c1 * prev + c2 * (bv[v] - au[v]) * inv_diag(dg[v]) : T(0);
      if (DOT) acc += (double)bv[v] * (double)o[v];
    }
    vstore<T, V>(out + pos, o);
    if (save) {
      T sv[V];
#pragma unroll
      for (int v = 0; v < V; ++v) sv[v] = ok[v] ? uc[v] : T(0);
      vstore<T, V>(save + pos, sv);
    }
  }
};

// q = A p, accumulate p . q
template <class T, int V>
struct EpiPcgApply {
  static constexpr bool kReduce = true;
  static constexpr bool kBegin = false;
  T* q;
  __device__ void pre(size_t) {}
  __device__ void operator()(size_t pos, const T* au, const T* dg, const T* uc, const bool* ok, double& acc) const {
    T o[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      o[v] = ok[v] ? au[v] : T(0);
      acc += (double)uc[v] * (double)o[v];
    }
    vstore<T, V>(q + pos, o);
  }
};

// r = b - A x (fp64 outer residual), accumulate r . r; b is the constant
// bconst, or the vector bvec when given
template <class T, int V>
struct EpiTrueResidual {
  static constexpr bool kReduce = true;
  static constexpr bool kBegin = false;
  T bconst;
  T* r;
  const T* bvec = nullptr;
  T bl[V];
  __device__ void pre(size_t pos) {
    if (bvec) vload<T, V>(bvec + pos, bl);
  }
  __device__ void operator()(size_t pos, const T* au, const T* dg, const T* uc, const bool* ok, double& acc) const {
    T o[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      o[v] = ok[v] ? (bvec ? bl[v] : bconst) - au[v] : T(0);
      acc += (double)o[v] * (double)o[v];
    }
    vstore<T, V>(r + pos, o);
  }
};

// fp64 refinement step with the correction applied on the fly: the operand
// is u_new = u + d (fp32 d), and the kernel writes u_new to a second buffer,
// the fp64 residual r = bconst - A u_new demoted to fp32 (the next inner
// right-hand side), and the fp64 partial sums of r . r.
template <class T, int V>
struct EpiRefine {
  static constexpr bool kReduce = true;
  static constexpr bool kBegin = false;
  T bconst;
  T* uout;
  float* rin;
  const T* bvec = nullptr;   // the right-hand side vector, if not the constant bconst
  T bl[V];
  __device__ void pre(size_t pos) {
    if (bvec) vload<T, V>(bvec + pos, bl);
  }
  __device__ void operator()(size_t pos, const T* au, const T* dg, const T* uc, const bool* ok, double& acc) const {
    T us[V];
    float f[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const T r = ok[v] ? (bvec ? bl[v] : bconst) - au[v] : T(0);
      acc += (double)r * (double)r;
      f[v] = (float)r;
      us[v] = ok[v] ? uc[v] : T(0);
    }
    vstore<T, V>(uout + pos, us);
    vstore<float, V>(rin + pos, f);
  }
};

// x0 = 0 Chebyshev step: out = c2 D^-1 b (needs only the kappa window)
template <class T, int V>
struct EpiChebZero {
  static constexpr bool kReduce = false;
  static constexpr bool kBegin = false;
  const T* b;
  T* out;
  T c2;
  T bv[V];
  __device__ void pre(size_t pos) { vload<T, V>(b + pos, bv); }
  __device__ void operator()(size_t pos, const T* au, const T* dg, const T* uc, const bool* ok, double&) const {
    T o[V];
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = ok[v] ? c2 * bv[v] * inv_diag(dg[v]) : T(0);
    vstore<T, V>(out + pos, o);
  }
};

// One LDS row segment of the u window: the thread's V values by one vector
// read, the halos i0-1 and i0+V from the neighbouring lanes of the same row
// (the G <= 64 lanes of a row are consecutive lanes of one wave; the row
// ends are zero: u(-1) = u(n) = 0).  LDS rows are dense (n values, no halo
// cells): scalar halo reads at a 16-byte lane stride would put all lanes of
// a wave on a quarter of the LDS banks, and the padding would cost the LDS
// that a fourth workgroup per CU needs.
// whole-wave DPP shifts (GFX9 wave_shr:1 / wave_shl:1, full VALU rate):
// lane l receives lane l-1 (from_prev) or lane l+1 (from_next), 0 at the ends
__device__ __forceinline__ int dpp_prev_i(int x) { return __builtin_amdgcn_update_dpp(0, x, 0x138, 0xF, 0xF, true); }
__device__ __forceinline__ int dpp_next_i(int x) { return __builtin_amdgcn_update_dpp(0, x, 0x130, 0xF, 0xF, true); }
__device__ __forceinline__ float from_prev(float x) { return __int_as_float(dpp_prev_i(__float_as_int(x))); }
__device__ __forceinline__ float from_next(float x) { return __int_as_float(dpp_next_i(__float_as_int(x))); }
__device__ __forceinline__ double from_prev(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = dpp_prev_i((int)(v & 0xffffffffll)), hi = dpp_prev_i((int)(v >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
__device__ __forceinline__ double from_next(double x) {
  const long long v = __double_as_longlong(x);
  const int lo = dpp_next_i((int)(v & 0xffffffffll)), hi = dpp_next_i((int)(v >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Halo modes of the row exchange.  HALO_SELECT: a wave holds several rows;
// whole-wave shifts and a select of 0 at the row ends.  HALO_DPPROW: a row is
// exactly one 16-lane DPP row (G = 16): shifts within the DPP rows, whose ends
// receive 0 with no select.  HALO_WAVE: a row is exactly one wave (G = 64):
// whole-wave shifts, 0 at the wave ends with no select.
enum : int { HALO_SELECT = 0, HALO_DPPROW = 1, HALO_WAVE = 2 };
inline int halo_mode(int G) { return G == 16 ? HALO_DPPROW : (G == 64 ? HALO_WAVE : HALO_SELECT); }

template <int HALO>
__device__ __forceinline__ int halo_prev_i(int x) {
  if constexpr (HALO == HALO_DPPROW) return __builtin_amdgcn_update_dpp(0, x, 0x111, 0xF, 0xF, true);   // row_shr:1
  else return dpp_prev_i(x);
}
template <int HALO>
__device__ __forceinline__ int halo_next_i(int x) {
  if constexpr (HALO == HALO_DPPROW) return __builtin_amdgcn_update_dpp(0, x, 0x101, 0xF, 0xF, true);   // row_shl:1
  else return dpp_next_i(x);
}
template <int HALO, class T>
__device__ __forceinline__ T halo_prev(T x, int gx) {
  T v;
  if constexpr (sizeof(T) == 4) {
    v = __int_as_float(halo_prev_i<HALO>(__float_as_int(x)));
  } else {
    const long long w = __double_as_longlong(x);
    const int lo = halo_prev_i<HALO>((int)(w & 0xffffffffll)), hi = halo_prev_i<HALO>((int)(w >> 32));
    v = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  }
  if constexpr (HALO == HALO_SELECT) return gx == 0 ? T(0) : v;
  else return v;
}
template <int HALO, class T>
__device__ __forceinline__ T halo_next(T x, int gx, int G) {
  T v;
  if constexpr (sizeof(T) == 4) {
    v = __int_as_float(halo_next_i<HALO>(__float_as_int(x)));
  } else {
    const long long w = __double_as_longlong(x);
    const int lo = halo_next_i<HALO>((int)(w & 0xffffffffll)), hi = halo_next_i<HALO>((int)(w >> 32));
    v = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  }
  if constexpr (HALO == HALO_SELECT) return gx == G - 1 ? T(0) : v;
  else return v;
}

template <class T, int V, int HALO = HALO_SELECT>
__device__ __forceinline__ void lds_urow(const T* row, T* dst, int gx, int G) {
  vload<T, V>(row, dst + 1);
  dst[0] = halo_prev<HALO>(dst[V], gx);
  dst[V + 1] = halo_next<HALO>(dst[1], gx, G);
}

// kappa row segment: element i0-1 (zero for i0 = 0) and i0 .. i0+V-1
template <class T, int V, int HALO = HALO_SELECT>
__device__ __forceinline__ void lds_krow(const T* row, T* dst, int gx) {
  vload<T, V>(row, dst + 1);
  dst[0] = halo_prev<HALO>(dst[V], gx);
}

// The 8-element sum of kappa at each of the V nodes from the four kappa row
// segments around them (element layers dz = node plane -1 / +0, element rows
// dy likewise; column c = v holds the element left of node v, c = v + 1 the
// one right of it): pair sums over the two layers, then over the two rows,
// then over the two columns.  The stencil kernels and the on-the-fly
// smoothing operand take the diagonal from this same sequence, so they agree
// to the bit.
template <class T, int V>
__device__ __forceinline__ void ksum_from_rows(const T (&K)[2][2][V + 1], T (&Z)[2][V + 1], T* ks) {
  T C[V + 1];
#pragma unroll
  for (int c = 0; c <= V; ++c) {
    Z[0][c] = K[0][0][c] + K[1][0][c];
    Z[1][c] = K[0][1][c] + K[1][1][c];
    C[c] = Z[0][c] + Z[1][c];
  }
#pragma unroll
  for (int v = 0; v < V; ++v) ks[v] = C[v] + C[v + 1];
}

// Q1 row pieces of the V nodes i0 .. i0+V-1 of row j, plane k, from the LDS
// tile: Kd (d = 0, 1) point at element row j-1 of element layers k-1 and k at
// column i0 (element row j one row further); Um, U0, Up at node row j-1 of
// planes k-1, k, k+1 (rows j, j+1 further).  ks: the 8-element sum; fr: the
// 20 neighbours (12 edge diagonals and 8 corners) each times the sum of kappa
// over the elements it shares with the node (two elements for an edge
// diagonal, one for a corner); uc: the centre values.  A u = h (ks uc / 3 -
// fr / 12).  The kappa pair sums are shared by the V nodes of the segment.
template <class T, int V, int HALO, bool CHAIN = false>
__device__ __forceinline__ void q1_gather(const T* K0, const T* K1, const T* Um, const T* U0, const T* Up, int rsh,
                                          int gx, int G, T* ks, T* fr, T* uc) {
  T K[2][2][V + 1];
#pragma unroll
  for (int dy = 0; dy < 2; ++dy) {
    lds_krow<T, V, HALO>(K0 + (dy << rsh), K[0][dy], gx);
    lds_krow<T, V, HALO>(K1 + (dy << rsh), K[1][dy], gx);
  }
  T Z[2][V + 1];
  ksum_from_rows<T, V>(K, Z, ks);
  {
    // plane k: the edge diagonals (i +- 1, j +- 1), two element layers each
    T Rm[V + 2], Rp[V + 2];
    lds_urow<T, V, HALO>(U0, Rm, gx, G);
    vload<T, V>(U0 + (1 << rsh), uc);
    lds_urow<T, V, HALO>(U0 + (2 << rsh), Rp, gx, G);
#pragma unroll
    for (int v = 0; v < V; ++v)
      fr[v] = Z[0][v] * Rm[v] + Z[0][v + 1] * Rm[v + 2] + Z[1][v] * Rp[v] + Z[1][v + 1] * Rp[v + 2];
  }
#pragma unroll
  for (int dz = 0; dz < 2; ++dz) {
    // plane k -+ 1: edge diagonals (i +- 1, j) over the two element rows,
    // (i, j +- 1) over the two element columns, and the four corners
    const T* U = dz ? Up : Um;
    T Q[3][V + 2];
#pragma unroll
    for (int dy = 0; dy < 3; ++dy) lds_urow<T, V, HALO>(U + (dy << rsh), Q[dy], gx, G);
    if constexpr (CHAIN) {
      // one fused multiply-add per neighbour into the running sums, row by
      // row (fewer instructions; more registers live)
#pragma unroll
      for (int v = 0; v < V; ++v) {
        fr[v] = fma(K[dz][0][v] + K[dz][0][v + 1], Q[0][v + 1], fr[v]);
        fr[v] = fma(K[dz][0][v], Q[0][v], fr[v]);
        fr[v] = fma(K[dz][0][v + 1], Q[0][v + 2], fr[v]);
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        fr[v] = fma(K[dz][0][v] + K[dz][1][v], Q[1][v], fr[v]);
        fr[v] = fma(K[dz][0][v + 1] + K[dz][1][v + 1], Q[1][v + 2], fr[v]);
      }
#pragma unroll
      for (int v = 0; v < V; ++v) {
        fr[v] = fma(K[dz][1][v] + K[dz][1][v + 1], Q[2][v + 1], fr[v]);
        fr[v] = fma(K[dz][1][v], Q[2][v], fr[v]);
        fr[v] = fma(K[dz][1][v + 1], Q[2][v + 2], fr[v]);
      }
    } else {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const T y0 = K[dz][0][v] + K[dz][1][v], y1 = K[dz][0][v + 1] + K[dz][1][v + 1];
        const T x0 = K[dz][0][v] + K[dz][0][v + 1], x1 = K[dz][1][v] + K[dz][1][v + 1];
        fr[v] += y0 * Q[1][v] + y1 * Q[1][v + 2] + x0 * Q[0][v + 1] + x1 * Q[2][v + 1] +
                 (K[dz][0][v] * Q[0][v] + K[dz][0][v + 1] * Q[0][v + 2] + K[dz][1][v] * Q[2][v] +
                  K[dz][1][v + 1] * Q[2][v + 2]);
      }
    }
  }
}

// N consecutive values (N = 1 or an aligned vector)
template <class T, int N>
__device__ __forceinline__ void nload(const T* p, T* dst) {
  if constexpr (N == 1) dst[0] = *p;
  else vload<T, N>(p, dst);
}

template <class T, int N>
__device__ __forceinline__ void nstore(T* p, const T* src) {
  if constexpr (N == 1) p[0] = src[0];
  else vstore<T, N>(p, src);
}

// PCG update fused with the first Chebyshev step (zero iterate) of the
// preconditioner that follows it: x += alpha p, r -= alpha q, sum r.r, and
// z = c2 D^-1 r with the updated r (needs only the kappa window).
template <class T, int V>
struct EpiPcgUpdateZero {
  static constexpr bool kReduce = true;
  static constexpr bool kBegin = true;
  T* x;
  const T* p;
  T* r;
  const T* q;
  T* z;
  const double* alpha;
  T c2;
  T a = T(0);
  T xv[V], pv[V], rv[V], qv[V];
  __device__ void begin(uint32_t b) { a = (T)alpha[b]; }
  __device__ void pre(size_t pos) {
    vload<T, V>(x + pos, xv);
    vload<T, V>(p + pos, pv);
    vload<T, V>(r + pos, rv);
    vload<T, V>(q + pos, qv);
  }
  __device__ void operator()(size_t pos, const T* au, const T* dg, const T* uc, const bool* ok, double& acc) {
    T zo[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      xv[v] = xv[v] + a * pv[v];
      rv[v] = rv[v] - a * qv[v];
      acc += (double)rv[v] * (double)rv[v];
      zo[v] = ok[v] ? c2 * rv[v] * inv_diag(dg[v]) : T(0);
    }
    vstore<T, V>(x + pos, xv);
    vstore<T, V>(r + pos, rv);
    vstore<T, V>(z + pos, zo);
  }
};

// PCG update without the iterate (the fused direction step applies x += alpha p
// one iteration later): r -= alpha q, sum r.r, and z = c2 D^-1 r with the
// updated r (the zero-iterate step of the following V-cycle).
template <class T, int V>
struct EpiPcgRUpdateZero {
  static constexpr bool kReduce = true;
  static constexpr bool kBegin = true;
  T* r;
  const T* q;
  T* z;
  const double* alpha;
  T c2;
  T a = T(0);
  T rv[V], qv[V];
  __device__ void begin(uint32_t b) { a = (T)alpha[b]; }
  __device__ void pre(size_t pos) {
    vload<T, V>(r + pos, rv);
    vload<T, V>(q + pos, qv);
  }
  __device__ void operator()(size_t pos, const T* au, const T* dg, const T* uc, const bool* ok, double& acc) {
    T zo[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      rv[v] = rv[v] - a * qv[v];
      acc += (double)rv[v] * (double)rv[v];
      zo[v] = ok[v] ? c2 * rv[v] * inv_diag(dg[v]) : T(0);
    }
    vstore<T, V>(r + pos, rv);
    vstore<T, V>(z + pos, zo);
  }
};

// The conjugate direction fused with the operator apply (operand OP_DIR:
// p = z + beta p_old staged on the fly): writes p into the other direction
// buffer (neighbouring workgroups still read p_old), q = A p, the partial
// sums of p . q, and applies the previous iteration's x += alpha p_old (alpha
// is still that iteration's value when this kernel runs).  On a sample's
// first direction there is no previous update, and an iterate marked fresh
// (pstate bit 2) is written rather than updated.
template <class T, int V>
struct EpiDirApply {
  static constexpr bool kReduce = true;
  static constexpr bool kBegin = true;
  T* x;
  T* p0;
  T* p1;
  T* q;
  const int* pstate;
  const double* alpha;
  T a = T(0);
  const T* pold = nullptr;
  T* pnew = nullptr;
  bool prev = false, fresh = false;
  T xv[V], pv[V];
  __device__ void pre(size_t pos) {
    if (prev) {
      if (!fresh) vload<T, V>(x + pos, xv);
      vload<T, V>(pold + pos, pv);
    }
  }
  // the same with p_old at the thread's own nodes already in registers (the
  // LDS engine stages them): no second read of p_old
  template <class W>
  __device__ void pre_own(size_t pos, const W& pown) {
    if (prev) {
      if (!fresh) vload<T, V>(x + pos, xv);
#pragma unroll
      for (int v = 0; v < V; ++v) pv[v] = pown[v];
    }
  }
  __device__ void begin(uint32_t b) {
    const int ps = pstate[b];
    prev = (ps & 2) == 0;
    fresh = (ps & 4) != 0;
    a = (T)alpha[b];
    pold = (ps & 1) ? p1 : p0;
    pnew = (ps & 1) ? p0 : p1;
  }
  __device__ void operator()(size_t pos, const T* au, const T* dg, const T* uc, const bool* ok, double& acc) const {
    T pn[V], o[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      pn[v] = ok[v] ? uc[v] : T(0);
      o[v] = ok[v] ? au[v] : T(0);
      acc += (double)pn[v] * (double)o[v];
    }
    vstore<T, V>(pnew + pos, pn);
    vstore<T, V>(q + pos, o);
    if (prev) {
      // a fresh iterate is written, not updated (it holds no value yet)
      T xn[V];
#pragma unroll
      for (int v = 0; v < V; ++v) xn[v] = fresh ? a * pv[v] : xv[v] + a * pv[v];
      vstore<T, V>(x + pos, xn);
    }
  }
};

// --------------------------------------------------------- z-march engine
// PF: issue the loads of the next plane step before computing the current one
// (one more plane of registers, more memory-level parallelism per wave).
// PRO: the operand is u + P xc, with xc on the n/2 mesh (stride cstride) and P
// the trilinear prolongation: the coarse-grid correction of a V-cycle is
// applied while its first post-smoothing step reads the iterate, instead of
// by a separate pass that reads and writes the fine vector.  A sliding window
// of two coarse planes x three coarse rows (the parents of the thread's three
// fine rows) is kept in registers; a new coarse plane is loaded every second
// fine plane.
// ADDD: the operand is u + d with d an fp32 vector in the same layout (u may
// be null: zero).
template <class T, int V, bool NEED_U, bool PF, bool PRO, bool ADDD, class Epi>
__global__ void __launch_bounds__(256) k_zmarch(ZGeom g, size_t stride, T h, const T* __restrict__ u,
                                                const T* __restrict__ kap, const int* __restrict__ active,
                                                double* __restrict__ partial, uint32_t pstride, Epi epi,
                                                const T* __restrict__ xc, size_t cstride,
                                                const float* __restrict__ dadd) {
  static_assert(!(PRO && (PF || !NEED_U)), "the fused prolongation uses the plain u window");
  static_assert(!(ADDD && (PF || PRO || !NEED_U)), "the added vector uses the plain u window");
  const uint32_t per = g.parts();
  const uint32_t lin = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t b = lin / per;
  const uint32_t part = lin - b * per;
  if (active && !active[b]) return;
  const int rb = (int)(part % (uint32_t)g.row_blocks), zb = (int)(part / (uint32_t)g.row_blocks);
  const int n = g.n, n2 = n * n;
  const int gx = (int)threadIdx.x % g.G, jr = (int)threadIdx.x / g.G;
  const int j = 1 + rb * g.rows + jr;
  const int i0 = gx * V;
  const int k0 = 1 + zb * g.zlen;
  int k1 = k0 + g.zlen;
  if (k1 > n) k1 = n;
  const bool valid = jr < g.rows && j <= n - 1 && k0 < k1;
  double acc = 0.0;
  if constexpr (Epi::kBegin) epi.begin(b);
  if (valid) {
    const T* ub = u ? u + (size_t)b * stride : nullptr;
    const float* db = ADDD ? dadd + (size_t)b * stride : nullptr;
    const T* kb = kap + (size_t)b * n2 * n;
    bool ok[V];
#pragma unroll
    for (int v = 0; v < V; ++v) ok[v] = (i0 + v) != 0;
    T U[3][3][V + 2];
    T K[2][2][V + 1];
    T PU[PF ? 3 : 1][V + 2];
    T PK[PF ? 2 : 1][V + 1];
    auto load_urow = [&](T* dst, int r, int kk) {
      const size_t off = (size_t)n * (j - 1 + r) + (size_t)n2 * kk;
      if (!ADDD || ub) {
        const T* row = ub + off;
        dst[0] = i0 > 0 ? row[i0 - 1] : T(0);
        vload<T, V>(row + i0, dst + 1);
        dst[V + 1] = row[i0 + V];   // position n is the next row's zero
      } else {
#pragma unroll
        for (int c = 0; c < V + 2; ++c) dst[c] = T(0);
      }
      if (ADDD) {
        const float* drow = db + off;
        float dv[V];
        vload<float, V>(drow + i0, dv);
        dst[0] += i0 > 0 ? (T)drow[i0 - 1] : T(0);
#pragma unroll
        for (int v = 0; v < V; ++v) dst[1 + v] += (T)dv[v];
        dst[V + 1] += (T)drow[i0 + V];
      }
    };
    auto load_krow = [&](T* dst, int r, int ez) {
      const T* row = kb + (size_t)n * (j - 1 + r) + (size_t)n2 * ez;
      dst[0] = i0 > 0 ? row[i0 - 1] : T(0);
      vload<T, V>(row + i0, dst + 1);
    };
    // ---- fused prolongation (PRO)
    // Coarse values I0-1 .. I0+V/2 (I0 = i0/2) of coarse rows JA .. JA+2,
    // JA = (j-1)/2 rounded down; the third row is needed only for even j.
    // Fine row j-1+r, fine plane kk: even index -> one coarse line, odd ->
    // the mean of two; positions outside the interior read coarse zeros.
    constexpr int CW = V / 2 + 2;
    T C[2][3][PRO ? CW : 1];
    int cK = 0;
    const int nc = n >> 1, nc2 = nc * nc;
    const bool jodd = (j & 1) != 0;
    const int JA = (j - 1) >> 1;
    const T* cb = PRO ? xc + (size_t)b * cstride : nullptr;
    auto load_cplane = [&](int slot, int K) {
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        T* dst = C[slot][s];
        if (K > nc || (s == 2 && jodd)) {
#pragma unroll
          for (int q = 0; q < CW; ++q) dst[q] = T(0);
          continue;
        }
        const T* row = cb + (size_t)nc * (JA + s) + (size_t)nc2 * K + (i0 >> 1);
        dst[0] = i0 > 0 ? row[-1] : T(0);
        nload<T, V / 2>(row, dst + 1);
        dst[V / 2 + 1] = row[V / 2];
      }
    };
    auto cshift = [&](int kk) {   // make the window hold coarse planes kk/2 and kk/2 + 1
      if ((kk >> 1) > cK) {
#pragma unroll
        for (int s = 0; s < 3; ++s)
#pragma unroll
          for (int q = 0; q < CW; ++q) C[0][s][q] = C[1][s][q];
        ++cK;
        load_cplane(1, cK + 1);
      }
    };
    auto add_pro = [&](T (*rows)[V + 2], int kk) {   // rows[r] += (P xc)(row j-1+r, plane kk)
      const bool kodd = (kk & 1) != 0;
      T P[3][CW];
#pragma unroll
      for (int s = 0; s < 3; ++s)
#pragma unroll
        for (int q = 0; q < CW; ++q) P[s][q] = kodd ? T(0.5) * (C[0][s][q] + C[1][s][q]) : C[0][s][q];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        T L[CW];
#pragma unroll
        for (int q = 0; q < CW; ++q) {
          const T mid01 = T(0.5) * (P[0][q] + P[1][q]), mid12 = T(0.5) * (P[1][q] + P[2][q]);
          const T a = r == 0 ? P[0][q] : (r == 1 ? mid01 : P[1][q]);    // j odd
          const T c = r == 0 ? mid01 : (r == 1 ? P[1][q] : mid12);      // j even
          L[q] = jodd ? a : c;
        }
#pragma unroll
        for (int t = 0; t < V + 2; ++t)
          rows[r][t] += (t & 1) ? L[(t + 1) / 2] : T(0.5) * (L[t / 2] + L[t / 2 + 1]);
      }
    };
    if (PRO) {
      cK = (k0 - 1) >> 1;
      load_cplane(0, cK);
      load_cplane(1, cK + 1);
    }
    if (NEED_U) {
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        load_urow(U[0][r], r, k0 - 1);
        load_urow(U[1][r], r, k0);
      }
      if (PRO) {
        add_pro(U[0], k0 - 1);
        cshift(k0);
        add_pro(U[1], k0);
      }
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) load_krow(K[0][r], r, k0 - 1);
    if (PF) {
      if (NEED_U)
#pragma unroll
        for (int r = 0; r < 3; ++r) load_urow(PU[r], r, k0 + 1);
#pragma unroll
      for (int r = 0; r < 2; ++r) load_krow(PK[r], r, k0);
    }
    const T third = T(1) / T(3), twelfth = T(1) / T(12);
    for (int k = k0; k < k1; ++k) {
      epi.pre((size_t)b * stride + i0 + (size_t)n * j + (size_t)n2 * k);
      if (PF) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < V + 2; ++c)
            if (NEED_U) U[2][r][c] = PU[r][c];
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
          for (int c = 0; c < V + 1; ++c) K[1][r][c] = PK[r][c];
        if (k + 1 < k1) {
          if (NEED_U)
#pragma unroll
            for (int r = 0; r < 3; ++r) load_urow(PU[r], r, k + 2);
#pragma unroll
          for (int r = 0; r < 2; ++r) load_krow(PK[r], r, k + 1);
        }
      } else {
        if (NEED_U) {
#pragma unroll
          for (int r = 0; r < 3; ++r) load_urow(U[2][r], r, k + 1);
          if (PRO) {
            cshift(k + 1);
            add_pro(U[2], k + 1);
          }
        }
#pragma unroll
        for (int r = 0; r < 2; ++r) load_krow(K[1][r], r, k);
      }
      T au[V], dg[V], uc[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        T ks = T(0), far = T(0);
#pragma unroll
        for (int sz = 0; sz < 2; ++sz)
#pragma unroll
          for (int sy = 0; sy < 2; ++sy)
#pragma unroll
            for (int sx = 0; sx < 2; ++sx) {
              const T kv = K[sz][sy][v + sx];
              ks += kv;
              if (NEED_U) {
                const T f = (U[1][2 * sy][v + 2 * sx] + U[2 * sz][1][v + 2 * sx]) +
                            (U[2 * sz][2 * sy][v + 1] + U[2 * sz][2 * sy][v + 2 * sx]);
                far += kv * f;
              }
            }
        uc[v] = NEED_U ? U[1][1][v + 1] : T(0);
        au[v] = h * (ks * uc[v] * third - far * twelfth);
        dg[v] = h * ks * third;
      }
      epi((size_t)b * stride + i0 + (size_t)n * j + (size_t)n2 * k, au, dg, uc, ok, acc);
      if (NEED_U) {
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
          for (int c = 0; c < V + 2; ++c) {
            U[0][r][c] = U[1][r][c];
            U[1][r][c] = U[2][r][c];
          }
      }
#pragma unroll
      for (int r = 0; r < 2; ++r)
#pragma unroll
        for (int c = 0; c < V + 1; ++c) K[0][r][c] = K[1][r][c];
    }
  }
  if (Epi::kReduce) {
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[(size_t)b * pstride + part] = acc;
  }
}

// ------------------------------------------------- LDS-tiled z-march engine
// One workgroup owns `rows` node rows (all n columns) of one sample and walks
// a chunk of planes.  Each plane step stages the next u plane ((rows + 2)
// rows: the tile and its two halo rows) and the next kappa plane ((rows + 1)
// element rows) into LDS rings with coalesced 16-byte loads that were issued
// one step earlier into registers, so the loads of plane k+2 are in flight
// while plane k is computed.  Every u and kappa value is read from HBM/L2
// once per workgroup (the register engine reads each u row three times), and
// the thread state is small, which leaves room for more waves.  The
// arithmetic per node is the register engine's.
//
// LDS rows: u row = [.., u(-1) = 0 at V-1, u(0..n-1) at V.., u(n) = 0 at V+n],
// stride n + 2V; kappa row = [.., 0 at V-1, kappa(0..n-1) at V..], stride n + V
// (the zero cells are written once and never overwritten).  u plane kk lives
// in ring slot kk mod 3, kappa plane ez in slot ez mod KP.  PRO adds P xc to
// each staged u vector (same operation order as the register engine).
//
// Operand modes (the value staged for a u position):
//   OP_PLAIN  u
//   OP_ADDD   u + d (fp32 d in the same layout; u may be null: zero), with d
//             optionally completed by the update its solve still owes
//   OP_Z1     c2 D^-1 u: the first smoothing step from a zero iterate of a
//             V-cycle whose right-hand side is u, formed while staging so
//             that step is never stored.  D of a staged node needs the kappa
//             planes kk-1, kk of its u plane and one more element row on
//             each side, so the kappa ring holds KP = 4 planes (staged three
//             planes ahead of the computed one instead of one) and R + 3 rows.
//   OP_DIR    z + beta p_old: the next conjugate direction, from z = u and the
//             sample's current direction p_old (the buffer p[pstate & 1]);
//             for a sample's first direction (pstate & 2) p_old is not read and
//             the operand is z.
enum : int { OP_PLAIN = 0, OP_ADDD = 1, OP_Z1 = 2, OP_DIR = 3 };

template <class T>
struct OpArgs {
  // per-sample choice of the u operand: u1 where (ustate[b] & 8), u otherwise
  // (may be null: u for every sample)
  const T* u1 = nullptr;
  const int* ustate = nullptr;
  const float* d = nullptr;       // OP_ADDD
  // OP_ADDD: the update a fused-direction solve still owes d (may be null):
  // d + alpha p with p the solve's current direction (fp32 buffers q0/q1 by
  // dstate bit 0); alpha p alone when d was never written (dstate bit 2); none
  // when the solve took no step (bit 1)
  const float* q0 = nullptr;
  const float* q1 = nullptr;
  const int* dstate = nullptr;
  const double* dalpha = nullptr;
  T c2 = T(0);                    // OP_Z1
  const T* p0 = nullptr;          // OP_DIR: the two direction buffers
  const T* p1 = nullptr;
  const int* pstate = nullptr;    // OP_DIR: per sample, bit 0 = buffer of p_old, bit 1 = first direction
  const double* beta = nullptr;   // OP_DIR
};

template <int OP> struct ZOp {
  static constexpr int KOFF = OP == OP_Z1 ? 1 : 0;   // extra kappa rows on each side
  static constexpr int KP = OP == OP_Z1 ? 4 : 2;     // kappa ring planes
  static constexpr int LEAD = OP == OP_Z1 ? 3 : 1;   // kappa plane stored at step k: k + LEAD
};

// LDS row strides: dense rows of n values (u) and n elements (kappa); the
// kernels index rows by shifts, n being a power of two
template <class T>
__host__ __device__ inline int zlds_urs(int n) { return n; }
template <class T>
__host__ __device__ inline int zlds_krs(int n) { return n; }
// LDS of a k_zlds workgroup: u ring of 3 planes x (rows + 2) rows, kappa
// ring of KP planes x (rows + 1 + 2 KOFF) rows; with the fused prolongation
// a ring of 2 coarse planes x (rows / 2 + 2) rows of n / 2 values
template <class T>
__host__ __device__ inline int zlds_crows(int rows) { return rows / 2 + 2; }
template <class T, int OP = OP_PLAIN, bool PRO = false>
inline size_t zlds_bytes(const ZGeom& g) {
  return ((size_t)3 * (g.rows + 2) * zlds_urs<T>(g.n) +
          (size_t)ZOp<OP>::KP * (g.rows + 1 + 2 * ZOp<OP>::KOFF) * zlds_krs<T>(g.n) +
          (PRO ? (size_t)2 * zlds_crows<T>(g.rows) * (g.n / 2) : 0)) * sizeof(T);
}
// the staging covers every row with two vectors per thread
// and the rings fit the 64 KiB of LDS a workgroup may take without opting in;
// a row is at most one wave (its halos move by DPP)
template <class T, int OP = OP_PLAIN, bool PRO = false>
inline bool zlds_ok(const ZGeom& g) {
  return g.G >= 1 && g.G <= 64 && (g.G & (g.G - 1)) == 0 && (g.rows + 2) * g.G <= 2 * g.threads && (g.rows + 1 + 2 * ZOp<OP>::KOFF) * g.G <= 2 * g.threads &&
         zlds_bytes<T, OP, PRO>(g) <= 65536 && (!PRO || g.zc == 1 || g.zlen % 2 == 0);   // PRO: chunks start odd
}

// c2 D^-1 b for the V staged nodes c*V .. c*V+V-1 of row jj, plane kk, in u
// (b on entry); D from the kappa ring (element planes kk-1, kk in slots s0,
// s1; element row ey in ring row ey - krow0) with the operation order of the
// stencil kernels' diagonal and of EpiChebZero, so the value is the one that
// step would have stored; 0 on boundary nodes.  The branch is uniform over
// the lanes of a row, which is what the DPP halo exchange needs.
template <class T, int V, int HALO>
__device__ __forceinline__ void z1_form(T* u, const T* Kl, int KR, int rsh, int krow0, int s0, int s1, int jj,
                                        int kk, int n, int c, T h, T c2) {
  if (jj < 1 || jj > n - 1 || kk < 1 || kk > n - 1) {
#pragma unroll
    for (int v = 0; v < V; ++v) u[v] = T(0);
    return;
  }
  const int sl[2] = {s0, s1};
  T K[2][2][V + 1], Z[2][V + 1], ks[V];
#pragma unroll
  for (int dz = 0; dz < 2; ++dz)
#pragma unroll
    for (int dy = 0; dy < 2; ++dy)
      lds_krow<T, V, HALO>(Kl + ((sl[dz] * KR + jj - 1 + dy - krow0) << rsh) + c * V, K[dz][dy], c);
  ksum_from_rows<T, V>(K, Z, ks);
  const T third = T(1) / T(3);
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const T dg = h * ks[v] * third;
    u[v] = (c * V + v) != 0 ? c2 * u[v] * inv_diag(dg) : T(0);
  }
}

template <class T, int V, bool NEED_U, bool PRO, int OP, class Epi, int HALO, int NC = 0>
__global__ void __launch_bounds__(256) k_zlds(ZGeom g, size_t stride, T h, const T* __restrict__ u,
                                              const T* __restrict__ kap, const int* __restrict__ active,
                                              double* __restrict__ partial, uint32_t pstride, Epi epi,
                                              const T* __restrict__ xc, size_t cstride, OpArgs<T> op) {
  static_assert(!PRO || NEED_U, "the fused prolongation needs the u operand");
  static_assert(OP == OP_PLAIN || NEED_U, "operand modes need the u operand");
  static_assert(OP != OP_ADDD || !PRO, "the added vector needs the plain u operand");
  constexpr bool ADDD = OP == OP_ADDD, Z1 = OP == OP_Z1, DIR = OP == OP_DIR;
  constexpr int KOFF = ZOp<OP>::KOFF, KP = ZOp<OP>::KP, LEAD = ZOp<OP>::LEAD;
  typedef typename Vec<float, V>::type fvt;
  typedef typename Vec<T, V>::type vt;
  extern __shared__ __align__(16) unsigned char zsmem[];
  const uint32_t per = g.parts();
  const uint32_t lin = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t b = lin / per;
  const uint32_t part = lin - b * per;
  if (active && !active[b]) return;   // uniform over the workgroup
  const int rb = (int)(part % (uint32_t)g.row_blocks), zb = (int)(part / (uint32_t)g.row_blocks);
  // NC > 0: the mesh size known at compile time (G = NC / V: the launcher
  // checks), so LDS row offsets fold into the instructions' immediate offsets
  const int n = NC ? NC : g.n, n2 = n * n, G = NC ? NC / V : g.G, R = g.rows;
  const int gsh = __builtin_ctz((unsigned)G);   // G is a power of two
  const int UR = R + 2, KR = R + 1 + 2 * KOFF;
  const int URS = zlds_urs<T>(n), KRS = zlds_krs<T>(n);
  const int rsh = __builtin_ctz((unsigned)n);   // LDS rows are n values, n a power of two
  T* Ul = reinterpret_cast<T*>(zsmem);        // [3][UR][URS]:  u rows j0-1 .. j0+R
  T* Kl = Ul + 3 * UR * URS;                   // [KP][KR][KRS]: kappa rows krow0 ..
  T* Cl = Kl + KP * KR * KRS;                  // PRO: [2][CR][n/2]: coarse rows crow0 ..
  const int tid = (int)threadIdx.x, nthr = (int)blockDim.x;
  const int j0 = 1 + rb * R;
  const int krow0 = j0 - 1 - KOFF;
  const int k0 = 1 + zb * g.zlen;
  int k1 = k0 + g.zlen;
  if (k1 > n) k1 = n;
  // last kappa plane staged: the computed planes need k1-1; OP_Z1 also forms
  // the operand on u plane k1
  const int kmax = Z1 ? (k1 < n - 1 ? k1 : n - 1) : k1 - 1;
  const int gx = tid & (G - 1), jr = tid >> gsh;
  const int j = j0 + jr, i0 = gx * V;
  const bool valid = jr < R && j <= n - 1 && k0 < k1;
  // a row fits in one wave (zlds_ok): halos by DPP, no branch in the gather
  const T* ub = (NEED_U && u) ? u + (size_t)b * stride : nullptr;
  if (NEED_U && op.ustate && (op.ustate[b] & 8)) ub = op.u1 + (size_t)b * stride;
  const float* db = ADDD ? op.d + (size_t)b * stride : nullptr;
  const T* kb = kap + (size_t)b * n2 * n;
  const T* cb = PRO ? xc + (size_t)b * cstride : nullptr;
  const int nc = n >> 1, nc2 = nc * nc;
  // OP_DIR: the sample's previous direction (absent for its first one) and beta
  bool dir_prev = false;
  T dbeta = T(0);
  const T* pob = nullptr;
  if constexpr (DIR) {
    const int ps = op.pstate[b];
    dir_prev = (ps & 2) == 0;
    dbeta = (T)op.beta[b];
    pob = ((ps & 1) ? op.p1 : op.p0) + (size_t)b * stride;
  }
  // OP_ADDD with an owed update: whether d is read, whether alpha p is added
  bool d_read = true, d_owe = false;
  float d_a = 0.0f;
  const float* dqb = nullptr;
  if constexpr (ADDD) {
    if (op.dstate) {
      const int ps = op.dstate[b];
      d_owe = (ps & 2) == 0;
      d_read = (ps & 4) == 0;
      d_a = (float)op.dalpha[b];
      dqb = ((ps & 1) ? op.q1 : op.q0) + (size_t)b * stride;
    }
  }
  if constexpr (Epi::kBegin) epi.begin(b);

  // staging: up to two 16-byte vectors per thread per plane for u and kappa;
  // a thread stages the same (row, column) positions on every plane
  vt pu[2], pk[2];
  fvt pd[ADDD ? 2 : 1], pq[ADDD ? 2 : 1];
  vt pp[DIR ? 2 : 1];
  // OP_DIR: p_old at the thread's own nodes of the next plane to finish (and
  // of the first plane, in the prologue)
  vt pown{}, pown0{};
  // staged u vector m of this thread: the first nthr by thread id, the rest
  // (a tile taller than the workgroup) by the last threads, so that extra
  // work (the OP_Z1 / PRO operand) does not pile onto wave 0, which stages the
  // extra kappa vectors; ubase is a multiple of G, so a row stays in one wave
  const int ubase = 2 * nthr - UR * G;
  // OP_DIR: the map is rotated by one row, so that a thread's first vector is
  // its own row j (tile row jr + 1) and the p_old it stages there serves its
  // x update as well; the extra vectors take tile rows R + 1 and 0
  auto uv = [&](int m) {
    int v = m == 0 ? tid : (tid >= ubase ? nthr + tid - ubase : 1 << 30);
    if constexpr (DIR) {
      if (v < UR * G) {
        v += G;
        if (v >= UR * G) v -= UR * G;
      }
    }
    return v;
  };
  // PRO: the coarse planes of the correction in an LDS ring of two planes
  // (plane C in slot C & 1), rows crow0 .. crow0 + CR - 1: the parents
  // (jj >> 1, (jj + 1) >> 1) of the staged fine rows jj = j0-1 .. j0+R.  A
  // lane reads the V/2 coarse values under its fine vector from LDS and the
  // next one from the neighbouring lane.  Coarse plane C is first needed by
  // fine plane 2C-1 and last by 2C+1; it is stored in the step that stages
  // fine plane 2C-2, over plane C-2 (last needed by fine plane 2C-3).
  constexpr int H = V / 2;
  const int CR = zlds_crows<T>(R), crow0 = (j0 - 1) >> 1;
  T pc[2][PRO ? H : 1];
  auto fetch_c = [&](int K) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int v = tid + m * nthr;
      const int r = v >> gsh, c = v & (G - 1);
      if (v < CR * G && crow0 + r <= nc)
        nload<T, H>(cb + (size_t)nc2 * K + (size_t)nc * (crow0 + r) + c * H, pc[m]);
    }
  };
  auto store_c = [&](int K) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int v = tid + m * nthr;
      const int r = v >> gsh, c = v & (G - 1);
      if (v < CR * G && crow0 + r <= nc) nstore<T, H>(Cl + (((K & 1) * CR + r) << (rsh - 1)) + c * H, pc[m]);
    }
  };
  auto fetch_u = [&](int kk) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int v = uv(m);
      const int r = v >> gsh, c = v & (G - 1);
      const int jj = j0 - 1 + r;
      if (v < UR * G && jj <= n) {
        const size_t off = (size_t)n2 * kk + (size_t)n * jj + c * V;
        if (!ADDD || ub) pu[m] = *reinterpret_cast<const vt*>(ub + off);
        else pu[m] = vt{};
        if (ADDD) {
          pd[ADDD ? m : 0] = d_read ? *reinterpret_cast<const fvt*>(db + off) : fvt{};
          if (d_owe) pq[ADDD ? m : 0] = *reinterpret_cast<const fvt*>(dqb + off);
        }
        if (DIR && dir_prev) pp[DIR ? m : 0] = *reinterpret_cast<const vt*>(pob + off);
      }
    }
  };
  // form the operand of the plane kk fetched last, in registers (the loads
  // were in flight meanwhile): OP_Z1 from kappa planes kk-1, kk (already in
  // the ring), then PRO adds the correction from the coarse window fetched
  // with it.  Done before the barrier that precedes put_u, so it overlaps the
  // other waves' stencil work instead of stalling the workgroup.
  auto prep_u = [&](int kk) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int v = uv(m);
      const int r = v >> gsh, c = v & (G - 1);
      const int jj = j0 - 1 + r;
      if (v < UR * G && jj <= n) {
        if (Z1) {
          T w[V];
#pragma unroll
          for (int t = 0; t < V; ++t) w[t] = pu[m][t];
          z1_form<T, V, HALO>(w, Kl, KR, rsh, krow0, (kk - 1) & (KP - 1), kk & (KP - 1), jj, kk, n, c, h, op.c2);
#pragma unroll
          for (int t = 0; t < V; ++t) pu[m][t] = w[t];
        }
        if (PRO) {
          // fine nodes c*V .. c*V+V-1 of row jj, plane kk: coarse values
          // c*H .. c*H+H of rows jj >> 1, (jj + 1) >> 1 on planes kk >> 1,
          // (kk + 1) >> 1 (the last value of a row is the zero boundary)
          const bool kodd = (kk & 1) != 0, jodd = (jj & 1) != 0;
          T W[2][2][H + 1];   // [plane][row][q]
#pragma unroll
          for (int pz = 0; pz < 2; ++pz)
#pragma unroll
            for (int jy = 0; jy < 2; ++jy) {
              const int K = (kk + pz) >> 1, J = (jj + jy) >> 1;
              nload<T, H>(Cl + (((K & 1) * CR + J - crow0) << (rsh - 1)) + c * H, W[pz][jy]);
              W[pz][jy][H] = halo_next<HALO>(W[pz][jy][0], c, G);
            }
          constexpr int CQ = H + 1;
          T L[CQ];
#pragma unroll
          for (int q = 0; q < CQ; ++q) {
            const T P0 = kodd ? T(0.5) * (W[0][0][q] + W[1][0][q]) : W[0][0][q];
            const T P1 = kodd ? T(0.5) * (W[0][1][q] + W[1][1][q]) : W[0][1][q];
            L[q] = jodd ? T(0.5) * (P0 + P1) : P0;
          }
#pragma unroll
          for (int t = 0; t < V; ++t)
            pu[m][t] += (t & 1) ? T(0.5) * (L[(t - 1) / 2] + L[(t + 1) / 2]) : L[t / 2];
        }
        if (ADDD) {
          // the completed correction in fp32, as the separate update would store it
          fvt dd = pd[ADDD ? m : 0];
          if (d_owe) dd = d_read ? dd + d_a * pq[ADDD ? m : 0] : d_a * pq[ADDD ? m : 0];
#pragma unroll
          for (int t = 0; t < V; ++t) pu[m][t] += (T)dd[t];
        }
        if (DIR && dir_prev) pu[m] = pu[m] + dbeta * pp[DIR ? m : 0];
      }
    }
  };
  auto put_u = [&](int slot) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int v = uv(m);
      const int r = v >> gsh, c = v & (G - 1);
      if (v < UR * G && j0 - 1 + r <= n) *reinterpret_cast<vt*>(Ul + ((slot * UR + r) << rsh) + c * V) = pu[m];
    }
  };
  auto store_u = [&](int slot, int kk) {
    prep_u(kk);
    put_u(slot);
  };
  auto fetch_k = [&](int ez) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int v = tid + m * nthr;
      const int r = v >> gsh, c = v & (G - 1);
      const int ey = krow0 + r;
      if (v < KR * G && ey >= 0 && ey <= n - 1)
        pk[m] = *reinterpret_cast<const vt*>(kb + (size_t)n2 * ez + (size_t)n * ey + c * V);
    }
  };
  auto store_k = [&](int ez) {
    const int slot = ez & (KP - 1);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int v = tid + m * nthr;
      const int r = v >> gsh, c = v & (G - 1);
      const int ey = krow0 + r;
      if (v < KR * G && ey >= 0 && ey <= n - 1)
        *reinterpret_cast<vt*>(Kl + ((slot * KR + r) << rsh) + c * V) = pk[m];
    }
  };

  double acc = 0.0;
  if (k0 < k1) {
    // prologue: u planes k0-1, k0, k0+1 and kappa planes up to k0 + LEAD - 1
    // into LDS; then the loads of u plane k0+2 and kappa plane k0 + LEAD are
    // left in flight
    // PRO: coarse planes cb0, cb0 + 1 for fine planes k0-1 .. k0+1 (k0 is odd)
    const int cb0 = (k0 - 1) >> 1;
    if (PRO) {
      fetch_c(cb0); store_c(cb0);
      fetch_c(cb0 + 1); store_c(cb0 + 1);
    }
    if (Z1) {
      // the operand of u plane kk needs kappa planes kk-1, kk
      for (int ez = k0 - 2; ez <= k0 + 1; ++ez)
        if (ez >= 0 && ez <= kmax) { fetch_k(ez); store_k(ez); }
      __syncthreads();
      fetch_u(k0 - 1); store_u((k0 - 1) % 3, k0 - 1);
      fetch_u(k0); store_u(k0 % 3, k0);
      fetch_u(k0 + 1); store_u((k0 + 1) % 3, k0 + 1);
      __syncthreads();   // kappa plane k0-2 is no longer read: its slot takes plane k0+2
      if (k0 + 2 <= kmax) { fetch_k(k0 + 2); store_k(k0 + 2); }
    } else {
      if (PRO) __syncthreads();
      if (NEED_U) {
        fetch_u(k0 - 1); store_u((k0 - 1) % 3, k0 - 1);
        fetch_u(k0); store_u(k0 % 3, k0);
        if constexpr (DIR) pown0 = pp[0];
        fetch_u(k0 + 1); store_u((k0 + 1) % 3, k0 + 1);
        if constexpr (DIR) pown = pp[0];
      }
      fetch_k(k0 - 1); store_k(k0 - 1);
      fetch_k(k0); store_k(k0);
      if (PRO) __syncthreads();   // coarse plane cb0 is no longer read
    }
    // coarse plane cb0 + 2 (first needed by fine plane k0 + 2) over cb0
    if (PRO && k0 + 2 <= k1) { fetch_c(cb0 + 2); store_c(cb0 + 2); }
    // the epilogue's own operands of plane k0 first: waiting for them later
    // then leaves the staging loads behind them in flight
    const size_t pos0 = (size_t)b * stride + i0 + (size_t)n * j + (size_t)n2 * k0;
    if (valid) {
      if constexpr (DIR) epi.pre_own(pos0, pown0);
      else epi.pre(pos0);
    }
    if (NEED_U && k0 + 2 <= k1) fetch_u(k0 + 2);
    if (k0 + LEAD <= kmax) fetch_k(k0 + LEAD);
    __syncthreads();
    bool ok[V];
#pragma unroll
    for (int v = 0; v < V; ++v) ok[v] = (i0 + v) != 0;
    int sm = (k0 - 1) % 3, s0 = k0 % 3, sp = (k0 + 1) % 3;   // u slots of planes k-1, k, k+1
    const T third = T(1) / T(3), h12 = h * (T(1) / T(12));
    for (int k = k0; k < k1; ++k) {
      if (valid) {
        // the Q1 row from the LDS tile (see q1_gather); without the u
        // operand only the diagonal is needed
        const int km = (k - 1) & (KP - 1), kc = k & (KP - 1);
        T far[V], ksum[V], uc[V];
        if (NEED_U) {
          q1_gather<T, V, HALO, true>(Kl + ((km * KR + jr + KOFF) << rsh) + i0, Kl + ((kc * KR + jr + KOFF) << rsh) + i0,
                                Ul + ((sm * UR + jr) << rsh) + i0, Ul + ((s0 * UR + jr) << rsh) + i0,
                                Ul + ((sp * UR + jr) << rsh) + i0, rsh, gx, G, ksum, far, uc);
        } else {
          T K[2][2][V + 1], Z[2][V + 1];
#pragma unroll
          for (int dy = 0; dy < 2; ++dy) {
            lds_krow<T, V, HALO>(Kl + ((km * KR + jr + dy + KOFF) << rsh) + i0, K[0][dy], gx);
            lds_krow<T, V, HALO>(Kl + ((kc * KR + jr + dy + KOFF) << rsh) + i0, K[1][dy], gx);
          }
          ksum_from_rows<T, V>(K, Z, ksum);
#pragma unroll
          for (int v = 0; v < V; ++v) {
            far[v] = T(0);
            uc[v] = T(0);
          }
        }
        T au[V], dg[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
          au[v] = h12 * fma(ksum[v] * uc[v], T(4), -far[v]);   // h (ks uc / 3 - fr / 12)
          dg[v] = h * ksum[v] * third;
        }
        epi(pos0 + (size_t)n2 * (k - k0), au, dg, uc, ok, acc);
      }
      if (k + 1 < k1) {
        // u plane k+2 (OP_Z1: from kappa planes k+1, k+2, stored in earlier
        // steps; kappa plane k+3 takes the slot of plane k-1 below)
        if (NEED_U && k + 2 <= k1) prep_u(k + 2);
        // every thread is done with u plane k-1 and kappa plane k-1
        __syncthreads();
        if (NEED_U && k + 2 <= k1) put_u(sm);   // plane k+2 takes the slot of plane k-1
        if (k + LEAD <= kmax) store_k(k + LEAD);
        // PRO: coarse plane (k + 4) / 2 with fine plane k + 2 (k even), fetched
        // in the step before
        if (PRO && ((k - k0) & 1) && k + 3 <= k1) store_c((k + 4) >> 1);
        if (valid) {
          if constexpr (DIR) epi.pre_own(pos0 + (size_t)n2 * (k + 1 - k0), pown);
          else epi.pre(pos0 + (size_t)n2 * (k + 1 - k0));
        }
        // OP_DIR: p_old of plane k + 2 (prepared above) for the next step
        if constexpr (DIR) pown = pp[0];
        if (NEED_U && k + 3 <= k1) fetch_u(k + 3);
        if (k + LEAD + 1 <= kmax) fetch_k(k + LEAD + 1);
        if (PRO && !((k - k0) & 1) && k + 4 <= k1) fetch_c((k + 5) >> 1);
        __syncthreads();
        const int t = sm; sm = s0; s0 = sp; sp = t;
      }
    }
  }
  if (Epi::kReduce) {
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[(size_t)b * pstride + part] = acc;
  }
}

// ------------------------------------- residual fused with the restriction
// bc = P^T (b - A x) on the n/2 mesh without writing the fine residual.  The
// workgroup's LDS tile is the one of k_zlds plus one row: it evaluates the
// residual t on its node rows j0 .. j0+R (row j0+R is the first row of the next
// tile, recomputed here) and on planes k0 .. k1 (plane k1 likewise), one
// plane at a time into LDS.  Every coarse node (I, J, K) with 2J in
// [j0+1, j0+R-1] and 2K in [k0+1, k1-1] has its whole 3x3x3 support in that
// range (j0 and k0 are odd, R and the chunk length even), so each coarse node
// is produced by exactly one workgroup: a thread owning (I, J) adds the
// in-plane full-weighting sum of t, weighted 1/2 from odd fine planes and 1
// from even ones, and stores the coarse value when plane 2K+1 is done.
// With Z1 the operand x is c2 D^-1 b, formed while staging (see OP_Z1), so a
// V-cycle level's zero-start pre-smoothing step costs no pass of its own.
template <class T, bool Z1 = false>
inline size_t resr_bytes(const ZGeom& g) {
  constexpr int KOFF = Z1 ? 1 : 0, KP = Z1 ? 4 : 2;
  return ((size_t)3 * (g.rows + 3) * zlds_urs<T>(g.n) + (size_t)KP * (g.rows + 2 + 2 * KOFF) * zlds_krs<T>(g.n) +
          (size_t)(g.rows + 1) * zlds_urs<T>(g.n)) * sizeof(T);
}

// Geometry of k_resr: the tiles of k_zlds.  (Adding threads so that the
// extra residual row of a full tile takes no second pass measured slower on
// the 64^3 batch: 320 threads, 9.8 -> 15.6 ms per step.)
// (14-row tiles, which keep every residual row in one pass, measured slower
// here: 9.6 -> 10.2 ms per 64^3 x 1024 step, from the extra tiles' staging)
template <class T>
inline ZGeom resr_geom(int n, int B) { return zgeom<T>(n, B); }

// usable when every tile and chunk starts on an odd index and the staging
// fits two vectors per thread
template <class T, bool Z1 = false>
inline bool resr_ok(const ZGeom& g) {
  return g.n >= 4 && g.G >= 1 && g.G <= 64 && (g.G & (g.G - 1)) == 0 && g.rows % 2 == 0 && (g.zc == 1 || g.zlen % 2 == 0) &&
         g.threads <= 256 && (g.rows + 3) * g.G <= 2 * g.threads && (g.rows + 2 + (Z1 ? 2 : 0)) * g.G <= 2 * g.threads &&
         (g.rows + 1) * g.G <= 2 * g.threads - (g.threads >= 192 ? g.threads / 2 : 0) && resr_bytes<T, Z1>(g) <= 65536;
}

// UPD (with Z1): the PCG residual update that ends the previous iteration is
// done here: the right-hand side is r = r_old - alpha q, formed while staging
// r_old and q (and again at the thread's own nodes, by the same fma), written
// at the tile's own nodes into the other residual buffer, with the partial
// sums of r . r; on a sample's first iteration (pstate bit 1) r = r_old and
// nothing is written.  The buffers are bf (R0) and upd.r1 (R1), selected by
// pstate bit 3.
template <class T>
struct ResrUpd {
  const T* q = nullptr;
  T* r1 = nullptr;
  const int* pstate = nullptr;
  const double* alpha = nullptr;
  double* partial = nullptr;
  uint32_t pstride = 0;
};

template <class T>
__device__ __forceinline__ T rupd(T r, T a, T q) { return fma(-a, q, r); }

// fp32 without the update: held to 128 VGPRs (no spill), so that four
// workgroups fit a CU with the 39 KB of LDS of the pre-smoothed form
template <class T, int V, bool Z1, bool UPD>
constexpr int resr_min_waves() { return sizeof(T) == 4 && !UPD ? 4 : 1; }

template <class T, int V, bool Z1, bool UPD, int HALO, int RW, int NC = 0>
__global__ void __launch_bounds__(256, (resr_min_waves<T, V, Z1, UPD>())) k_resr(ZGeom g, size_t stride, T h, const T* __restrict__ x,
                                              const T* __restrict__ bf, const T* __restrict__ kap,
                                              const int* __restrict__ active, T* __restrict__ bc, size_t cstride,
                                              T c2, ResrUpd<T> upd) {
  static_assert(!UPD || Z1, "the residual update is fused into the pre-smoothed form");
  typedef typename Vec<T, V>::type vt;
  constexpr int KOFF = Z1 ? 1 : 0, KP = Z1 ? 4 : 2, LEAD = Z1 ? 3 : 1;
  extern __shared__ __align__(16) unsigned char zsmem[];
  const uint32_t per = g.parts();
  const uint32_t lin = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t b = lin / per;
  const uint32_t part = lin - b * per;
  if (active && !active[b]) return;   // uniform over the workgroup
  const int rb = (int)(part % (uint32_t)g.row_blocks), zb = (int)(part / (uint32_t)g.row_blocks);
  // NC > 0: the mesh size known at compile time (256 threads, G = NC / V,
  // R = 256 / G: the launcher checks), so LDS row offsets fold into the
  // instructions' immediate offsets
  const int n = NC ? NC : g.n, n2 = n * n, G = NC ? NC / V : g.G, R = NC ? 256 / (NC / V) : g.rows;
  const int gsh = __builtin_ctz((unsigned)G);   // G is a power of two
  const int UR = R + 3, KR = R + 2 + 2 * KOFF, TR = R + 1;
  const int URS = zlds_urs<T>(n), KRS = zlds_krs<T>(n);
  const int rsh = __builtin_ctz((unsigned)n);   // LDS rows are n values, n a power of two
  T* Ul = reinterpret_cast<T*>(zsmem);        // [3][UR][URS]:  u rows j0-1 .. j0+R+1
  T* Kl = Ul + 3 * UR * URS;                   // [KP][KR][KRS]: kappa rows j0-1-KOFF .. j0+R+KOFF
  T* Tl = Kl + KP * KR * KRS;                  // [TR][URS]:     t rows j0 .. j0+R
  const int tid = (int)threadIdx.x, nthr = (int)blockDim.x;
  const int j0 = 1 + rb * R;
  const int krow0 = j0 - 1 - KOFF;
  const int k0 = 1 + zb * g.zlen;
  int k1 = k0 + g.zlen;
  if (k1 > n) k1 = n;
  const int kt1 = k1 < n - 1 ? k1 : n - 1;    // last residual plane
  // last kappa plane staged: the residual planes need kt1; Z1 also forms the
  // operand on u plane kt1 + 1
  const int kmax = Z1 ? (kt1 + 1 < n - 1 ? kt1 + 1 : n - 1) : kt1;
  // halos by DPP (a row fits in one wave: resr_ok); with the extra rows of a
  // tile spread over the waves this measured faster than LDS halo reads
  // (8.7 vs 9.4 ms per 64^3 x 1024 step)
  const T* ub = (Z1 ? bf : x) + (size_t)b * stride;
  const T* bb = bf + (size_t)b * stride;
  const T* kb = kap + (size_t)b * n2 * n;
  const int nc = n >> 1, nc2 = nc * nc;
  // element offset within a sample's array as a 32-bit byte offset on the
  // sample's (uniform) base, so that a per-lane address takes one register:
  // rows are at most 64 vectors (resr_ok), so a sample's array is at most
  // 256^3 fp32 or 128^3 fp64 values
  auto at = [](auto* base, uint32_t off) {
    typedef std::remove_reference_t<decltype(*base)> E;
    return reinterpret_cast<E*>(reinterpret_cast<std::conditional_t<std::is_const_v<E>, const char*, char*>>(base) +
                                off * (uint32_t)sizeof(E));
  };
  T* bcb = bc + (size_t)b * cstride;
  // UPD: r_old in R[par], r written to R[1 - par] unless this is the first
  // iteration; q and alpha of the previous iteration
  bool upd_on = false;
  T ua = T(0);
  const T* qb = nullptr;
  T* rnb = nullptr;
  if constexpr (UPD) {
    const int ps = upd.pstate[b];
    const bool par = (ps & 8) != 0;
    upd_on = (ps & 2) == 0;
    ua = (T)upd.alpha[b];
    const T* rold = (par ? (const T*)upd.r1 : bf) + (size_t)b * stride;
    ub = rold;
    bb = rold;
    qb = upd.q + (size_t)b * stride;
    rnb = (par ? const_cast<T*>(bf) : upd.r1) + (size_t)b * stride;
  }
  double racc = 0.0;   // UPD: sum of r . r over the tile's own nodes

  vt pu[2], pk[2], pq[UPD ? 2 : 1];
  // staged u vector m: extras on the last threads (see k_zlds)
  const int ubase = 2 * nthr - UR * G;
  auto uv = [&](int m) { return m == 0 ? tid : (tid >= ubase ? nthr + tid - ubase : 1 << 30); };
  auto fetch_u = [&](int kk) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int v = uv(m);
      const int r = v >> gsh, c = v & (G - 1);
      const int jj = j0 - 1 + r;
      if (v < UR * G && jj <= n) {
        const uint32_t off = (uint32_t)(n2 * kk + n * jj + c * V);
        pu[m] = *reinterpret_cast<const vt*>(at(ub, off));
        if (UPD && upd_on) pq[UPD ? m : 0] = *reinterpret_cast<const vt*>(at(qb, off));
      }
    }
  };
  // Z1: the operand of the plane kk fetched last, in registers, before the
  // barrier that precedes put_u (see k_zlds)
  auto prep_u = [&](int kk) {
    if (!Z1) return;
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int v = uv(m);
      const int r = v >> gsh, c = v & (G - 1);
      const int jj = j0 - 1 + r;
      if (v < UR * G && jj <= n) {
        T w[V];
#pragma unroll
        for (int t = 0; t < V; ++t) w[t] = (UPD && upd_on) ? rupd(pu[m][t], ua, pq[UPD ? m : 0][t]) : pu[m][t];
        z1_form<T, V, HALO>(w, Kl, KR, rsh, krow0, (kk - 1) & (KP - 1), kk & (KP - 1), jj, kk, n, c, h, c2);
#pragma unroll
        for (int t = 0; t < V; ++t) pu[m][t] = w[t];
      }
    }
  };
  auto put_u = [&](int slot) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int v = uv(m);
      const int r = v >> gsh, c = v & (G - 1);
      if (v < UR * G && j0 - 1 + r <= n) *reinterpret_cast<vt*>(Ul + ((slot * UR + r) << rsh) + c * V) = pu[m];
    }
  };
  auto store_u = [&](int slot, int kk) {
    prep_u(kk);
    put_u(slot);
  };
  auto fetch_k = [&](int ez) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int v = tid + m * nthr;
      const int r = v >> gsh, c = v & (G - 1);
      const int ey = krow0 + r;
      if (v < KR * G && ey >= 0 && ey <= n - 1)
        pk[m] = *reinterpret_cast<const vt*>(at(kb, (uint32_t)(n2 * ez + n * ey + c * V)));
    }
  };
  auto store_k = [&](int ez) {
    const int slot = ez & (KP - 1);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int v = tid + m * nthr;
      const int r = v >> gsh, c = v & (G - 1);
      const int ey = krow0 + r;
      if (v < KR * G && ey >= 0 && ey <= n - 1)
        *reinterpret_cast<vt*>(Kl + ((slot * KR + r) << rsh) + c * V) = pk[m];
    }
  };

  const int tbase = nthr >= 192 ? nthr / 2 : 0;
  // A full tile has one row more to compute than threads (R G = nthr).  A
  // second pass of vector tasks for it would fall on one wave, which every
  // wave then waits for at the plane's barrier; where the row is 64 RW nodes
  // (RW = 1, 2; the launcher checks) it is one pass of one wave instead (RW
  // nodes per lane, halos by whole-wave shifts), on the wave below the one
  // that forms the extra staged u vectors.  Each node's arithmetic is the
  // vector task's.
  const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  constexpr int VX = RW;   // nodes per lane of the row's pass; 0: two passes of vector tasks
  const bool row_wave = RW != 0;
  const int xw = (ubase >> 6) > 0 ? (ubase >> 6) - 1 : 0;

  // coarse node owned by this thread: coarse row Jf + (tid / nc), column tid % nc
  const int Jf = (j0 + 1) >> 1;
  const int Jlast = (j0 + R - 1) >> 1 < nc - 1 ? (j0 + R - 1) >> 1 : nc - 1;
  const int cJ = Jf + (tid >> __builtin_ctz((unsigned)nc)), cI = tid & (nc - 1);   // nc a power of two
  const bool owner = tid < (R / 2) * nc && cJ <= Jlast;
  T cacc = T(0);

  if (k0 < k1) {
    if (Z1) {
      for (int ez = k0 - 2; ez <= k0 + 1; ++ez)
        if (ez >= 0 && ez <= kmax) { fetch_k(ez); store_k(ez); }
      __syncthreads();
      fetch_u(k0 - 1); store_u((k0 - 1) % 3, k0 - 1);
      fetch_u(k0); store_u(k0 % 3, k0);
      fetch_u(k0 + 1); store_u((k0 + 1) % 3, k0 + 1);
      __syncthreads();   // kappa plane k0-2 is no longer read: its slot takes plane k0+2
      if (k0 + 2 <= kmax) { fetch_k(k0 + 2); store_k(k0 + 2); }
    } else {
      fetch_u(k0 - 1); store_u((k0 - 1) % 3, k0 - 1);
      fetch_u(k0); store_u(k0 % 3, k0);
      fetch_u(k0 + 1); store_u((k0 + 1) % 3, k0 + 1);
      fetch_k(k0 - 1); store_k(k0 - 1);
      fetch_k(k0); store_k(k0);
    }
    if (k0 + 2 <= kt1 + 1) fetch_u(k0 + 2);
    if (k0 + LEAD <= kmax) fetch_k(k0 + LEAD);
    __syncthreads();
    int sm = (k0 - 1) % 3, s0 = k0 % 3, sp = (k0 + 1) % 3;
    const T h12 = h * (T(1) / T(12));
    for (int kk = k0; kk <= kt1; ++kk) {
      const int km = (kk - 1) & (KP - 1), kc = kk & (KP - 1);
      // residual of rows j0 .. j0+R on plane kk into LDS
      // the residual of VV nodes i0 = gx VV .. of tile row jr; a row is GG
      // lanes of VV nodes (halo mode HH)
      auto task_row = [&](auto vv, auto hh, int jr, int gx, int GG) {
        constexpr int VV = decltype(vv)::value, HH = decltype(hh)::value;
        const int j = j0 + jr, i0 = gx * VV;
        T far[VV], ksum[VV], uc[VV];
        q1_gather<T, VV, HH>(Kl + ((km * KR + jr + KOFF) << rsh) + i0, Kl + ((kc * KR + jr + KOFF) << rsh) + i0,
                             Ul + ((sm * UR + jr) << rsh) + i0, Ul + ((s0 * UR + jr) << rsh) + i0,
                             Ul + ((sp * UR + jr) << rsh) + i0, rsh, gx, GG, ksum, far, uc);
        T bv[VV], t[VV];
        const uint32_t own = (uint32_t)(i0 + n * j + n2 * kk);
        vload<T, VV>(at(bb, own), bv);
        if (UPD) {
          if (upd_on) {
            T qv[VV];
            vload<T, VV>(at(qb, own), qv);
#pragma unroll
            for (int v = 0; v < VV; ++v) bv[v] = rupd(bv[v], ua, qv[v]);
          }
          // the tile's own nodes: rows j0 .. j0+R-1, planes k0 .. k1-1
          if (jr < R && kk < k1) {
            if (upd_on) vstore<T, VV>(at(rnb, own), bv);
#pragma unroll
            for (int v = 0; v < VV; ++v) racc += (double)bv[v] * (double)bv[v];
          }
        }
#pragma unroll
        for (int v = 0; v < VV; ++v)   // b - h (ks uc / 3 - fr / 12)
          t[v] = (i0 + v) != 0 ? fma(-h12, fma(ksum[v] * uc[v], T(4), -far[v]), bv[v]) : T(0);
        vstore<T, VV>(Tl + (jr << rsh) + i0, t);
      };
      if (row_wave) {
        // rows j0 .. j0+R-1 one task per thread; row j0+R on wave xw alone,
        // one lane per VX nodes
        if (j0 + (tid >> gsh) <= n - 1) task_row(Ic<V>(), Ic<HALO>(), tid >> gsh, tid & (G - 1), G);
        __builtin_amdgcn_sched_barrier(0);   // the two passes' registers are not live at once
        if (wave == xw && j0 + R <= n - 1) {
          task_row(Ic<(VX > 0 ? VX : 1)>(), Ic<HALO_WAVE>(), R, lane, 64);
        }
      } else {
        // tasks: one per thread, the extra rows of a full tile (TR * G - nthr
        // tasks, at most nthr) on the threads from tbase on, i.e. not on the
        // waves that stage the extra u and kappa vectors
#pragma unroll 1
        for (int q = 0; q < 2; ++q) {
          const int task = q == 0 ? tid : (tid >= tbase ? nthr + tid - tbase : TR * G);
          if (task >= TR * G) continue;
          const int jr = task >> gsh;
          if (j0 + jr > n - 1) continue;
          task_row(Ic<V>(), Ic<HALO>(), jr, task & (G - 1), G);
        }
      }
      if (kk + 1 <= kt1) prep_u(kk + 2);   // kappa planes kk+1, kk+2 are in the ring
      __syncthreads();
      // in-plane full weighting of t at the owned coarse node, folded over planes
      if (owner) {
        // t at fine columns 2I, 2I+1 by one aligned pair read per row (lanes
        // at consecutive pairs: no LDS bank conflicts); column 2I-1 is the
        // previous lane's second value (coarse column I-1 of the same coarse
        // row, an owner too), passed by a whole-wave shift, except on a
        // wave's first lane, where a coarse row wider than a wave (nc > 64)
        // continues from the previous wave: read from LDS there
        typedef typename Vec<T, 2>::type t2;
        const int jr = 2 * cJ - j0;   // tile row of fine row 2J
        T r2 = T(0);
#pragma unroll
        for (int dy = -1; dy <= 1; ++dy) {
          const T* row = Tl + ((jr + dy) << rsh) + 2 * cI;
          const t2 pr = *reinterpret_cast<const t2*>(row);
          T left = from_prev(pr[1]);
          if (nc > 64 && lane == 0 && cI > 0) left = row[-1];
          r2 += (dy == 0 ? T(1) : T(0.5)) * (T(0.5) * (left + pr[1]) + pr[0]);
        }
        if (cI == 0) r2 = T(0);
        if (kk & 1) {
          // odd plane 2K+1 closes coarse plane K (from the second odd plane on)
          // and opens plane K+1
          const int K = (kk - 1) >> 1;
          if (kk > k0 && K <= nc - 1) *at(bcb, (uint32_t)(cI + nc * cJ + nc2 * K)) = cacc + T(0.5) * r2;
          cacc = T(0.5) * r2;
        } else {
          cacc += r2;
        }
      }
      if (kk + 1 <= kt1) {
        // u plane kk-1 and kappa plane kk-1 are no longer read
        put_u(sm);   // u plane kk+2
        if (kk + LEAD <= kmax) store_k(kk + LEAD);
        if (kk + 3 <= kt1 + 1) fetch_u(kk + 3);
        if (kk + LEAD + 1 <= kmax) fetch_k(kk + LEAD + 1);
      }
      __syncthreads();
      const int tu = sm; sm = s0; s0 = sp; sp = tu;
    }
  }
  if constexpr (UPD) {
    racc = block_sum(racc);
    if (threadIdx.x == 0) upd.partial[(size_t)b * upd.pstride + part] = racc;
  }
}

// the corrected smoothing step with its operand formed on the fly stages two
// rows more than it computes: tall-tile geometry (see zgeom_tall)
template <class T, bool PRO, int OP>
inline ZGeom zlds_geom(int n, int B) { return (PRO && OP == OP_Z1) ? zgeom_tall<T>(n, B) : zgeom<T>(n, B); }

template <class T, bool NEED_U, bool PRO, int OP, class Epi>
hipError_t zlaunch_lds(int n, int B, const T* u, const T* xc, const T* kap, const int* active, double* partial,
                       uint32_t pstride, Epi epi, uint32_t* nparts, hipStream_t st, OpArgs<T> op = {}) {
  constexpr int V = ZV<T>::V;
  const ZGeom g = zlds_geom<T, PRO, OP>(n, B);
  if (!zlds_ok<T, OP, PRO>(g)) return hipErrorInvalidValue;
  if (nparts) *nparts = g.parts();
  const uint32_t blocks = g.parts() * (uint32_t)B;
  const size_t lds = zlds_bytes<T, OP, PRO>(g);
  const size_t cs = PRO ? grid_stride(n / 2) : 0;
  switch (halo_mode(g.G)) {
    case HALO_DPPROW:
      if constexpr (sizeof(T) == 4) {
        if (n == 64) {   // the fp32 64^3 mesh: its row size compiled in
          k_zlds<T, V, NEED_U, PRO, OP, Epi, HALO_DPPROW, 64><<<dim3(blocks), dim3(g.threads), lds, st>>>(
              g, grid_stride(n), T(1) / T(n), u, kap, active, partial, pstride, epi, xc, cs, op);
          break;
        }
      }
      k_zlds<T, V, NEED_U, PRO, OP, Epi, HALO_DPPROW><<<dim3(blocks), dim3(g.threads), lds, st>>>(
          g, grid_stride(n), T(1) / T(n), u, kap, active, partial, pstride, epi, xc, cs, op);
      break;
    case HALO_WAVE:
      k_zlds<T, V, NEED_U, PRO, OP, Epi, HALO_WAVE><<<dim3(blocks), dim3(g.threads), lds, st>>>(
          g, grid_stride(n), T(1) / T(n), u, kap, active, partial, pstride, epi, xc, cs, op);
      break;
    default:
      k_zlds<T, V, NEED_U, PRO, OP, Epi, HALO_SELECT><<<dim3(blocks), dim3(g.threads), lds, st>>>(
          g, grid_stride(n), T(1) / T(n), u, kap, active, partial, pstride, epi, xc, cs, op);
  }
  return hipGetLastError();
}

// the LDS engine when selected and its staging covers the tile (the register
// engine otherwise)
template <class T>
inline bool use_lds(int n, int B, int var, int bit) {
  return (var & bit) && (bit == ZVAR_LDS_PRO ? zlds_ok<T, OP_PLAIN, true>(zgeom<T>(n, B)) : zlds_ok<T>(zgeom<T>(n, B)));
}

template <class T, bool NEED_U, class Epi>
hipError_t zlaunch(int n, int B, const T* u, const T* kap, const int* active, double* partial, uint32_t pstride,
                   Epi epi, uint32_t* nparts, int var, hipStream_t st) {
  if (use_lds<T>(n, B, var, ZVAR_LDS))
    return zlaunch_lds<T, NEED_U, false, OP_PLAIN, Epi>(n, B, u, nullptr, kap, active, partial, pstride, epi, nparts,
                                                        st);
  constexpr int V = ZV<T>::V;
  const ZGeom g = zgeom<T>(n, B);
  if (g.G < 1) return hipErrorInvalidValue;
  if (nparts) *nparts = g.parts();
  const uint32_t blocks = g.parts() * (uint32_t)B;
  if (var & ZVAR_PREFETCH)
    k_zmarch<T, V, NEED_U, true, false, false, Epi><<<dim3(blocks), dim3(g.threads), 0, st>>>(
        g, grid_stride(n), T(1) / T(n), u, kap, active, partial, pstride, epi, nullptr, 0, nullptr);
  else
    k_zmarch<T, V, NEED_U, false, false, false, Epi><<<dim3(blocks), dim3(g.threads), 0, st>>>(
        g, grid_stride(n), T(1) / T(n), u, kap, active, partial, pstride, epi, nullptr, 0, nullptr);
  return hipGetLastError();
}

// the operand is u + d (d fp32, same layout; u may be null)
template <class T, class Epi>
hipError_t zlaunch_addd(int n, int B, const T* u, const float* d, const T* kap, const int* active, double* partial,
                        uint32_t pstride, Epi epi, uint32_t* nparts, int var, hipStream_t st) {
  if (use_lds<T>(n, B, var, ZVAR_LDS)) {
    OpArgs<T> op;
    op.d = d;
    return zlaunch_lds<T, true, false, OP_ADDD, Epi>(n, B, u, nullptr, kap, active, partial, pstride, epi, nparts, st,
                                                     op);
  }
  constexpr int V = ZV<T>::V;
  const ZGeom g = zgeom<T>(n, B);
  if (g.G < 1) return hipErrorInvalidValue;
  if (nparts) *nparts = g.parts();
  const uint32_t blocks = g.parts() * (uint32_t)B;
  k_zmarch<T, V, true, false, false, true, Epi><<<dim3(blocks), dim3(g.threads), 0, st>>>(
      g, grid_stride(n), T(1) / T(n), u, kap, active, partial, pstride, epi, nullptr, 0, d);
  return hipGetLastError();
}

// the operand is u + P xc (xc on the n/2 mesh); plain register window or LDS
template <class T, class Epi>
hipError_t zlaunch_pro(int n, int B, const T* u, const T* xc, const T* kap, const int* active, double* partial,
                       uint32_t pstride, Epi epi, uint32_t* nparts, hipStream_t st, int var) {
  if (use_lds<T>(n, B, var, ZVAR_LDS_PRO))
    return zlaunch_lds<T, true, true, OP_PLAIN, Epi>(n, B, u, xc, kap, active, partial, pstride, epi, nparts, st);
  constexpr int V = ZV<T>::V;
  const ZGeom g = zgeom<T>(n, B);
  if (g.G < 1) return hipErrorInvalidValue;
  if (nparts) *nparts = g.parts();
  const uint32_t blocks = g.parts() * (uint32_t)B;
  k_zmarch<T, V, true, false, true, false, Epi><<<dim3(blocks), dim3(g.threads), 0, st>>>(
      g, grid_stride(n), T(1) / T(n), u, kap, active, partial, pstride, epi, xc, grid_stride(n / 2), nullptr);
  return hipGetLastError();
}

// --------------------------------------------- fallback for meshes below V
// One thread per node (used for fp32 on the 2^3 mesh only).
struct Node {
  uint32_t b, s;
  bool ok;
};

__device__ __forceinline__ Node node_of_thread(int n, uint32_t nchunk) {
  Node nd;
  nd.b = blockIdx.x / nchunk;
  const uint32_t c = blockIdx.x - nd.b * nchunk;
  const uint32_t n2 = (uint32_t)n * n;
  const uint32_t p = n2 + c * kBlock + threadIdx.x;
  const uint32_t lg = (uint32_t)ilog2(n);
  const uint32_t i = p & (n - 1), j = (p >> lg) & (n - 1);
  nd.ok = (p < n2 * (uint32_t)n) && i != 0 && j != 0;
  nd.s = p;
  return nd;
}

inline uint32_t chunks_of(int n) { return (uint32_t)(((size_t)(n - 1) * n * n + kBlock - 1) / kBlock); }

template <class T>
__device__ __forceinline__ void q1_row(const T* __restrict__ u, const T* __restrict__ kap, int n, uint32_t s, T h,
                                       T& au, T& diag) {
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
  au = h * (ks * u0 * (T(1) / T(3)) - far * (T(1) / T(12)));
  diag = h * ks * (T(1) / T(3));
}

// mode 0 apply, 1 residual, 2 cheb zero, 3 cheb (no xo), 4 cheb with xo, 5 pcg apply+dot
template <class T>
__global__ void __launch_bounds__(kBlock) k_small(int mode, int n, uint32_t nchunk, size_t stride, T h,
                                                  const T* __restrict__ kap, const T* __restrict__ u,
                                                  const T* __restrict__ b, const T* xo, T* out, T c1, T c2,
                                                  const int* __restrict__ active, double* partial,
                                                  uint32_t pstride) {
  const Node nd = node_of_thread(n, nchunk);
  if (active && !active[nd.b]) return;
  double acc = 0.0;
  if (nd.ok) {
    const size_t ne = (size_t)n * n * n;
    const size_t g = nd.b * stride + nd.s;
    T au = T(0), dg = T(0);
    q1_row(u ? u + nd.b * stride : b + nd.b * stride, kap + nd.b * ne, n, nd.s, h, au, dg);
    switch (mode) {
      case 0: out[g] = au; break;
      case 1: out[g] = b[g] - au; break;
      case 2: out[g] = c2 * b[g] / dg; break;
      case 3: out[g] = u[g] + c1 * u[g] + c2 * (b[g] - au) / dg; break;
      case 4: out[g] = u[g] + c1 * (u[g] - xo[g]) + c2 * (b[g] - au) / dg; break;
      default: out[g] = au; acc = (double)u[g] * (double)au; break;
    }
  }
  if (mode == 5) {
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[(size_t)nd.b * pstride + (blockIdx.x - nd.b * nchunk)] = acc;
  }
}

template <class T>
hipError_t small_launch(int mode, int n, int B, const T* kap, const T* u, const T* b, const T* xo, T* out, double c1,
                        double c2, const int* active, double* partial, uint32_t pstride, uint32_t* nparts,
                        hipStream_t st) {
  const uint32_t nc = chunks_of(n);
  if (nparts) *nparts = nc;
  k_small<T><<<dim3(nc * (uint32_t)B), kBlock, 0, st>>>(mode, n, nc, grid_stride(n), T(1) / T(n), kap, u, b, xo, out,
                                                       T(c1), T(c2), active, partial, pstride);
  return hipGetLastError();
}

template <class T>
inline bool use_small(int n) { return n < ZV<T>::V || n < 2; }

// ------------------------------------------------------ transfer kernels
// full weighting: coarse node (I,J,K) gathers fine (2I+dx, 2J+dy, 2K+dz) with
// weights prod_d (dx == 0 ? 1 : 1/2).  A thread owns two coarse nodes I0, I0+1
// (I0 even) of one coarse row: per fine row it needs fine x 2I0-1 .. 2I0+3, one
// aligned 4-vector and one halo value.
template <class T>
__global__ void __launch_bounds__(kBlock) k_restrict(int nc, uint32_t nchunk, size_t sc, size_t sf,
                                                     const T* __restrict__ rf, T* __restrict__ bc,
                                                     const int* __restrict__ active) {
  const uint32_t logical = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t b = logical / nchunk, c = logical - b * nchunk;
  if (active && !active[b]) return;
  const uint32_t n2 = (uint32_t)nc * nc;
  const uint32_t p = n2 + 2 * (c * kBlock + threadIdx.x);
  if (p >= n2 * (uint32_t)nc) return;
  const int lg = ilog2(nc);
  const uint32_t I0 = p & (nc - 1), J = (p >> lg) & (nc - 1), K = p >> (2 * lg);
  if (J == 0) return;
  const int nf = 2 * nc;
  const T* r = rf + b * sf;
  const size_t f2 = (size_t)nf * nf;
  T a0 = T(0), a1 = T(0);
#pragma unroll
  for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
    for (int dy = -1; dy <= 1; ++dy) {
      const T w = (dy == 0 ? T(1) : T(0.5)) * (dz == 0 ? T(1) : T(0.5));
      const T* row = r + (size_t)nf * (2 * J + dy) + f2 * (2 * K + dz) + 2 * I0;
      T f[5];
      f[0] = I0 > 0 ? row[-1] : T(0);
      vload<T, 4>(row, f + 1);
      a0 += w * (T(0.5) * (f[0] + f[2]) + f[1]);
      a1 += w * (T(0.5) * (f[2] + f[4]) + f[3]);
    }
  T o[2] = {I0 > 0 ? a0 : T(0), a1};
  vstore<T, 2>(bc + b * sc + p, o);
}

// trilinear interpolation from the n/2 grid added to the fine values; a
// thread owns V consecutive fine nodes of one row (vector load/store of xf).
template <class T, int V>
__global__ void __launch_bounds__(kBlock) k_prolong_add(int nf, uint32_t nchunk, size_t sf, size_t sc,
                                                        const T* __restrict__ xc, T* __restrict__ xf,
                                                        const int* __restrict__ active) {
  const uint32_t logical = xcd_remap(blockIdx.x, gridDim.x);
  const uint32_t b = logical / nchunk, c = logical - b * nchunk;
  if (active && !active[b]) return;
  const uint32_t n2 = (uint32_t)nf * nf;
  const uint32_t p = n2 + (c * kBlock + threadIdx.x) * V;   // first of V fine positions
  if (p >= n2 * (uint32_t)nf) return;
  const int lg = ilog2(nf);
  const uint32_t i0 = p & (nf - 1), j = (p >> lg) & (nf - 1), k = p >> (2 * lg);
  if (j == 0) return;
  const int nc = nf / 2, c2 = nc * nc;
  const T* cb = xc + b * sc;
  // coarse x values covering fine i0-1 .. i0+V: coarse i0/2 .. i0/2 + V/2
  const uint32_t jl = j >> 1, jh = (j + 1) >> 1, kl = k >> 1, kh = (k + 1) >> 1;
  const T wj = (j & 1) ? T(0.5) : T(1), wk = (k & 1) ? T(0.5) : T(1);
  T cx[V / 2 + 1];
#pragma unroll
  for (int q = 0; q <= V / 2; ++q) cx[q] = T(0);
  auto add_row = [&](uint32_t jj, uint32_t kk, T w) {
    const T* row = cb + nc * jj + c2 * kk + (i0 >> 1);
#pragma unroll
    for (int q = 0; q <= V / 2; ++q) cx[q] += w * row[q];
  };
  // rows/planes: even index -> one coarse line with weight 1, odd -> two with 1/2
  if (k & 1) {
    if (j & 1) { add_row(jl, kl, wj * wk); add_row(jh, kl, wj * wk); add_row(jl, kh, wj * wk); add_row(jh, kh, wj * wk); }
    else { add_row(jl, kl, wk); add_row(jl, kh, wk); }
  } else {
    if (j & 1) { add_row(jl, kl, wj); add_row(jh, kl, wj); }
    else add_row(jl, kl, T(1));
  }
  T xv[V];
  vload<T, V>(xf + b * sf + p, xv);
#pragma unroll
  for (int v = 0; v < V; ++v) {
    const uint32_t i = i0 + v;
    if (i == 0) continue;
    const int q = v >> 1;   // coarse offset of i >> 1 relative to i0 >> 1
    xv[v] += (i & 1) ? T(0.5) * (cx[q] + cx[q + 1]) : cx[q];
  }
  vstore<T, V>(xf + b * sf + p, xv);
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
                                                    T* __restrict__ kc, const int* __restrict__ active) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= total) return;
  const int lg = __builtin_ctz((unsigned)nc);   // nc is a power of two
  const int64_t nce = (int64_t)nc * nc * nc;
  const int64_t b = t >> (3 * lg), E = t & (nce - 1);
  if (active && !active[b]) return;
  const int nf = 2 * nc;
  const int EX = (int)(E & (nc - 1)), EY = (int)((E >> lg) & (nc - 1)), EZ = (int)(E >> (2 * lg));
  const T* f = kf + b * nce * 8 + 2 * EX + (int64_t)nf * 2 * EY + (int64_t)nf * nf * 2 * EZ;
  const int64_t f2 = (int64_t)nf * nf;
  const T s = ((f[0] + f[1]) + (f[nf] + f[nf + 1])) + ((f[f2] + f[f2 + 1]) + (f[f2 + nf] + f[f2 + nf + 1]));
  kc[t] = s * T(0.125);
}

template <class Ts, class Td>
__global__ void __launch_bounds__(kBlock) k_convert(size_t count, const Ts* __restrict__ src, Td* __restrict__ dst) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < count) dst[t] = (Td)src[t];
}

}  // namespace

template <class T>
hipError_t launch_apply(int n, int B, const T* kap, const T* u, T* y, const int* active, hipStream_t st, int var) {
  if (use_small<T>(n))
    return small_launch<T>(0, n, B, kap, u, nullptr, nullptr, y, 0, 0, active, nullptr, 0, nullptr, st);
  return zlaunch<T, true>(n, B, u, kap, active, nullptr, 0, EpiApply<T, ZV<T>::V>{y}, nullptr, var, st);
}

template <class T>
hipError_t launch_residual(int n, int B, const T* kap, const T* b, const T* x, T* r, const int* active,
                           hipStream_t st, int var) {
  if (use_small<T>(n))
    return small_launch<T>(1, n, B, kap, x, b, nullptr, r, 0, 0, active, nullptr, 0, nullptr, st);
  return zlaunch<T, true>(n, B, x, kap, active, nullptr, 0, EpiResidual<T, ZV<T>::V>{b, r}, nullptr, var, st);
}

template <class T>
hipError_t launch_cheb(int n, int B, const T* kap, const T* b, const T* x, const T* xo, T* out, double c1,
                       double c2, bool zero_x, bool use_xo, const int* active, hipStream_t st, SolveState* dot,
                       uint32_t* nparts, int var) {
  constexpr int V = ZV<T>::V;
  if (use_small<T>(n)) {
    if (dot) return hipErrorInvalidValue;   // the fused r.z is only used on meshes with n >= V
    return small_launch<T>(zero_x ? 2 : (use_xo ? 4 : 3), n, B, kap, zero_x ? nullptr : x, b, xo, out, c1, c2,
                           active, nullptr, 0, nullptr, st);
  }
  if (zero_x) {
    if (dot) return hipErrorInvalidValue;
    return zlaunch<T, false>(n, B, nullptr, kap, active, nullptr, 0, EpiChebZero<T, V>{b, out, T(c2)}, nullptr, var,
                             st);
  }
  if (dot) {
    if (use_xo)
      return zlaunch<T, true>(n, B, x, kap, active, dot->partial, dot->pstride,
                              EpiCheb<T, V, true, true>{b, xo, out, T(c1), T(c2)}, nparts, var, st);
    return zlaunch<T, true>(n, B, x, kap, active, dot->partial, dot->pstride,
                            EpiCheb<T, V, false, true>{b, xo, out, T(c1), T(c2)}, nparts, var, st);
  }
  if (use_xo)
    return zlaunch<T, true>(n, B, x, kap, active, nullptr, 0, EpiCheb<T, V, true, false>{b, xo, out, T(c1), T(c2)},
                            nullptr, var, st);
  return zlaunch<T, true>(n, B, x, kap, active, nullptr, 0, EpiCheb<T, V, false, false>{b, xo, out, T(c1), T(c2)},
                          nullptr, var, st);
}

template <class T>
hipError_t launch_cheb_prolong(int n, int B, const T* kap, const T* b, const T* x, const T* xc, T* out, T* save,
                               double c2, const int* active, hipStream_t st, SolveState* dot, uint32_t* nparts,
                               int var) {
  constexpr int V = ZV<T>::V;
  if (use_small<T>(n) || n < 4) return hipErrorInvalidValue;
  if (dot)
    return zlaunch_pro<T>(n, B, x, xc, kap, active, dot->partial, dot->pstride,
                          EpiCheb<T, V, false, true>{b, nullptr, out, T(0), T(c2), save}, nparts, st, var);
  return zlaunch_pro<T>(n, B, x, xc, kap, active, nullptr, 0,
                        EpiCheb<T, V, false, false>{b, nullptr, out, T(0), T(c2), save}, nullptr, st, var);
}

template <class T>
bool presmooth_usable(int n, int B) {
  const ZGeom g = zlds_geom<T, true, OP_Z1>(n, B);
  return n >= 4 && !use_small<T>(n) && resr_ok<T, true>(resr_geom<T>(n, B)) && zlds_ok<T, OP_Z1, true>(g);
}

template <class T>
hipError_t launch_cheb_prolong_presmoothed(int n, int B, const T* kap, const T* b, const T* xc, T* out, double c2,
                                           const int* active, hipStream_t st, SolveState* dot, uint32_t* nparts,
                                           const T* b1, const int* bstate) {
  constexpr int V = ZV<T>::V;
  if (!presmooth_usable<T>(n, B)) return hipErrorInvalidValue;
  OpArgs<T> op;
  op.c2 = T(c2);
  op.u1 = b1;
  op.ustate = bstate;
  if (dot)
    return zlaunch_lds<T, true, true, OP_Z1>(
        n, B, b, xc, kap, active, dot->partial, dot->pstride,
        EpiCheb<T, V, false, true>{b, nullptr, out, T(0), T(c2), nullptr, b1, bstate}, nparts, st, op);
  return zlaunch_lds<T, true, true, OP_Z1>(
      n, B, b, xc, kap, active, nullptr, 0, EpiCheb<T, V, false, false>{b, nullptr, out, T(0), T(c2), nullptr, b1, bstate},
      nullptr, st, op);
}

template <class T>
hipError_t launch_pcg_update_zero(int n, int B, const T* kap, T* x, const T* p, T* r, const T* q, T* z, double c2,
                                  SolveState s, uint32_t* nparts, hipStream_t st, int var) {
  if (use_small<T>(n)) return hipErrorInvalidValue;
  return zlaunch<T, false>(n, B, nullptr, kap, s.active, s.partial, s.pstride,
                           EpiPcgUpdateZero<T, ZV<T>::V>{x, p, r, q, z, s.alpha, T(c2)}, nparts, var, st);
}

template <class T>
bool dir_usable(int n, int B) {
  const ZGeom g = zgeom<T>(n, B);
  return n >= 4 && !use_small<T>(n) && zlds_ok<T, OP_DIR>(g);
}

template <class T>
hipError_t launch_pcg_dir_apply(int n, int B, const T* kap, const T* z, T* x, T* p0, T* p1, T* q, const int* pstate,
                                SolveState s, uint32_t* nparts, hipStream_t st) {
  if (!dir_usable<T>(n, B)) return hipErrorInvalidValue;
  OpArgs<T> op;
  op.p0 = p0;
  op.p1 = p1;
  op.pstate = pstate;
  op.beta = s.beta;
  return zlaunch_lds<T, true, false, OP_DIR>(n, B, z, nullptr, kap, s.active, s.partial, s.pstride,
                                             EpiDirApply<T, ZV<T>::V>{x, p0, p1, q, pstate, s.alpha}, nparts, st, op);
}

template <class T>
hipError_t launch_pcg_rupdate_zero(int n, int B, const T* kap, T* r, const T* q, T* z, double c2, SolveState s,
                                   uint32_t* nparts, hipStream_t st, int var) {
  if (use_small<T>(n)) return hipErrorInvalidValue;
  return zlaunch<T, false>(n, B, nullptr, kap, s.active, s.partial, s.pstride,
                           EpiPcgRUpdateZero<T, ZV<T>::V>{r, q, z, s.alpha, T(c2)}, nparts, var, st);
}

template <class T>
hipError_t launch_pcg_apply_dot(int n, int B, const T* kap, const T* p, T* q, SolveState s, uint32_t* nparts,
                                hipStream_t st, int var) {
  if (use_small<T>(n))
    return small_launch<T>(5, n, B, kap, p, nullptr, nullptr, q, 0, 0, s.active, s.partial, s.pstride, nparts, st);
  return zlaunch<T, true>(n, B, p, kap, s.active, s.partial, s.pstride, EpiPcgApply<T, ZV<T>::V>{q}, nparts, var, st);
}

hipError_t launch_refine(int n, int B, const double* kap, double bconst, const double* u, const float* d,
                         double* uout, float* rin, SolveState s, uint32_t* nparts, hipStream_t st, int var,
                         const double* bvec) {
  return zlaunch_addd<double>(n, B, u, d, kap, s.active, s.partial, s.pstride,
                              EpiRefine<double, ZV<double>::V>{bconst, uout, rin, bvec}, nparts, var, st);
}

bool refine_owed_usable(int n, int B, int var) {
  return use_lds<double>(n, B, var, ZVAR_LDS) && zlds_ok<double, OP_ADDD>(zgeom<double>(n, B));
}

hipError_t launch_refine_owed(int n, int B, const double* kap, double bconst, const double* u, const float* d,
                              const float* p0, const float* p1, SolveState inner, double* uout, float* rin,
                              SolveState s, uint32_t* nparts, hipStream_t st, const double* bvec) {
  if (!zlds_ok<double, OP_ADDD>(zgeom<double>(n, B))) return hipErrorInvalidValue;
  OpArgs<double> op;
  op.d = d;
  op.q0 = p0;
  op.q1 = p1;
  op.dstate = inner.pstate;
  op.dalpha = inner.alpha;
  return zlaunch_lds<double, true, false, OP_ADDD>(n, B, u, nullptr, kap, s.active, s.partial, s.pstride,
                                                   EpiRefine<double, ZV<double>::V>{bconst, uout, rin, bvec}, nparts, st,
                                                   op);
}

hipError_t launch_true_residual(int n, int B, const double* kap, double bconst, const double* x, double* r,
                                SolveState s, uint32_t* nparts, hipStream_t st, int var, const double* bvec) {
  return zlaunch<double, true>(n, B, x, kap, s.active, s.partial, s.pstride,
                               EpiTrueResidual<double, ZV<double>::V>{bconst, r, bvec}, nparts, var, st);
}

template <class T>
bool resr_usable(int n, int B) { return resr_ok<T>(resr_geom<T>(n, B)); }

template <class T, int V, bool Z1, bool UPD>
void resr_dispatch(const ZGeom& g, uint32_t blocks, size_t lds, hipStream_t st, size_t stride, T h, const T* x,
                   const T* bf, const T* kap, const int* active, T* bc, size_t cstride, T c2, ResrUpd<T> upd) {
  // the extra row of a full tile in one pass of one wave where it is 64 or
  // 128 nodes and narrower than a row of vector tasks
  const bool full = g.rows * g.G == g.threads;
  const int rw = full && g.n == 64 && V > 1 ? 1 : (full && g.n == 128 && V > 2 ? 2 : 0);
  const int halo = halo_mode(g.G);
#define MLMC_RESR(H, RWV)                                                                                          \
  k_resr<T, V, Z1, UPD, H, RWV><<<dim3(blocks), dim3(g.threads), lds, st>>>(g, stride, h, x, bf, kap, active, bc, \
                                                                           cstride, c2, upd)
  // rows of 16 vectors are 64 fp32 (or 32 fp64) nodes, rows of 32 vectors
  // 128 fp32 (or 64 fp64) nodes
  constexpr int RW_SELECT = sizeof(T) == 4 ? 2 : 1;
  if (halo == HALO_DPPROW) {
    if constexpr (sizeof(T) == 4) {
      if (rw == 1) {
        if (g.n == 64 && g.threads == 256 && g.rows == 16) {
          k_resr<T, V, Z1, UPD, HALO_DPPROW, 1, 64><<<dim3(blocks), dim3(g.threads), lds, st>>>(
              g, stride, h, x, bf, kap, active, bc, cstride, c2, upd);
          return;
        }
        MLMC_RESR(HALO_DPPROW, 1);
        return;
      }
    }
    MLMC_RESR(HALO_DPPROW, 0);
  } else if (halo == HALO_WAVE) {
    MLMC_RESR(HALO_WAVE, 0);
  } else if (rw == RW_SELECT) {
    MLMC_RESR(HALO_SELECT, RW_SELECT);
  } else {
    MLMC_RESR(HALO_SELECT, 0);
  }
#undef MLMC_RESR
}

template <class T>
hipError_t launch_residual_restrict(int n, int B, const T* kap, const T* b, const T* x, T* bc, const int* active,
                                   hipStream_t st, bool presmooth, double c2) {
  constexpr int V = ZV<T>::V;
  const ZGeom g = resr_geom<T>(n, B);
  const uint32_t blocks = g.parts() * (uint32_t)B;
  if (presmooth) {
    if (!presmooth_usable<T>(n, B)) return hipErrorInvalidValue;
    resr_dispatch<T, V, true, false>(g, blocks, resr_bytes<T, true>(g), st, grid_stride(n), T(1) / T(n), nullptr, b,
                                     kap, active, bc, grid_stride(n / 2), T(c2), ResrUpd<T>{});
    return hipGetLastError();
  }
  if (!resr_ok<T>(g)) return hipErrorInvalidValue;
  resr_dispatch<T, V, false, false>(g, blocks, resr_bytes<T, false>(g), st, grid_stride(n), T(1) / T(n), x, b, kap,
                                    active, bc, grid_stride(n / 2), T(0), ResrUpd<T>{});
  return hipGetLastError();
}

template <class T>
hipError_t launch_residual_restrict_update(int n, int B, const T* kap, const T* r0, T* r1, const T* q, T* bc,
                                          SolveState s, double c2, uint32_t* nparts, hipStream_t st) {
  constexpr int V = ZV<T>::V;
  const ZGeom g = resr_geom<T>(n, B);
  if (!presmooth_usable<T>(n, B)) return hipErrorInvalidValue;
  if (nparts) *nparts = g.parts();
  ResrUpd<T> u;
  u.q = q;
  u.r1 = r1;
  u.pstate = s.pstate;
  u.alpha = s.alpha;
  u.partial = s.partial;
  u.pstride = s.pstride;
  const uint32_t blocks = g.parts() * (uint32_t)B;
  resr_dispatch<T, V, true, true>(g, blocks, resr_bytes<T, true>(g), st, grid_stride(n), T(1) / T(n), nullptr, r0, kap,
                                  s.active, bc, grid_stride(n / 2), T(c2), u);
  return hipGetLastError();
}

template <class T>
hipError_t launch_restrict(int nf, int B, const T* rf, T* bc, const int* active, hipStream_t st) {
  const int nc = nf / 2;
  const uint32_t ch = (uint32_t)(((size_t)(nc - 1) * nc * nc / 2 + kBlock - 1) / kBlock);
  k_restrict<T><<<dim3(ch * (uint32_t)B), kBlock, 0, st>>>(nc, ch, grid_stride(nc), grid_stride(nf), rf, bc, active);
  return hipGetLastError();
}

template <class T>
hipError_t launch_prolong_add(int nf, int B, const T* xc, T* xf, const int* active, hipStream_t st) {
  constexpr int V = 4;   // 4 fine nodes per thread (needs nf >= 4)
  const size_t pos = (size_t)(nf - 1) * nf * nf / V;
  const uint32_t ch = (uint32_t)((pos + kBlock - 1) / kBlock);
  k_prolong_add<T, V><<<dim3(ch * (uint32_t)B), kBlock, 0, st>>>(nf, ch, grid_stride(nf), grid_stride(nf / 2), xc,
                                                                 xf, active);
  return hipGetLastError();
}

template <class T>
hipError_t launch_coarsest(int B, const T* kap, const T* b, T* x, const int* active, hipStream_t st) {
  k_coarsest<T><<<dim3((B + 63) / 64), 64, 0, st>>>(B, grid_stride(2), kap, b, x, active);
  return hipGetLastError();
}

template <class T>
hipError_t launch_coarsen(int nf, int B, const T* kf, T* kc, hipStream_t st, const int* active) {
  const int nc = nf / 2;
  const int64_t total = (int64_t)B * nc * nc * nc;
  k_coarsen<T><<<dim3((unsigned)((total + kBlock - 1) / kBlock)), kBlock, 0, st>>>(nc, total, kf, kc, active);
  return hipGetLastError();
}

template <class Ts, class Td>
hipError_t launch_convert(size_t count, const Ts* src, Td* dst, hipStream_t st) {
  if (!count) return hipSuccess;
  k_convert<Ts, Td><<<dim3((unsigned)((count + kBlock - 1) / kBlock)), kBlock, 0, st>>>(count, src, dst);
  return hipGetLastError();
}

#define MLMC_INST(T)                                                                                    \
  template hipError_t launch_apply<T>(int, int, const T*, const T*, T*, const int*, hipStream_t, int); \
  template hipError_t launch_residual<T>(int, int, const T*, const T*, const T*, T*, const int*,       \
                                         hipStream_t, int);                                            \
  template hipError_t launch_cheb<T>(int, int, const T*, const T*, const T*, const T*, T*, double,     \
                                     double, bool, bool, const int*, hipStream_t, SolveState*,         \
                                     uint32_t*, int);                                                  \
  template hipError_t launch_cheb_prolong<T>(int, int, const T*, const T*, const T*, const T*, T*, T*,   \
                                             double, const int*, hipStream_t, SolveState*, uint32_t*,   \
                                             int);                                                      \
  template hipError_t launch_pcg_update_zero<T>(int, int, const T*, T*, const T*, T*, const T*, T*,     \
                                                double, SolveState, uint32_t*, hipStream_t, int);      \
  template hipError_t launch_pcg_apply_dot<T>(int, int, const T*, const T*, T*, SolveState, uint32_t*, \
                                              hipStream_t, int);                                       \
  template hipError_t launch_restrict<T>(int, int, const T*, T*, const int*, hipStream_t);             \
  template bool resr_usable<T>(int, int);                                                              \
  template hipError_t launch_residual_restrict<T>(int, int, const T*, const T*, const T*, T*, const int*, \
                                                  hipStream_t, bool, double);                          \
  template bool presmooth_usable<T>(int, int);                                                         \
  template bool dir_usable<T>(int, int);                                                               \
  template hipError_t launch_pcg_dir_apply<T>(int, int, const T*, const T*, T*, T*, T*, T*, const int*,  \
                                              SolveState, uint32_t*, hipStream_t);                     \
  template hipError_t launch_pcg_rupdate_zero<T>(int, int, const T*, T*, const T*, T*, double, SolveState, \
                                                 uint32_t*, hipStream_t, int);                         \
  template hipError_t launch_cheb_prolong_presmoothed<T>(int, int, const T*, const T*, const T*, T*, double, \
                                                         const int*, hipStream_t, SolveState*, uint32_t*, \
                                                         const T*, const int*);                            \
  template hipError_t launch_residual_restrict_update<T>(int, int, const T*, const T*, T*, const T*, T*,  \
                                                         SolveState, double, uint32_t*, hipStream_t);      \
  template hipError_t launch_prolong_add<T>(int, int, const T*, T*, const int*, hipStream_t);          \
  template hipError_t launch_coarsest<T>(int, const T*, const T*, T*, const int*, hipStream_t);        \
  template hipError_t launch_coarsen<T>(int, int, const T*, T*, hipStream_t, const int*);
MLMC_INST(float)
MLMC_INST(double)
#undef MLMC_INST
template hipError_t launch_convert<double, float>(size_t, const double*, float*, hipStream_t);
template hipError_t launch_convert<float, double>(size_t, const float*, double*, hipStream_t);

}  // namespace mlmc
