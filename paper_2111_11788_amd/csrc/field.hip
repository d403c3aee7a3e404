// K2: log-normal KLE coefficient on fp64 MFMA.
//
// kappa_b(e) = exp( sum_m Xi[b][m] Phi[e][m] ),  Xi[b][m] = xi_b,m sqrt(lambda_m),
// Phi[e][m] = phi_i(x_e) phi_j(y_e) phi_k(z_e) for mode m = (i, j, k) evaluated
// at the element centroid (the KLE of the log-field in Sec. 5.2).  The sum is
// a dense [B x M] . [M x n^3] contraction; Phi is never stored in HBM -- each
// workgroup builds its [elements x modes] tile in LDS from the separable 1D
// tables tab[x][q] = phi_q((x + 1/2)/n) and feeds it to
// v_mfma_f64_16x16x4_f64 with the xi tile.  exp (and the optional fp32 copy)
// is applied in the epilogue, so g never round-trips through memory.
//
// Operand layout of v_mfma_f64_16x16x4_f64 (64 lanes, checked on gfx950 with a
// probe of encoded operands): lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16]; accumulator element r of lane l holds D[l / 16 + 4 r][l % 16].
// Rows = samples, columns = elements, K = modes.  An optional row map sends
// row r to batch slot rowmap[r] (xi read from and kappa written to that slot).
// The default evaluation for 64^3 to 256^3 meshes factorises the same sum
// over the three axes and keeps only the final per-plane contraction, a
// [n x K1] . [K1 x n] product, on the same instruction (k_field_plane_mfma).
#include <algorithm>

#include "common.hpp"
#include "kernels.hpp"

namespace mlmc {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kKc = 16;   // modes per LDS stage (4 MFMA k-steps)

// BS samples x BE elements per workgroup of 4 waves; each wave owns a
// 16-sample x 64-element strip (four 16x16 accumulator tiles).
template <int BS>
__global__ void __launch_bounds__(256) k_field(int n, int M, int64_t count,
                                               const double* __restrict__ xi,
                                               const double* __restrict__ sqrtlam,
                                               const int* __restrict__ triples,
                                               const double* __restrict__ tab, int K1,
                                               double* __restrict__ kappa, float* __restrict__ kappa32,
                                               const int* __restrict__ rowmap) {
  constexpr int WS = BS / 16;          // waves along samples
  constexpr int WE = 4 / WS;           // waves along elements
  constexpr int BE = 64 * WE;          // elements per workgroup
  __shared__ double xs[BS][kKc + 1];
  __shared__ double ph[BE][kKc + 1];

  // The tile's BE elements are consecutive and n is a power of two, so the
  // tile covers TR = max(1, BE / n) whole or partial x-rows; the y-z factor
  // phi_j(y) phi_k(z) of a mode is shared by every element of a row.
  // TR = min(BE / n, n^2) <= 32 over all powers of two n (n = 8: 32 rows)
  __shared__ double wyz[32][kKc];
  const int ne = n * n * n;                  // <= 2^27 for the meshes in use
  const int e0 = (int)blockIdx.x * BE;
  const int64_t s0 = (int64_t)blockIdx.y * BS;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ws = wave % WS, we = wave / WS;
  const int lg = 31 - __clz(n);
  const int TR = BE > n ? (BE / n < n * n ? BE / n : n * n) : 1;
  const int row0 = e0 >> lg;                 // first x-row (ey + n ez) of the tile

  d4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};

  for (int m0 = 0; m0 < M; m0 += kKc) {
    // stage Xi (scaled by sqrt(lambda)), the y-z factors of the tile rows,
    // then the Phi tile = phi_i(x) * y-z factor
    for (int q = tid; q < BS * kKc; q += 256) {
      const int r = q / kKc, c = q % kKc;
      const int64_t s = s0 + r;
      const int m = m0 + c;
      const int64_t row = (s < count && rowmap) ? rowmap[s] : s;
      xs[r][c] = (s < count && m < M) ? xi[row * M + m] * sqrtlam[m] : 0.0;
    }
    for (int q = tid; q < TR * kKc; q += 256) {
      const int tr = q / kKc, c = q % kKc;
      const int m = m0 + c;
      const int xr = row0 + tr;              // x-row index ey + n ez
      double v = 0.0;
      if (m < M && xr < n * n) {
        const int ey = xr & (n - 1), ez = xr >> lg;
        v = tab[ey * K1 + triples[3 * m + 1]] * tab[ez * K1 + triples[3 * m + 2]];
      }
      wyz[tr][c] = v;
    }
    __syncthreads();
    for (int q = tid; q < BE * kKc; q += 256) {
      const int r = q / kKc, c = q % kKc;
      const int e = e0 + r;
      const int m = m0 + c;
      double v = 0.0;
      if (e < ne && m < M) v = tab[(e & (n - 1)) * K1 + triples[3 * m]] * wyz[(e >> lg) - row0][c];
      ph[r][c] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kKc; kk += 4) {
      const double a = xs[16 * ws + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double b = ph[64 * we + 16 * t + (lane & 15)][kk + (lane >> 4)];
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[t], 0, 0, 0);
      }
    }
    __syncthreads();
  }

#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t e = (int64_t)e0 + 64 * we + 16 * t + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t s = s0 + 16 * ws + (lane >> 4) + 4 * r;
      if (s < count && e < ne) {
        const int64_t row = rowmap ? rowmap[s] : s;
        const double k = exp(acc[t][r]);
        kappa[row * (int64_t)ne + e] = k;
        if (kappa32) kappa32[row * (int64_t)ne + e] = (float)k;
      }
    }
  }
}

// ---------------------------------------------------------------- bf16 MFMA
// The same contraction with bf16 operands and fp32 accumulation on
// v_mfma_f32_16x16x32_bf16 (gfx950): lane l supplies A[l % 16][8 (l / 16) + v]
// and B[8 (l / 16) + v][l % 16], v = 0..7, and accumulator element r holds
// D[4 (l / 16) + r][l % 16] (checked on gfx950 with a probe of one-hot
// operands).  Xi sqrt(lambda) and Phi are formed in fp64 and rounded to bf16
// (unit roundoff 2^-8), so |g - g_exact| <= (2 u + u^2 + M 2^-24) sum_m
// |Xi_m Phi_m|; kappa = exp(g) is evaluated in fp64 from the fp32 sum.  This
// changes the coefficient field itself (a model perturbation of up to ~1% in
// kappa for |g| of a few units), not just the route to it.
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
constexpr int kKb = 32;        // modes per stage (one MFMA k-step)
constexpr int kKbPad = 40;     // LDS row pitch in bf16 (16-byte aligned rows)

template <int BS>
__global__ void __launch_bounds__(256) k_field_bf16(int n, int M, int64_t count,
                                                    const double* __restrict__ xi,
                                                    const double* __restrict__ sqrtlam,
                                                    const int* __restrict__ triples,
                                                    const double* __restrict__ tab, int K1,
                                                    double* __restrict__ kappa, float* __restrict__ kappa32,
                                                    const int* __restrict__ rowmap) {
  constexpr int WS = BS / 16;
  constexpr int WE = 4 / WS;
  constexpr int BE = 64 * WE;
  __shared__ __align__(16) __bf16 xs[BS][kKbPad];
  __shared__ __align__(16) __bf16 ph[BE][kKbPad];
  __shared__ double wyz[32][kKb];
  const int ne = n * n * n;
  const int e0 = (int)blockIdx.x * BE;
  const int64_t s0 = (int64_t)blockIdx.y * BS;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ws = wave % WS, we = wave / WS;
  const int lg = 31 - __clz(n);
  const int TR = BE > n ? (BE / n < n * n ? BE / n : n * n) : 1;
  const int row0 = e0 >> lg;

  f4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = f4{0.f, 0.f, 0.f, 0.f};

  for (int m0 = 0; m0 < M; m0 += kKb) {
    for (int q = tid; q < BS * kKb; q += 256) {
      const int r = q / kKb, c = q % kKb;
      const int64_t s = s0 + r;
      const int m = m0 + c;
      const int64_t row = (s < count && rowmap) ? rowmap[s] : s;
      xs[r][c] = (__bf16)(float)((s < count && m < M) ? xi[row * M + m] * sqrtlam[m] : 0.0);
    }
    for (int q = tid; q < TR * kKb; q += 256) {
      const int tr = q / kKb, c = q % kKb;
      const int m = m0 + c;
      const int xr = row0 + tr;
      double v = 0.0;
      if (m < M && xr < n * n) {
        const int ey = xr & (n - 1), ez = xr >> lg;
        v = tab[ey * K1 + triples[3 * m + 1]] * tab[ez * K1 + triples[3 * m + 2]];
      }
      wyz[tr][c] = v;
    }
    __syncthreads();
    for (int q = tid; q < BE * kKb; q += 256) {
      const int r = q / kKb, c = q % kKb;
      const int e = e0 + r;
      const int m = m0 + c;
      double v = 0.0;
      if (e < ne && m < M) v = tab[(e & (n - 1)) * K1 + triples[3 * m]] * wyz[(e >> lg) - row0][c];
      ph[r][c] = (__bf16)(float)v;
    }
    __syncthreads();
    const bf8 a = *reinterpret_cast<const bf8*>(&xs[16 * ws + (lane & 15)][8 * (lane >> 4)]);
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const bf8 b = *reinterpret_cast<const bf8*>(&ph[64 * we + 16 * t + (lane & 15)][8 * (lane >> 4)]);
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
    }
    __syncthreads();
  }

#pragma unroll
  for (int t = 0; t < 4; ++t) {
    const int64_t e = (int64_t)e0 + 64 * we + 16 * t + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t s = s0 + 16 * ws + 4 * (lane >> 4) + r;
      if (s < count && e < ne) {
        const int64_t row = rowmap ? rowmap[s] : s;
        const double k = exp((double)acc[t][r]);
        kappa[row * (int64_t)ne + e] = k;
        if (kappa32) kappa32[row * (int64_t)ne + e] = (float)k;
      }
    }
  }
}

// ------------------------------------------------------------ separable form
// The modes are products phi_i(x) phi_j(y) phi_k(z), so on one x-row of
// elements (fixed ey, ez)
//   g[s][ex] = sum_a phi_a(x_ex) H[s][a],
//   H[s][a]  = sum over the modes m with x-factor a of xi[s][m] sqrt(lambda_m) phi_j(y) phi_k(z):
// M products per sample and row, then K1 (distinct x-factors, <= 16 for 512
// modes at correlation length 0.1) per element, against M per element for the
// dense contraction.  A workgroup takes S samples and R consecutive x-rows:
// it stages the samples' xi in x-grouped mode order into LDS once, then per
// row forms w (the row's y-z factors, sqrt(lambda) included), H and the row's
// elements.  Every sum runs in a fixed order, so a sample's field does not
// depend on its batch.
constexpr int kSepRows = 16;   // x-rows per workgroup

__global__ void __launch_bounds__(256) k_field_sep(int n, int M, int K1, int S, int64_t count,
                                                   const double* __restrict__ xi,
                                                   const double* __restrict__ sqrtlam,
                                                   const int* __restrict__ triples,
                                                   const int* __restrict__ xperm, const int* __restrict__ xoff,
                                                   const double* __restrict__ tab, double* __restrict__ kappa,
                                                   float* __restrict__ kappa32, const int* __restrict__ rowmap) {
  extern __shared__ double fsm[];
  double* X = fsm;            // [S][M]: xi of the block, x-grouped order
  double* w = X + S * M;      // [M]
  double* H = w + M;          // [S][K1]
  double* T = H + S * K1;     // [K1][n]: phi_a(x_ex), transposed so a row's lanes read consecutive words
  const int lg = 31 - __clz(n);
  const int nrows = n * n;
  const int row0 = (int)blockIdx.x * kSepRows;
  const int64_t s0 = (int64_t)blockIdx.y * S;
  const int tid = (int)threadIdx.x;
  for (int q = tid; q < S * M; q += 256) {
    const int s = q / M, p = q - (q / M) * M;
    double v = 0.0;
    if (s0 + s < count) {
      const int64_t r = rowmap ? rowmap[s0 + s] : s0 + s;
      v = xi[r * M + xperm[p]];
    }
    X[q] = v;
  }
  for (int q = tid; q < K1 * n; q += 256) {
    const int a = q >> lg, ex = q & (n - 1);
    T[q] = tab[ex * K1 + a];
  }
  const int64_t ne = (int64_t)n * n * n;
  for (int row = row0; row < row0 + kSepRows && row < nrows; ++row) {
    const int ey = row & (n - 1), ez = row >> lg;
    __syncthreads();   // X staged; the previous row's H no longer read
    for (int p = tid; p < M; p += 256) {
      const int m = xperm[p];
      w[p] = sqrtlam[m] * (tab[ey * K1 + triples[3 * m + 1]] * tab[ez * K1 + triples[3 * m + 2]]);
    }
    __syncthreads();
    for (int q = tid; q < S * K1; q += 256) {
      const int s = q / K1, a = q - (q / K1) * K1;
      const double* x = X + s * M;
      double hv = 0.0;
      for (int p = xoff[a]; p < xoff[a + 1]; ++p) hv += x[p] * w[p];
      H[q] = hv;
    }
    __syncthreads();
    for (int q = tid; q < S * n; q += 256) {
      const int s = q >> lg, ex = q & (n - 1);
      if (s0 + s >= count) continue;
      const double* hs = H + s * K1;
      double g = 0.0;
      for (int a = 0; a < K1; ++a) g += hs[a] * T[a * n + ex];
      const int64_t r = rowmap ? rowmap[s0 + s] : s0 + s;
      const double k = exp(g);
      const int64_t e = (int64_t)row * n + ex;
      kappa[r * ne + e] = k;
      if (kappa32) kappa32[r * ne + e] = (float)k;
    }
  }
}

// ------------------------------------------ separable form, one z-plane per workgroup
// The same sum factorised over all three axes: on the element plane ez of
// sample s,
//   A[a][b]   = sum over the modes m = (a, b, c) of sqrt(lambda_m) xi[s][m] phi_c(z_ez)
//   B[ey][a]  = sum_b A[a][b] phi_b(y_ey)
//   g[ey][ex] = sum_a B[ey][a] phi_a(x_ex)
// so an element costs K1 multiply-adds and the exponential, and the plane's
// M + n K1^2 other products are shared by its n^2 elements.  The element
// contraction g = B Phi_x (n x K1 by K1 x n, K1 padded to a multiple of 4
// with zeros) runs on v_mfma_f64_16x16x4f64: wave w owns the 16-column tiles
// w, w + 4, ... (CTW = n / 64 of them) and keeps their Phi_x operands in
// registers (lane l: phi_{4 ks + l/16} of column 16 t + l % 16); B is formed
// RB rows at a time into LDS (odd row pitch), and per 16-row tile the wave
// loads its A operands once and runs KS k-steps per column tile; the
// accumulator's rows (l/16 + 4 r) and column (l % 16) go through exp to
// kappa.  Every sum runs in a fixed order (A over the modes in x-grouped
// order, B over b, g in the MFMA's k-steps), so a sample's field does not
// depend on its batch.  (The same form with the element sums on the VALU
// measured 706 / 902 us against 574 / 612 us here for 64^3 x 1024 / 256^3 x 16.)
template <int KS, int CTW>
__global__ void __launch_bounds__(256) k_field_plane_mfma(int n, int M, int K1, int RB, int64_t count,
                                                          const double* __restrict__ xi,
                                                          const double* __restrict__ sqrtlam,
                                                          const int* __restrict__ triples,
                                                          const int* __restrict__ xperm,
                                                          const int* __restrict__ xoff,
                                                          const double* __restrict__ tab,
                                                          double* __restrict__ kappa, float* __restrict__ kappa32,
                                                          const int* __restrict__ rowmap) {
  constexpr int KP = 4 * KS, KPS = KP + 1;
  extern __shared__ double fsm[];
  double* wv = fsm;                                   // [M] sqrt(lambda) xi phi_c(z), x-grouped order
  double* A = wv + M;                                 // [K1][K1]
  double* Bm = A + K1 * K1;                           // [RB][KPS]
  int* bv = reinterpret_cast<int*>(Bm + RB * KPS);    // [M] y-factor of each mode
  const int ez = (int)blockIdx.x;
  const int64_t s = (int64_t)blockIdx.y;
  if (s >= count) return;
  const int64_t r = rowmap ? rowmap[s] : s;
  const int tid = (int)threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int p = tid; p < M; p += 256) {
    const int m = xperm[p];
    const int b = triples[3 * m + 1], c = triples[3 * m + 2];
    wv[p] = sqrtlam[m] * xi[r * M + m] * tab[ez * K1 + c];
    bv[p] = b;
  }
  double ph[CTW][KS];
#pragma unroll
  for (int t = 0; t < CTW; ++t)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int a = 4 * ks + (lane >> 4), ex = 16 * (wave + 4 * t) + (lane & 15);
      ph[t][ks] = a < K1 ? tab[ex * K1 + a] : 0.0;
    }
  __syncthreads();
  for (int q = tid; q < K1 * K1; q += 256) {
    const int a = q / K1, b = q - a * K1;
    double acc = 0.0;
    for (int p = xoff[a]; p < xoff[a + 1]; ++p)
      if (bv[p] == b) acc += wv[p];
    A[q] = acc;
  }
  const int64_t ne = (int64_t)n * n * n;
  double* kr = kappa + r * ne + (int64_t)ez * n * n;
  float* kr32 = kappa32 ? kappa32 + r * ne + (int64_t)ez * n * n : nullptr;
  for (int y0 = 0; y0 < n; y0 += RB) {
    __syncthreads();   // A formed; the previous rows' B no longer read
    for (int q = tid; q < RB * KP; q += 256) {
      const int yr = q / KP, a = q - yr * KP;
      double acc = 0.0;
      if (a < K1) {
        const double* ty = tab + (y0 + yr) * K1;
        const double* Aa = A + a * K1;
        for (int b = 0; b < K1; ++b) acc = fma(Aa[b], ty[b], acc);
      }
      Bm[yr * KPS + a] = acc;
    }
    __syncthreads();
    for (int rt = 0; rt < RB / 16; ++rt) {
      double av[KS];
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) av[ks] = Bm[(16 * rt + (lane & 15)) * KPS + 4 * ks + (lane >> 4)];
#pragma unroll
      for (int t = 0; t < CTW; ++t) {
        d4 acc = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[ks], ph[t][ks], acc, 0, 0, 0);
        const int ex = 16 * (wave + 4 * t) + (lane & 15);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int64_t e = (int64_t)(y0 + 16 * rt + (lane >> 4) + 4 * q) * n + ex;
          const double k = exp(acc[q]);
          kr[e] = k;
          if (kr32) kr32[e] = (float)k;
        }
      }
    }
  }
}

template <int KS, int CTW>
void launch_field_plane_mfma(int n, int M, int K1, int64_t count, const double* xi, const double* sqrtlam,
                             const int* triples, const int* xperm, const int* xoff, const double* tab,
                             double* kappa, float* kappa32, const int* rowmap, hipStream_t st) {
  constexpr int KPS = 4 * KS + 1;
  // B rows per pass: a power of two of 16 rows or more within 2048 values
  int RB = 16;
  while (RB * 2 <= n && RB * 2 * KPS <= 2048) RB *= 2;
  const size_t lds = ((size_t)M + (size_t)K1 * K1 + (size_t)RB * KPS) * sizeof(double) + (size_t)M * sizeof(int);
  dim3 grid((unsigned)n, (unsigned)count);
  k_field_plane_mfma<KS, CTW><<<grid, dim3(256), lds, st>>>(n, M, K1, RB, count, xi, sqrtlam, triples, xperm, xoff,
                                                            tab, kappa, kappa32, rowmap);
}

template <int KS>
void launch_field_plane_mfma_n(int n, int M, int K1, int64_t count, const double* xi, const double* sqrtlam,
                               const int* triples, const int* xperm, const int* xoff, const double* tab,
                               double* kappa, float* kappa32, const int* rowmap, hipStream_t st) {
  if (n == 64) launch_field_plane_mfma<KS, 1>(n, M, K1, count, xi, sqrtlam, triples, xperm, xoff, tab, kappa, kappa32, rowmap, st);
  else if (n == 128) launch_field_plane_mfma<KS, 2>(n, M, K1, count, xi, sqrtlam, triples, xperm, xoff, tab, kappa, kappa32, rowmap, st);
  else launch_field_plane_mfma<KS, 4>(n, M, K1, count, xi, sqrtlam, triples, xperm, xoff, tab, kappa, kappa32, rowmap, st);
}

}  // namespace

hipError_t launch_field(int n, int M, int64_t count, const double* xi, const double* sqrtlam,
                        const int* triples, const double* tab, int K1, double* kappa,
                        float* kappa32, hipStream_t st, const int* rowmap, bool bf16, const int* xperm,
                        const int* xoff) {
  if (count <= 0) return hipSuccess;
  const int64_t ne = (int64_t)n * n * n;
  if (!bf16 && xperm && xoff && (n == 64 || n == 128 || n == 256) && K1 <= 32 && M <= 2048 && count <= 65535) {
    // one workgroup per sample and element plane (at most 48 KiB of LDS)
    if (K1 <= 8) launch_field_plane_mfma_n<2>(n, M, K1, count, xi, sqrtlam, triples, xperm, xoff, tab, kappa, kappa32, rowmap, st);
    else if (K1 <= 16) launch_field_plane_mfma_n<4>(n, M, K1, count, xi, sqrtlam, triples, xperm, xoff, tab, kappa, kappa32, rowmap, st);
    else launch_field_plane_mfma_n<8>(n, M, K1, count, xi, sqrtlam, triples, xperm, xoff, tab, kappa, kappa32, rowmap, st);
    return hipGetLastError();
  }
  if (!bf16 && xperm && xoff) {
    // samples per workgroup: as many as fit 64 KiB of LDS with the row's
    // factors and the transposed x-table, at most 32 (more workgroups per CU
    // measured faster than larger blocks)
    const int64_t room = (65536 / (int64_t)sizeof(double) - M - (int64_t)K1 * n) / (M + K1);
    int S = (int)std::min<int64_t>({32, room, count});
    const size_t lds = ((size_t)S * M + M + (size_t)S * K1 + (size_t)K1 * n) * sizeof(double);
    if (S >= 1 && (count + S - 1) / S <= 65535) {   // grid y within the launch limit
      dim3 grid((unsigned)(((int64_t)n * n + kSepRows - 1) / kSepRows), (unsigned)((count + S - 1) / S));
      k_field_sep<<<grid, dim3(256), lds, st>>>(n, M, K1, S, count, xi, sqrtlam, triples, xperm, xoff, tab, kappa,
                                                 kappa32, rowmap);
      return hipGetLastError();
    }
    // the block's coefficients and sums exceed the LDS of a workgroup: the dense form
  }
  if (bf16) {
    if (count >= 48) {
      dim3 grid((unsigned)((ne + 63) / 64), (unsigned)((count + 63) / 64));
      k_field_bf16<64><<<grid, dim3(256), 0, st>>>(n, M, count, xi, sqrtlam, triples, tab, K1, kappa, kappa32,
                                                   rowmap);
    } else {
      dim3 grid((unsigned)((ne + 255) / 256), (unsigned)((count + 15) / 16));
      k_field_bf16<16><<<grid, dim3(256), 0, st>>>(n, M, count, xi, sqrtlam, triples, tab, K1, kappa, kappa32,
                                                   rowmap);
    }
    return hipGetLastError();
  }
  if (count >= 48) {
    dim3 grid((unsigned)((ne + 63) / 64), (unsigned)((count + 63) / 64));
    k_field<64><<<grid, dim3(256), 0, st>>>(n, M, count, xi, sqrtlam, triples, tab, K1, kappa, kappa32, rowmap);
  } else {
    dim3 grid((unsigned)((ne + 255) / 256), (unsigned)((count + 15) / 16));
    k_field<16><<<grid, dim3(256), 0, st>>>(n, M, count, xi, sqrtlam, triples, tab, K1, kappa, kappa32, rowmap);
  }
  return hipGetLastError();
}

}  // namespace mlmc
