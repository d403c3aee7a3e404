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

  const int64_t ne = (int64_t)n * n * n;
  const int64_t e0 = (int64_t)blockIdx.x * BE;
  const int64_t s0 = (int64_t)blockIdx.y * BS;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int ws = wave % WS, we = wave / WS;
  const int n2 = n * n;

  d4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};

  for (int m0 = 0; m0 < M; m0 += kKc) {
    // stage Xi (scaled by sqrt(lambda)) and the Phi tile
    for (int q = tid; q < BS * kKc; q += 256) {
      const int r = q / kKc, c = q % kKc;
      const int64_t s = s0 + r;
      const int m = m0 + c;
      const int64_t row = (s < count && rowmap) ? rowmap[s] : s;
      xs[r][c] = (s < count && m < M) ? xi[row * M + m] * sqrtlam[m] : 0.0;
    }
    for (int q = tid; q < BE * kKc; q += 256) {
      const int r = q / kKc, c = q % kKc;
      const int64_t e = e0 + r;
      const int m = m0 + c;
      double v = 0.0;
      if (e < ne && m < M) {
        const int ex = (int)(e % n), ey = (int)((e / n) % n), ez = (int)(e / n2);
        const int* t3 = triples + 3 * m;
        v = tab[ex * K1 + t3[0]] * tab[ey * K1 + t3[1]] * tab[ez * K1 + t3[2]];
      }
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
    const int64_t e = e0 + 64 * we + 16 * t + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t s = s0 + 16 * ws + (lane >> 4) + 4 * r;
      if (s < count && e < ne) {
        const int64_t row = rowmap ? rowmap[s] : s;
        const double k = exp(acc[t][r]);
        kappa[row * ne + e] = k;
        if (kappa32) kappa32[row * ne + e] = (float)k;
      }
    }
  }
}

}  // namespace

hipError_t launch_field(int n, int M, int64_t count, const double* xi, const double* sqrtlam,
                        const int* triples, const double* tab, int K1, double* kappa,
                        float* kappa32, hipStream_t st, const int* rowmap) {
  if (count <= 0) return hipSuccess;
  const int64_t ne = (int64_t)n * n * n;
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
