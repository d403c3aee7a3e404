// K1: counter-based draw of the KLE coefficients xi on the device.
//
// Every coefficient is a pure function of (seed, level, sample index): the
// paper puts the randomness in omega (Sec. 2.1) and distributes samples as
// contiguous index ranges (Sec. 4.2), so a sample can be drawn anywhere, in
// any batch, and always gets the same xi.
//
// Generator: Philox4x64 with 10 rounds (Salmon, Moraes, Dror, Shaw, SC'11),
// key (seed, 0), counter (sample, level, block, 0).  Each 64-bit word becomes
// the uniform ((w >> 12) + 1/2) 2^-52 (exact, strictly inside (0,1)); uniforms
// (u0, u1) and (u2, u3) of a block give two Box-Muller pairs
//   z = sqrt(-2 log ua) cos(2 pi ub),  z' = sqrt(-2 log ua) sin(2 pi ub).
// log, sin and cos are evaluated by fixed operation sequences written here
// (no fused multiply-add anywhere in this file), so the normals are a
// reproducible function of the Philox bits:
//   log u   = e ln2_hi + (2 s P(s^2) + e ln2_lo), u = m 2^e, m in [sqrt(1/2), sqrt 2),
//             s = (m - 1)/(m + 1), P the atanh series sum_{k<12} z^k / (2k+1)
//   sin(pi r), cos(pi r), |r| <= 1/4: Taylor series in r whose coefficients
//             follow c_k = -c_{k-1} pi^2 / ((2k)(2k+1)), d_k = -d_{k-1} pi^2 /
//             ((2k-1)(2k)) from c_0 = pi, d_0 = 1 (11 terms each)
//   2 pi u  = pi (q/2 + r), q = rint(4u), r = 2u - q/2, quadrant q mod 4.
#pragma clang fp contract(off)

#include "common.hpp"
#include "kernels.hpp"

namespace mlmc {
namespace {

constexpr uint64_t kPhiloxM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t kPhiloxM1 = 0xCA5A826395121157ull;
constexpr uint64_t kPhiloxW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kPhiloxW1 = 0xBB67AE8584CAA73Bull;

struct Block4 { uint64_t w[4]; };

__device__ __forceinline__ Block4 philox4x64_10(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                               uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r) { k0 += kPhiloxW0; k1 += kPhiloxW1; }
    const uint64_t hi0 = __umul64hi(kPhiloxM0, c0), lo0 = kPhiloxM0 * c0;
    const uint64_t hi1 = __umul64hi(kPhiloxM1, c2), lo1 = kPhiloxM1 * c2;
    const uint64_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
  }
  return Block4{{c0, c1, c2, c3}};
}

__device__ __forceinline__ double to_uniform(uint64_t w) {
  return ((double)(w >> 12) + 0.5) * 0x1.0p-52;
}

// ln 2 split as in fdlibm: the high part has 32 trailing zero bits, so
// e * ln2_hi is exact for |e| < 2^20.
constexpr double kLn2Hi = 0x1.62e42fee00000p-1;
constexpr double kLn2Lo = 0x1.a39ef35793c76p-33;

__device__ double fixed_log(double u) {
  const uint64_t bits = (uint64_t)__double_as_longlong(u);
  int e = (int)((bits >> 52) & 0x7FF) - 1023;
  double m = __longlong_as_double((long long)((bits & 0x000FFFFFFFFFFFFFull) | 0x3FF0000000000000ull));
  const double sqrt2 = __dsqrt_rn(2.0);
  if (m > sqrt2) { m = m * 0.5; e += 1; }
  const double s = (m - 1.0) / (m + 1.0);
  const double z = s * s;
  double p = 1.0 / 23.0;
#pragma unroll
  for (int k = 10; k >= 0; --k) p = p * z + 1.0 / (double)(2 * k + 1);
  const double logm = 2.0 * (s * p);
  const double ef = (double)e;
  return ef * kLn2Hi + (logm + ef * kLn2Lo);
}

struct TrigCoeffs { double s[11]; double c[11]; };

__device__ __forceinline__ TrigCoeffs trig_coeffs() {
  TrigCoeffs t;
  const double pi = 3.141592653589793115997963468544185161590576171875;  // double nearest pi
  const double pi2 = pi * pi;
  t.s[0] = pi;
  t.c[0] = 1.0;
#pragma unroll
  for (int k = 1; k < 11; ++k) {
    t.s[k] = -t.s[k - 1] * pi2 / (double)((2 * k) * (2 * k + 1));
    t.c[k] = -t.c[k - 1] * pi2 / (double)((2 * k - 1) * (2 * k));
  }
  return t;
}

__device__ void fixed_sincos_2pi(double u, const TrigCoeffs& tc, double* sv, double* cv) {
  const double t = 2.0 * u;
  const double q = __builtin_rint(4.0 * u);
  const double r = t - 0.5 * q;
  const double r2 = r * r;
  double ps = tc.s[10], pc = tc.c[10];
#pragma unroll
  for (int k = 9; k >= 0; --k) {
    ps = ps * r2 + tc.s[k];
    pc = pc * r2 + tc.c[k];
  }
  const double sr = r * ps, cr = pc;
  switch (((int)q) & 3) {
    case 0: *sv = sr; *cv = cr; break;
    case 1: *sv = cr; *cv = -sr; break;
    case 2: *sv = -sr; *cv = -cr; break;
    default: *sv = -cr; *cv = sr; break;
  }
}

// The four normals of Philox block (sample, level, j, stream): two Box-Muller
// pairs.  Stream 0 draws xi, stream 2 the forcing's xi_f (stream 1 is the
// pause model's).
__device__ __forceinline__ void block_normals(uint64_t seed, uint64_t sample, uint64_t level, int j, double* z,
                                              uint64_t stream = 0) {
  const Block4 b = philox4x64_10(sample, level, (uint64_t)j, stream, seed, 0ull);
  const TrigCoeffs tc = trig_coeffs();
#pragma unroll
  for (int p = 0; p < 2; ++p) {
    const double ua = to_uniform(b.w[2 * p]), ub = to_uniform(b.w[2 * p + 1]);
    const double rad = __dsqrt_rn(-2.0 * fixed_log(ua));
    double sv, cv;
    fixed_sincos_2pi(ub, tc, &sv, &cv);
    z[2 * p] = rad * cv;
    z[2 * p + 1] = rad * sv;
  }
}

// One thread per (sample, Philox block); xi row-major [count][M].
__global__ void __launch_bounds__(kBlock) k_draw_xi(uint64_t seed, uint64_t level, uint64_t first,
                                                    int64_t count, int M, double* __restrict__ xi,
                                                    uint64_t stream) {
  const int nblk = (M + 3) >> 2;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= count * nblk) return;
  const int64_t s = tid / nblk;
  const int j = (int)(tid - s * nblk);
  double z[4];
  block_normals(seed, first + (uint64_t)s, level, j, z, stream);
  double* out = xi + s * M + 4 * j;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (4 * j + q < M) out[q] = z[q];
}

// Serving form: row r draws sample ids[r] of level lv[r] into row slots[r] of xi.
__global__ void __launch_bounds__(kBlock) k_draw_xi_rows(uint64_t seed, int64_t count, int M,
                                                         const uint64_t* __restrict__ ids,
                                                         const int* __restrict__ lv,
                                                         const int* __restrict__ slots,
                                                         double* __restrict__ xi) {
  const int nblk = (M + 3) >> 2;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= count * nblk) return;
  const int64_t r = tid / nblk;
  const int j = (int)(tid - r * nblk);
  double z[4];
  block_normals(seed, ids[r], (uint64_t)lv[r], j, z);
  double* out = xi + (int64_t)slots[r] * M + 4 * j;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (4 * j + q < M) out[q] = z[q];
}

// Pause model: sample i of level lv takes a + w u microseconds, u the uniform
// of word 0 of block (i, lv, 0, 1) (word 3 = 1 keeps these blocks apart from
// the xi blocks).  One thread per sample of the level; out[s] for sample s.
__global__ void __launch_bounds__(kBlock) k_pause_draw(uint64_t seed, uint64_t lv, int64_t count, double a,
                                                       double w, double* __restrict__ out) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= count) return;
  const Block4 b = philox4x64_10((uint64_t)s, lv, 0ull, 1ull, seed, 0ull);
  out[s] = a + w * to_uniform(b.w[0]);
}

}  // namespace

hipError_t launch_pause_draw(uint64_t seed, int level, int64_t count, double a, double w, double* out,
                             hipStream_t st) {
  if (count <= 0) return hipSuccess;
  k_pause_draw<<<dim3((unsigned)((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, st>>>(seed, (uint64_t)level,
                                                                                          count, a, w, out);
  return hipGetLastError();
}

hipError_t launch_draw_xi_rows(uint64_t seed, int64_t count, int M, const uint64_t* ids, const int* lv,
                               const int* slots, double* xi, hipStream_t st) {
  const int64_t total = count * ((M + 3) / 4);
  if (total <= 0) return hipSuccess;
  k_draw_xi_rows<<<dim3((unsigned)((total + kBlock - 1) / kBlock)), dim3(kBlock), 0, st>>>(seed, count, M, ids, lv,
                                                                                           slots, xi);
  return hipGetLastError();
}

hipError_t launch_draw_xi(uint64_t seed, int level, uint64_t first, int64_t count, int M,
                          double* xi, hipStream_t st, int stream) {
  const int64_t total = count * ((M + 3) / 4);
  if (total <= 0) return hipSuccess;
  const int64_t grid = (total + kBlock - 1) / kBlock;
  k_draw_xi<<<dim3((unsigned)grid), dim3(kBlock), 0, st>>>(seed, (uint64_t)level, first, count, M, xi,
                                                           (uint64_t)stream);
  return hipGetLastError();
}

}  // namespace mlmc
