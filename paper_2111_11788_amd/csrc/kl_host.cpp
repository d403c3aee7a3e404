// Host setup of the Karhunen-Loeve expansion (done once per context).
//
// The log-field has zero mean and covariance sigma2 exp(-|x - y| / l_c) along
// each axis (the exponential-covariance KLE of Sec. 5.2, read as separable in
// 3D).  1D eigenpairs on [0, 1] (Ghanem & Spanos, ch. 2), c = 1/l_c, a = 1/2:
//   cos-type: omega in (2k pi, 2k pi + pi), c cos(omega a) = omega sin(omega a),
//             phi(x) = cos(omega (x - a)) / sqrt(a + sin(2 omega a) / (2 omega))
//   sin-type: omega in (2k pi + pi, 2k pi + 2 pi), omega cos(omega a) = -c sin(omega a),
//             phi(x) = sin(omega (x - a)) / sqrt(a - sin(2 omega a) / (2 omega))
//   lambda = 2 c / (omega^2 + c^2), ordered by increasing omega.
// 3D modes (i, j, k) have eigenvalue sigma2 lambda_i lambda_j lambda_k; the M
// kept are those with the largest products (lambda_a lambda_b) lambda_c over
// the sorted indices a <= b <= c (so permutations tie exactly), ties broken
// by (i, j, k) in lexicographic order.
#include "kl_host.hpp"

#include <algorithm>
#include <cmath>
#include <tuple>

namespace mlmc {
namespace {

template <class F>
double bisect_root(F f, double lo, double hi) {
  double flo = f(lo);
  for (int it = 0; it < 4000; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (!(mid > lo && mid < hi)) break;
    const double fm = f(mid);
    if (fm == 0.0) return mid;
    if ((fm > 0.0) == (flo > 0.0)) {
      lo = mid;
      flo = fm;
    } else {
      hi = mid;
    }
  }
  return 0.5 * (lo + hi);
}

}  // namespace

void kl1d_pairs(double corr_len, int count, std::vector<double>& omega, std::vector<double>& lambda,
                std::vector<int>& parity) {
  const double c = 1.0 / corr_len, a = 0.5, pi = M_PI;
  omega.clear();
  lambda.clear();
  parity.clear();
  for (int k = 0; (int)omega.size() < count; ++k) {
    const double w0 = bisect_root([&](double w) { return c * std::cos(w * a) - w * std::sin(w * a); },
                                  2.0 * k * pi, 2.0 * k * pi + pi);
    omega.push_back(w0);
    parity.push_back(0);
    if ((int)omega.size() < count) {
      const double w1 = bisect_root([&](double w) { return w * std::cos(w * a) + c * std::sin(w * a); },
                                    2.0 * k * pi + pi, 2.0 * k * pi + 2.0 * pi);
      omega.push_back(w1);
      parity.push_back(1);
    }
  }
  for (double w : omega) lambda.push_back(2.0 * c / (w * w + c * c));
}

double kl1d_phi(double omega, int parity, double x) {
  const double a = 0.5, s = x - a;
  if (parity == 0) return std::cos(omega * s) / std::sqrt(a + std::sin(2.0 * omega * a) / (2.0 * omega));
  return std::sin(omega * s) / std::sqrt(a - std::sin(2.0 * omega * a) / (2.0 * omega));
}

static double product3(const std::vector<double>& lam, int i, int j, int k) {
  int v[3] = {i, j, k};
  std::sort(v, v + 3);
  return (lam[v[0]] * lam[v[1]]) * lam[v[2]];
}

KLModes kl_select(double corr_len, double sigma2, int M) {
  KLModes out;
  int kmax = 4;
  std::vector<std::tuple<double, int, int, int>> cand;
  std::vector<double> om, lam;
  std::vector<int> par;
  for (;;) {
    kl1d_pairs(corr_len, kmax + 1, om, lam, par);
    cand.clear();
    for (int i = 0; i < kmax; ++i)
      for (int j = 0; j < kmax; ++j)
        for (int k = 0; k < kmax; ++k) cand.emplace_back(-product3(lam, i, j, k), i, j, k);
    std::sort(cand.begin(), cand.end());
    if ((int)cand.size() >= M) {
      const double mth = -std::get<0>(cand[M - 1]);
      const double bound = (lam[0] * lam[0]) * lam[kmax];
      if (bound < mth) break;
    }
    kmax *= 2;
  }
  int need = 0;
  for (int m = 0; m < M; ++m) {
    const auto& t = cand[m];
    out.triples.push_back(std::get<1>(t));
    out.triples.push_back(std::get<2>(t));
    out.triples.push_back(std::get<3>(t));
    out.lambda.push_back(sigma2 * -std::get<0>(t));
    need = std::max({need, std::get<1>(t) + 1, std::get<2>(t) + 1, std::get<3>(t) + 1});
  }
  out.omega.assign(om.begin(), om.begin() + need);
  out.lambda1d.assign(lam.begin(), lam.begin() + need);
  out.parity.assign(par.begin(), par.begin() + need);
  return out;
}

std::vector<double> kl_centroid_table(const KLModes& md, int n) {
  const int K1 = (int)md.omega.size();
  std::vector<double> tab((size_t)n * K1);
  for (int x = 0; x < n; ++x)
    for (int q = 0; q < K1; ++q)
      tab[(size_t)x * K1 + q] = kl1d_phi(md.omega[q], md.parity[q], (x + 0.5) / n);
  return tab;
}

}  // namespace mlmc
