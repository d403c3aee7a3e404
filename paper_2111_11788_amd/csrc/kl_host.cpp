// Host setup of the Karhunen-Loeve expansion (done once per context).
//
// The log-field has zero mean and covariance sigma2 exp(-|x - y| / l_c) along
// each axis (the exponential-covariance KLE of Sec. 5.2, read as separable in
// 3D), so its eigenpairs are products of the 1D eigenpairs of the kernel
// exp(-|x - y| / l_c) on [0, 1] (Ghanem & Spanos, ch. 2).  With c = 1/l_c and
// theta = omega / 2 (the half-interval frequency), the 1D frequencies are the
// roots of
//   cos-type:  theta sin(theta) = (c/2) cos(theta),  theta in (k pi, k pi + pi/2)
//   sin-type:  theta cos(theta) = -(c/2) sin(theta), theta in (k pi + pi/2, k pi + pi)
// one of each per k, with lambda = 2 c / (omega^2 + c^2) (decreasing in omega)
// and phi = cos(omega (x - 1/2)) or sin(omega (x - 1/2)) over the square root
// of its squared integral over [0, 1], 1/2 + sin(omega) / (2 omega) or
// 1/2 - sin(omega) / (2 omega).  Each root is found by Newton's iteration
// kept inside its bracket (a bisection step whenever Newton would leave it).
//
// 3D modes (i, j, k) have eigenvalue sigma2 lambda_i lambda_j lambda_k; the M
// kept are those with the largest products (lambda_a lambda_b) lambda_c over
// the sorted indices a <= b <= c (so permutations tie exactly), ties broken
// by (i, j, k) in lexicographic order.  They are enumerated best first: a
// max-heap over sorted index triples, whose successors (one index raised,
// order kept) have products no larger, yields the sorted triples in
// non-increasing product; each stands for its distinct permutations.
#include "kl_host.hpp"

#include <algorithm>
#include <cmath>
#include <limits>
#include <queue>
#include <set>
#include <tuple>

namespace mlmc {
namespace {

// root of f in (lo, hi) where f(lo) and f(hi) differ in sign; df = f'
template <class F, class D>
double newton_bracketed(F f, D df, double lo, double hi) {
  const bool rising = f(lo) < 0.0;
  double x = 0.5 * (lo + hi);
  for (int it = 0; it < 200; ++it) {
    const double fx = f(x);
    if (fx == 0.0) return x;
    // keep the bracket: the root lies above x where f(x) has the sign of f(lo)
    if ((fx < 0.0) == rising) lo = x;
    else hi = x;
    const double d = df(x);
    double next = d != 0.0 ? x - fx / d : 0.5 * (lo + hi);
    if (!(next > lo && next < hi)) next = 0.5 * (lo + hi);
    if (std::fabs(next - x) <= 2.0 * std::numeric_limits<double>::epsilon() * std::fabs(x) || next == x)
      return next;
    x = next;
  }
  return x;
}

struct Roots1D {
  double c;
  std::vector<double> omega, lambda;
  std::vector<int> parity;
  // extend to at least `count` eigenpairs in order of increasing omega
  void grow(int count) {
    const double pi = M_PI, h = 0.5 * c;
    while ((int)omega.size() < count) {
      const int idx = (int)omega.size();
      const int k = idx / 2;
      double theta;
      if (idx % 2 == 0) {
        theta = newton_bracketed([&](double t) { return t * std::sin(t) - h * std::cos(t); },
                                 [&](double t) { return std::sin(t) + t * std::cos(t) + h * std::sin(t); },
                                 k * pi, k * pi + 0.5 * pi);
      } else {
        theta = newton_bracketed([&](double t) { return t * std::cos(t) + h * std::sin(t); },
                                 [&](double t) { return std::cos(t) - t * std::sin(t) + h * std::cos(t); },
                                 k * pi + 0.5 * pi, (k + 1) * pi);
      }
      const double w = 2.0 * theta;
      omega.push_back(w);
      parity.push_back(idx % 2);
      lambda.push_back(2.0 * c / (w * w + c * c));
    }
  }
};

}  // namespace

void kl1d_pairs(double corr_len, int count, std::vector<double>& omega, std::vector<double>& lambda,
                std::vector<int>& parity) {
  Roots1D r{1.0 / corr_len, {}, {}, {}};
  r.grow(count);
  omega = r.omega;
  lambda = r.lambda;
  parity = r.parity;
}

double kl1d_phi(double omega, int parity, double x) {
  const double s = x - 0.5, half_sinc = std::sin(omega) / (2.0 * omega);
  if (parity == 0) return std::cos(omega * s) / std::sqrt(0.5 + half_sinc);
  return std::sin(omega * s) / std::sqrt(0.5 - half_sinc);
}

KLModes kl_select(double corr_len, double sigma2, int M) {
  Roots1D r{1.0 / corr_len, {}, {}, {}};
  typedef std::tuple<int, int, int> Tri;   // sorted a <= b <= c
  auto prod = [&](const Tri& t) {
    r.grow(std::get<2>(t) + 1);
    return (r.lambda[std::get<0>(t)] * r.lambda[std::get<1>(t)]) * r.lambda[std::get<2>(t)];
  };
  // heap entries: (product, triple); larger products first, then smaller triples
  typedef std::pair<double, Tri> Ent;
  auto worse = [](const Ent& x, const Ent& y) {
    if (x.first != y.first) return x.first < y.first;
    return x.second > y.second;
  };
  std::priority_queue<Ent, std::vector<Ent>, decltype(worse)> heap(worse);
  std::set<Tri> seen;
  auto push = [&](int a, int b, int c) {
    const Tri t(a, b, c);
    if (seen.insert(t).second) heap.emplace(prod(t), t);
  };
  push(0, 0, 0);
  // (product, i, j, k) of every permutation of the sorted triples taken so
  // far; all those with the M-th largest product are taken, then ordered
  std::vector<std::tuple<double, int, int, int>> got;
  double last = 0.0;
  while (!heap.empty()) {
    const Ent e = heap.top();
    if ((int)got.size() >= M && e.first < last) break;
    heap.pop();
    last = e.first;
    int v[3] = {std::get<0>(e.second), std::get<1>(e.second), std::get<2>(e.second)};
    do {
      got.emplace_back(-e.first, v[0], v[1], v[2]);
    } while (std::next_permutation(v, v + 3));
    if (v[0] < v[1]) push(v[0] + 1, v[1], v[2]);
    if (v[1] < v[2]) push(v[0], v[1] + 1, v[2]);
    push(v[0], v[1], v[2] + 1);
  }
  std::sort(got.begin(), got.end());
  KLModes out;
  int need = 0;
  for (int m = 0; m < M && m < (int)got.size(); ++m) {
    const auto& t = got[m];
    const int i = std::get<1>(t), j = std::get<2>(t), k = std::get<3>(t);
    out.triples.insert(out.triples.end(), {i, j, k});
    out.lambda.push_back(sigma2 * -std::get<0>(t));
    need = std::max({need, i + 1, j + 1, k + 1});
  }
  r.grow(need);
  out.omega.assign(r.omega.begin(), r.omega.begin() + need);
  out.lambda1d.assign(r.lambda.begin(), r.lambda.begin() + need);
  out.parity.assign(r.parity.begin(), r.parity.begin() + need);
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
