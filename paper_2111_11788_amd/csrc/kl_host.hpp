// Host-side Karhunen-Loeve setup (1D eigenpairs, 3D mode selection, tables).
#pragma once

#include <vector>

namespace mlmc {

struct KLModes {
  std::vector<int> triples;      // [M][3] 1D mode index per axis
  std::vector<double> lambda;    // [M] sigma2 * lambda_i lambda_j lambda_k
  std::vector<double> omega;     // 1D frequencies of every index used
  std::vector<double> lambda1d;  // 1D eigenvalues
  std::vector<int> parity;       // 0: cos-type, 1: sin-type
};

void kl1d_pairs(double corr_len, int count, std::vector<double>& omega, std::vector<double>& lambda,
                std::vector<int>& parity);
double kl1d_phi(double omega, int parity, double x);
KLModes kl_select(double corr_len, double sigma2, int M);
// tab[x * K1 + q] = phi_q((x + 1/2) / n)
std::vector<double> kl_centroid_table(const KLModes& md, int n);

}  // namespace mlmc
