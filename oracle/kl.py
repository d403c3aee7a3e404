"""Karhunen-Loeve expansion of the log-diffusion field (oracle side).

The paper's diffusion coefficient is log-normal, given by a KLE whose Gaussian
field has zero mean and an exponential covariance (Sec. 5.2).  It does not
print the eigenpairs; they are the textbook solution (Ghanem & Spanos,
"Stochastic finite elements", ch. 2) of

    int_0^1 exp(-|x - y| / l_c) phi(y) dy = lambda phi(x)

on [0, 1].  With c = 1/l_c, a = 1/2 and s = x - 1/2:
  even (cos) modes: omega in (2k pi, 2k pi + pi) solves c cos(w a) - w sin(w a) = 0,
                    phi = cos(w s) / sqrt(a + sin(2 w a) / (2 w))
  odd  (sin) modes: omega in (2k pi + pi, 2k pi + 2 pi) solves w cos(w a) + c sin(w a) = 0,
                    phi = sin(w s) / sqrt(a - sin(2 w a) / (2 w))
  lambda = 2 c / (omega^2 + c^2)
Modes are ordered by decreasing lambda (increasing omega, even and odd
alternating).  Roots are found by plain bisection down to adjacent doubles.

3D (reading of "separable exponential covariance"): the covariance is
sigma2 * prod_d exp(-|dx_d| / l_c), so its eigenpairs are products
lambda_(ijk) = sigma2 * lambda_i lambda_j lambda_k (product taken in sorted
index order so that permutations tie exactly) and phi_(ijk) = phi_i phi_j phi_k.
The M modes kept are those with the M largest unscaled products
(lambda_a lambda_b) lambda_c (a <= b <= c the sorted indices), ties broken by
(i, j, k) lexicographic; sigma2 only scales the kept values.
"""
from __future__ import annotations

import math
from typing import List, Tuple

import numpy as np


def _bisect(f, lo: float, hi: float) -> float:
    flo = f(lo)
    for _ in range(2000):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi:
            break
        fm = f(mid)
        if fm == 0.0:
            return mid
        if (fm > 0) == (flo > 0):
            lo, flo = mid, fm
        else:
            hi = mid
    return 0.5 * (lo + hi)


def kl_1d(corr_len: float, n_modes: int):
    """First n_modes 1D eigenpairs: (omega[n], lam[n], parity[n]) parity 0 = cos.

    Pinned by a Nystrom discretisation of the integral operator, by
    orthonormality of the phi, and by the trace identity sum(lambda) = 1.
    """
    c = 1.0 / corr_len
    a = 0.5
    omegas, lams, par = [], [], []
    k = 0
    while len(omegas) < n_modes:
        # even root in (2k pi, 2k pi + pi)
        lo, hi = 2 * k * math.pi, 2 * k * math.pi + math.pi
        w = _bisect(lambda w: c * math.cos(w * a) - w * math.sin(w * a), lo, hi)
        omegas.append(w); par.append(0)
        if len(omegas) < n_modes:
            lo, hi = 2 * k * math.pi + math.pi, 2 * k * math.pi + 2 * math.pi
            w = _bisect(lambda w: w * math.cos(w * a) + c * math.sin(w * a), lo, hi)
            omegas.append(w); par.append(1)
        k += 1
    om = np.array(omegas)
    lam = 2.0 * c / (om * om + c * c)
    return om, lam, np.array(par, dtype=np.int64)


def phi_1d(omega: float, parity: int, x: np.ndarray) -> np.ndarray:
    """Normalised 1D eigenfunction evaluated at x in [0, 1]."""
    a = 0.5
    s = np.asarray(x, dtype=np.float64) - a
    if parity == 0:
        return np.cos(omega * s) / math.sqrt(a + math.sin(2 * omega * a) / (2 * omega))
    return np.sin(omega * s) / math.sqrt(a - math.sin(2 * omega * a) / (2 * omega))


def lambda_product(lam: np.ndarray, i: int, j: int, k: int) -> float:
    a, b, cc = sorted((i, j, k))
    return (lam[a] * lam[b]) * lam[cc]


def lambda3(lam: np.ndarray, sigma2: float, i: int, j: int, k: int) -> float:
    return sigma2 * lambda_product(lam, i, j, k)


def select_modes(corr_len: float, sigma2: float, n_modes: int):
    """The M largest separable 3D modes.

    Returns (triples int64 [M, 3], lam3 float64 [M], omega, lam1d, parity) where
    the 1D arrays cover every index appearing in a triple.
    Pin: the selection is checked against brute-force enumeration and the
    tie structure of permuted triples.
    """
    kmax = 4
    while True:
        om, lam, par = kl_1d(corr_len, kmax + 1)
        cand: List[Tuple[float, int, int, int]] = []
        for i in range(kmax):
            for j in range(kmax):
                for k in range(kmax):
                    cand.append((-lambda_product(lam, i, j, k), i, j, k))
        cand.sort()
        if len(cand) >= n_modes:
            mth = -cand[n_modes - 1][0]
            # any triple using an index >= kmax has product <= lam0^2 lam_kmax
            bound = (lam[0] * lam[0]) * lam[kmax]
            if bound < mth:
                break
        kmax *= 2
    chosen = cand[:n_modes]
    triples = np.array([[t[1], t[2], t[3]] for t in chosen], dtype=np.int64)
    lam3 = np.array([sigma2 * -t[0] for t in chosen])
    need = int(triples.max()) + 1
    return triples, lam3, om[:need], lam[:need], par[:need]


def nystrom_eigs(corr_len: float, npts: int = 2000) -> np.ndarray:
    """Eigenvalues of the midpoint-rule Nystrom matrix (pin for kl_1d)."""
    x = (np.arange(npts) + 0.5) / npts
    cmat = np.exp(-np.abs(x[:, None] - x[None, :]) / corr_len) / npts
    return np.sort(np.linalg.eigvalsh(cmat))[::-1]
