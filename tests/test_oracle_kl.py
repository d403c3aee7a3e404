"""Pins for the KL eigenpairs and 3D mode selection (oracle.kl, oracle.field)."""
import itertools
import math

import numpy as np
import pytest

from oracle import field, kl


@pytest.mark.parametrize("lc", [0.5, 0.3, 0.2, 0.1])
def test_eigenvalues_match_nystrom(lc):
    _, lam, _ = kl.kl_1d(lc, 6)
    ny = kl.nystrom_eigs(lc, 2000)[:6]
    assert np.allclose(lam, ny, rtol=2e-5)


@pytest.mark.parametrize("lc", [0.5, 0.1])
def test_integral_equation_residual(lc):
    # int_0^1 exp(-|x-y|/lc) phi(y) dy = lambda phi(x), Gauss-Legendre split at x
    om, lam, par = kl.kl_1d(lc, 8)
    gx, gw = np.polynomial.legendre.leggauss(60)
    for q in range(8):
        for x in (0.0, 0.137, 0.5, 0.91):
            tot = 0.0
            for a, b in ((0.0, x), (x, 1.0)):
                if b <= a:
                    continue
                y = 0.5 * (b - a) * gx + 0.5 * (a + b)
                tot += 0.5 * (b - a) * np.sum(gw * np.exp(-np.abs(x - y) / lc) * kl.phi_1d(om[q], par[q], y))
            assert abs(tot - lam[q] * kl.phi_1d(om[q], par[q], np.array([x]))[0]) < 1e-12


def test_orthonormal():
    om, lam, par = kl.kl_1d(0.3, 12)
    gx, gw = np.polynomial.legendre.leggauss(200)
    y = 0.5 * (gx + 1.0)
    P = np.stack([kl.phi_1d(om[q], par[q], y) for q in range(12)])
    G = (P * (0.5 * gw)[None, :]) @ P.T
    assert np.abs(G - np.eye(12)).max() < 1e-13


def test_trace_and_order():
    om, lam, par = kl.kl_1d(0.5, 4000)
    assert np.all(np.diff(lam) < 0)
    assert np.all(np.diff(om) > 0)
    assert list(par[:6]) == [0, 1, 0, 1, 0, 1]
    # sum of all eigenvalues = int_0^1 C(x,x) dx = 1; tail ~ 2c/(pi^2 * 4000)
    assert abs(lam.sum() - 1.0) < 1e-3


def test_sign_convention():
    om, lam, par = kl.kl_1d(0.4, 4)
    assert kl.phi_1d(om[0], 0, np.array([0.5]))[0] > 0
    eps = 1e-6
    d = kl.phi_1d(om[1], 1, np.array([0.5 + eps]))[0] - kl.phi_1d(om[1], 1, np.array([0.5 - eps]))[0]
    assert d > 0


@pytest.mark.parametrize("lc,M", [(0.5, 8), (0.3, 64), (0.2, 128)])
def test_mode_selection_brute_force(lc, M):
    triples, lam3, om, lam1, par = kl.select_modes(lc, 1.0, M)
    _, lam, _ = kl.kl_1d(lc, 24)
    cand = sorted((-kl.lambda3(lam, 1.0, i, j, k), i, j, k)
                  for i, j, k in itertools.product(range(24), repeat=3))
    want = np.array([c[1:] for c in cand[:M]])
    assert np.array_equal(triples, want)
    # permuted triples tie bit-exactly
    for t, l in zip(triples, lam3):
        for p in itertools.permutations(t):
            assert kl.lambda3(lam, 1.0, *p) == l


def test_c1_cut_through_three_way_tie():
    # M = 8 at l_c = 0.5: (000), 3x(001), 3x(002), then one of the (011)-type
    triples, lam3, *_ = kl.select_modes(0.5, 1.0, 8)
    assert triples[-1].tolist() == [0, 1, 1]
    assert lam3[-1] == pytest.approx(0.021957, abs=1e-6)


def test_field_constant_when_sigma_zero():
    xi = np.random.default_rng(0).standard_normal((3, 8))
    k = field.kappa(8, 0.5, 0.0, 8, xi)
    assert np.all(k == 1.0)


def test_field_pointwise_definition():
    # g at one element centroid equals the direct sum over modes
    n, lc, s2, M = 8, 0.3, 1.3, 10
    xi = np.random.default_rng(1).standard_normal((2, M))
    g = field.log_field(n, lc, s2, M, xi)
    triples, lam3, om, lam1, par = kl.select_modes(lc, s2, M)
    ex, ey, ez = 3, 6, 1
    c = (np.array([ex, ey, ez]) + 0.5) / n
    val = 0.0
    for m in range(M):
        ph = 1.0
        for d in range(3):
            q = triples[m, d]
            ph *= kl.phi_1d(om[q], par[q], np.array([c[d]]))[0]
        val += math.sqrt(lam3[m]) * ph * xi[1, m]
    assert abs(g[1, ex + n * (ey + n * ez)] - val) < 1e-14


def test_field_variance_matches_truncated_covariance():
    # Var g(x) = sum_m lambda_m phi_m(x)^2 (truncated KLE), checked by sampling
    n, lc, s2, M = 4, 0.5, 1.0, 8
    xi = np.random.default_rng(2).standard_normal((40000, M))
    g = field.log_field(n, lc, s2, M, xi)
    tab, triples, lam3 = field.centroid_tables(n, lc, s2, M)
    e = 1 + n * (2 + n * 3)
    phi = tab[1, triples[:, 0]] * tab[2, triples[:, 1]] * tab[3, triples[:, 2]]
    assert g[:, e].var() == pytest.approx(np.sum(lam3 * phi ** 2), rel=0.03)
