"""Pins for the Q1 discretisation, Jacobi-PCG and QoI of the oracle."""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle import fe, pcg
from workloads import element_field


def _khat_by_quadrature():
    # int_[0,1]^3 grad N_a . grad N_b with 3x3x3 Gauss (exact for this degree)
    gx, gw = np.polynomial.legendre.leggauss(3)
    t, w = 0.5 * (gx + 1), 0.5 * gw
    off = fe.local_offsets()
    K = np.zeros((8, 8))
    for (x, wx), (y, wy), (z, wz) in itertools.product(zip(t, w), zip(t, w), zip(t, w)):
        p = np.array([x, y, z])
        g = np.zeros((8, 3))
        for a in range(8):
            val = np.where(off[a] == 1, p, 1 - p)
            for d in range(3):
                dv = 1.0 if off[a][d] == 1 else -1.0
                g[a, d] = dv * np.prod(np.delete(val, d))
        K += wx * wy * wz * g @ g.T
    return K


def test_khat_against_quadrature_and_structure():
    K = fe.khat()
    assert np.abs(K - _khat_by_quadrature()).max() < 1e-15
    off = fe.local_offsets()
    for a in range(8):
        for b in range(8):
            ham = int(np.sum(off[a] != off[b]))
            want = {0: 1 / 3, 1: 0.0, 2: -1 / 12, 3: -1 / 12}[ham]
            assert abs(K[a, b] - want) < 1e-16
    assert np.abs(K.sum(axis=1)).max() < 1e-16


def test_constant_kappa_stencil():
    n = 8
    h = 1.0 / n
    A = fe.assemble(n, np.ones(n ** 3))
    g = fe.interior_index(n, 4, 3, 5)
    row = A.getrow(g)
    ijk = fe.interior_ijk(n)
    for c, v in zip(row.indices, row.data):
        d = np.abs(ijk[c] - np.array([4, 3, 5]))
        nz = int((d != 0).sum())
        want = {0: 8 * h / 3, 2: -h / 6, 3: -h / 12}[nz]
        assert abs(v - want) < 1e-16
    assert row.nnz == 1 + 12 + 8          # face neighbours are structurally zero
    assert abs(row.data.sum()) < 1e-15


def _assemble_element_loop(n, kap):
    # brute-force element-by-element COO assembly (independent of fe.assemble)
    K = fe.khat()
    off = fe.local_offsets()
    h = 1.0 / n
    A = np.zeros(((n - 1) ** 3, (n - 1) ** 3))
    for e, (ex, ey, ez) in enumerate(fe.element_ijk(n)):
        nodes = [np.array([ex, ey, ez]) + off[a] for a in range(8)]
        for a in range(8):
            for b in range(8):
                pa, pb = nodes[a], nodes[b]
                if np.all((pa >= 1) & (pa <= n - 1)) and np.all((pb >= 1) & (pb <= n - 1)):
                    A[fe.interior_index(n, *pa), fe.interior_index(n, *pb)] += h * kap[e] * K[a, b]
    return A


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_assembly_matches_element_loop(n):
    kap = element_field(n, 1, seed=10 + n)[0]
    A = fe.assemble(n, kap).toarray()
    B = _assemble_element_loop(n, kap)
    assert np.abs(A - B).max() <= 1e-15 * np.abs(B).max()


@pytest.mark.parametrize("n", [2, 3, 4])
def test_spd_symmetric_gershgorin(n):
    kap = element_field(n, 1, seed=20 + n)[0]
    A = fe.assemble(n, kap)
    assert (A != A.T).nnz == 0                      # bitwise symmetric
    dense = A.toarray()
    np.linalg.cholesky(dense)
    assert np.linalg.eigvalsh(dense).min() > 0
    d = np.sqrt(dense.diagonal())
    ev = np.linalg.eigvalsh(dense / d[:, None] / d[None, :])
    assert ev.min() > 0 and ev.max() <= 2.0 + 1e-12


def test_two_cubed_closed_form():
    # one unknown: u = h^3 / ((h/3) sum kappa) = 0.75 / sum kappa
    kap = element_field(2, 1, seed=5)[0]
    A = fe.assemble(2, kap)
    u = fe.load_constant(2) / A.diagonal()
    assert u[0] == pytest.approx(0.75 / kap.sum(), rel=1e-15)
    q = fe.qoi_weights(2, 0) @ (fe.load_constant(2) / fe.assemble(2, np.ones(8)).diagonal())
    assert q == pytest.approx(0.01171875, rel=1e-15)


@pytest.mark.parametrize("n", [3, 4])
def test_pcg_matches_dense_and_scipy(n):
    kap = element_field(n, 1, seed=30 + n)[0]
    A = fe.assemble(n, kap)
    b = fe.load_constant(n)
    x, it, rel = pcg.jacobi_pcg(A, b, 1e-13, 500)
    xd = np.linalg.solve(A.toarray(), b)
    assert rel <= 1e-13
    assert np.abs(x - xd).max() <= 1e-11 * np.abs(xd).max()
    xs, info = spla.cg(A, b, rtol=1e-13, atol=0.0, maxiter=500)
    assert info == 0 and np.abs(xs - xd).max() <= 1e-11 * np.abs(xd).max()


def test_pcg_true_residual_and_cap():
    n = 8
    kap = element_field(n, 1, seed=3)[0]
    A = fe.assemble(n, kap)
    b = fe.load_constant(n)
    x, it, rel = pcg.jacobi_pcg(A, b, 1e-10, 1000)
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)
    _, it2, rel2 = pcg.jacobi_pcg(A, b, 1e-10, 3)
    assert it2 == 3 and rel2 > 1e-10


def _mms(n):
    s = lambda x: np.sin(np.pi * x)
    f = lambda x, y, z: 3 * np.pi ** 2 * s(x) * s(y) * s(z)
    A = fe.assemble(n, np.ones(n ** 3))
    b = fe.load_function(n, f)
    u = spla.spsolve(A.tocsc(), b)
    return fe.l2_error(n, u, lambda x, y, z: s(x) * s(y) * s(z))


def test_manufactured_solution_l2_second_order():
    errs = [_mms(n) for n in (4, 8, 16)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert rates[0] > 1.85 and rates[1] > 1.95


def _continuum_average(terms=4001):
    # mean of the solution of -lap u = 1 on the unit cube, u = 0 on the boundary,
    # from its sine series: sum over odd i, j, k of
    # 512 / (pi^8 i^2 j^2 k^2 (i^2 + j^2 + k^2)); the k-sum is done in closed form,
    # sum_{k odd} 1/(k^2 (k^2 + a^2)) = (pi^2/8 - pi tanh(pi a / 2) / (4 a)) / a^2
    o = np.arange(1, terms, 2, dtype=np.float64)
    I, J = np.meshgrid(o, o, indexing="ij")
    a = np.sqrt(I ** 2 + J ** 2)
    inner = (np.pi ** 2 / 8 - np.pi * np.tanh(np.pi * a / 2) / (4 * a)) / a ** 2
    return float(np.sum(512.0 / (np.pi ** 8 * I ** 2 * J ** 2) * inner))


def test_domain_average_converges_to_continuum():
    ref = _continuum_average()
    assert ref == pytest.approx(0.02016850032, abs=1e-11)
    errs = []
    for n in (8, 16, 32):
        A = fe.assemble(n, np.ones(n ** 3))
        u, _, _ = pcg.jacobi_pcg(A, fe.load_constant(n), 1e-13, 5000)
        errs.append(abs(fe.qoi_weights(n, 0) @ u - ref))
    assert 3.5 < errs[0] / errs[1] < 4.5 and 3.5 < errs[1] / errs[2] < 4.5


def test_subcube_weights_integrate_trilinear_exactly():
    # for a trilinear function the FE interpolant is exact; the subcube mean of
    # (1+x)(2+y)(3-z) over [1/4,3/4]^3 is 1.5 * 2.5 * 2.5
    n = 12
    ijk = fe.interior_ijk(n)
    x, y, z = (ijk / n).T
    u = (1 + x) * (2 + y) * (3 - z)
    assert fe.qoi_weights(n, 1) @ u == pytest.approx(1.5 * 2.5 * 2.5, rel=1e-14)
    assert fe.qoi_weights(n, 1).sum() == pytest.approx(1.0, rel=1e-14)


def test_index_maps():
    n = 6
    ijk = fe.interior_ijk(n)
    assert ijk.shape == ((n - 1) ** 3, 3)
    assert np.array_equal(fe.interior_index(n, ijk[:, 0], ijk[:, 1], ijk[:, 2]), np.arange((n - 1) ** 3))
    e = fe.element_ijk(n)
    assert np.array_equal(e[:, 0] + n * (e[:, 1] + n * e[:, 2]), np.arange(n ** 3))
