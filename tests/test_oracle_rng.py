"""Pins for the oracle's counter-based draw of xi (oracle.rng)."""
import numpy as np
import pytest
from scipy import stats

from oracle import rng


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((5, 7, 11, 13), (123456789, 987)),
    ((2**64 - 2, 3, 2**63, 1), (20211123, 0)),
    ((1, 4, 9, 0), (2**64 - 1, 2**64 - 1)),
])
def test_philox_matches_numpy(ctr, key):
    # numpy's Philox is an independent 4x64-10 implementation that increments
    # its counter before producing a block: its first block is for ctr + 1.
    v = sum(int(w) << (64 * q) for q, w in enumerate(ctr))
    v = (v - 1) % 2**256
    prev = np.array([(v >> (64 * q)) & (2**64 - 1) for q in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=prev, key=np.array(key, dtype=np.uint64))
    want = [int(v) for v in bg.random_raw(4)]
    assert list(rng.philox4x64(ctr, key)) == want


def test_uniform_endpoints_exact():
    w = np.array([0, 2**64 - 1, 2**12, 2**63], dtype=np.uint64)
    u = rng.uniforms(w)
    assert u[0] == 2.0 ** -53
    assert u[1] == 1.0 - 2.0 ** -53
    assert u[2] == 1.5 * 2.0 ** -52
    assert u[3] == 0.5 + 2.0 ** -53
    assert np.all((u > 0) & (u < 1))


def _ulps(a, b):
    return np.abs(np.asarray(a).view(np.int64) - np.asarray(b).view(np.int64))


def test_fixed_log_within_4ulp_of_libm():
    w = np.random.default_rng(3).integers(0, 2**63, size=100000, dtype=np.uint64) * np.uint64(2)
    u = np.concatenate([rng.uniforms(w), [2.0 ** -53, 0.5, 1.0 - 2.0 ** -53, np.sqrt(0.5)]])
    assert _ulps(rng.fixed_log(u), np.log(u)).max() <= 4


def test_fixed_sincos_against_long_double():
    w = np.random.default_rng(4).integers(0, 2**63, size=100000, dtype=np.uint64) * np.uint64(2)
    u = rng.uniforms(w)
    s, c = rng.fixed_sincos_2pi(u)
    ul = u.astype(np.longdouble)
    two_pi = np.longdouble("6.283185307179586476925286766559005768")
    assert np.abs(s - np.sin(two_pi * ul)).max() < 4e-16
    assert np.abs(c - np.cos(two_pi * ul)).max() < 4e-16
    # quadrant points are exact
    s, c = rng.fixed_sincos_2pi(np.array([0.25, 0.5, 0.75]))
    assert list(s) == [1.0, 0.0, -1.0] and list(c) == [0.0, -1.0, 0.0]


def test_normals_distribution():
    z = rng.draw_xi(99, 2, 1000, 2500, 8).ravel()
    assert abs(z.mean()) < 0.03 and abs(z.std() - 1.0) < 0.03
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_xi_counter_layout():
    # xi depends on (seed, level, sample index) only: a sub-range reproduces
    # the same rows, another level or seed gives different rows.
    a = rng.draw_xi(7, 1, 0, 6, 13)
    b = rng.draw_xi(7, 1, 3, 2, 13)
    assert np.array_equal(a[3:5], b)
    assert not np.array_equal(a, rng.draw_xi(7, 2, 0, 6, 13))
    assert not np.array_equal(a, rng.draw_xi(8, 1, 0, 6, 13))
    # first normal of a sample is sqrt(-2 log u0) cos(2 pi u1) of block 0
    w = rng.philox4x64((4, 1, 0, 0), (7, 0))
    u = rng.uniforms(np.array(w, dtype=np.uint64))
    z0 = np.sqrt(-2.0 * np.log(u[0])) * np.cos(2 * np.pi * u[1])
    assert abs(a[4, 0] - z0) < 1e-14 * max(1.0, abs(z0))
