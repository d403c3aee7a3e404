"""Pins of the oracle's random forcing (eq. model with a random f, Sec. 2.1):
the stream-2 draw against numpy's Philox, and the load vector of an
elementwise-constant f against the constant load, a Gauss-quadrature load and
a brute-force corner count."""
import numpy as np
import pytest

from oracle import fe, rng


def test_forcing_stream_matches_numpy_philox():
    seed, level, i, j = 5, 2, 3, 1
    v = (i + (level << 64) + (j << 128) + (2 << 192) - 1) % 2**256
    prev = np.array([(v >> (64 * q)) & (2**64 - 1) for q in range(4)], dtype=np.uint64)
    bg = np.random.Philox(counter=prev, key=np.array([seed, 0], dtype=np.uint64))
    want = [int(x) for x in bg.random_raw(4)]
    got = rng.raw_words(seed, level, i, 1, 8, stream=2)[0, 4:8]
    assert [int(x) for x in got] == want
    # a different stream from xi
    assert not np.array_equal(rng.draw_xi(seed, level, i, 1, 8, stream=2), rng.draw_xi(seed, level, i, 1, 8))


@pytest.mark.parametrize("n", [2, 4, 8])
def test_unit_forcing_is_the_constant_load(n):
    assert np.array_equal(fe.load_elements(n, np.ones(n ** 3)), fe.load_constant(n))


@pytest.mark.parametrize("n", [4, 8])
def test_elementwise_load_equals_gauss_quadrature(n):
    # 3x3x3 Gauss is exact for (constant f) x (trilinear hat) on each element
    r = np.random.default_rng(n)
    F = np.exp(r.standard_normal(n ** 3))
    h = 1.0 / n

    def f(x, y, z):
        ex = np.floor(x / h).astype(int)
        ey = np.floor(y / h).astype(int)
        ez = np.floor(z / h).astype(int)
        return F[ex + n * (ey + n * ez)]

    a = fe.load_elements(n, F)
    b = fe.load_function(n, f)
    assert np.allclose(a, b, rtol=1e-13, atol=0)


def test_elementwise_load_brute_force():
    n = 4
    r = np.random.default_rng(1)
    F = r.random(n ** 3)
    h3 = (1.0 / n) ** 3
    b = np.zeros((n - 1) ** 3)
    for ez in range(n):
        for ey in range(n):
            for ex in range(n):
                for dz in (0, 1):
                    for dy in (0, 1):
                        for dx in (0, 1):
                            i, j, k = ex + dx, ey + dy, ez + dz
                            if 1 <= i <= n - 1 and 1 <= j <= n - 1 and 1 <= k <= n - 1:
                                b[(i - 1) + (n - 1) * ((j - 1) + (n - 1) * (k - 1))] += F[ex + n * (ey + n * ez)] * h3 / 8
    assert np.allclose(fe.load_elements(n, F), b, rtol=1e-14, atol=0)
