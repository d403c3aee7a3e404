"""The library's host-side KLE setup (root finding and mode selection, its own
algorithm: bracketed Newton iteration and a best-first enumeration) against
the oracle's (bisection and exhaustive candidate sort), on the CPU."""
import numpy as np
import pytest

import paper_2111_11788_amd as mm
from oracle import kl


# (the oracle's exhaustive candidate list grows as the cube of the 1D index
# range, which for long correlation lengths and thousands of modes takes
# minutes: 4096 modes only at short ones)
CASES = [(corr, M) for corr in (1.0, 0.5, 0.3, 0.25, 0.2, 0.15, 0.1, 0.05, 0.02)
         for M in (1, 2, 7, 8, 13, 40, 64, 130, 256, 512, 1000)] + [(0.1, 4096), (0.05, 4096), (0.02, 4096)]


@pytest.mark.parametrize("corr,M", CASES)
def test_selection_matches_the_oracle(corr, M):
    tri, lam, om = mm.kl_modes(corr, 1.7, M)
    t2, l2, om2, lam1, par = kl.select_modes(corr, 1.7, M)
    assert np.array_equal(tri, t2)
    assert np.allclose(lam, l2, rtol=1e-14, atol=0)
    assert len(om) == len(om2)
    assert np.allclose(om, om2, rtol=2e-15, atol=0)


def test_roots_solve_their_equations():
    # each frequency solves its transcendental equation to rounding, lies in
    # its bracket, and the brackets alternate cos / sin type
    _, _, om = mm.kl_modes(0.07, 1.0, 4096)
    c = 1.0 / 0.07
    for q, w in enumerate(om):
        k = q // 2
        th = w / 2
        if q % 2 == 0:
            assert k * np.pi < th < k * np.pi + np.pi / 2
            res = c * np.cos(th) - w * np.sin(th)
        else:
            assert k * np.pi + np.pi / 2 < th < (k + 1) * np.pi
            res = w * np.cos(th) + c * np.sin(th)
        # rounding of theta (relative eps) moves the residual by about its
        # derivative, (c + w) theta
        assert abs(res) <= 8 * np.finfo(float).eps * (c + w) * (1 + th), (q, res)


def test_bad_arguments_are_rejected():
    for args in [(0.0, 1.0, 8), (-1.0, 1.0, 8), (float("nan"), 1.0, 8), (0.3, -1.0, 8), (0.3, 1.0, 0),
                 (0.3, 1.0, 4097)]:
        with pytest.raises(mm.MLMCError):
            mm.kl_modes(*args)
