"""Plain definitions of the geometric-multigrid pieces (oracle side).

The paper's solver was algebraic multigrid from a library (Sec. 5.2); the GPU
library uses a matrix-free geometric V-cycle instead.  These pieces do not
change the converged discrete solution (the oracle's answer comes from
Jacobi-PCG alone); they exist so that the GPU multigrid kernels can be
compared element by element with an independent statement of what they
compute.  Every operator here is an explicit sparse matrix.

  coarse kappa   kappa_{2h}[E] = mean of the 8 children of E (rediscretisation)
  prolongation   P: trilinear interpolation from the n/2 grid to the n grid,
                 zero boundary values; restriction is P^T
  Chebyshev      smoothing polynomial in D^-1 A on [lo, hi] (Saad, Iterative
                 Methods, Alg. 12.1), three-term form:
                   theta = (hi+lo)/2, delta = (hi-lo)/2, sigma = theta/delta
                   x1 = x0 + (1/theta) D^-1 (b - A x0)
                   rho_0 = 1/sigma, rho_k = 1/(2 sigma - rho_{k-1})
                   x_{k+1} = x_k + rho_k rho_{k-1} (x_k - x_{k-1})
                                 + (2 rho_k / delta) D^-1 (b - A x_k)
  V-cycle        pre-smooth (degree s, x0 = 0), residual, restrict, recurse,
                 prolong and add, post-smooth (degree s); exact solve at n = 2.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import fe


def coarsen_kappa(n: int, kap: np.ndarray) -> np.ndarray:
    """[..., n^3] -> [..., (n/2)^3]: arithmetic mean of the 8 children."""
    kap = np.asarray(kap, dtype=np.float64)
    lead = kap.shape[:-1]
    k = kap.reshape(lead + (n // 2, 2, n // 2, 2, n // 2, 2))   # ez, cz, ey, cy, ex, cx
    s = k.sum(axis=(-1, -3, -5))
    return (s / 8.0).reshape(lead + ((n // 2) ** 3,))


def prolongation(n: int) -> sp.csr_matrix:
    """P [(n-1)^3 x (n/2-1)^3]: fine node value = trilinear interpolant.

    Coarse node (I, J, K) sits at fine node (2I, 2J, 2K); a fine node gets
    weight prod_d w(i_d - 2 I_d), w(0) = 1, w(+-1) = 1/2 from each coarse node.
    """
    nc = n // 2
    ijk = fe.interior_ijk(n)
    rows, cols, vals = [], [], []
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                d = np.array([dx, dy, dz])
                c2 = ijk + d[None, :]            # candidate 2*coarse coordinate
                even = np.all(c2 % 2 == 0, axis=1)
                C = c2 // 2
                ok = even & np.all((C >= 1) & (C <= nc - 1), axis=1)
                w = np.prod(np.where(d == 0, 1.0, 0.5))
                rows.append(np.nonzero(ok)[0])
                cols.append(fe.interior_index(nc, C[ok, 0], C[ok, 1], C[ok, 2]))
                vals.append(np.full(ok.sum(), w))
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(ijk.shape[0], (nc - 1) ** 3))
    P.sort_indices()
    return P


def chebyshev(A, dinv: np.ndarray, b: np.ndarray, x0: np.ndarray, degree: int,
              lo: float, hi: float) -> np.ndarray:
    """Chebyshev-Jacobi smoothing of A x = b from x0 (three-term form above)."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    sigma = theta / delta
    xprev = x0
    x = x0 + (1.0 / theta) * (dinv * (b - A @ x0))
    rho = 1.0 / sigma
    for _ in range(1, degree):
        rho_new = 1.0 / (2.0 * sigma - rho)
        xn = x + (rho_new * rho) * (x - xprev) + (2.0 * rho_new / delta) * (dinv * (b - A @ x))
        xprev, x, rho = x, xn, rho_new
    return x


def chebyshev_polynomial(lam: np.ndarray, degree: int, lo: float, hi: float) -> np.ndarray:
    """Error-propagation polynomial T_s((theta - lam)/delta) / T_s(theta/delta)."""
    theta = 0.5 * (hi + lo)
    delta = 0.5 * (hi - lo)
    t = np.polynomial.chebyshev.Chebyshev.basis(degree)
    return t((theta - lam) / delta) / t(theta / delta)


class Hierarchy:
    """Rediscretised operators A_l on n, n/2, ..., 2 with their P_l."""

    def __init__(self, n: int, kap: np.ndarray):
        self.ns, self.As, self.Ps, self.kaps = [], [], [], []
        k = np.asarray(kap, dtype=np.float64)
        m = n
        while True:
            self.ns.append(m)
            self.kaps.append(k)
            self.As.append(fe.assemble(m, k))
            if m == 2:
                break
            self.Ps.append(prolongation(m))
            k = coarsen_kappa(m, k)
            m //= 2

    def vcycle(self, b: np.ndarray, degree: int, lo_ratio: float, hi: float, lvl: int = 0):
        A = self.As[lvl]
        if self.ns[lvl] == 2:
            return b / A.diagonal()
        dinv = 1.0 / A.diagonal()
        lo = hi / lo_ratio
        x = chebyshev(A, dinv, b, np.zeros_like(b), degree, lo, hi)
        r = b - A @ x
        P = self.Ps[lvl]
        xc = self.vcycle(P.T @ r, degree, lo_ratio, hi, lvl + 1)
        x = x + P @ xc
        return chebyshev(A, dinv, b, x, degree, lo, hi)
