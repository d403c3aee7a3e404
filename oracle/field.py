"""Log-normal diffusion coefficient on a mesh (oracle side).

kappa(x, omega) = exp(g(x, omega)),  g = sum_m sqrt(lambda_m) phi_m(x) xi_m
(KLE of a zero-mean Gaussian field, Sec. 5.2), truncated to the M modes of
``kl.select_modes``.  Reading: one coefficient per Q1 element, evaluated at
the element centroid c_e = ((ex + 1/2) h, (ey + 1/2) h, (ez + 1/2) h),
element index e = ex + n (ey + n ez).
"""
from __future__ import annotations

import numpy as np

from . import kl


def centroid_tables(n: int, corr_len: float, sigma2: float, n_modes: int):
    """1D tables tab[x, q] = phi_q((x + 1/2)/n), the mode triples and lambda."""
    triples, lam3, om, lam1, par = kl.select_modes(corr_len, sigma2, n_modes)
    xc = (np.arange(n) + 0.5) / n
    tab = np.stack([kl.phi_1d(om[q], par[q], xc) for q in range(len(om))], axis=1)
    return tab, triples, lam3


def mode_plane(tab, triples, lam3, ez: int) -> np.ndarray:
    """sqrt(lambda_m) phi_m(c_e) for the n^2 elements of layer ez: [n^2, M]."""
    n = tab.shape[0]
    phi = (tab[:, triples[:, 0]][None, :, :]          # ex on axis 1
           * tab[:, triples[:, 1]][:, None, :]        # ey on axis 0
           * tab[ez, triples[:, 2]][None, None, :])   # ez fixed
    return phi.reshape(n * n, len(lam3)) * np.sqrt(lam3)[None, :]


def log_field(n: int, corr_len: float, sigma2: float, n_modes: int, xi: np.ndarray) -> np.ndarray:
    """g[b, e] for xi[b, M]; evaluated one element layer (fixed ez) at a time."""
    xi = np.asarray(xi, dtype=np.float64)
    tab, triples, lam3 = centroid_tables(n, corr_len, sigma2, n_modes)
    g = np.empty((xi.shape[0], n ** 3))
    for ez in range(n):
        g[:, ez * n * n:(ez + 1) * n * n] = xi @ mode_plane(tab, triples, lam3, ez).T
    return g


def kappa(n: int, corr_len: float, sigma2: float, n_modes: int, xi: np.ndarray) -> np.ndarray:
    """kappa[b, e] = exp(g[b, e])."""
    return np.exp(log_field(n, corr_len, sigma2, n_modes, xi))
