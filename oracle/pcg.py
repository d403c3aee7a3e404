"""Jacobi-preconditioned conjugate gradients (oracle side).

Hestenes-Stiefel PCG with M = diag(A) and x0 = 0.  Stopping rule (reading of
"relative residual"; the paper does not state its solver tolerance): iterate
until the recurrence residual satisfies ||r_k||_2 <= rtol ||b||_2, then
recompute the true residual b - A x; accept if ||b - A x||_2 <= rtol ||b||_2,
otherwise continue from the true residual; give up after max_iter iterations.
"""
from __future__ import annotations

import numpy as np


def jacobi_pcg(A, b: np.ndarray, rtol: float, max_iter: int):
    """Returns (x, iterations, true relative residual)."""
    b = np.asarray(b, dtype=np.float64)
    dinv = 1.0 / A.diagonal()
    x = np.zeros_like(b)
    r = b.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, 0.0
    z = dinv * r
    p = z.copy()
    rz = r @ z
    it = 0
    while it < max_iter:
        q = A @ p
        alpha = rz / (p @ q)
        x = x + alpha * p
        r = r - alpha * q
        it += 1
        if np.linalg.norm(r) <= rtol * bnorm:
            r = b - A @ x
            if np.linalg.norm(r) <= rtol * bnorm:
                break
            z = dinv * r
            p = z.copy()
            rz = r @ z
            continue
        z = dinv * r
        rz_new = r @ z
        p = z + (rz_new / rz) * p
        rz = rz_new
    rel = np.linalg.norm(b - A @ x) / bnorm
    return x, it, rel
