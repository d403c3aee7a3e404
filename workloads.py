"""Seeded synthetic workloads shared by the tests, the bench and the oracle.

This module holds workload *definitions* only: mesh sizes, KLE parameters,
seeds, sample counts, solver tolerances, and seeded generators of plain random
arrays used as inputs in step-level parity tests.  It contains none of the
method's arithmetic (no Philox, no KL eigenpairs, no operator, no solver), so
both the CPU oracle and the HIP path can consume it without sharing code.

The five workloads imitate the shapes of the paper's 3D Poisson experiment
(Sec. 5.2: log-normal KLE diffusion with exponential covariance, meshes that
double per level, sample counts that fall geometrically with the level as in
the sample-scaling law of Sec. 5) on the unit cube with f = 1 and homogeneous
Dirichlet data.  The random-domain geometry of that experiment is replaced by
the cube.
"""
from __future__ import annotations

import dataclasses
from typing import Optional, Tuple

import numpy as np

DEFAULT_SEED = 20211123


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    n0: int                  # elements per side of the coarsest MLMC level
    levels: int              # number of MLMC levels (L + 1); n_l = n0 * 2**l
    sigma2: float            # variance of the Gaussian log-field
    corr_len: float          # correlation length of exp(-|dx|/corr_len)
    n_modes: int             # number of 3D KL modes M (length of xi)
    seed: int = DEFAULT_SEED
    qoi: int = 0             # 0: domain average of u; 1: average over [1/4,3/4]^3
    rtol: float = 1e-8       # true relative residual ||b-Ax||/||b||
    max_iter: int = 2000
    n_per_level: Tuple[int, ...] = ()
    batch: int = 0           # samples per batched solve (0: whole level)
    precision: int = 0       # 0: fp64; 1: fp32 GMG inner solve in fp64 refinement
    solver: int = 0          # 0: GMG-PCG; 1: Jacobi-PCG
    forcing: int = 0         # 0: f = 1; 1: log-normal random f (own KLE coefficients)
    eps: Optional[float] = None  # target RMSE for the allocation formula

    def n(self, level: int) -> int:
        return self.n0 << level

    @staticmethod
    def dofs(n: int) -> int:
        return (n - 1) ** 3


# Plain MLMC in fp64: 4^3, 8^3, 16^3, N = (200, 50, 12), Jacobi-PCG to 1e-10.
C1 = Workload("plain-mlmc-4-8-16", n0=4, levels=3, sigma2=1.0, corr_len=0.5,
              n_modes=8, qoi=0, rtol=1e-10, n_per_level=(200, 50, 12),
              solver=1, precision=0)

# Single-level batched solve at 64^3, 1024 samples, M = 64, corr 0.3, GMG-PCG
# to 1e-8, subcube QoI.  fp64 and mixed precision are both run on it.
C2 = Workload("batched-64cube-1024", n0=64, levels=1, sigma2=1.0, corr_len=0.3,
              n_modes=64, qoi=1, rtol=1e-8, n_per_level=(1024,), batch=1024,
              solver=0, precision=1)

# Full MLMC on 8^3 .. 128^3 (5 levels), M = 128, corr 0.2, pilot of 32 per
# level then the optimal allocation for RMSE 1e-3, mixed precision.
C3 = Workload("mlmc-5level-8-128", n0=8, levels=5, sigma2=1.0, corr_len=0.2,
              n_modes=128, qoi=0, rtol=1e-8, n_per_level=(32, 32, 32, 32, 32),
              solver=0, precision=1, eps=1e-3)

# Serving mix 16^3 .. 256^3, M = 256, level weights proportional to 16^(4-l).
C4 = Workload("serving-16-256", n0=16, levels=5, sigma2=1.0, corr_len=0.2,
              n_modes=256, qoi=0, rtol=1e-8, solver=0, precision=2)

# Largest single-GPU stress: 256^3, sigma2 = 2, corr 0.1, M = 512, batches of 4..16.
C5 = Workload("stress-256cube", n0=256, levels=1, sigma2=2.0, corr_len=0.1,
              n_modes=512, qoi=0, rtol=1e-8, n_per_level=(16,), batch=16,
              solver=0, precision=1)

ALL = (C1, C2, C3, C4, C5)


def grid_vector(n: int, batch: int, seed: int) -> np.ndarray:
    """Seeded random values on the interior nodes of an n^3 mesh.

    Returns float64 [batch, (n-1)^3] in the canonical interior ordering
    g = (i-1) + (n-1)*((j-1) + (n-1)*(k-1)), uniform in [-1, 1).
    """
    rng = np.random.default_rng(seed)
    return rng.uniform(-1.0, 1.0, size=(batch, (n - 1) ** 3))


def element_field(n: int, batch: int, seed: int, spread: float = 2.0) -> np.ndarray:
    """Seeded positive per-element coefficients exp(U(-spread, spread)).

    Returns float64 [batch, n^3], element e = ex + n*(ey + n*ez).
    """
    rng = np.random.default_rng(seed)
    return np.exp(rng.uniform(-spread, spread, size=(batch, n ** 3)))


def normals(batch: int, m: int, seed: int) -> np.ndarray:
    """Seeded N(0,1) coefficients used where a test feeds xi in directly."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(size=(batch, m))
