"""CPU oracle for the MLMC finite-element hot path -- TEST INFRASTRUCTURE ONLY.

A plain, slow, fp64 NumPy/SciPy implementation of what the GPU library
computes, written from the paper (Badia, Hampton, Principe, "A massively
parallel implementation of multilevel Monte Carlo for finite element models")
and from textbook definitions where the paper leaves a step unstated.  It
shares no code, constants generator or table with the HIP library and never
imports it.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it; the product path never does.

Modules
  rng    Philox4x64-10 counter-based draw of the KLE coefficients xi
  kl     1D exponential-covariance KL eigenpairs, separable 3D mode selection
  field  log-normal diffusion coefficient at element centroids
  fe     Q1 mesh index maps, assembled CSR operator, load vector, QoI weights
  gmg    plain definitions of the multigrid pieces (coarse kappa, transfers,
         Chebyshev-Jacobi smoothing) used by step-level parity tests
  pcg    Jacobi-preconditioned conjugate gradients (the oracle's solver)
  mlmc   per-sample level differences Y_l, running statistics, allocation,
         the telescoping MLMC estimator
  pause  pause-model durations and the step schedule of the scheduler stress

Functions without an independent pin say "parity unpinned" in their docstring.
"""
