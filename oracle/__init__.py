"""FP64 CPU oracle for mini-batch sparse kernel k-means -- TEST INFRASTRUCTURE.

This package is the slow, plain, obviously-correct statement of what the
method computes (Ferrarotti, Decherchi, Rocchia, "Distributed Kernel K-Means
for Large Scale Clustering": Sec. 2 Eq. 1-7, Sec. 3.1 Eq. 8-13, Sec. 3.2
Eq. 14-18).  It exists only to check the HIP library against.  Only the tests,
the smoke check of the package entry file and the CPU-baseline leg of the
benchmark may import it; the library and its Python binding never do.

It shares no code with the HIP path.  It consumes the seeded inputs of
``kkm_inputs`` (datasets and the method's random draws), which hold none of
the method's arithmetic.

Modules
-------
kernels    -- linear, Gaussian (RBF) and RMSD-superposition kernel functions
kkm        -- the paper's mini-batch / landmark algorithm (fit, assign, cost)
reference  -- textbook routines the method must reduce to (exact kernel
              k-means, Lloyd, brute force over all partitions)
metrics    -- clustering accuracy (majority vote) and NMI

Every function is pinned by tests/test_oracle_*.py against something other
than itself (closed forms, invariants, special cases, brute force).
"""
from . import kernels, kkm, reference, metrics  # noqa: F401
