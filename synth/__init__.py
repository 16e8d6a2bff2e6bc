"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.

This package generates matrices with prescribed spectra and sparse matrices
with prescribed structure.  It holds none of the randomized PCA's own
arithmetic (no sketching, renormalization, projection or SVD of a sketch) and
none of its random test matrices: those are drawn by the method from its own
counter-based generator.

  dense    -- A = U diag(sigma) V^T with Haar-distributed U, V (NumPy on the
              host, or torch on a device for the large workloads), the
              spectra used by the paper's dense experiments (Section 7) and
              by the workloads of this project, and the exact spectrum of the
              column-centered construction.
"""

from . import dense  # noqa: F401
