"""FP64 CPU oracle for the randomized PCA of Szlam, Kluger and Tygert,
"An implementation of a randomized algorithm for principal component
analysis" (ACM TOMS, 2014; arXiv:1412.3510).

TEST INFRASTRUCTURE ONLY.  Nothing in the library path may import, call or
link anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP path (``paper_1412_3510_amd``); both sides take their inputs from the
seeded generators in ``synth``, and the random test matrix is reproduced here
from the published Philox4x32-10 definition rather than taken from the GPU.

Each function is written from the paper's description, in its order and
notation, in plain NumPy/SciPy float64.  LAPACK (through numpy/scipy) serves
only as a primitive: matrix products, LU with partial pivoting, Householder
QR, Cholesky, and the SVD of small matrices.

Modules
  philox    -- Philox4x32-10 counter-based generator and the Gaussian map.
  rsvd      -- randomized SVD / PCA with power iterations (Sections 2 and 5).
  nystrom   -- shift-stabilized Nystrom method for PSD matrices (Section 3).
  spectral  -- spectral-norm error: exact and randomized power method
               (Section 4).
  precision -- bfloat16 and E4M3 (column-scaled) copies of A for the
               precision form of the range finder.

Parity status: every function is pinned by CPU tests in ``tests/`` against
brute force, closed forms and invariants; see the header of each module.
"""

from . import philox, precision, rsvd, nystrom, spectral  # noqa: F401
