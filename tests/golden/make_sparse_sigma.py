"""Writes sparse_1e6_sigma.json: sigma_{k+1} (k = 20) of the 10^6 x 10^6 sparse
test matrix (10 entries per row, seed 1004), estimated by the FP64 oracle with
l = 60 and its = 8 (the matrix has no closed-form spectrum).  Calls only
``oracle`` and ``synth``.  Run from the repository root:
    python tests/golden/make_sparse_sigma.py
"""

import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import philox, rsvd  # noqa: E402
from synth import sparse  # noqa: E402

M = N = 1000000
K, SEED_A, SEED = 20, 1004, 2004


def main():
    rp, ci, va = sparse.random_rows(M, N, 10, SEED_A)
    A = sparse.to_scipy(M, N, rp, ci, va)
    lr = 60
    _, S, _ = rsvd.rsvd(A, lr, lr, 8, philox.omega(SEED + 1, N, lr))
    out = {"m": M, "n": N, "per_row": 10, "seed_A": SEED_A, "seed": SEED, "k": K,
           "l_ref": lr, "its_ref": 8, "sigma_k_plus_1": float(S[K]),
           "sigma_top": [float(x) for x in S[:K + 1]]}
    with open(os.path.join(HERE, "sparse_1e6_sigma.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
