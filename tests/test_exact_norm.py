"""The exact spectral-norm residual the benchmark and the full-size tests gate on
(``bench.exact_residual_norm``, float64 Gram matrices through PyTorch) equals
the oracle's ||A - U diag(S) V^T||_2 from a full SVD of the residual (Section
4's measure), on the host, for tall, wide, centered and symmetric cases."""

import numpy as np
import pytest
import torch

from bench import exact_residual_norm
from oracle import spectral


@pytest.mark.parametrize("m,n,center", [(300, 40, False), (300, 40, True), (35, 260, False),
                                        (35, 260, True), (70, 70, False)])
def test_matches_full_svd(m, n, center):
    rng = np.random.default_rng(m * n)
    A = rng.standard_normal((m, n)).astype(np.float32)
    k = 6
    U = np.linalg.qr(rng.standard_normal((m, k)))[0].astype(np.float32)
    V = np.linalg.qr(rng.standard_normal((n, k)))[0].astype(np.float32)
    S = np.sort(rng.uniform(1, 3, k))[::-1]
    want = spectral.spectral_err_exact(A, U, S, V, center=center)
    got = exact_residual_norm(torch.from_numpy(A), torch.from_numpy(U), S, torch.from_numpy(V),
                              center=center, chunk=64)
    assert got == pytest.approx(want, rel=1e-12)


def test_symmetric_residual_and_small_errors():
    rng = np.random.default_rng(3)
    n, k = 90, 5
    X = np.linalg.qr(rng.standard_normal((n, n)))[0]
    lam = np.exp(-np.arange(n) / 4.0)
    A = ((X * lam) @ X.T).astype(np.float32)
    A = 0.5 * (A + A.T)
    U = X[:, :k].astype(np.float32)
    L = lam[:k]
    want = spectral.spectral_err_exact(A, U, L, None)
    got = exact_residual_norm(torch.from_numpy(A), torch.from_numpy(U), L, None)
    assert got == pytest.approx(want, rel=1e-10)
    # ||E|| ~ lambda_{k+1} = e^-1.25 here, far above the float32 rounding of A
    assert got == pytest.approx(lam[k], rel=1e-5)
