"""Pins for the oracle's spectral-norm error (Section 4)."""

import numpy as np
import pytest

from oracle import philox, rsvd, spectral
from synth import dense


def _approx(m, n, k, seed, which=1):
    sig = dense.spectrum_paper(which, k, min(m, n), rng=np.random.default_rng(seed))
    A = dense.dense(m, n, sig, seed=seed, dtype=np.float64)
    U, S, V = rsvd.rsvd(A, k, k + 2, 1, philox.omega(seed, n, k + 2))
    return A, U, S, V


def test_exact_norm_is_largest_singular_value_of_residual():
    A, U, S, V = _approx(70, 50, 5, 1)
    E = A - (U * S) @ V.T
    assert spectral.spectral_err_exact(A, U, S, V) == pytest.approx(
        np.linalg.svd(E, compute_uv=False)[0], rel=1e-13)


@pytest.mark.parametrize("which", [1, 3, 5, 6])
def test_power_estimate_lower_bound_and_convergence(which):
    A, U, S, V = _approx(150, 90, 8, which, which)
    exact = spectral.spectral_err_exact(A, U, S, V)
    X0 = philox.omega(99, 90, 4, stream=philox.STREAM_SPECTRAL)
    prev = 0.0
    for iters in (1, 3, 10, 200):
        est = spectral.spectral_err_power(A, U, S, V, X0, iters)
        assert est <= exact * (1 + 1e-12)
        assert est >= exact / 2          # Kuczynski-Wozniakowski, w.h.p.
        assert est >= prev * (1 - 1e-9)  # subspace iteration is monotone here
        prev = est
    assert est == pytest.approx(exact, rel=1e-8)


def test_zero_residual():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((30, 20))
    U, S, Vt = np.linalg.svd(A, full_matrices=False)
    X0 = philox.omega(1, 20, 4, stream=1)
    assert spectral.spectral_err_power(A, U, S, Vt.T, X0, 5) < 1e-12
    assert spectral.spectral_err_exact(A, U, S, Vt.T) < 1e-12


def test_psd_and_centered_residuals():
    rng = np.random.default_rng(3)
    G = rng.standard_normal((40, 40))
    A = G @ G.T
    w, X = np.linalg.eigh(A)
    U, L = X[:, ::-1][:, :5], w[::-1][:5]
    assert spectral.spectral_err_exact(A, U, L) == pytest.approx(w[::-1][5], rel=1e-10)
    B = rng.standard_normal((50, 30)) + 2.0
    Bc = B - B.mean(axis=0)
    U, S, Vt = np.linalg.svd(Bc, full_matrices=False)
    assert spectral.spectral_err_exact(B, U[:, :3], S[:3], Vt[:3].T, center=True) == \
        pytest.approx(S[3], rel=1e-10)
    X0 = philox.omega(4, 30, 4, stream=1)
    est = spectral.spectral_err_power(B, U[:, :3], S[:3], Vt[:3].T, X0, 300, center=True)
    assert est == pytest.approx(S[3], rel=1e-6)


def test_orth_pos_unique_factor():
    rng = np.random.default_rng(4)
    X = rng.standard_normal((25, 4))
    Q = spectral.orth_pos(X)
    R = Q.T @ X
    assert np.all(np.diag(R) > 0)
    np.testing.assert_allclose(np.tril(R, -1), 0, atol=1e-12)
    np.testing.assert_allclose(Q.T @ Q, np.eye(4), atol=1e-13)
    # Cholesky QR gives the same factor
    C = np.linalg.cholesky(X.T @ X)
    np.testing.assert_allclose(Q, X @ np.linalg.inv(C.T), atol=1e-12)
