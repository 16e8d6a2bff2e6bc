"""Pins for the oracle's shift-stabilized Nystrom method (Section 3)."""

import numpy as np
import pytest

from oracle import nystrom, philox, spectral
from synth import dense


def _psd_rank(n, r, seed):
    lam = np.zeros(n)
    lam[:r] = np.exp(-np.arange(1, r + 1) / 3.0)
    return dense.psd(n, lam, seed, dtype=np.float64), lam


@pytest.mark.parametrize("its", [0, 1, 2])
def test_exact_when_rank_at_most_l(its):
    n, r, k, l = 80, 12, 10, 15
    A, lam = _psd_rank(n, r, 1)
    U, L, nu, retries = nystrom.eig_psd(A, k, l, its, philox.omega(2, n, l), u_A=2.0 ** -52)
    np.testing.assert_allclose(L, lam[:k], rtol=1e-9, atol=1e-12)
    assert spectral.spectral_err_exact(A, U, L) < 1e-9 + lam[k]
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-12)


def test_full_width_is_exact_eigendecomposition():
    n, k = 40, 30
    rng = np.random.default_rng(5)
    G = rng.standard_normal((n, n))
    A = G @ G.T / n
    w, X = np.linalg.eigh(A)
    w, X = w[::-1], X[:, ::-1]
    U, L, nu, _ = nystrom.eig_psd(A, k, n, 1, philox.omega(3, n, n), u_A=2.0 ** -52)
    np.testing.assert_allclose(L, w[:k], rtol=1e-9)
    P1, P2 = U @ U.T, X[:, :k] @ X[:, :k].T
    assert np.linalg.norm(P1 - P2, 2) < 1e-8


def test_unshifted_bounds_loewner_and_interlacing():
    # For the exact Nystrom approximation A_hat = (AQ)(Q*AQ)^+(AQ)*,
    # A - A_hat is PSD, hence lambda_hat_j <= lambda_j.
    n, k, l = 120, 10, 14
    lam = dense.spectrum_exp(n)
    A = dense.psd(n, lam, seed=7, dtype=np.float64)
    U, L = nystrom.eig_psd_sqrt(A, l, l, 1, philox.omega(4, n, l))
    Ahat = (U * L) @ U.T
    ev = np.linalg.eigvalsh(A - Ahat)
    assert ev.min() > -1e-10
    assert np.all(L <= lam[:l] + 1e-12)


def test_shifted_and_square_root_forms_agree():
    n, k, l = 200, 15, 20
    lam = dense.spectrum_exp(n)
    A = dense.psd(n, lam, seed=8, dtype=np.float64)
    om = philox.omega(5, n, l)
    U1, L1, nu, _ = nystrom.eig_psd(A, k, l, 2, om)
    U2, L2 = nystrom.eig_psd_sqrt(A, k, l, 2, om)
    assert nu > 0
    np.testing.assert_allclose(L1, L2, atol=20 * nu)
    # error close to the best possible
    err = spectral.spectral_err_exact(A, U1, L1)
    assert lam[k] * (1 - 1e-9) <= err <= 1.2 * lam[k]


def test_shift_retry_and_failure():
    # An indefinite matrix makes Q* (A + nu I) Q indefinite until nu exceeds
    # the negative eigenvalue: the shift is multiplied by 10 per retry.
    n, l = 60, 8
    lam = np.linspace(1.0, 0.1, n)
    lam[0] = -10.0
    A = dense.psd(n, lam, seed=9, dtype=np.float64)
    om = philox.omega(6, n, l)
    Q = nystrom.range_psd(A, l, 2, om)
    assert np.linalg.eigvalsh(Q.T @ A @ Q)[0] < -9.0
    nu0 = nystrom.shift0(A @ Q, n, 2.0 ** -24)
    need = int(np.ceil(np.log10(10.0 / nu0)))
    _, _, nu, retries = nystrom.eig_psd(A, 4, l, 2, om)
    assert 1 <= retries <= need + 1
    assert nu == pytest.approx(nu0 * 10.0 ** retries)
    with pytest.raises(np.linalg.LinAlgError):
        nystrom.eig_psd(A, 4, l, 2, om, max_retries=retries - 1)


def test_float32_input_error_near_optimal():
    n, k, l = 300, 20, 25
    lam = dense.spectrum_exp(n)
    A = dense.psd(n, lam, seed=3)
    U, L, nu, r = nystrom.eig_psd(A, k, l, 2, philox.omega(1, n, l))
    assert r == 0
    err = spectral.spectral_err_exact(A, U, L)
    assert err <= 1.1 * lam[k]


def test_range_matrix_enters_only_through_its_span():
    # the self-adjoint range finder normalizes after each product, so a
    # multiple of A gives the same Q; B1 = A Q always uses A
    n, k, l = 120, 6, 10
    lam = np.exp(-np.arange(1, n + 1) / 5.0)
    A = dense.psd(n, lam, seed=41).astype(np.float64)
    om = philox.omega(9, n, l)
    U0, L0, _, _ = nystrom.eig_psd(A, k, l, 2, om)
    U1, L1, _, _ = nystrom.eig_psd(A, k, l, 2, om, A_range=0.25 * A)
    np.testing.assert_allclose(L1, L0, rtol=1e-10)
    np.testing.assert_allclose(np.abs(U1.T @ U0), np.eye(k), atol=1e-8)


# ---- the self-adjoint (not necessarily definite) Rayleigh-Ritz eigenpairs

def _sym(n, lam, seed):
    return dense.psd(n, lam, seed, dtype=np.float64)  # V diag(lam) V^T for any signs


def test_eig_sym_exact_when_rank_at_most_l():
    # an indefinite matrix of rank 8 <= l: the sketch spans its range exactly
    n, k, l = 90, 6, 12
    lam = np.zeros(n)
    lam[:8] = [5.0, -4.0, 3.0, -2.5, 2.0, -1.0, 0.5, -0.25]
    A = _sym(n, lam, 31)
    U, L = nystrom.eig_sym(A, k, l, 2, philox.omega(3, n, l))
    want = lam[np.argsort(-np.abs(lam), kind="stable")][:k]
    np.testing.assert_allclose(L, want, rtol=1e-10)
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-12)
    np.testing.assert_allclose(A @ U, U * L, atol=1e-10)


def test_eig_sym_full_width_and_interlacing():
    rng = np.random.default_rng(8)
    n = 50
    G = rng.standard_normal((n, n))
    A = 0.5 * (G + G.T)
    w = np.linalg.eigvalsh(A)
    # l = n: every eigenpair exactly
    U, L = nystrom.eig_sym(A, n, n, 1, philox.omega(4, n, n))
    np.testing.assert_allclose(np.sort(L), w, atol=1e-10)
    # l < n: the Ritz values lie inside the spectrum (Cauchy interlacing for
    # Q* A Q): the j-th largest Ritz value is at most the j-th largest
    # eigenvalue, the j-th smallest at least the j-th smallest
    l = 12
    Q = nystrom.range_psd(A, l, 2, philox.omega(5, n, l))
    th = np.linalg.eigvalsh(Q.T @ A @ Q)
    assert np.all(th[::-1] <= w[::-1][:l] + 1e-12)
    assert np.all(th >= w[:l] - 1e-12)
    _, L2 = nystrom.eig_sym(A, 5, l, 2, philox.omega(5, n, l))
    th_by_mag = th[np.argsort(-np.abs(th), kind="stable")][:5]
    np.testing.assert_allclose(L2, th_by_mag, rtol=1e-12)


def test_eig_sym_on_psd_matches_rayleigh_ritz_bound():
    # on a PSD matrix the Rayleigh-Ritz values never exceed the Nystrom ones
    # (Nystrom's A_hat dominates Q Q* A Q Q* in the Loewner order)
    n, k, l = 150, 8, 12
    lam = dense.spectrum_exp(n)
    A = dense.psd(n, lam, seed=12, dtype=np.float64)
    om = philox.omega(6, n, l)
    _, Lrr = nystrom.eig_sym(A, k, l, 1, om)
    _, Lny = nystrom.eig_psd_sqrt(A, k, l, 1, om)
    assert np.all(Lrr <= Lny + 1e-12)
    assert np.all(Lny <= lam[:k] + 1e-12)


def test_sqrt_form_with_rounding_cut():
    # the cut sqrt(n) u ||B1||_F drops the null directions of a rank-10 A
    # (l = 20) and keeps the result exact
    n, r, k, l = 200, 10, 8, 20
    lam = np.zeros(n)
    lam[:r] = np.exp(-np.arange(1, r + 1) / 3.0)
    A = dense.psd(n, lam, seed=13, dtype=np.float64)
    U, L = nystrom.eig_psd_sqrt(A, k, l, 1, philox.omega(7, n, l), u_A=2.0 ** -16)
    np.testing.assert_allclose(L, lam[:k], rtol=1e-9)
