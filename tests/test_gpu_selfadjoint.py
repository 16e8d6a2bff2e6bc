"""Self-adjoint paths beyond the shifted Nystrom method, on the GPU.

  * rpca_eig_sym: Rayleigh-Ritz eigenpairs of a general (indefinite)
    symmetric A after the self-adjoint core loop of Section 5 -- eigenvalues
    (signed, by magnitude) within 1e-4 of the oracle's ``eig_sym`` on the same
    Omega, eigenvectors column by column where the eigenvalues are well
    separated, exact recovery when rank(A) <= l;
  * rpca_eig_psd with RPCA_NYSTROM_SQRT: Section 3's square-root
    stabilization (eigendecomposition of B2, regularized pseudoinverse cut at
    the shift's scale sqrt(n) u ||B1||_F, u = 2^-16 for the float32 path's
    products) against the oracle's ``eig_psd_sqrt`` with the same cut, also
    with rank(A) < l, and in a batch.
"""

import numpy as np
import pytest
import torch

from oracle import nystrom, philox, spectral
from synth import dense

pytestmark = pytest.mark.gpu
U_SPLIT = 2.0 ** -16


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return gpu_lib.Context()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _indefinite(n, seed, scale=10.0):
    # eigenvalues +-exp(-j/scale), alternating signs, distinct magnitudes
    j = np.arange(1, n + 1)
    lam = np.exp(-j / scale) * np.where(j % 2 == 0, -1.0, 1.0)
    return dense.psd(n, lam, seed), lam


@pytest.mark.parametrize("n,k,l,its", [(300, 10, 15, 2), (1000, 40, 50, 2), (2000, 100, 120, 2),
                                       (500, 5, 10, 0)])
def test_eig_sym_parity(ctx, n, k, l, its):
    A, lam = _indefinite(n, seed=n + k, scale=10.0 if l <= 64 else 25.0)
    U, L = ctx.eig_sym(_dev(A), k, l, its, seed=5, sync=True)
    U, L = U.cpu().numpy().astype(np.float64), L.cpu().numpy()
    U0, L0 = nystrom.eig_sym(A, k, l, its, philox.omega(5, n, l))
    np.testing.assert_allclose(L, L0, rtol=1e-4, atol=1e-6 * abs(L0[0]))
    assert np.linalg.norm(U.T @ U - np.eye(k), 2) < 1e-5
    # vectors where |lambda| is separated from its neighbours by 2% or more
    mag = np.abs(L0)
    gap = np.minimum(np.r_[np.inf, mag[:-1] - mag[1:]], np.r_[mag[:-1] - mag[1:], np.inf]) / mag
    sep = gap > 0.02
    if its > 0:
        assert np.all(np.abs(np.sum(U[:, sep] * U0[:, sep], axis=0)) > 1 - 1e-4)
        err = spectral.spectral_err_exact(A, U, L)
        err0 = spectral.spectral_err_exact(A, U0, L0)
        assert err <= err0 * (1 + 1e-3) + 1e-6 * mag[0]


def test_eig_sym_exact_for_rank_le_l(ctx):
    n, k, l = 400, 6, 12
    lam = np.zeros(n)
    lam[:8] = [5.0, -4.0, 3.0, -2.5, 2.0, -1.0, 0.5, -0.25]
    A = dense.psd(n, lam, seed=3)
    U, L = ctx.eig_sym(_dev(A), k, l, 2, seed=9, sync=True)
    np.testing.assert_allclose(L.cpu().numpy(), lam[:k], rtol=1e-5)
    U = U.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(A.astype(np.float64) @ U, U * lam[:k], atol=2e-5)


@pytest.mark.parametrize("n,k,l,its", [(300, 20, 25, 2), (1000, 10, 15, 1), (2000, 100, 120, 2)])
def test_eig_psd_sqrt_parity(ctx, n, k, l, its):
    lam = dense.spectrum_exp(n, scale=10.0 if l <= 64 else 30.0)
    A = dense.psd(n, lam, seed=n + 7)
    U, L = ctx.eig_psd(_dev(A), k, l, its, seed=11, sync=True, stabilize="sqrt")
    U, L = U.cpu().numpy(), L.cpu().numpy()
    U0, L0 = nystrom.eig_psd_sqrt(A, k, l, its, philox.omega(11, n, l), u_A=U_SPLIT)
    np.testing.assert_allclose(L, L0, rtol=1e-4)
    err = spectral.spectral_err_exact(A, U, L)
    assert err <= 1.1 * lam[k]
    assert np.linalg.norm(U.T.astype(np.float64) @ U - np.eye(k), 2) < 1e-5


def test_eig_psd_sqrt_rank_below_l(ctx):
    n, r, k, l = 300, 10, 8, 20
    lam = np.zeros(n)
    lam[:r] = np.exp(-np.arange(1, r + 1) / 3.0)
    A = dense.psd(n, lam, seed=22)
    U, L = ctx.eig_psd(_dev(A), k, l, 2, seed=14, sync=True, stabilize="sqrt")
    np.testing.assert_allclose(L.cpu().numpy(), lam[:k], rtol=1e-4)


def test_batched_sqrt_and_shift(ctx):
    n, k, l = 600, 10, 15
    lam = dense.spectrum_exp(n)
    A = _dev(dense.psd(n, lam, seed=5))
    outs = ctx.svd_batched([dict(kind="psd", A=A, k=k, l=l, seed=3, stabilize="sqrt"),
                            dict(kind="psd", A=A, k=k, l=l, seed=3)], sync=True)
    _, L0 = nystrom.eig_psd_sqrt(A.cpu().numpy(), k, l, 2, philox.omega(3, n, l), u_A=U_SPLIT)
    np.testing.assert_allclose(outs[0][1].cpu().numpy(), L0, rtol=1e-4)
    # the two stabilizations agree to O(nu)
    np.testing.assert_allclose(outs[1][1].cpu().numpy(), L0, rtol=1e-2)
