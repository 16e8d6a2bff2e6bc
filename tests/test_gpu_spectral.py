"""Parity of the spectral-error estimate (FP64 block power method, Section 4).

Both sides start from the same n x 4 Gaussian block (Philox stream 1) and
run the same number of X <- orth(E^T E X) steps, so the estimates agree up
to the rounding of float64 sums: 1e-7 relative is asked (the residuals here
are well conditioned, so rounding moves the estimate by far less).  Any
estimate is also checked against the exact ||E||_2 from a full SVD: it may
not exceed it (Rayleigh quotient), and after enough steps it meets it.
"""

import numpy as np
import pytest
import torch

from oracle import philox, spectral
from synth import dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return gpu_lib.Context()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _lowrank_case(m, n, k, seed, center=False):
    """A with a known spectrum and a rank-k approximation taken from a perturbed SVD."""
    r = min(m, n)
    sig = 1.0 / np.arange(1, r + 1) ** 1.2
    A = dense.dense(m, n, sig, seed=seed)
    Ad = A.astype(np.float64)
    if center:
        Ad = Ad - Ad.mean(axis=0, keepdims=True)
    U, S, Vt = np.linalg.svd(Ad, full_matrices=False)
    rng = np.random.default_rng(seed + 1)
    U = (U[:, :k] + 1e-3 * rng.standard_normal((m, k))).astype(np.float32)
    V = (Vt[:k].T + 1e-3 * rng.standard_normal((n, k))).astype(np.float32)
    return A, U, S[:k].copy(), V


@pytest.mark.parametrize("m,n,k,iters,center", [(2000, 300, 10, 20, False),
                                                (1500, 200, 7, 20, True),
                                                (333, 1001, 12, 10, False),
                                                (4099, 301, 5, 15, True),
                                                (64, 64, 0, 30, False)])
def test_spectral_matches_oracle(ctx, m, n, k, iters, center):
    A, U, S, V = _lowrank_case(m, n, k, seed=m + n, center=center)
    seed = 77 + k
    got = ctx.spectral_err(_dev(A), _dev(U), _dev(S), _dev(V), iters=iters, seed=seed,
                           center=center)
    X0 = philox.omega(seed, n, 4, stream=philox.STREAM_SPECTRAL)
    want = spectral.spectral_err_power(A, U, S, V, X0, iters, center=center)
    exact = spectral.spectral_err_exact(A, U, S, V, center=center)
    assert got == pytest.approx(want, rel=1e-7)
    assert got <= exact * (1 + 1e-9)
    assert got >= exact / 2


def test_spectral_unaligned_leading_dimension(ctx):
    # a column slice: ld = 403 is not a multiple of 4, so the scalar-load kernels run
    m, n, k = 1000, 400, 6
    A, U, S, V = _lowrank_case(m, n, k, seed=9)
    big = np.zeros((m, n + 3), dtype=np.float32)
    big[:, 1:n + 1] = A
    dA = _dev(big)[:, 1:n + 1]
    got = ctx.spectral_err(dA, _dev(U), _dev(S), _dev(V), iters=12, seed=5)
    X0 = philox.omega(5, n, 4, stream=philox.STREAM_SPECTRAL)
    want = spectral.spectral_err_power(A, U, S, V, X0, 12)
    assert got == pytest.approx(want, rel=1e-7)


def test_spectral_symmetric_residual(ctx):
    n, k = 300, 8
    lam = np.exp(-np.arange(1, n + 1) / 10.0)
    A = dense.psd(n, lam, seed=3)
    w, Q = np.linalg.eigh(A.astype(np.float64))
    U = Q[:, ::-1][:, :k].astype(np.float32)
    S = w[::-1][:k].copy()
    got = ctx.spectral_err(_dev(A), _dev(U), _dev(S), None, iters=25, seed=11)
    X0 = philox.omega(11, n, 4, stream=philox.STREAM_SPECTRAL)
    want = spectral.spectral_err_power(A, U, S, None, X0, 25)
    exact = spectral.spectral_err_exact(A, U, S, None)
    assert got == pytest.approx(want, rel=1e-7)
    assert got == pytest.approx(exact, rel=1e-3)


def test_spectral_converges_to_exact(ctx):
    m, n, k = 800, 120, 4
    A, U, S, V = _lowrank_case(m, n, k, seed=21)
    exact = spectral.spectral_err_exact(A, U, S, V)
    got = ctx.spectral_err(_dev(A), _dev(U), _dev(S), _dev(V), iters=200, seed=1)
    assert got == pytest.approx(exact, rel=1e-8)


def test_spectral_zero_residual(ctx):
    # A = U diag(S) V^T exactly in float64 arithmetic on float32 factors
    rng = np.random.default_rng(4)
    U = rng.standard_normal((200, 3)).astype(np.float32)
    V = rng.standard_normal((90, 3)).astype(np.float32)
    S = np.array([1.0, 0.5, 0.25])
    A = ((U.astype(np.float64) * S) @ V.T.astype(np.float64))
    A32 = A.astype(np.float32)
    got = ctx.spectral_err(_dev(A32), _dev(U), _dev(S), _dev(V), iters=10, seed=2)
    exact = spectral.spectral_err_exact(A32, U, S, V)
    assert got <= exact * (1 + 1e-6) + 1e-12
    assert got < 1e-5


def test_spectral_invalid_arguments(ctx, gpu_lib):
    A = torch.zeros(10, 3, device="cuda")
    U = torch.zeros(10, 1, device="cuda")
    S = torch.zeros(1, device="cuda", dtype=torch.float64)
    V = torch.zeros(3, 1, device="cuda")
    with pytest.raises(gpu_lib.RpcaError):
        ctx.spectral_err(A, U, S, V)            # min(m, n) < 4
    A = torch.zeros(10, 8, device="cuda")
    V = torch.zeros(8, 1, device="cuda")
    with pytest.raises(gpu_lib.RpcaError):
        ctx.spectral_err(A, U, S, None)         # symmetric residual needs a square A
    with pytest.raises(ValueError):
        ctx.spectral_err(A, U, S.float(), V)    # S must be float64
