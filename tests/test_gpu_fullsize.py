"""Parity at the full size of the timed workload, in the same launch path.

The 100000 x 4000 column-centered matrix (sigma_j = 1/j for j <= 50, then
1e-3 exp(-(j - 51)/200)) is built on the device exactly as the benchmark
builds it, and the library is called with the benchmark's k = 50, l = 60,
its = 2 and seed.  The FP64 oracle runs the same algorithm on the host copy
of the same float32 matrix with the same Gaussian test matrix:
  * singular values within 1e-4 relative of the oracle's;
  * the k-dimensional left and right subspaces within 1e-3 in the largest
    principal-angle sine (sigma_k / sigma_{k+1} = 20 here, so both are well
    determined);
  * the spectral error ||A_c - U S V^T||_2, computed exactly in float64 (the
    largest eigenvalue of E^T E, formed from the float32 A on the device with
    PyTorch products), between sigma_{k+1} of the centered matrix (closed
    form; Eckart-Young, less the float32 rounding of A, u ||A||_F < 1e-4
    sigma_{k+1}) and 1.1 sigma_{k+1};
  * the library's FP64 power estimate equal to the oracle's from the same
    start block, and below the exact norm (it is a lower bound).
"""

import numpy as np
import pytest
import torch

from bench import exact_residual_norm
from oracle import philox, rsvd, spectral
from synth import dense

pytestmark = pytest.mark.gpu

M, N, K, L, ITS, SEED, A_SEED = 100000, 4000, 50, 60, 2, 2002, 1002


@pytest.fixture(scope="module")
def workload(gpu_lib):
    A, _, csig = dense.dense_torch(M, N, dense.spectrum_tall(N), seed=A_SEED, device="cuda",
                                   center_spectrum=True)
    ctx = gpu_lib.Context()
    U, S, V = ctx.svd(A, K, L, ITS, SEED, center=True, sync=True)
    Ah = A.cpu().numpy()
    om = philox.omega(SEED, N, L)
    U0, S0, V0 = rsvd.rsvd(Ah, K, L, ITS, om, center=True)
    return dict(ctx=ctx, A=A, Ah=Ah, U=U, S=S, V=V, U0=U0, S0=S0, V0=V0, csig=csig)


def _max_sine(Q1, Q2):
    s = np.linalg.svd(Q1.T @ Q2, compute_uv=False)
    return float(np.sqrt(max(0.0, 1.0 - s.min() ** 2)))


def test_fullsize_singular_values(workload):
    S = workload["S"].cpu().numpy()
    S0 = workload["S0"]
    np.testing.assert_allclose(S, S0, rtol=1e-4)
    # the closed-form spectrum of the centered matrix bounds the Ritz values from above
    assert np.all(S <= workload["csig"][:K] * (1 + 1e-4))


def test_fullsize_subspaces(workload):
    U = workload["U"].cpu().numpy().astype(np.float64)
    V = workload["V"].cpu().numpy().astype(np.float64)
    assert _max_sine(U, workload["U0"]) < 1e-3
    assert _max_sine(V, workload["V0"]) < 1e-3
    assert np.linalg.norm(U.T @ U - np.eye(K), 2) < 1e-4
    assert np.linalg.norm(V.T @ V - np.eye(K), 2) < 1e-4


def test_fullsize_spectral_error(workload):
    w = workload
    iters = 3
    got = w["ctx"].spectral_err(w["A"], w["U"], w["S"], w["V"], iters=iters, seed=7, center=True)
    X0 = philox.omega(7, N, 4, stream=philox.STREAM_SPECTRAL)
    want = spectral.spectral_err_power(w["Ah"], w["U"].cpu().numpy(), w["S"].cpu().numpy(),
                                       w["V"].cpu().numpy(), X0, iters, center=True)
    assert got == pytest.approx(want, rel=1e-6)
    sk1 = w["csig"][K]
    exact = exact_residual_norm(w["A"], w["U"], w["S"], w["V"], center=True)
    print("err / sigma_{k+1} = %.6f (exact)" % (exact / sk1), flush=True)
    assert sk1 * (1 - 1e-4) <= exact <= 1.1 * sk1
    est = w["ctx"].spectral_err(w["A"], w["U"], w["S"], w["V"], iters=30, seed=8, center=True)
    assert 0.5 * exact <= est <= exact * (1 + 1e-6)
