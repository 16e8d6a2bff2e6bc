"""The fused schedule (RPCA_FUSED_ATA) on the GPU against the oracle's.

Renormalizing only after every second application, the acceleration Section 5
describes: ``its`` steps Z = A_c^T (A_c Z), each renormalized, then
Y = A_c Z orthonormalized and Rayleigh-Ritz.  The oracle runs the same
schedule in float64 (``oracle.rsvd.rsvd(..., fused=True)``); span invariance
lets its pivoted LU stand for the device's Cholesky QR.

The squared spectrum is what the schedule gives up accuracy on: a direction
j enters A^T A Z at sigma_j^2 / sigma_1^2 of the leading one.  The float32
cases keep sigma_l^2 / sigma_1^2 = 1/l far above the split-bfloat16
products' resolution (2^-16), where the device has no reason to differ from
the float64 oracle by more than on the standard schedule; the tolerances are
then the standard schedule's: singular values within 1e-4 relative, the
exact error no more than 0.1% above the oracle's.  Shapes: m not a multiple
of the 32-row panels, n not a multiple of 256-column blocks, n from 300 to
8100.
"""

import numpy as np
import pytest
import torch

from oracle import philox, precision, rsvd, spectral
from synth import dense, sparse

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return gpu_lib.Context()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _compare(A, out, k, l, its, seed, center=False, A_range=None, rel=1e-4):
    U, S, V = (t.cpu().numpy() for t in out)
    n = A.shape[1]
    U0, S0, V0 = rsvd.rsvd(A, k, l, its, philox.omega(seed, n, l), center=center,
                           A_range=A_range, fused=True)
    np.testing.assert_allclose(S, S0, rtol=rel)
    assert np.linalg.norm(U.T.astype(np.float64) @ U - np.eye(k), 2) < 1e-5
    assert np.linalg.norm(V.T.astype(np.float64) @ V - np.eye(k), 2) < 1e-5
    err = spectral.spectral_err_exact(A, U, S, V, center=center)
    err0 = spectral.spectral_err_exact(A, U0, S0, V0, center=center)
    assert err <= err0 * (1 + 1e-3) + 1e-6 * S0[0]
    return err, err0


# sigma_j = j^-1/2: sigma_l^2 / sigma_1^2 = 1/l >= 1/120, far above 2^-16
@pytest.mark.parametrize("m,n,k,l,its", [(3001, 300, 20, 30, 2), (300, 3001, 20, 30, 1),
                                         (5000, 1000, 50, 60, 3), (2003, 4000, 40, 60, 2),
                                         (1500, 8100, 20, 30, 1), (2000, 600, 90, 120, 2),
                                         (777, 333, 5, 12, 4)])
def test_fused_svd(ctx, m, n, k, l, its):
    sig = dense.spectrum_power(min(m, n), 0.5)
    A = dense.dense(m, n, sig, seed=m + 3 * n)
    seed = 51 + its
    out = ctx.svd(_dev(A), k, l, its, seed, fused=True, sync=True)
    _compare(A, out, k, l, its, seed)


def test_fused_svd_centered(ctx):
    m, n, k, l, its, seed = 6001, 700, 20, 30, 2, 8
    sig = dense.spectrum_power(n, 0.5)
    A = dense.dense(m, n, sig, seed=91) + np.float32(0.02)
    out = ctx.svd(_dev(A), k, l, its, seed, center=True, fused=True, sync=True)
    _compare(A, out, k, l, its, seed, center=True)


def test_fused_its0_is_the_plain_sketch(ctx):
    m, n, k, l = 2000, 500, 10, 20
    A = dense.dense(m, n, dense.spectrum_power(n, 0.5), seed=5)
    dA = _dev(A)
    a = ctx.svd(dA, k, l, 0, 3, sync=True)
    b = ctx.svd(dA, k, l, 0, 3, sync=True, fused=True)
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_fused_svd_bf16_copy(ctx, gpu_lib):
    # the precision form: A^T A Z from the bfloat16 copy, each operand rounded
    # to bfloat16 (oracle.precision.LowPrecisionA).  The device's float32
    # intermediates differ from the oracle's float64 ones by float32 rounding,
    # so an operand entry near a bfloat16 rounding boundary can round the
    # other way (one bfloat16 ulp, 2^-8): a perturbation of the sketched
    # span, to which a converged Ritz value responds at second order only.
    # So the k values here are converged: sigma_j = j^-1/2 up to k = 40, then
    # a drop to 1/50 of that, (sigma_{l+1} / sigma_k)^(2 (2 its + 1)) ~ 1e-18.
    m, n, k, l, its, seed = 20000, 1024, 40, 60, 2, 4243
    j = np.arange(1, n + 1, dtype=np.float64)
    sig = np.where(j <= k, j ** -0.5, 0.02 * j ** -0.5)
    A = dense.dense(m, n, sig, seed=78)
    dA = _dev(A)
    q, s = ctx.quantize(dA, "bf16")
    mat = gpu_lib.dense(q, col_scale=s, A_f32=dA)
    out = ctx.svd(q, k, l, its, seed, fused=True, sync=True, mat=mat)
    Al = precision.from_bf16_bits(q.view(torch.int16).cpu().numpy().view(np.uint16))
    _compare(A, out, k, l, its, seed, A_range=precision.LowPrecisionA(Al, None))


def test_fused_svd_sparse(ctx, gpu_lib):
    # a sparse A takes the two-read form of A^T A Z (CSR, then CSC)
    m, n, k, l, its, seed = 4000, 2500, 10, 16, 2, 77
    rp, ci, va = sparse.random_rows(m, n, 12, 21)
    cp, ri, vt = sparse.transpose(m, n, rp, ci, va)
    S = gpu_lib.csr(m, n, _dev(rp), _dev(ci), _dev(va), _dev(cp), _dev(ri), _dev(vt))
    out = ctx.svd(S, k, l, its, seed, fused=True, sync=True)
    A = sparse.to_scipy(m, n, rp, ci, va)
    Sv = out[1].cpu().numpy()
    _, S0, _ = rsvd.rsvd(A, k, l, its, philox.omega(seed, n, l), fused=True)
    np.testing.assert_allclose(Sv, S0, rtol=1e-4)


def test_fused_in_a_batch_equals_single_calls(ctx):
    # fused problems run on the batch's streams with the single-call kernels
    probs, single = [], []
    for i, (m, n) in enumerate([(3000, 400), (1000, 2000), (5000, 300)]):
        A = _dev(dense.dense(m, n, dense.spectrum_power(min(m, n), 0.5), seed=300 + i))
        probs.append(dict(A=A, k=10, l=16, its=2, seed=i, fused=True))
        single.append(ctx.svd(A, 10, 16, 2, i, fused=True, sync=True))
    outs = ctx.svd_batched(probs, sync=True)
    for (U, S, V), (U1, S1, V1) in zip(outs, single):
        assert torch.equal(S, S1) and torch.equal(U, U1) and torch.equal(V, V1)
