"""Precision form on the GPU: bfloat16 / E4M3 copies of A for the range finder.

  * rpca_quantize is bit-exact with the oracle's definition of the copies
    (round to nearest even; E4M3 column scales max |a| / 448).
  * The low-precision passes compute A8 X' (and A8^T Q') where X' is the
    operand rounded to bfloat16 (the high part of the packed split), in
    float32 arithmetic: every entry within (K + 2) 2^-24 (|A8| |X'|) of the
    float64 product of the same rounded operands (K terms accumulated in
    float32 after exact bfloat16 products).
  * Whole solves are compared with the oracle run with the same
    low-precision products (stored values times the operand rounded to
    bfloat16, ``oracle.precision.LowPrecisionA``) in the range finder and the
    float32 A in the Rayleigh-Ritz product: the two differ by float32
    rounding only, and singular values agree within 1e-4 relative for both
    copies, as on the float32 path; the bfloat16 solve meets
    err <= 1.1 sigma_{k+1}, the bound of the float32 path.  E4M3 claims no
    bound (its rounding can exceed sigma_{k+1}); its error must stay within 5%
    of the oracle's for the same E4M3 products.
"""

import numpy as np
import pytest
import torch

from oracle import nystrom, philox, precision, rsvd, spectral
from synth import dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return gpu_lib.Context()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _bf16_round(x):
    return precision.to_bf16(np.asarray(x, dtype=np.float32))


@pytest.mark.parametrize("m,n", [(1000, 512), (333, 77), (4099, 1040)])
def test_quantize_bit_exact(ctx, m, n):
    rng = np.random.default_rng(m + n)
    A = (rng.standard_normal((m, n)) * np.logspace(-4, 3, n)).astype(np.float32)
    A[:, 3] = 0.0
    dA = _dev(A)
    qb, _ = ctx.quantize(dA, "bf16")
    got = qb.view(torch.int16).cpu().numpy().view(np.uint16)
    np.testing.assert_array_equal(got, precision.to_bf16_bits(A))
    q8, s = ctx.quantize(dA, "fp8")
    codes, s0 = precision.to_e4m3(A)
    np.testing.assert_array_equal(s.cpu().numpy(), s0)
    np.testing.assert_array_equal(q8.view(torch.uint8).cpu().numpy(), codes)


def _lowp(ctx, gpu_lib, A, kind):
    dA = _dev(A)
    q, s = ctx.quantize(dA, kind)
    if kind == "bf16":
        Al = precision.from_bf16_bits(q.view(torch.int16).cpu().numpy().view(np.uint16))
        sh = np.ones(A.shape[1])
    else:
        Al = precision.e4m3_decode(q.view(torch.uint8).cpu().numpy())
        sh = s.cpu().numpy().astype(np.float64)
    mat = gpu_lib.dense(q, col_scale=s, A_f32=dA)
    return dA, q, s, mat, Al, sh


def _op(Al, sh, kind):
    return precision.LowPrecisionA(Al, None if kind == "bf16" else sh.astype(np.float32))


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
# 70001 and 66000 rows: the tall form of A X (one tile of 274 or 258 rows per
# workgroup).  40000 x 1040: the wide form of A^T Q (two 512-column tiles and
# a last one 16 columns wide)
@pytest.mark.parametrize("m,n,l", [(1000, 512, 12), (777, 320, 60), (300, 1024, 120),
                                   (4099, 256, 64), (70001, 400, 60), (130, 48, 33),
                                   (66000, 208, 120), (40000, 1040, 60), (40000, 1040, 120)])
def test_lowp_products(ctx, gpu_lib, kind, m, n, l):
    rng = np.random.default_rng(m + n + l)
    A = rng.standard_normal((m, n)).astype(np.float32)
    X = rng.standard_normal((n, l)).astype(np.float32)
    Q = rng.standard_normal((m, l)).astype(np.float32)
    dA, q, s, mat, A8, sh = _lowp(ctx, gpu_lib, A, kind)
    # Y = A X: the kernel sees A8 and bf16(fl(X_j s_j))
    Xs = (X * sh[:, None].astype(np.float32)).astype(np.float32) if kind == "fp8" else X
    Xb = _bf16_round(Xs)
    want = A8 @ Xb
    bound = (n + 2) * 2.0 ** -24 * (np.abs(A8) @ np.abs(Xb)) + 1e-30
    Y = ctx.matmul(q, _dev(X), mat=mat).cpu().numpy()
    assert np.all(np.abs(Y - want) <= bound)
    # Z = A^T Q: s_j (A8^T bf16(Q))_j, scaled in float32 at the end
    Qb = _bf16_round(Q)
    wz = (A8.T @ Qb) * sh[:, None]
    bz = (m + 3) * 2.0 ** -24 * (np.abs(A8.T) @ np.abs(Qb)) * sh[:, None] + 1e-30
    Z = ctx.matmul(q, _dev(Q), trans=True, mat=mat).cpu().numpy()
    assert np.all(np.abs(Z - wz) <= bz)


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_lowp_svd(ctx, gpu_lib, kind):
    m, n, k, l, its, seed = 20000, 1024, 50, 60, 2, 4242
    sig = dense.spectrum_tall(n)
    A, (Uf, _, _) = dense.dense(m, n, sig, seed=77, return_factors=True)
    csig = dense.centered_spectrum(Uf, sig)
    dA, q, s, mat, Al, sh = _lowp(ctx, gpu_lib, A, kind)
    U, S, V = ctx.svd(q, k, l, its, seed, center=True, sync=True, mat=mat)
    Uh, Sh, Vh = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
    err = spectral.spectral_err_exact(A, Uh, Sh, Vh, center=True)
    om = philox.omega(seed, n, l)
    U0, S0, V0 = rsvd.rsvd(A, k, l, its, om, center=True, A_range=_op(Al, sh, kind))
    err0 = spectral.spectral_err_exact(A, U0, S0, V0, center=True)
    np.testing.assert_allclose(Sh, S0, rtol=1e-4)
    if kind == "bf16":
        # the bound the float32 path meets
        assert err <= 1.1 * csig[k]
    else:
        # E4M3 rounding (2^-4) perturbs A by more than sigma_{k+1} here: no bound
        # is claimed, the result must match the oracle run on the same E4M3 products
        assert err <= 1.05 * err0
    # the GPU error estimate reads the float32 copy
    est = ctx.spectral_err(q, U, S, V, iters=30, seed=3, center=True, mat=mat)
    assert 0.5 * err <= est <= err * (1 + 1e-9)


def test_lowp_eig_psd(ctx, gpu_lib):
    n, k, l, its, seed = 1024, 10, 15, 2, 12
    lam = np.exp(-np.arange(1, n + 1) / 10.0)
    A = dense.psd(n, lam, seed=8)
    dA, q, s, mat, Al, sh = _lowp(ctx, gpu_lib, A, "bf16")
    U, L = ctx.eig_psd(q, k, l, its, seed=seed, sync=True, mat=mat)
    Lh = L.cpu().numpy()
    om = philox.omega(seed, n, l)
    # B1 = A Q reads the float32 A: the shift's unit roundoff is that of its
    # split-bfloat16 products
    U0, L0, _, _ = nystrom.eig_psd(A, k, l, its, om, A_range=precision.LowPrecisionA(Al),
                                   u_A=2.0 ** -16)
    err = spectral.spectral_err_exact(A, U.cpu().numpy(), Lh, None)
    err0 = spectral.spectral_err_exact(A, U0, L0, None)
    assert err <= 1.05 * err0
    np.testing.assert_allclose(Lh, L0, rtol=1e-4)


def test_lowp_shape_rules(ctx, gpu_lib):
    A = torch.randn(64, 40, device="cuda").to(torch.bfloat16)  # n % 8 == 0 is fine
    U, S, V = ctx.svd(A, 2, 4, 1, 1, sync=True)
    assert torch.isfinite(S).all()
    B = torch.zeros(64, 44, device="cuda", dtype=torch.bfloat16)  # n % 8 != 0
    with pytest.raises(gpu_lib.RpcaError):
        ctx.svd(B, 2, 4, 1, 1, sync=True)
    C = torch.zeros(64, 48, device="cuda", dtype=torch.float8_e4m3fn)
    with pytest.raises(gpu_lib.RpcaError):       # E4M3 needs column scales
        ctx.svd(C, 2, 4, 1, 1, sync=True)
