"""Parity of the HIP path with the FP64 oracle, called through the C ABI.

Tolerances:
  * Philox words: bit-exact; Omega: within one float32 ulp (both sides
    evaluate Box-Muller in float64 with their own libm, then round once).
  * A X, A^T X: every entry within (2^-15 + K 2^-24) (|A| |X|)_ij, the
    bound for bfloat16-split products (three bf16 products, dropped terms
    below 2^-16 relative each) accumulated in float32 over K terms.
  * singular values: 1e-4 relative to the oracle's, error <= 1.1 sigma_{k+1}.
"""

import numpy as np
import pytest
import torch

from oracle import nystrom, philox, rsvd, spectral
from synth import dense

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return gpu_lib.Context()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


# ---------------------------------------------------------------- Philox
# the device kernel writes tiles of 8 to 256 rows and up to 128 columns:
# 1001, 20001 and 300001 rows end on a ragged tile (blocks of four variates
# straddle columns where n % 4 != 0), 131 and 200 columns take two column
# tiles, 300001 rows take 256-row tiles
@pytest.mark.parametrize("n,l,seed,stream", [(500, 12, 2001, 0), (1001, 7, 2**40 + 3, 1),
                                             (33, 5, 0, 0), (301, 131, 77, 2), (9, 200, 3, 1),
                                             (20001, 33, 5, 0), (300001, 4, 11, 0)])
def test_gaussian_matches_oracle(ctx, n, l, seed, stream):
    om, w = ctx.gaussian(seed, n, l, stream=stream, words=True)
    torch.cuda.synchronize()
    nb = (n * l + 3) // 4
    want_w = philox.words(seed, stream, nb).reshape(-1).view(np.int32)
    np.testing.assert_array_equal(w.cpu().numpy(), want_w)
    want = philox.omega(seed, n, l, stream=stream)
    got = om.cpu().numpy()
    ulp = np.spacing(np.abs(want).astype(np.float32))
    assert np.all(np.abs(got - want) <= ulp)


# ---------------------------------------------------------------- products
def _product_bound(A, X, K):
    return (2.0 ** -15 + K * 2.0 ** -24) * (np.abs(A) @ np.abs(X)) + 1e-30


# n % 4 == 0 takes the LDS-DMA kernels, other n the register-staged ones;
# m >= 65536 takes the tall form of A X and, with n >= 1024, the wide form
# of A^T X (512-column tiles; at n = 1028 the last one 4 columns wide)
@pytest.mark.parametrize("m,n,l", [(1000, 500, 12), (777, 333, 60), (300, 1000, 120),
                                   (65, 97, 33), (4099, 257, 64), (4099, 260, 64),
                                   (131, 1028, 120), (70001, 400, 60), (33, 36, 30),
                                   (70001, 1028, 120)])
def test_ax_and_atx(ctx, m, n, l):
    rng = np.random.default_rng(m + n + l)
    A = rng.standard_normal((m, n)).astype(np.float32)
    X = rng.standard_normal((n, l)).astype(np.float32)
    Xt = rng.standard_normal((m, l)).astype(np.float32)
    dA = _dev(A)
    Y = ctx.matmul(dA, _dev(X)).cpu().numpy()
    A64 = A.astype(np.float64)
    ref = A64 @ X.astype(np.float64)
    assert np.all(np.abs(Y - ref) <= _product_bound(A64, X, n))
    Z = ctx.matmul(dA, _dev(Xt), trans=True).cpu().numpy()
    ref = A64.T @ Xt.astype(np.float64)
    assert np.all(np.abs(Z - ref) <= _product_bound(A64.T, Xt, m))


def test_centered_products(ctx):
    m, n, l = 901, 130, 20
    rng = np.random.default_rng(5)
    A = (rng.standard_normal((m, n)) + 3.0).astype(np.float32)
    X = rng.standard_normal((n, l)).astype(np.float32)
    Xt = rng.standard_normal((m, l)).astype(np.float32)
    Ac = A.astype(np.float64) - A.astype(np.float64).mean(axis=0)
    dA = _dev(A)
    Y = ctx.matmul(dA, _dev(X), center=True).cpu().numpy()
    ref = Ac @ X
    bound = _product_bound(A.astype(np.float64), X, n) * 4
    assert np.all(np.abs(Y - ref) <= bound)
    Z = ctx.matmul(dA, _dev(Xt), trans=True, center=True).cpu().numpy()
    ref = Ac.T @ Xt
    Xc = Xt - Xt.mean(axis=0)
    assert np.all(np.abs(Z - ref) <= _product_bound(np.abs(A.T), np.abs(Xc), m) * 4 + 1e-4)


# ---------------------------------------------------------------- renormalization
# 200000 x 120: the triangular solve takes its scalar-row form there
@pytest.mark.parametrize("rows,l", [(1000, 12), (5000, 60), (70000, 60), (3000, 120), (257, 33),
                                    (200000, 120)])
def test_lu_renorm(ctx, rows, l):
    rng = np.random.default_rng(rows + l)
    Y = (rng.standard_normal((rows, l)) @ np.diag(np.logspace(0, -3, l))).astype(np.float32)
    Q, piv = ctx.renorm(_dev(Y), "lu")
    Q = Q.cpu().numpy().astype(np.float64)
    piv = piv.cpu().numpy()
    assert len(set(piv.tolist())) == l and piv.min() >= 0 and piv.max() < rows
    # pivot rows form a unit lower triangular block (in pivot order)
    L11 = Q[piv]
    np.testing.assert_allclose(np.diag(L11), 1.0, atol=1e-5)
    assert np.max(np.abs(np.triu(L11, 1))) < 1e-5
    # same span as Y: Y = Q U for some U
    Uf = np.linalg.lstsq(Q, Y.astype(np.float64), rcond=None)[0]
    res = np.linalg.norm(Q @ Uf - Y) / np.linalg.norm(Y)
    assert res < 1e-5
    # tournament pivoting keeps |L| small
    assert np.max(np.abs(Q)) < 10.0
    assert np.linalg.matrix_rank(Q) == l


# 200000 x 70 (lp = 128): the zero pivots reach the scalar-row solve
@pytest.mark.parametrize("rows,l,rank", [(600, 10, 7), (200000, 70, 60)])
def test_lu_renorm_zero_pivots(ctx, rows, l, rank):
    rng = np.random.default_rng(1)
    Y = np.zeros((rows, l), np.float32)
    Y[:rank] = rng.standard_normal((rank, l))   # only `rank` nonzero rows: l - rank zero pivots
    Q, piv = ctx.renorm(_dev(Y), "lu")
    Q = Q.cpu().numpy().astype(np.float64)
    piv = piv.cpu().numpy()
    assert len(set(piv.tolist())) == l and piv.min() >= 0 and piv.max() < rows
    assert np.linalg.matrix_rank(Q) == l
    Uf = np.linalg.lstsq(Q, Y.astype(np.float64), rcond=None)[0]
    assert np.linalg.norm(Q @ Uf - Y) < 1e-5 * np.linalg.norm(Y)


@pytest.mark.parametrize("rows,l,cond", [(1000, 12, 1e2), (20000, 60, 1e4), (3000, 120, 1e3),
                                         (5000, 40, 1e9), (200000, 120, 1e3)])
def test_orth_renorm(ctx, rows, l, cond):
    rng = np.random.default_rng(int(cond) % 1000 + rows)
    Y = (rng.standard_normal((rows, l)) @ np.diag(np.logspace(0, -np.log10(cond), l))).astype(np.float32)
    Q, R = ctx.renorm(_dev(Y), "qr")
    Q = Q.cpu().numpy().astype(np.float64)
    R = R.cpu().numpy()
    assert np.linalg.norm(Q.T @ Q - np.eye(l), 2) < 5e-6
    # R = Q^T Y: upper triangular up to the rounding of Q
    assert np.max(np.abs(np.tril(R, -1))) < 1e-5 * np.abs(R).max()
    if cond < 1e8:
        res = np.linalg.norm(Q @ R - Y) / np.linalg.norm(Y)
        assert res < 1e-5


def test_orth_renorm_rank_deficient(ctx):
    rows, l = 800, 22
    rng = np.random.default_rng(2)
    Y = np.zeros((rows, l), np.float32)
    Y[:20] = rng.standard_normal((20, l))   # rank 20 < l
    Q, R = ctx.renorm(_dev(Y), "qr")
    Q = Q.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(Q.T @ Q - np.eye(l), 2) < 5e-6
    P = Q @ Q.T
    assert np.linalg.norm(P @ Y - Y) < 1e-5 * np.linalg.norm(Y)


@pytest.mark.parametrize("l", [5, 12, 33, 60, 120])
def test_small_svd(ctx, l):
    rng = np.random.default_rng(l)
    M = rng.standard_normal((l, l)) @ np.diag(np.logspace(0, -6, l)) @ rng.standard_normal((l, l))
    W, s, X = ctx.small_svd(_dev(M))
    W, s, X = W.cpu().numpy(), s.cpu().numpy(), X.cpu().numpy()
    s0 = np.linalg.svd(M, compute_uv=False)
    np.testing.assert_allclose(s, s0, rtol=1e-10, atol=1e-14 * s0[0])
    np.testing.assert_allclose(W @ np.diag(s) @ X.T, M, atol=1e-12 * s0[0])
    np.testing.assert_allclose(X.T @ X, np.eye(l), atol=1e-12)


# ---------------------------------------------------------------- end to end
def _check_svd(ctx, A, k, l, its, seed, center=False, rel=1e-4, err_factor=1.1, sk1=None,
               renorm="chol"):
    m, n = A.shape
    U, S, V = ctx.svd(_dev(A), k, l, its, seed, center=center, renorm=renorm)
    torch.cuda.synchronize()
    U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
    om = philox.omega(seed, n, l)
    U0, S0, V0 = rsvd.rsvd(A, k, l, its, om, center=center,
                           renorm="qr" if renorm == "orth" else "lu")
    np.testing.assert_allclose(S, S0, rtol=rel)
    assert np.linalg.norm(U.T.astype(np.float64) @ U - np.eye(k), 2) < 1e-5
    assert np.linalg.norm(V.T.astype(np.float64) @ V - np.eye(k), 2) < 1e-5
    err = spectral.spectral_err_exact(A, U, S, V, center=center)
    err0 = spectral.spectral_err_exact(A, U0, S0, V0, center=center)
    if sk1 is not None:
        assert err <= err_factor * sk1
    assert err <= err0 * (1 + 1e-3) + 1e-6 * S0[0]
    return U, S, V, U0, S0, V0


def test_svd_small_config(ctx):
    # 1000 x 500, sigma_j = 1/j (j <= 10) then 1e-2 exp(-(j-11)/50); k=10, l=12, its=2
    m, n, k = 1000, 500, 10
    sig = dense.spectrum_small(n)
    A = dense.dense(m, n, sig, seed=1001)
    U, S, V, U0, S0, V0 = _check_svd(ctx, A, k, k + 2, 2, 2001, sk1=sig[k])
    # distinct singular values: vectors agree column by column (same sign rule)
    assert np.max(np.abs(U - U0)) < 1e-3
    assert np.max(np.abs(V - V0)) < 1e-3


@pytest.mark.parametrize("m,n,k,l,its", [(3000, 200, 20, 30, 2), (200, 3000, 20, 30, 1),
                                         (4000, 400, 50, 60, 2), (2000, 300, 90, 120, 3),
                                         (500, 300, 5, 12, 0)])
def test_svd_shapes(ctx, m, n, k, l, its):
    sig = dense.spectrum_tall(min(m, n))
    A = dense.dense(m, n, sig, seed=m + n)
    # its = 0 is the plain sketch, which the paper finds inaccurate (Section 7):
    # only parity with the oracle is asked of it
    _check_svd(ctx, A, k, l, its, 7 + its, sk1=sig[k] if its > 0 else None, err_factor=1.2)


def test_svd_l120_vectors(ctx):
    # l = 120 (lp = 128): the small SVD rotates the columns in LDS and recovers
    # the rotations as W = M^T X diag(s)^-2 (sigma_l / sigma_1 ~ 7e-4 here);
    # the singular vectors must match the oracle's column by column
    m, n, k, l = 3000, 600, 30, 120
    sig = dense.spectrum_tall(n)
    A = dense.dense(m, n, sig, seed=4321)
    U, S, V, U0, S0, V0 = _check_svd(ctx, A, k, l, 2, 99, sk1=sig[k])
    assert np.max(np.abs(U - U0)) < 1e-4
    assert np.max(np.abs(V - V0)) < 1e-4


@pytest.mark.parametrize("m,n,k,l,its", [(3000, 200, 20, 30, 2), (200, 3000, 20, 30, 1),
                                         (4000, 400, 50, 60, 3), (2000, 300, 90, 120, 2)])
def test_svd_lu_renorm(ctx, m, n, k, l, its):
    # pivoted LU (tournament) between applications, the paper's choice; the
    # default renormalization (one Cholesky QR pass) spans the same space
    sig = dense.spectrum_tall(min(m, n))
    A = dense.dense(m, n, sig, seed=m + n + 2)
    _check_svd(ctx, A, k, l, its, 27 + its, sk1=sig[k], err_factor=1.2, renorm="lu")


@pytest.mark.parametrize("m,n,k,l,its", [(3000, 200, 20, 30, 2), (4000, 400, 50, 60, 3),
                                         (2000, 300, 90, 120, 2)])
def test_svd_orth_renorm(ctx, m, n, k, l, its):
    # Cholesky QR after every application; the oracle uses Householder QR there
    sig = dense.spectrum_tall(min(m, n))
    A = dense.dense(m, n, sig, seed=m + n + 1)
    _check_svd(ctx, A, k, l, its, 17 + its, sk1=sig[k], err_factor=1.2, renorm="orth")


def test_svd_centered(ctx):
    m, n, k, l = 6000, 300, 20, 30
    sig = dense.spectrum_tall(n)
    A, (U0, s0, V0) = dense.dense(m, n, sig, seed=42, return_factors=True)
    A = A + np.float32(0.01)
    cs = np.linalg.svd(A.astype(np.float64) - A.astype(np.float64).mean(axis=0), compute_uv=False)
    _check_svd(ctx, A, k, l, 2, 3, center=True, sk1=cs[k])


@pytest.mark.parametrize("size,k", [(30, 20), (30, 21), (100, 50)])
def test_svd_propack_fixtures(ctx, size, k):
    A = dense.propack_diag(size).astype(np.float32)
    l = k + 2
    U, S, V = ctx.svd(_dev(A), k, l, 2, size + k)
    S = S.cpu().numpy()
    want = np.diag(A)[:k].astype(np.float64)
    # the products carry 16 significant bits per operand (bf16 hi + lo), so a
    # diagonal matrix, whose entries of B = Q* A are sums of few terms, shows
    # the per-product error 3 * 2^-18 ~ 1.1e-5 (times a small sum of |q|)
    np.testing.assert_allclose(S, want, atol=3e-5)
    U = U.cpu().numpy().astype(np.float64)
    assert np.linalg.norm(U.T @ U - np.eye(k), 2) < 1e-5


# ---------------------------------------------------------------- Nystrom
@pytest.mark.parametrize("n,k,l,its", [(300, 20, 25, 2), (1000, 10, 15, 1), (700, 40, 45, 2),
                                       (500, 5, 10, 0)])
def test_eig_psd(ctx, n, k, l, its):
    lam = dense.spectrum_exp(n)
    A = dense.psd(n, lam, seed=n + k)
    U, L = ctx.eig_psd(_dev(A), k, l, its, 99)
    U, L = U.cpu().numpy(), L.cpu().numpy()
    U0, L0, nu, _ = nystrom.eig_psd(A, k, l, its, philox.omega(99, n, l), u_A=2.0 ** -16)
    np.testing.assert_allclose(L, L0, rtol=1e-4, atol=1e-6 * L0[0])
    err = spectral.spectral_err_exact(A, U, L)
    err0 = spectral.spectral_err_exact(A, U0, L0)
    assert err <= err0 * 1.001 + 1e-6
    assert np.linalg.norm(U.T.astype(np.float64) @ U - np.eye(k), 2) < 1e-5


def test_eig_psd_rejects_nonsquare(ctx, gpu_lib):
    A = torch.zeros(10, 12, device="cuda")
    with pytest.raises(gpu_lib.RpcaError):
        ctx.eig_psd(A, 2, 4)


def test_invalid_arguments(ctx, gpu_lib):
    A = torch.zeros(10, 12, device="cuda")
    with pytest.raises(gpu_lib.RpcaError) as e:
        ctx.svd(A, 5, 4)
    assert e.value.status == 1
    with pytest.raises(gpu_lib.RpcaError):
        ctx.svd(A, 5, 11)
    with pytest.raises(gpu_lib.RpcaError) as e:
        ctx.svd(torch.zeros(300, 300, device="cuda"), 100, 130)
    assert e.value.status == 2
