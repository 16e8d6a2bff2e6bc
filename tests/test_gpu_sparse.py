"""Sparse A (CSR for A X, CSC for A^T X) on the GPU, against the FP64 oracle.

  * products: every entry within (K + 1) 2^-24 (|A| |X|) of the float64 product,
    K = the most entries in a row (float32 sums of K float32 products);
  * whole solves: singular values within 1e-4 relative of the oracle's (the
    same algorithm and test matrix in float64 on the same float32 values), and
    the error within 1.1 sigma_{k+1}, sigma_{k+1} taken from the oracle run
    at l = 60, its = 8 (the sparse workload has no closed-form spectrum);
  * the GPU power estimate equals the oracle's from the same start block.
The largest case is the 10^6 x 10^6 matrix with 10 entries per row
(k = 20, l = 30, its = 4), with float32 and with bfloat16 values (the
oracle then runs on the rounded values).
"""

import numpy as np
import pytest
import torch

from oracle import philox, rsvd, spectral
from synth import sparse

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return gpu_lib.Context()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _make(gpu_lib, m, n, per_row, seed, bf16=False):
    rp, ci, va = sparse.random_rows(m, n, per_row, seed)
    cp, ri, vt = sparse.transpose(m, n, rp, ci, va)
    if bf16:
        va = torch.from_numpy(va).to(torch.bfloat16).float().numpy()
        vt = torch.from_numpy(vt).to(torch.bfloat16).float().numpy()
    A = sparse.to_scipy(m, n, rp, ci, va)
    dt = torch.bfloat16 if bf16 else torch.float32
    S = gpu_lib.csr(m, n, _dev(rp), _dev(ci), _dev(va).to(dt), _dev(cp), _dev(ri), _dev(vt).to(dt))
    return A, S


@pytest.mark.parametrize("m,n,l,bf16", [(3000, 2000, 30, False), (1001, 4000, 60, False),
                                        (5000, 777, 120, False), (2000, 2000, 12, True)])
def test_sparse_products(ctx, gpu_lib, m, n, l, bf16):
    A, S = _make(gpu_lib, m, n, 10, seed=m + l, bf16=bf16)
    rng = np.random.default_rng(l)
    X = rng.standard_normal((n, l)).astype(np.float32)
    Q = rng.standard_normal((m, l)).astype(np.float32)
    Ad = A.astype(np.float64)
    Aa = abs(Ad)
    Y = ctx.matmul(S, _dev(X)).cpu().numpy()
    assert np.all(np.abs(Y - Ad @ X) <= 11 * 2.0 ** -24 * (Aa @ np.abs(X)) + 1e-30)
    Kt = int(np.diff(A.tocsc().indptr).max())
    Z = ctx.matmul(S, _dev(Q), trans=True).cpu().numpy()
    assert np.all(np.abs(Z - Ad.T @ Q) <= (Kt + 1) * 2.0 ** -24 * (Aa.T @ np.abs(Q)) + 1e-30)
    # centered A^T Q = A^T (Q - 1 mean(Q))
    Zc = ctx.matmul(S, _dev(Q), trans=True, center=True).cpu().numpy()
    Qc = Q.astype(np.float64) - Q.astype(np.float64).mean(axis=0)
    assert np.allclose(Zc, Ad.T @ Qc, rtol=1e-4, atol=1e-5 * np.abs(Ad.T @ Qc).max())


def _reference_sk1(A, k, seed):
    m, n = A.shape
    lr = min(60, m, n)
    _, Sref, _ = rsvd.rsvd(A, lr, lr, 8, philox.omega(seed + 1, n, lr))
    return Sref[k]


def _check(ctx, A, S, k, l, its, seed, iters=30, sk1=None):
    m, n = A.shape
    U, Sv, V = ctx.svd(S, k, l, its, seed, sync=True)
    Uh, Sh, Vh = U.cpu().numpy(), Sv.cpu().numpy(), V.cpu().numpy()
    U0, S0, V0 = rsvd.rsvd(A, k, l, its, philox.omega(seed, n, l))
    np.testing.assert_allclose(Sh, S0, rtol=1e-4)
    assert np.linalg.norm(Uh.T.astype(np.float64) @ Uh - np.eye(k), 2) < 1e-5
    assert np.linalg.norm(Vh.T.astype(np.float64) @ Vh - np.eye(k), 2) < 1e-5
    # reference sigma_{k+1}: the oracle with more oversampling and iterations
    if sk1 is None:
        sk1 = _reference_sk1(A, k, seed)
    est = ctx.spectral_err(S, U, Sv, V, iters=iters, seed=5)
    X0 = philox.omega(5, n, 4, stream=philox.STREAM_SPECTRAL)
    want = spectral.spectral_err_power(A, Uh, Sh, Vh, X0, iters)
    assert est == pytest.approx(want, rel=1e-6)
    assert est <= 1.1 * sk1
    return est / sk1


@pytest.mark.parametrize("m,n,k,l,its", [(20000, 15000, 20, 30, 4), (8000, 30000, 10, 16, 2)])
def test_sparse_svd(ctx, gpu_lib, m, n, k, l, its):
    A, S = _make(gpu_lib, m, n, 10, seed=m + n)
    _check(ctx, A, S, k, l, its, seed=21)


def test_sparse_svd_full_size(ctx, gpu_lib):
    import json
    import os
    m = n = 1000000
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "sparse_1e6_sigma.json")))
    assert ref["m"] == m and ref["seed_A"] == 1004 and ref["seed"] == 2004
    A, S = _make(gpu_lib, m, n, 10, seed=1004)
    ratio = _check(ctx, A, S, 20, 30, 4, seed=2004, iters=10, sk1=ref["sigma_k_plus_1"])
    print("err / sigma_{k+1} = %.4f" % ratio)


@pytest.mark.parametrize("m,n,k,l,its", [(20000, 15000, 20, 30, 4), (8000, 30000, 10, 16, 2)])
def test_sparse_svd_bf16_values(ctx, gpu_lib, m, n, k, l, its):
    # bfloat16 values (widened exactly to float32 in the gather): the oracle
    # runs on the same rounded values, so the float32 tolerance holds
    A, S = _make(gpu_lib, m, n, 10, seed=m + n, bf16=True)
    _check(ctx, A, S, k, l, its, seed=23)


def test_sparse_svd_full_size_bf16_values(ctx, gpu_lib):
    import json
    import os
    m = n = 1000000
    ref = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                      "sparse_1e6_sigma.json")))
    A, S = _make(gpu_lib, m, n, 10, seed=1004, bf16=True)
    # sigma_{k+1} of the float32-valued matrix; bfloat16 rounding of the values
    # (2^-9 relative each) moves it by far less than the 10% margin
    ratio = _check(ctx, A, S, 20, 30, 4, seed=2004, iters=10, sk1=ref["sigma_k_plus_1"])
    print("bf16 values: err / sigma_{k+1} = %.4f" % ratio)


def test_sparse_rejects_missing_transpose(ctx, gpu_lib):
    m, n = 100, 80
    rp, ci, va = sparse.random_rows(m, n, 5, seed=1)
    S = gpu_lib.csr(m, n, _dev(rp), _dev(ci), _dev(va))
    with pytest.raises(gpu_lib.RpcaError):
        ctx.svd(S, 5, 8, 1, 1, sync=True)
