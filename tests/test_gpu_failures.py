"""Failure handling and the flags of the C ABI, on the GPU.

Every condition here is forced from the host and every kernel ends normally:
  * an indefinite "PSD" matrix makes the Nystrom shift (Section 3) grow by 10
    per retry; the device retry count equals the oracle's for the same shift
    rule (u = 2^-16, the unit roundoff of the split-bfloat16 float32
    products), and with the retry cap below that count the call reports
    RPCA_ERR_NOT_PSD -- synchronously with RPCA_SYNC, else at rpca_sync --
    in single calls and per problem in batches (persistent launch and
    streams);
  * a NaN or an infinity in A ends in RPCA_ERR_NUMERICAL (every device loop
    is bounded: the LU tournament's levels and steps, at most 60 Jacobi
    sweeps, at most 30 shift retries);
  * a workspace cap gives RPCA_ERR_NO_MEMORY before anything is launched;
  * RPCA_DETERMINISTIC ignores the autotune table;
  * Nystrom at 64 < l <= 128 and with rank(A) < l against the oracle.
"""

import numpy as np
import pytest
import torch

from oracle import nystrom, philox
from synth import dense

pytestmark = pytest.mark.gpu

NOT_PSD, NUMERICAL, NO_MEMORY = 5, 6, 3
U_SPLIT = 2.0 ** -16  # unit roundoff of the float32 path's products


@pytest.fixture()
def ctx(gpu_lib):
    c = gpu_lib.Context()
    yield c
    c.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _indefinite(n=60):
    lam = np.linspace(1.0, 0.1, n)
    lam[0] = -10.0
    return dense.psd(n, lam, seed=9)


def _oracle_retries(A, l, its, seed):
    om = philox.omega(seed, A.shape[0], l)
    _, _, nu, retries = nystrom.eig_psd(A.astype(np.float64), 4, l, its, om, u_A=U_SPLIT)
    Q = nystrom.range_psd(A.astype(np.float64), l, its, om)
    lmin = np.linalg.eigvalsh(Q.T @ A.astype(np.float64) @ Q)[0]
    # the retry that succeeds clears -lmin by a margin the float32 rounding cannot close
    assert nu / 10.0 < -lmin * 0.9 and nu > -lmin * 1.1
    return retries


def test_indefinite_retries_then_not_psd(ctx, gpu_lib):
    A = _indefinite()
    l, its, seed = 8, 2, 6
    need = _oracle_retries(A, l, its, seed)
    assert need >= 2
    dA = _dev(A)
    U, L = ctx.eig_psd(dA, 4, l, its, seed=seed, sync=True)
    assert ctx.stats()["shift_retries"] == need
    assert torch.isfinite(L).all()
    ctx.set_nystrom_retries(need - 1)
    with pytest.raises(gpu_lib.RpcaError) as e:
        ctx.eig_psd(dA, 4, l, its, seed=seed, sync=True)
    assert e.value.status == NOT_PSD
    # without RPCA_SYNC the failure surfaces at the next synchronizing call, once
    ctx.eig_psd(dA, 4, l, its, seed=seed)
    with pytest.raises(gpu_lib.RpcaError) as e:
        ctx.sync()
    assert e.value.status == NOT_PSD
    ctx.sync()
    ctx.set_nystrom_retries(need)
    ctx.eig_psd(dA, 4, l, its, seed=seed, sync=True)


@pytest.mark.parametrize("mode", [0, 1])  # persistent launch, streams
def test_batched_not_psd_per_problem(ctx, gpu_lib, mode):
    A = _indefinite()
    l, its, seed = 8, 2, 6
    need = _oracle_retries(A, l, its, seed)
    good = dense.psd(80, dense.spectrum_exp(80), seed=3)
    ctx.set_batch_mode(mode)
    ctx.set_nystrom_retries(need - 1)
    probs = [dict(kind="psd", A=_dev(good), k=5, l=10, its=2, seed=1),
             dict(kind="psd", A=_dev(A), k=4, l=l, its=its, seed=seed),
             dict(kind="svd", A=_dev(good[:, :40].copy()), k=5, l=10, its=2, seed=2)]
    outs = ctx.svd_batched(probs)
    assert ctx.batch_status(3) == [0, NOT_PSD, 0]
    with pytest.raises(gpu_lib.RpcaError) as e:
        ctx.sync()
    assert e.value.status == NOT_PSD
    # the healthy problems are intact: the oracle's eigenvalues
    om = philox.omega(1, 80, 10)
    _, L0, _, _ = nystrom.eig_psd(good.astype(np.float64), 5, 10, 2, om, u_A=U_SPLIT)
    np.testing.assert_allclose(outs[0][1].cpu().numpy(), L0, rtol=1e-4)
    # with the default cap every problem succeeds, and RPCA_SYNC reports nothing
    ctx.set_nystrom_retries(10)
    ctx.svd_batched(probs, sync=True)
    assert ctx.batch_status(3) == [0, 0, 0]


@pytest.mark.parametrize("where", ["nan", "inf"])
def test_non_finite_input(ctx, gpu_lib, where):
    rng = np.random.default_rng(4)
    A = rng.standard_normal((300, 120)).astype(np.float32)
    A[17, 33] = np.nan if where == "nan" else np.inf
    dA = _dev(A)
    with pytest.raises(gpu_lib.RpcaError) as e:
        ctx.svd(dA, 5, 10, 2, 1, sync=True)
    assert e.value.status == NUMERICAL
    # asynchronous: reported once, by the next synchronizing call
    ctx.svd(dA, 5, 10, 2, 1)
    with pytest.raises(gpu_lib.RpcaError) as e:
        ctx.sync()
    assert e.value.status == NUMERICAL
    ctx.sync()
    S = (A[:120] + A[:120].T) / 2
    with pytest.raises(gpu_lib.RpcaError) as e:
        ctx.eig_psd(_dev(np.ascontiguousarray(S)), 4, 8, 2, seed=1, sync=True)
    assert e.value.status == NUMERICAL
    # a batch: the non-finite problem alone is flagged
    good = rng.standard_normal((200, 64)).astype(np.float32)
    ctx.svd_batched([dict(A=_dev(good), k=4, l=8, seed=1), dict(A=dA, k=4, l=8, seed=1)])
    assert ctx.batch_status(2) == [0, NUMERICAL]
    with pytest.raises(gpu_lib.RpcaError):
        ctx.sync()


def test_workspace_limit(ctx, gpu_lib):
    rng = np.random.default_rng(5)
    A = _dev(rng.standard_normal((4000, 300)).astype(np.float32))
    U = torch.full((4000, 10), 7.0, device="cuda")
    S = torch.full((10,), 7.0, device="cuda", dtype=torch.float64)
    V = torch.full((300, 10), 7.0, device="cuda")
    ctx.set_workspace_limit(4096)
    with pytest.raises(gpu_lib.RpcaError) as e:
        ctx.svd(A, 10, 12, 2, 1, out=(U, S, V))
    assert e.value.status == NO_MEMORY
    torch.cuda.synchronize()
    assert bool((U == 7.0).all()) and bool((S == 7.0).all()) and bool((V == 7.0).all())
    with pytest.raises(gpu_lib.RpcaError) as e:
        ctx.svd_batched([dict(A=A, k=10, l=12, seed=1)])
    assert e.value.status == NO_MEMORY
    ctx.set_workspace_limit(0)
    ctx.svd(A, 10, 12, 2, 1, out=(U, S, V), sync=True)
    assert torch.isfinite(S).all()


def test_deterministic_ignores_the_tune_table(gpu_lib, tmp_path):
    m, n, k, l = 20000, 1000, 20, 60
    A = dense.dense(m, n, dense.spectrum_tall(n), seed=12)
    dA = _dev(A)
    plain = gpu_lib.Context()
    U0, S0, V0 = plain.svd(dA, k, l, 2, 5, sync=True)
    tuned = gpu_lib.Context()
    # a stored configuration other than the built-in one for this shape class
    # (ceil log2 m = 15, ceil log2 n = 10, lp = 64, float32)
    (tmp_path / "t.txt").write_text("15 10 64 0 4 2 4 2 256\n")
    tuned.tune_load(str(tmp_path / "t.txt"))
    U1, S1, V1 = tuned.svd(dA, k, l, 2, 5, sync=True, deterministic=True)
    assert torch.equal(S0, S1) and torch.equal(U0, U1) and torch.equal(V0, V1)
    U2, S2, V2 = tuned.svd(dA, k, l, 2, 5, sync=True)
    np.testing.assert_allclose(S2.cpu().numpy(), S0.cpu().numpy(), rtol=1e-5)
    plain.close()
    tuned.close()


def test_eig_psd_l120(ctx):
    n, k, l, its, seed = 2000, 100, 120, 2, 31
    lam = np.exp(-np.arange(1, n + 1) / 30.0)
    A = dense.psd(n, lam, seed=21)
    U, L = ctx.eig_psd(_dev(A), k, l, its, seed=seed, sync=True)
    U0, L0, _, r0 = nystrom.eig_psd(A, k, l, its, philox.omega(seed, n, l), u_A=U_SPLIT)
    assert ctx.stats()["shift_retries"] == r0
    np.testing.assert_allclose(L.cpu().numpy(), L0, rtol=1e-4)
    Uh = U.cpu().numpy().astype(np.float64)
    # eigenvectors of the well-separated leading eigenvalues, column by column
    lead = slice(0, 60)
    np.testing.assert_allclose(np.abs(np.sum(Uh[:, lead] * U0[:, lead], axis=0)), 1.0, atol=1e-4)


def test_eig_psd_rank_below_l(ctx):
    # rank 10 < l = 20: Q* A Q is singular and the shift alone makes it definite
    n, r, k, l, its, seed = 300, 10, 8, 20, 2, 14
    lam = np.zeros(n)
    lam[:r] = np.exp(-np.arange(1, r + 1) / 3.0)
    A = dense.psd(n, lam, seed=22)
    U, L = ctx.eig_psd(_dev(A), k, l, its, seed=seed, sync=True)
    U0, L0, nu0, r0 = nystrom.eig_psd(A, k, l, its, philox.omega(seed, n, l), u_A=U_SPLIT)
    assert ctx.stats()["shift_retries"] == r0
    np.testing.assert_allclose(L.cpu().numpy(), L0, rtol=1e-4)
    np.testing.assert_allclose(L0, lam[:k], rtol=1e-6)
