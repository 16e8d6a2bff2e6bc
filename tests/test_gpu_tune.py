"""The autotuner (rpca_tune) and its table, on the GPU, through the C ABI.

  * rpca_tune times every candidate configuration (for lp = 64: five forms
    of the A X kernel, the tall one among them, five of the A^T X kernel,
    the wide one among them, three tournament block heights) and reports a
    choice the launchers support;
  * every configuration the autotuner can choose, forced through a loaded
    table, gives solves that match the FP64 oracle: singular values within
    1e-4 relative, orthonormal factors, spectral error no worse than the
    oracle's (the configurations change tile shapes and summation order,
    not the method);
  * the table survives save / clear / load; a malformed file is rejected and
    leaves the table as it was; a low-precision copy tunes the tournament
    only; sparse A is unsupported.
"""

import numpy as np
import pytest
import torch

from oracle import philox, rsvd, spectral
from synth import dense, sparse

pytestmark = pytest.mark.gpu

M, N, K, L, ITS, SEED = 20000, 400, 50, 60, 2, 31


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return gpu_lib.Context()


@pytest.fixture(scope="module")
def case():
    sig = dense.spectrum_tall(N)
    A = dense.dense(M, N, sig, seed=777)
    U0, S0, V0 = rsvd.rsvd(A, K, L, ITS, philox.omega(SEED, N, L))
    err0 = spectral.spectral_err_exact(A, U0, S0, V0)
    return A, torch.from_numpy(A).cuda(), S0, err0


def _class(m, n, lp, dtype=0):
    # ceil log2 of m and n, the padded l and the dtype code
    return "%d %d %d %d" % ((m - 1).bit_length(), (n - 1).bit_length(), lp, dtype)


def _check_solve(ctx, case):
    A, dA, S0, err0 = case
    U, S, V = ctx.svd(dA, K, L, ITS, SEED, sync=True)
    U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
    np.testing.assert_allclose(S, S0, rtol=1e-4)
    assert np.linalg.norm(U.T.astype(np.float64) @ U - np.eye(K), 2) < 1e-5
    assert np.linalg.norm(V.T.astype(np.float64) @ V - np.eye(K), 2) < 1e-5
    err = spectral.spectral_err_exact(A, U, S, V)
    assert err <= err0 * (1 + 1e-3) + 1e-6 * S0[0]


def test_tune_reports_a_choice(ctx, case):
    _, dA, _, _ = case
    ctx.tune_clear()
    r = ctx.tune(dA, L, reps=2)
    assert r["candidates"] == 5 + 5 + 3
    assert (r["ax_waves"], r["ax_ring"]) in ((16, 0), (8, 4), (4, 2), (4, 3), (4, 4))
    assert (r["atx_waves"], r["atx_ring"]) in ((16, 0), (8, 4), (4, 2), (4, 3), (4, 4))
    assert r["lu_rows"] in (256, 512, 1024)
    assert r["ms_ax"] > 0 and r["ms_atx"] > 0 and r["ms_lu"] > 0
    assert ctx.tune_count() == 1
    _check_solve(ctx, case)


@pytest.mark.parametrize("cfg", [(8, 4, 8, 4, 512), (4, 2, 4, 3, 256), (4, 4, 4, 2, 1024),
                                 (4, 3, 8, 4, 256), (8, 4, 4, 4, 1024), (16, 0, 8, 4, 512),
                                 (16, 0, 4, 2, 256), (16, 0, 16, 0, 512), (4, 3, 16, 0, 256)])
def test_forced_configuration_matches_oracle(ctx, case, tmp_path, cfg):
    path = tmp_path / "tune.txt"
    path.write_text("# forced\n%s %d %d %d %d %d\n" % ((_class(M, N, 64),) + cfg))
    ctx.tune_clear()
    ctx.tune_load(str(path))
    assert ctx.tune_count() == 1
    try:
        _check_solve(ctx, case)
    finally:
        ctx.tune_clear()


@pytest.mark.parametrize("cfg", ["8 3 8 3", "16 0 8 3", "16 0 16 0"])
def test_forced_8wave_lp128_matches_oracle(ctx, tmp_path, cfg):
    # l = 120 (lp = 128): the 8-wave forms of both passes (3-stage rings), the
    # tall A X with the 8-wave A^T X, or the tall and the wide forms, forced
    # for this shape class, against the oracle
    m, n, k, l = 20000, 1024, 100, 120
    sig = dense.spectrum_tall(n)
    A = dense.dense(m, n, sig, seed=778)
    U0, S0, V0 = rsvd.rsvd(A, k, l, ITS, philox.omega(SEED, n, l))
    err0 = spectral.spectral_err_exact(A, U0, S0, V0)
    path = tmp_path / "tune128.txt"
    path.write_text("# forced\n%s %s 512\n" % (_class(m, n, 128), cfg))
    ctx.tune_clear()
    ctx.tune_load(str(path))
    try:
        U, S, V = ctx.svd(torch.from_numpy(A).cuda(), k, l, ITS, SEED, sync=True)
    finally:
        ctx.tune_clear()
    U, S, V = U.cpu().numpy(), S.cpu().numpy(), V.cpu().numpy()
    np.testing.assert_allclose(S, S0, rtol=1e-4)
    assert np.linalg.norm(U.T.astype(np.float64) @ U - np.eye(k), 2) < 1e-5
    assert np.linalg.norm(V.T.astype(np.float64) @ V - np.eye(k), 2) < 1e-5
    err = spectral.spectral_err_exact(A, U, S, V)
    assert err <= err0 * (1 + 1e-3) + 1e-6 * S0[0]


def test_tune_table_round_trip(ctx, case, tmp_path, gpu_lib):
    _, dA, _, _ = case
    ctx.tune_clear()
    ctx.tune(dA, L, reps=1)
    ctx.tune(dA[:, :200].contiguous(), 30, reps=1)
    assert ctx.tune_count() == 2
    p1, p2 = tmp_path / "a.txt", tmp_path / "b.txt"
    ctx.tune_save(str(p1))
    ctx.tune_clear()
    assert ctx.tune_count() == 0
    ctx.tune_load(str(p1))
    assert ctx.tune_count() == 2
    ctx.tune_save(str(p2))
    assert p1.read_text() == p2.read_text()
    # malformed lines: too few fields, a padded l that does not exist
    for bad in ("17 9 64 0 4 2\n", "17 9 48 0 4 2 4 2 512\n", "x\n"):
        p3 = tmp_path / "bad.txt"
        p3.write_text("# table\n" + bad)
        with pytest.raises(gpu_lib.RpcaError):
            ctx.tune_load(str(p3))
        assert ctx.tune_count() == 2
    ctx.tune_clear()


def test_tune_low_precision_and_sparse(ctx, case, gpu_lib):
    _, dA, _, _ = case
    q, _ = ctx.quantize(dA, "bf16")
    ctx.tune_clear()
    r = ctx.tune(q, L, reps=1, mat=gpu_lib.dense(q, A_f32=dA))
    assert r["candidates"] == 3
    assert r["ax_waves"] == 0 and r["atx_waves"] == 0 and r["lu_rows"] in (256, 512, 1024)
    ctx.tune_clear()
    rp, ci, va = sparse.random_rows(300, 200, 5, seed=3)
    cp, ri, vt = sparse.transpose(300, 200, rp, ci, va)
    dev = [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in (rp, ci, va, cp, ri, vt)]
    S = gpu_lib.csr(300, 200, *dev)
    with pytest.raises(gpu_lib.RpcaError):
        ctx.tune(S, 10)
