"""The persistent batched launch on the GPU (rpca_svd_batched for dense
float32 problems with m, n <= 8192 and l <= 64: one workgroup per problem).

Each problem is checked against the FP64 oracle on the same Omega:
  * singular values (eigenvalues) within 1e-4 relative;
  * U and V orthonormal to 1e-5;
  * where the exact residual is affordable, an error within 0.1% of the
    oracle's own rank-k error.
The batch is solved twice: every problem on one workgroup, and with the
problems above the batch's average load split over teams of workgroups
(shared passes, Gram matrices and solves by row ranges).  It mixes shapes
that exercise every edge of the single-workgroup routines: l <= 32 and 32 < l <= 64 (one or two MFMA column blocks), row
counts and column counts that are not multiples of the tiles (64 for the
K chunks, 256 for the row and column tiles), wide and tall A, its = 0, the
centered form, Cholesky QR in place of LU, an A whose row stride is odd (the
unaligned load path), a rank-deficient A (zero LU pivots, shifted Cholesky
QR with completion), the zero matrix, l = min(m, n), a single row or column
(l = k = 1), and the largest shape (8192 x 2048).  The same batch solved on
streams (mode 1) agrees to rounding, and a call mixing persistent problems
with one too large for it (m > 8192, solved on a stream) matches the oracle.
"""

import numpy as np
import pytest
import torch

from oracle import nystrom, philox, rsvd, spectral
from synth import dense

pytestmark = pytest.mark.gpu

# (kind, m, n, k, l, its, center, renorm, special)
CASES = [
    ("svd", 1000, 500, 10, 12, 2, False, "chol", None),
    ("svd", 3000, 200, 20, 30, 2, False, "lu", None),
    ("svd", 200, 3000, 20, 30, 1, False, "lu", None),
    ("svd", 4000, 400, 50, 60, 2, False, "chol", None),
    ("svd", 777, 333, 40, 45, 2, True, "chol", None),
    ("svd", 777, 333, 40, 45, 2, True, "lu", None),
    ("svd", 500, 300, 5, 12, 0, False, "lu", None),
    ("svd", 3000, 200, 20, 30, 2, False, "orth", None),
    ("svd", 300, 70, 8, 64, 3, False, "chol", None),
    ("svd", 100, 64, 10, 64, 2, False, "lu", None),
    ("svd", 257, 129, 12, 33, 2, True, "chol", "odd_ld"),
    ("svd", 600, 400, 5, 20, 2, False, "lu", "rank5"),
    ("svd", 600, 400, 5, 20, 2, False, "chol", "rank5"),
    ("svd", 300, 200, 5, 10, 1, False, "lu", "zero"),
    ("svd", 300, 200, 5, 10, 1, False, "chol", "zero"),
    ("svd", 8192, 2048, 40, 45, 2, False, "chol", None),
    ("psd", 300, 300, 20, 25, 2, False, "lu", None),
    ("psd", 1000, 1000, 10, 15, 1, False, "chol", None),
    ("psd", 700, 700, 40, 45, 2, False, "chol", None),
    ("psd", 500, 500, 5, 10, 0, False, "lu", None),
    ("psd", 2500, 2500, 30, 35, 2, False, "orth", None),
    ("psd", 200, 200, 3, 20, 0, False, "chol", None),
    ("svd", 1, 300, 1, 1, 1, False, "chol", None),
    ("svd", 500, 1, 1, 1, 2, False, "lu", None),
]


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return gpu_lib.Context()


def _matrix(i, case):
    kind, m, n, k, l, its, center, renorm, special = case
    if kind == "psd":
        return dense.psd(n, dense.spectrum_exp(n), seed=300 + i)
    if special == "rank5":
        sig = np.zeros(min(m, n))
        sig[:5] = [5.0, 4.0, 3.0, 2.0, 1.0]
        return dense.dense(m, n, sig, seed=300 + i)
    if special == "zero":
        return np.zeros((m, n), dtype=np.float32)
    A = dense.dense(m, n, dense.spectrum_tall(min(m, n)), seed=300 + i)
    if center:
        A = A + np.float32(0.05)
    return A


def _device(A, special):
    t = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    if special == "odd_ld":  # row stride n + 1: the unaligned path
        m, n = A.shape
        w = torch.zeros(m, n + 1, device="cuda", dtype=torch.float32)
        w[:, :n] = t
        return w[:, :n]
    return t


def _problems():
    host, probs = [], []
    for i, case in enumerate(CASES):
        kind, m, n, k, l, its, center, renorm, special = case
        A = _matrix(i, case)
        host.append(A)
        probs.append(dict(A=_device(A, special), k=k, l=l, its=its, seed=900 + i,
                          center=center, renorm=renorm, kind=kind))
    return host, probs


# (max_parts, min_parts): (1, 1) every problem on one workgroup; (8, 4)
# every problem that can be split (min(m, n) >= 128, no LU renormalization)
# over a team of 2 to 8 workgroups
SPLITS = {"whole": (1, 1), "split": (8, 4)}


@pytest.fixture(scope="module", params=["whole", "split"])
def batch(ctx, request):
    host, probs = _problems()
    ctx.set_batch_split(*SPLITS[request.param])
    try:
        outs = ctx.svd_batched(probs, sync=True)
        assert ctx.batch_status(len(probs)) == [0] * len(probs)
    finally:
        ctx.set_batch_split()
    return host, probs, [[t.cpu().numpy() for t in o] for o in outs], request.param


def _orth_err(X):
    X = X.astype(np.float64)
    return np.linalg.norm(X.T @ X - np.eye(X.shape[1]), 2)


@pytest.mark.parametrize("i", range(len(CASES)))
def test_persistent_matches_oracle(batch, i):
    host, probs, outs, _ = batch
    kind, m, n, k, l, its, center, renorm, special = CASES[i]
    A = host[i]
    om = philox.omega(900 + i, n, l)
    print("case", CASES[i], flush=True)
    if kind == "psd":
        U, L = outs[i]
        U0, L0, _, _ = nystrom.eig_psd(A, k, l, its, om, u_A=2.0 ** -16)
        np.testing.assert_allclose(L, L0, rtol=1e-4, atol=1e-6 * L0[0])
        assert _orth_err(U) < 1e-5
        if n <= 1000:
            err = spectral.spectral_err_exact(A, U, L)
            err0 = spectral.spectral_err_exact(A, U0, L0)
            assert err <= err0 * 1.001 + 1e-6
        return
    U, S, V = outs[i]
    U0, S0, V0 = rsvd.rsvd(A, k, l, its, om, center=center,
                           renorm="qr" if renorm == "orth" else "lu")
    if special == "zero":
        assert np.all(S == 0.0)
        return
    if special == "rank5":
        np.testing.assert_allclose(S, S0, rtol=1e-4, atol=1e-6 * S0[0])
    else:
        np.testing.assert_allclose(S, S0, rtol=1e-4)
    assert _orth_err(U) < 1e-5
    assert _orth_err(V) < 1e-5
    if m * n <= 3000 * 500:
        err = spectral.spectral_err_exact(A, U, S, V, center=center)
        err0 = spectral.spectral_err_exact(A, U0, S0, V0, center=center)
        # when l >= min(m, n) the oracle's error is ~0 and what remains is the
        # rounding of the float32 factors, about 2^-24 sqrt(m + n) sigma_1
        floor = 2e-7 * np.sqrt(m + n) if l >= min(m, n) else 1e-6
        assert err <= err0 * (1 + 1e-3) + floor * S0[0]


def test_persistent_agrees_with_streams(ctx, batch):
    host, probs, outs, _ = batch
    ctx.set_batch_mode(1)
    try:
        ref = ctx.svd_batched(probs, sync=True)
    finally:
        ctx.set_batch_mode(0)
    for i, (o, r) in enumerate(zip(outs, ref)):
        if CASES[i][8] == "zero":
            continue
        S, S_ref = o[1], r[1].cpu().numpy()
        np.testing.assert_allclose(S, S_ref, rtol=1e-5, atol=1e-7 * S_ref[0])


def test_persistent_repeat_bit_identical(ctx, batch):
    # the same batch again, another batch in between (the table is rewritten by
    # every call):
    # bit-identical results every time
    host, probs, outs, split = batch
    small = [probs[0], probs[5], probs[13]]
    ctx.set_batch_split(*SPLITS[split])
    try:
        for rep in range(2):
            again = ctx.svd_batched(probs, sync=True)
            for o, a in zip(outs, again):
                for x, y in zip(o, a):
                    assert np.array_equal(x, y.cpu().numpy()), "repeat %d" % rep
            ctx.svd_batched(small, sync=True)
    finally:
        ctx.set_batch_split()


def test_split_changes_rounding_only(ctx):
    # the same problems whole and split: the split ones sum their partial
    # products in another order, so they differ in the last bits (which shows
    # the split happened) and agree to rounding
    host, probs = _problems()
    ctx.set_batch_split(1)
    whole = ctx.svd_batched(probs, sync=True)
    ctx.set_batch_split(8, 4)
    split = ctx.svd_batched(probs, sync=True)
    ctx.set_batch_split()
    differ = 0
    for i, (a, b) in enumerate(zip(whole, split)):
        if CASES[i][8] == "zero":
            continue
        S0, S1 = a[1].cpu().numpy(), b[1].cpu().numpy()
        np.testing.assert_allclose(S1, S0, rtol=1e-5, atol=1e-7 * S0[0])
        differ += int(not np.array_equal(S0, S1) or not torch.equal(a[0], b[0]))
    assert differ >= 8


def test_split_wait_limit_reports_timeout(ctx, gpu_lib):
    # a wait limit of one poll, forced from the host: a share that arrives
    # first stops waiting at once and its problem reports RPCA_ERR_TIMEOUT
    # (every kernel still ends normally); the problems solved whole are not
    # affected, and with the default limit the batch is clean again
    TIMEOUT = 7
    host, probs = _problems()
    big = [i for i, c in enumerate(CASES) if min(c[1], c[2]) >= 1000 and c[7] != "lu"]
    assert len(big) >= 3
    ctx.set_batch_split(8, 4, 1)
    try:
        ctx.svd_batched(probs)
        st = ctx.batch_status(len(probs))
        with pytest.raises(gpu_lib.RpcaError) as e:
            ctx.sync()
        assert e.value.status == TIMEOUT
    finally:
        ctx.set_batch_split()
    assert set(st) <= {0, TIMEOUT} and sum(s == TIMEOUT for s in st) >= 1
    small = [i for i, c in enumerate(CASES) if min(c[1], c[2]) < 128 or c[7] == "lu"]
    assert all(st[i] == 0 for i in small)
    ctx.svd_batched(probs, sync=True)
    assert ctx.batch_status(len(probs)) == [0] * len(probs)


def test_batch_split_rejects_bad_values(ctx, gpu_lib):
    for args in ((0, 1, 0), (17, 1, 0), (4, 5, 0), (4, 0, 0), (4, 2, -1)):
        with pytest.raises(gpu_lib.RpcaError):
            ctx.set_batch_split(*args)


def test_persistent_and_streams_in_one_call(ctx):
    # m > 8192 goes to a stream, the others to the persistent launch
    shapes = [("svd", 700, 300, 10, 15), ("svd", 9000, 100, 10, 15), ("psd", 400, 400, 10, 15)]
    host, probs = [], []
    for i, (kind, m, n, k, l) in enumerate(shapes):
        A = (dense.psd(n, dense.spectrum_exp(n), seed=700 + i) if kind == "psd"
             else dense.dense(m, n, dense.spectrum_tall(min(m, n)), seed=700 + i))
        host.append(A)
        probs.append(dict(A=torch.from_numpy(A).cuda(), k=k, l=l, its=2, seed=800 + i, kind=kind))
    outs = ctx.svd_batched(probs, sync=True)
    for (kind, m, n, k, l), A, o in zip(shapes, host, outs):
        om = philox.omega(800 + shapes.index((kind, m, n, k, l)), n, l)
        if kind == "psd":
            _, L0, _, _ = nystrom.eig_psd(A, k, l, 2, om, u_A=2.0 ** -16)
            np.testing.assert_allclose(o[1].cpu().numpy(), L0, rtol=1e-4, atol=1e-6 * L0[0])
        else:
            _, S0, _ = rsvd.rsvd(A, k, l, 2, om)
            np.testing.assert_allclose(o[1].cpu().numpy(), S0, rtol=1e-4)


def test_batch_mode_rejects_bad_value(ctx, gpu_lib):
    with pytest.raises(gpu_lib.RpcaError):
        ctx.set_batch_mode(2)
