"""Pins of the oracle's low-precision copies (oracle/precision.py)."""

import numpy as np
import pytest
import torch

from oracle import precision as pr


def test_e4m3_table_closed_form():
    v = pr.e4m3_values()
    assert v[0x7E] == 448.0                   # 1.75 * 2^8, the largest finite value
    assert v[0x08] == 2.0 ** -6               # smallest normal
    assert v[0x01] == 2.0 ** -9               # smallest subnormal
    assert v[0x07] == 7 * 2.0 ** -9           # largest subnormal
    assert v[0x38] == 1.0                     # exponent field 7 = bias
    assert v[0x77] == 240.0                   # 1.875 * 2^7
    assert np.isnan(v[0x7F]) and np.isnan(v[0xFF])
    assert v[0x80] == 0.0 and np.signbit(v[0x80])
    pos = v[:0x7F]
    assert np.all(np.diff(pos) > 0)           # codes order the values
    np.testing.assert_array_equal(v[0x80:0xFF], -v[:0x7F])


def test_e4m3_matches_torch_table():
    t = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).double().numpy()
    v = pr.e4m3_values()
    np.testing.assert_array_equal(np.isnan(v), np.isnan(t))
    np.testing.assert_array_equal(v[~np.isnan(v)], t[~np.isnan(t)])


def test_e4m3_rounding_brute_force():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.uniform(-448, 448, 3000), rng.standard_normal(3000) * 0.02])
    pos = pr.e4m3_values()[:0x7F]
    mids = (pos[:-1] + pos[1:]) / 2
    x = np.concatenate([x, mids, -mids]).astype(np.float32).astype(np.float64)
    codes = pr.e4m3_encode(x)
    got = pr.e4m3_decode(codes)
    for xi, gi, ci in zip(x, got, codes):
        d = np.abs(pos - abs(xi))
        best = np.flatnonzero(d == d.min())
        want = best[0] if len(best) == 1 else best[best % 2 == 0][0]  # tie: even code
        assert (ci & 0x7F) == want and abs(gi) == pos[want]
        assert np.signbit(gi) == np.signbit(xi) or gi == 0


def test_e4m3_matches_torch_conversion():
    rng = np.random.default_rng(2)
    x = np.clip(rng.standard_normal(200000) * 60, -448, 448).astype(np.float32)
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(pr.e4m3_encode(x), want)


def test_e4m3_scaled_copy_error():
    rng = np.random.default_rng(3)
    A = (rng.standard_normal((300, 70)) * np.logspace(-3, 2, 70)).astype(np.float32)
    A[:, 5] = 0.0
    codes, s = pr.to_e4m3(A)
    assert s[5] == 1.0 and np.all(codes[:, 5] & 0x7F == 0)
    # each column reaches 448 in magnitude at its largest entry
    dec = pr.e4m3_decode(codes)
    cols = [j for j in range(70) if j != 5]
    np.testing.assert_allclose(np.abs(dec[:, cols]).max(axis=0), 448.0)
    B = pr.from_e4m3(codes, s)
    # relative rounding 2^-4 for normal values; subnormal steps 2^-9 s_j
    err = np.abs(B - A)
    assert np.all(err <= np.maximum(2.0 ** -4 * np.abs(A), 2.0 ** -10 * s[None, :] * 1.0001))


def test_bf16_rounding():
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -7, -(1 + 2 ** -8), 3.0e38,
                  1e-40], dtype=np.float32)
    got = pr.to_bf16(x)
    # 1 + 2^-8 is a tie -> even fraction (1.0); 1 + 3 2^-8 is a tie -> 1 + 2^-6
    np.testing.assert_array_equal(got[:5], [1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -1.0])
    rng = np.random.default_rng(4)
    y = (rng.standard_normal(100000) * 10.0 ** rng.uniform(-20, 20, 100000)).astype(np.float32)
    b = pr.to_bf16(y)
    assert np.all(np.abs(b - y) <= 2.0 ** -8 * np.abs(y.astype(np.float64)))  # u = 2^-8
    want = torch.from_numpy(y).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(pr.to_bf16_bits(y), want)


# ---- the low-precision products of the precision form -------------------

def _torch_bf16(x):
    """bfloat16 rounding by PyTorch (an implementation independent of the oracle's)."""
    import torch
    return torch.tensor(np.asarray(x, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _lowp_pair(kind, m, n, seed):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((m, n)) * np.logspace(-2, 1, n)).astype(np.float32)
    if kind == "bf16":
        return A, pr.LowPrecisionA(pr.to_bf16(A))
    codes, s = pr.to_e4m3(A)
    return A, pr.LowPrecisionA(pr.e4m3_decode(codes), s)


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_lowp_products_brute_force(kind):
    import math
    m, n, l = 9, 7, 3
    A, op = _lowp_pair(kind, m, n, 3)
    rng = np.random.default_rng(4)
    X = rng.standard_normal((n, l))
    Q = rng.standard_normal((m, l))
    vals = op.values
    s = np.ones(n, dtype=np.float32) if op.scales is None else op.scales
    # Y = A X: operand diag(s) X formed in float32, rounded to bfloat16 by torch
    Xs = _torch_bf16(np.float32(1) * X.astype(np.float32) * s[:, None])
    Y = np.array([[math.fsum(vals[i, j] * Xs[j, c] for j in range(n)) for c in range(l)]
                  for i in range(m)])
    np.testing.assert_allclose(op.matmul(X), Y, rtol=1e-14, atol=0)
    # Z = A^T Q: the column scale applied after the sum
    Qb = _torch_bf16(Q)
    Z = np.array([[float(s[j]) * math.fsum(vals[i, j] * Qb[i, c] for i in range(m))
                   for c in range(l)] for j in range(n)])
    np.testing.assert_allclose(op.rmatmul(Q), Z, rtol=1e-14, atol=0)


def test_lowp_product_exact_for_representable_operands():
    A, op = _lowp_pair("bf16", 40, 30, 5)
    X = pr.to_bf16(np.random.default_rng(6).standard_normal((30, 4)).astype(np.float32))
    np.testing.assert_allclose(op.matmul(X), op.values @ X, rtol=1e-15)
    # a perturbation below half a bfloat16 ulp rounds away, one above does not
    tiny = X * (1 + 2.0 ** -10)
    np.testing.assert_array_equal(pr.bf16_operand(tiny), X)
    big = X * (1 + 2.0 ** -7)
    assert np.all(pr.bf16_operand(big)[X != 0] != X[X != 0])


def test_lowp_scales_act_on_the_right_side():
    # the E4M3 copy stands for A8 diag(s): both products agree with that matrix
    # up to the operand's bfloat16 rounding (2^-8 relative per term)
    A, op = _lowp_pair("fp8", 200, 64, 7)
    D = op.dense()
    rng = np.random.default_rng(8)
    X = rng.standard_normal((64, 5))
    Q = rng.standard_normal((200, 5))
    bound = 2.0 ** -8 * (np.abs(D) @ np.abs(X)) * 1.001
    assert np.all(np.abs(op.matmul(X) - D @ X) <= bound)
    bound_t = 2.0 ** -8 * (np.abs(D.T) @ np.abs(Q)) * 1.001
    assert np.all(np.abs(op.rmatmul(Q) - D.T @ Q) <= bound_t)
    # the bound is tight enough to see a dropped scale (s_j spans 1e-2 .. 10 / 448)
    assert not np.all(np.abs(op.values @ X - D @ X) <= bound)
    assert not np.all(np.abs(op.values.T @ Q - D.T @ Q) <= bound_t)


@pytest.mark.parametrize("center", [False, True])
def test_lowp_range_finder_recovers_rank_le_l(center):
    # rank(A) = 6 <= l: the rounded operand moves only the basis of the sketch,
    # whose span stays range(A); B = Q* A on the exact A then gives the exact SVD
    from oracle import philox, rsvd
    m, n, r, k, l = 300, 80, 6, 5, 10
    rng = np.random.default_rng(9)
    sig = np.linspace(1.0, 0.2, r)
    U0 = np.linalg.qr(rng.standard_normal((m, r)))[0]
    V0 = np.linalg.qr(rng.standard_normal((n, r)))[0]
    A = pr.to_bf16(((U0 * sig) @ V0.T).astype(np.float32))  # bfloat16-exact
    op = pr.LowPrecisionA(A)
    _, S, _ = rsvd.rsvd(A, k, l, 2, philox.omega(3, n, l), center=center, A_range=op)
    Ac = A - A.mean(axis=0) if center else A
    np.testing.assert_allclose(S, np.linalg.svd(Ac, compute_uv=False)[:k], rtol=1e-10)
    # with rank > l the rounding does show: the result differs from the exact-operand run
    B = rng.standard_normal((m, n)).astype(np.float32)
    opb = pr.LowPrecisionA(pr.to_bf16(B))
    om = philox.omega(3, n, l)
    _, S1, _ = rsvd.rsvd(B, k, l, 1, om, A_range=opb)
    _, S2, _ = rsvd.rsvd(B, k, l, 1, om, A_range=opb.dense())
    assert np.max(np.abs(S1 - S2) / S2) > 1e-6
