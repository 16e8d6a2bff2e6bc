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
