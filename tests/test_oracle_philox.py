"""Pins for the oracle's Philox4x32-10 stream and Gaussian map.

Known-answer vectors are not available here, so the generator is pinned by
what the method needs from it (Section 2: i.i.d. standard normal entries;
Section 5: robustness to the generator's quality) and by the closed forms of
its constants.  Its agreement with the device generator is a GPU parity test.
"""

from decimal import Decimal, getcontext

import numpy as np
import pytest
from scipy import stats

from oracle import philox


def test_weyl_constants_closed_form():
    # The key schedule adds the fractional parts of the golden ratio and of
    # sqrt(3), scaled by 2^32 and truncated.
    getcontext().prec = 60
    phi_frac = (Decimal(5).sqrt() - 1) / 2
    s3_frac = Decimal(3).sqrt() - 1
    assert int(phi_frac * 2 ** 32) == int(philox.W0)
    assert int(s3_frac * 2 ** 32) == int(philox.W1)


def test_multipliers_odd():
    # Odd multipliers make each round a bijection of the counter.
    assert int(philox.M0) % 2 == 1 and int(philox.M1) % 2 == 1


def test_round_is_bijection():
    # One round is invertible: recover the input from the output.
    rng = np.random.default_rng(0)
    c = rng.integers(0, 2 ** 32, size=(4, 5000), dtype=np.uint64)
    k0, k1 = 0x12345678, 0x9ABCDEF0
    o = [x.astype(np.uint64) for x in philox.philox4x32(*c, k0, k1, rounds=1)]
    inv0 = pow(int(philox.M0), -1, 2 ** 32)
    inv1 = pow(int(philox.M1), -1, 2 ** 32)
    c0 = (o[3] * np.uint64(inv0)) & philox.MASK32
    c2 = (o[1] * np.uint64(inv1)) & philox.MASK32
    hi0 = (c0 * philox.M0) >> np.uint64(32)
    hi1 = (c2 * philox.M1) >> np.uint64(32)
    c1 = o[0] ^ hi1 ^ np.uint64(k0)
    c3 = o[2] ^ hi0 ^ np.uint64(k1)
    for a, b in zip((c0, c1, c2, c3), c):
        np.testing.assert_array_equal(a, b)


def test_bit_balance_and_word_uniformity():
    w = philox.words(seed=2024, stream=0, nblocks=1 << 16).reshape(-1)
    n = w.size
    bits = ((w[:, None] >> np.arange(32, dtype=np.uint32)) & 1).astype(np.float64)
    p = bits.mean(axis=0)
    assert np.all(np.abs(p - 0.5) < 6 * 0.5 / np.sqrt(n))
    # chi-square on the top byte
    counts = np.bincount((w >> 24).astype(np.int64), minlength=256)
    chi2 = ((counts - n / 256) ** 2 / (n / 256)).sum()
    assert stats.chi2.sf(chi2, 255) > 1e-4


def test_avalanche():
    # Flipping one counter bit flips about half of the 128 output bits.
    rng = np.random.default_rng(1)
    t = rng.integers(0, 2 ** 31, size=4096, dtype=np.uint64)
    z = np.zeros_like(t)
    a = philox.philox4x32(t, z, z, z, 7, 11)
    flips = []
    for bit in (0, 13, 31):
        b = philox.philox4x32(t ^ np.uint64(1 << bit), z, z, z, 7, 11)
        d = sum(np.unpackbits((x ^ y).view(np.uint8)).sum() for x, y in zip(a, b))
        flips.append(d / (128 * t.size))
    assert np.all(np.abs(np.array(flips) - 0.5) < 0.01)
    # a single round does not mix: this separates ten rounds from one
    a1 = philox.philox4x32(t, z, z, z, 7, 11, rounds=1)
    b1 = philox.philox4x32(t ^ np.uint64(1), z, z, z, 7, 11, rounds=1)
    d1 = sum(np.unpackbits((x ^ y).view(np.uint8)).sum() for x, y in zip(a1, b1))
    assert d1 / (128 * t.size) < 0.3


def test_streams_and_seeds_differ():
    a = philox.words(5, 0, 64)
    b = philox.words(5, 1, 64)
    c = philox.words(6, 0, 64)
    assert not np.array_equal(a, b) and not np.array_equal(a, c)


def test_gaussian_moments_and_ks():
    z = philox.normals(seed=77, stream=0, count=1 << 20).astype(np.float64)
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1) < 5 * np.sqrt(2 / n)
    assert abs(stats.skew(z)) < 5 * np.sqrt(6 / n)
    assert abs(stats.kurtosis(z)) < 5 * np.sqrt(24 / n)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the two members of a Box-Muller pair are uncorrelated
    zz = z.reshape(-1, 2)
    assert abs(np.corrcoef(zz[:, 0], zz[:, 1])[0, 1]) < 5 / np.sqrt(n / 2)


def test_gaussian_float32_rounding():
    # rounded once from float64
    w = philox.words(3, 0, 256)
    z0, _ = philox.box_muller(w[:, 0], w[:, 1])
    got = philox.normals(3, 0, 1024).reshape(-1, 4)[:, 0]
    np.testing.assert_array_equal(got, z0.astype(np.float32))


@pytest.mark.parametrize("n,l", [(7, 3), (16, 4), (33, 5)])
def test_omega_layout(n, l):
    z = philox.normals(11, 0, n * l)
    om = philox.omega(11, n, l)
    assert om.shape == (n, l) and om.dtype == np.float32
    for i in range(n):
        for j in range(l):
            assert om[i, j] == z[j * n + i]


def test_uniform_map_closed_form_and_law():
    # the uniform test matrix of Section 5: v = (x + 1/2) 2^-31 - 1 per word
    w = philox.words(11, 0, 1000).reshape(-1)
    v = philox.uniforms(11, 0, 4000)
    # closed form at the extremes and the midpoint, and exactness of the map
    assert np.float32((0 + 0.5) * 2.0 ** -31 - 1.0) == np.float32(-1.0)
    assert np.float32((2.0 ** 32 - 0.5) * 2.0 ** -31 - 1.0) == np.float32(1.0)
    assert np.float32((2.0 ** 31 + 0.5) * 2.0 ** -31 - 1.0) == np.float32(2.0 ** -32)
    np.testing.assert_array_equal(v, ((w.astype(np.float64) + 0.5) / 2.0 ** 31 - 1.0)
                                  .astype(np.float32))
    big = philox.uniforms(12, 0, 400000).astype(np.float64)
    assert abs(big.mean()) < 5e-3
    assert abs(big.var() - 1.0 / 3.0) < 5e-3
    assert big.min() >= -1.0 and big.max() <= 1.0
    from scipy import stats
    assert stats.kstest(big, "uniform", args=(-1.0, 2.0)).pvalue > 1e-3
    om = philox.omega_uniform(12, 100, 7)
    np.testing.assert_array_equal(om[:, 2], philox.uniforms(12, 0, 700)[200:300])


def test_uniform_omega_serves_the_range_finder():
    # Section 5: the algorithm does not depend on the generator's law; with a
    # uniform Omega the error stays near sigma_{k+1}, as with the Gaussian one
    from oracle import rsvd, spectral
    from synth import dense
    m, n, k, l = 400, 200, 10, 12
    sig = dense.spectrum_small(n)
    A = dense.dense(m, n, sig, seed=5)
    U, S, V = rsvd.rsvd(A, k, l, 2, philox.omega_uniform(3, n, l))
    assert spectral.spectral_err_exact(A, U, S, V) <= 1.1 * sig[k]
