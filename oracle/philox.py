"""Philox4x32-10 and the Gaussian test matrix (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper draws the random test vectors with i.i.d. standard normal entries
(Section 2, the range-finder paragraph) and notes that the algorithm does not
depend on the quality of the generator (Section 5).  No generator is named,
so this project fixes one that two independent implementations can reproduce
bit for bit: the counter-based Philox4x32-10 of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11), written here from that
paper's definition:

  * state: a 128-bit counter (c0, c1, c2, c3) and a 64-bit key (k0, k1),
    all 32-bit words;
  * one round: (hi0, lo0) = M0 * c0 and (hi1, lo1) = M1 * c2 as 64-bit
    products, then (c0, c1, c2, c3) <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0);
  * between rounds the key is bumped by the Weyl constants (W0, W1);
  * ten rounds.

Mapping to the test matrix (fixed by this project):
  * key   = (seed mod 2^32, seed >> 32);
  * counter for block t = (t mod 2^32, t >> 32, stream, 0);
  * block t yields the normal variates z[4t .. 4t+3]: words (x0, x1) give
    (z0, z1) and (x2, x3) give (z2, z3) by the Box-Muller transform
        u = (x + 1/2) * 2^-32,  r = sqrt(-2 ln u_a),  theta = 2*pi*u_b,
        (z_even, z_odd) = (r cos theta, r sin theta),
    evaluated in float64 and rounded once to float32;
  * the n-by-l test matrix is Omega[i, j] = z[j*n + i] (column-major order
    of the stream);
  * the uniform alternative of Section 5 maps each word on its own,
    v = (x + 1/2) 2^-31 - 1, exact in float64 and rounded once to float32,
    and Omega[i, j] = v[j*n + i] (``omega_uniform``).

Pins (tests/test_oracle_philox.py): the Weyl constants against their closed
forms (golden ratio and sqrt(3)), bijectivity of the round on a small word
sample, bit balance and avalanche of the output, uniformity of the words
(chi-square), and the first four moments and a Kolmogorov-Smirnov test of the
Gaussian map.  Published known-answer vectors are not used.

Parity unpinned: the exact Philox4x32-10 word stream is not checked against
the generator's published known-answer vectors (none are available here).
These pins would not catch, say, a permutation of the output words; the
method itself only needs i.i.d. N(0, 1) draws, which the statistical pins
cover.  The library's generator is an independent implementation compared
with this one bit for bit.
"""

import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)  # floor(2^32 * (golden ratio - 1))
W1 = np.uint64(0xBB67AE85)  # floor(2^32 * (sqrt(3) - 1))
ROUNDS = 10
TWO_PI = 6.283185307179586  # float64 nearest to 2*pi
TWO_M32 = 2.0 ** -32

# stream identifiers used by the library
STREAM_OMEGA = 0
STREAM_SPECTRAL = 1


def philox4x32(c0, c1, c2, c3, k0, k1, rounds=ROUNDS):
    """Apply ``rounds`` Philox4x32 rounds to counters (c0..c3) under key (k0, k1).

    Arguments are array-likes of 32-bit values (any integer dtype); returns a
    tuple of four uint32 arrays.
    """
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.asarray(c1, dtype=np.uint64)
    c2 = np.asarray(c2, dtype=np.uint64)
    c3 = np.asarray(c3, dtype=np.uint64)
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * c0  # < 2^64, exact in uint64
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def words(seed, stream, nblocks, first_block=0):
    """The raw 32-bit words of blocks first_block .. first_block+nblocks-1.

    Returns a uint32 array of shape (nblocks, 4).
    """
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    t = np.arange(first_block, first_block + nblocks, dtype=np.uint64)
    x = philox4x32(t & MASK32, t >> np.uint64(32),
                   np.full_like(t, int(stream) & 0xFFFFFFFF), np.zeros_like(t),
                   seed & 0xFFFFFFFF, seed >> 32)
    return np.stack(x, axis=1)


def box_muller(xa, xb):
    """Map word pairs to a pair of standard normals (float64, not yet rounded)."""
    ua = (xa.astype(np.float64) + 0.5) * TWO_M32
    ub = (xb.astype(np.float64) + 0.5) * TWO_M32
    r = np.sqrt(-2.0 * np.log(ua))
    th = TWO_PI * ub
    return r * np.cos(th), r * np.sin(th)


def normals(seed, stream, count):
    """z[0 .. count-1] of the given stream, float32."""
    nb = (int(count) + 3) // 4
    w = words(seed, stream, nb)
    z = np.empty((nb, 4), dtype=np.float64)
    z[:, 0], z[:, 1] = box_muller(w[:, 0], w[:, 1])
    z[:, 2], z[:, 3] = box_muller(w[:, 2], w[:, 3])
    return z.reshape(-1)[:count].astype(np.float32)


def omega(seed, n, l, stream=STREAM_OMEGA):
    """The n-by-l Gaussian test matrix Omega[i, j] = z[j*n + i], float32."""
    z = normals(seed, stream, n * l)
    return z.reshape(l, n).T.copy()


def uniforms(seed, stream, count):
    """v[0 .. count-1]: word e of the stream (block e // 4, word e % 4) mapped
    to (x + 1/2) 2^-31 - 1 in (-1, 1), exact in float64, rounded once to
    float32 (Section 5: uniform draws on [-1, 1] serve as well as normal
    ones, from the fastest generator at hand)."""
    nb = (int(count) + 3) // 4
    w = words(seed, stream, nb).reshape(-1)[:count]
    return ((w.astype(np.float64) + 0.5) * 2.0 ** -31 - 1.0).astype(np.float32)


def omega_uniform(seed, n, l, stream=STREAM_OMEGA):
    """The n-by-l uniform test matrix Omega[i, j] = v[j*n + i], float32."""
    return uniforms(seed, stream, n * l).reshape(l, n).T.copy()
