"""Low-precision copies of A (oracle side): bfloat16 and E4M3 with column scales.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper's cost is the number of passes over A and the bytes each pass
moves (Section 2: A has far more entries than any other matrix).  The
precision form of this project runs the range finder on a rounded copy of A
and the Rayleigh-Ritz product on the float32 A; the copies are defined here
from the number formats themselves:

  * bfloat16: 1 sign, 8 exponent (bias 127), 7 fraction bits -- float32 with
    the low 16 bits rounded away, to nearest, ties to an even fraction;
  * E4M3 (the OCP 8-bit floating-point format): 1 sign, 4 exponent (bias 7),
    3 fraction bits; exponent field 0 holds subnormals f * 2^-9; the code
    S.1111.111 is NaN and there are no infinities, so the largest finite value
    is 1.75 * 2^8 = 448.  Rounding is to the nearest value, ties to the even
    code.  Column j is stored as a_ij / s_j with s_j = max_i |a_ij| / 448
    (s_j = 1 for a zero column), so A = A8 diag(s).

The products of the range finder with such a copy are matrix-core
products of two bfloat16 operands: the copy's values and the other operand
rounded to bfloat16.  That rounding belongs to the definition of the
precision form (``LowPrecisionA``): Y = A X is A_s bf16(diag(s) X) and
A* Q is diag(s) A_s* bf16(Q), where A_s holds the stored values (bfloat16, or
decoded E4M3) and s the column scales (all ones for bfloat16); the operand is
held in float32 (diag(s) X formed in float32) before it is rounded, and the
products are exact sums (float64 here).  The Rayleigh-Ritz product reads the
float32 A and its operand is not rounded.

Pins (tests/test_oracle_precision.py): the E4M3 value table against its
closed-form corner values (448, 2^-6, 2^-9, 240, ...), monotonicity and
symmetry; rounding against brute force over the table (nearest value, ties
to even) and against PyTorch's own float8_e4m3fn and bfloat16 conversions
(independent library routines); bfloat16 ties and relative error 2^-8; the
low-precision products against brute-force sums over operands rounded by
PyTorch's bfloat16 conversion, exactness for operands that bfloat16
represents, the side the column scales act on, and exact recovery of a
matrix of rank <= l when the range finder reads a rounded copy.
"""

import numpy as np

E4M3_MAX = 448.0


def e4m3_values():
    """float64 value of each of the 256 E4M3 codes (NaN for 0x7F and 0xFF)."""
    codes = np.arange(256)
    sign = np.where(codes & 0x80, -1.0, 1.0)
    e = (codes >> 3) & 0xF
    f = codes & 0x7
    mag = np.where(e == 0, f * 2.0 ** -9, (1.0 + f / 8.0) * 2.0 ** (e - 7.0))
    val = sign * mag
    val[(codes & 0x7F) == 0x7F] = np.nan
    return val


def e4m3_encode(x):
    """Codes (uint8) of the E4M3 values nearest to x (ties to the even code),
    saturating at +-448."""
    x = np.asarray(x, dtype=np.float64)
    table = e4m3_values()[:0x7F]  # non-negative finite values, increasing with the code
    a = np.minimum(np.abs(x), E4M3_MAX)
    hi = np.searchsorted(table, a, side="left")  # table[hi] >= a
    hi = np.minimum(hi, 0x7E)
    lo = np.maximum(hi - 1, 0)
    dlo = a - table[lo]
    dhi = table[hi] - a
    pick_hi = (dhi < dlo) | ((dhi == dlo) & (hi % 2 == 0))
    code = np.where(pick_hi, hi, lo).astype(np.uint8)
    # the sign is kept, also when the magnitude rounds to zero (-0 is 0x80)
    code = np.where(np.signbit(x), code | 0x80, code).astype(np.uint8)
    return code


def e4m3_decode(codes):
    return e4m3_values()[np.asarray(codes, dtype=np.int64)]


def e4m3_scales(A):
    """s_j = max_i |a_ij| / 448, 1 for a zero column (float32 arithmetic, as stored)."""
    A = np.asarray(A, dtype=np.float32)
    amax = np.abs(A).max(axis=0)
    s = np.where(amax > 0, amax / np.float32(E4M3_MAX), np.float32(1.0)).astype(np.float32)
    return s


def to_e4m3(A):
    """(codes m x n uint8, scales n float32) with A ~ decode(codes) diag(scales).

    The quotient a_ij / s_j is formed in float32, as a float32 matrix and a
    float32 scale divide."""
    A = np.asarray(A, dtype=np.float32)
    s = e4m3_scales(A)
    q = (A / s[None, :]).astype(np.float32)
    return e4m3_encode(q), s


def from_e4m3(codes, s):
    """The matrix the E4M3 copy stands for, float64: decode(codes) diag(s)."""
    return e4m3_decode(codes) * np.asarray(s, dtype=np.float64)[None, :]


def to_bf16_bits(A):
    """uint16 bfloat16 codes of float32 A, round to nearest, ties to even."""
    b = np.asarray(A, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = (b + 0x7FFF + lsb) >> 16
    return r.astype(np.uint16)


def from_bf16_bits(bits):
    """float64 values of bfloat16 codes."""
    u = np.asarray(bits, dtype=np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def to_bf16(A):
    """float64 values of bfloat16(A)."""
    return from_bf16_bits(to_bf16_bits(A))


def bf16_operand(X):
    """The operand of a low-precision product: X held in float32, then rounded
    to bfloat16 (nearest even); float64 values."""
    return to_bf16(np.asarray(X, dtype=np.float32))


class LowPrecisionA:
    """A bfloat16 or E4M3 copy of an m x n A as the range finder applies it.

    values -- m x n stored values (bfloat16 values, or decoded E4M3 codes)
    scales -- length-n float32 column scales (E4M3), None for bfloat16

    matmul(X)  = A_s bf16(fl32(diag(s) X))      (Y = A X)
    rmatmul(Q) = diag(s) A_s^T bf16(fl32(Q))    (Z = A* Q)
    both summed exactly (float64).
    """

    def __init__(self, values, scales=None):
        self.values = np.asarray(values, dtype=np.float64)
        self.scales = None if scales is None else np.asarray(scales, dtype=np.float32)
        self.shape = self.values.shape

    def dense(self):
        """The matrix the copy stands for, A_s diag(s), in float64."""
        if self.scales is None:
            return self.values
        return self.values * self.scales.astype(np.float64)[None, :]

    def matmul(self, X):
        X32 = np.asarray(X, dtype=np.float32)
        if self.scales is not None:
            X32 = (X32 * self.scales[:, None]).astype(np.float32)
        return self.values @ bf16_operand(X32)

    def rmatmul(self, Q):
        Z = self.values.T @ bf16_operand(Q)
        if self.scales is not None:
            Z = Z * self.scales.astype(np.float64)[:, None]
        return Z
