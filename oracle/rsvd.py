"""Randomized SVD / PCA with renormalized power iterations (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows the paper's Section 2 (formulas (i1)-(i4) and (approx), the power
iteration with A A* A, renormalization after every application of A or A*)
and Section 5 (LU with partial pivoting in all but the last renormalization,
QR in the last; centering by subtracting the column means; applying A* as the
adjoint of Q* A), in float64 with the test matrix Omega passed in.

Readings of the paper taken here (the paper leaves these open):
  * l columns are sketched and the top k Ritz triplets are returned;
  * ``its`` counts the extra A* A applications: Y = A Omega, then ``its``
    times Z = A* Q, Y = A Q, i.e. 2*its + 1 applications before the
    Rayleigh-Ritz product B = Q* A (its = 0 is the plain sketch);
  * renormalization by LU returns the permuted unit lower factor P L
    (MATLAB's two-output ``[L, U] = lu(Y)``); the U factor is discarded;
  * a zero pivot leaves its column of L equal to the unit vector of the
    pivot row (LAPACK getrf behaviour), so span(P L) contains span(Y);
  * the last renormalization is an unpivoted Householder QR (the paper says
    pivoting is not needed there);
  * centering means PCA of A_c = A - 1 c with c the row vector of column
    means; here A_c is formed explicitly (the plain definition);
  * singular values are sorted in descending order; each left singular
    vector is signed so that its entry of largest magnitude is positive, and
    the matching right singular vector gets the same sign.

Pins (tests/test_oracle_rsvd.py): exact truncated SVD when l = min(m, n) or
rank(A) <= l (brute force with numpy.linalg.svd, including the paper's
diag(1,1,1,.999 x 17, 0, ...) matrices from Section 6); the closed-form
spectrum of a centered construction; Cauchy interlacing and Eckart-Young
bounds; orthonormality; equality of the LU and Householder variants (span
invariance); near-optimal error on the six spectra of Section 7.  The
schedule that renormalizes only after every second application (``fused``):
exact at full width, the same range as the standard schedule where float64
loses nothing by squaring, and the accuracy Section 5 says it gives up where
the squared spectrum passes float64's resolution.
"""

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sps


def lu_renorm(Y):
    """P L from the partial-pivoting LU of the tall matrix Y (U discarded).

    Section 5: an LU decomposition renormalizes Q after each multiplication
    with A, except in the last iteration.
    """
    PL, _ = sla.lu(np.asarray(Y, dtype=np.float64), permute_l=True)
    return PL


def qr_renorm(Y):
    """Orthonormal Q from the economy Householder QR of Y (Section 5, last step)."""
    Q, _ = np.linalg.qr(np.asarray(Y, dtype=np.float64), mode="reduced")
    return Q


def sign_fix(U, V=None):
    """Sign each column of U so that its largest-magnitude entry is positive."""
    idx = np.argmax(np.abs(U), axis=0)
    s = np.sign(U[idx, np.arange(U.shape[1])])
    s[s == 0] = 1.0
    U = U * s
    if V is None:
        return U
    return U, V * s


def rsvd(A, k, l, its, omega, center=False, renorm="lu", A_range=None, fused=False):
    """Rank-k approximation U diag(S) V^T of A (or of its column-centered form).

    A       -- m x n array (the exact values the device sees; upcast to float64),
               or a scipy.sparse matrix
    omega   -- n x l test matrix (float32 values from ``oracle.philox.omega``)
    renorm  -- "lu" (the paper's choice) or "qr" (Householder everywhere; equal
               to "lu" in exact arithmetic by span invariance)
    A_range -- optional operator the range finder applies instead of A: an
               m x n array (applied exactly), or an object with
               ``matmul(X)`` = A X and ``rmatmul(Q)`` = A* Q (the precision
               form's low-precision copy, ``oracle.precision.LowPrecisionA``);
               the Rayleigh-Ritz product B = Q* A always uses A
    fused   -- renormalize only after every second application (the
               acceleration Section 5 describes and does not adopt): starting
               from Q = omega, ``its`` times Z = A* (A Q) with no
               renormalization between the two products, then Z renormalized;
               then Y = A Q, orthonormalized by QR, and Rayleigh-Ritz as
               usual.  The range is (A A*)^its A omega as without ``fused``;
               its = 0 is the plain sketch either way

    Returns (U m x k, S length k, V n x k), all float64.
    """
    if sps.issparse(A):
        # a sparse A is only ever multiplied (Section 8); the centered sparse
        # form is not asked of the oracle
        if center or A_range is not None:
            raise ValueError("sparse A: no centering or range matrix")
        A = sps.csr_matrix(A, dtype=np.float64)
    else:
        A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    if not (1 <= k <= l <= min(m, n)):
        raise ValueError("need 1 <= k <= l <= min(m, n)")
    op = hasattr(A_range, "matmul")
    R = A if A_range is None else (A_range if op else np.asarray(A_range, dtype=np.float64))
    if R.shape != A.shape:
        raise ValueError("A_range must have the shape of A")
    if center:
        # PCA after subtracting from each column its mean (Section 2).
        A = A - A.mean(axis=0, keepdims=True)
        if not op:
            R = A if A_range is None else R - R.mean(axis=0, keepdims=True)
    omega = np.asarray(omega, dtype=np.float64)
    mid = lu_renorm if renorm == "lu" else qr_renorm

    def apply(X):  # A X (centered: the column means of the product removed)
        if not op:
            return R @ X
        Y = R.matmul(X)
        return Y - Y.mean(axis=0, keepdims=True) if center else Y

    def apply_t(Q):  # A* Q, as (Q* A)* for an array; A_c* Q = A* (Q - 1 mean(Q))
        if not op:
            return np.asarray(Q.T @ R).T
        return R.rmatmul(Q - Q.mean(axis=0, keepdims=True) if center else Q)

    if fused and its > 0:
        Q = omega
        for it in range(1, its + 1):
            # A* A Q with no renormalization in between (Section 5, last
            # paragraph: renormalizing only in the odd-numbered iterations)
            Q = mid(apply_t(apply(Q)))
        # the last application is followed by the orthonormalizing QR
        Q = qr_renorm(apply(Q))
        return _rayleigh_ritz(A, Q, k)

    # Apply A to l random vectors (Section 2, range finder).
    Y = apply(omega)
    Q = qr_renorm(Y) if its == 0 else mid(Y)
    for it in range(1, its + 1):
        # Apply A* as (Q* A)* without forming A* (Section 5).
        Z = apply_t(Q)
        Q = mid(Z)
        Y = apply(Q)
        # LU in all but the last iteration, QR in the last (Section 5).
        Q = mid(Y) if it < its else qr_renorm(Y)

    return _rayleigh_ritz(A, Q, k)


def _rayleigh_ritz(A, Q, k):
    """Top k of B = Q* A and U = Q W (formulas (i2)-(i4)), signs fixed."""
    # B = Q* A, formula (i2); its SVD W Sigma V* = B, formula (i3).
    B = np.asarray(Q.T @ A)
    W, S, Vt = np.linalg.svd(B, full_matrices=False)
    # U = Q W, formula (i4).
    U = Q @ W
    V = Vt.T
    U, S, V = U[:, :k], S[:k], V[:, :k]
    U, V = sign_fix(U, V)
    return U, S, V
