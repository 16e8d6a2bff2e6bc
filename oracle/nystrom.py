"""Shift-stabilized Nystrom method for PSD matrices (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Follows the paper's Section 3 (formulas (start), (second), (Cholesky),
(pseudo), the SVD of F, and (finish), after Halko, Martinsson and Tropp's
Algorithm 5.5), with the stabilization the paper's own codes use: add a
multiple nu of the identity before the Cholesky factorization and subtract it
afterwards.  The orthonormal Q comes from the self-adjoint core loop of
Section 5 (A applied ``its`` times, LU after all but the last application,
QR after the last).

Readings of the paper taken here:
  * its = 0 means Q = qr(Omega) (the loop body never runs);
  * the shift is nu = sqrt(n) * u_A * ||B1||_F with u_A the unit roundoff of
    the arithmetic B1 = A Q is computed in (2^-24 for float32 products,
    2^-16 for the device's float32 path, whose products carry about 16
    significant bits); if the Cholesky factor does not exist, nu is
    multiplied by 10, at most ``max_retries`` times;
  * the shift enters as B1_nu = B1 + nu Q = (A + nu I) Q, and the computed
    eigenvalues are max(S^2 - nu, 0);
  * C is the upper triangular factor with C* C = B2 (MATLAB ``chol``), and
    F = B1_nu C^-1 is formed by a triangular solve;
  * the eigenvalues are sorted in descending order and each eigenvector is
    signed so that its largest-magnitude entry is positive.

The alternative of the paper (a self-adjoint square root of B2 from its
eigendecomposition, with a regularized pseudoinverse) is ``eig_psd_sqrt``;
in exact arithmetic both give the same approximation A_hat = B1 B2^+ B1*.
For a self-adjoint A that is not definite, ``eig_sym`` gives the
Rayleigh-Ritz eigenpairs Q W diag(lambda) (Q W)* with B2 = Q* A Q =
W diag(lambda) W*, Q from the same core loop.

Pins (tests/test_oracle_nystrom.py): exactness when rank(A) <= l; the
eigenvalue bounds lambda_hat_j <= lambda_j and A - A_hat >= 0 (Loewner order)
for the unshifted form; agreement of the shifted-Cholesky and square-root
forms up to O(nu); brute force with numpy.linalg.eigh.
"""

import numpy as np
import scipy.linalg as sla

from .rsvd import lu_renorm, qr_renorm, sign_fix


def range_psd(A, l, its, omega):
    """Orthonormal Q (n x l) from the self-adjoint core loop of Section 5.

    A is an array (applied exactly) or an object whose ``matmul(X)`` is A X
    (the precision form's low-precision copy, ``oracle.precision``)."""
    if not hasattr(A, "matmul"):
        A = np.asarray(A, dtype=np.float64)
    Q = np.asarray(omega, dtype=np.float64)
    if its == 0:
        return qr_renorm(Q)
    for it in range(1, its + 1):
        Q = A.matmul(Q) if hasattr(A, "matmul") else A @ Q
        Q = lu_renorm(Q) if it < its else qr_renorm(Q)
    return Q


def shift0(B1, n, u_A):
    """Initial Nystrom shift nu = sqrt(n) * u_A * ||B1||_F."""
    return float(np.sqrt(n) * u_A * np.linalg.norm(B1))


def eig_psd(A, k, l, its, omega, u_A=2.0 ** -24, max_retries=10, A_range=None):
    """Rank-k approximation U diag(lam) U^T of the PSD matrix A.

    ``A_range`` (optional) is what the range finder applies instead of A (an
    array, or the precision form's low-precision copy with its rounded
    operand, see ``oracle.precision``); B1 = A Q always uses A.  ``u_A`` is
    the unit roundoff of the product B1 = A Q that the shift has to dominate.
    Returns (U n x k, lam length k, nu used, retries).
    Raises np.linalg.LinAlgError if the shifted B2 is never positive definite.
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[0]
    if A.shape != (n, n):
        raise ValueError("A must be square")
    if not (1 <= k <= l <= n):
        raise ValueError("need 1 <= k <= l <= n")
    Q = range_psd(A if A_range is None else A_range, l, its, omega)
    B1 = A @ Q                                   # (start)
    nu = shift0(B1, n, u_A)
    for retry in range(max_retries + 1):
        B1nu = B1 + nu * Q                       # (A + nu I) Q
        B2 = Q.T @ B1nu                          # (second)
        B2 = 0.5 * (B2 + B2.T)
        try:
            C = sla.cholesky(B2, lower=False)    # (Cholesky): C* C = B2
            break
        except np.linalg.LinAlgError:
            if retry == max_retries:
                raise
            nu *= 10.0
    # (pseudo): F = B1 C^-1, i.e. solve F C = B1_nu.
    F = sla.solve_triangular(C, B1nu.T, trans="T", lower=False).T
    U, S, _ = np.linalg.svd(F, full_matrices=False)
    lam = np.maximum(S ** 2 - nu, 0.0)            # (finish), then remove the shift
    U = sign_fix(U[:, :k])
    return U, lam[:k], nu, retry


def eig_psd_sqrt(A, k, l, its, omega, rcond=1e-13, u_A=None):
    """The self-adjoint square-root form of Section 3 (no shift).

    C = B2^(1/2) from the eigendecomposition of B2, F = B1 C^+ with the
    pseudoinverse regularized by discarding the eigenvalues below
    rcond * max, or, when ``u_A`` is given, below the shift's scale
    sqrt(n) u_A ||B1||_F (the size of the rounding B2 carries when B1 = A Q is
    computed with unit roundoff u_A).
    """
    A = np.asarray(A, dtype=np.float64)
    Q = range_psd(A, l, its, omega)
    B1 = A @ Q
    B2 = Q.T @ B1
    B2 = 0.5 * (B2 + B2.T)
    w, X = np.linalg.eigh(B2)
    if u_A is None:
        keep = w > rcond * max(w.max(), 0.0)
    else:
        keep = w > shift0(B1, A.shape[0], u_A)
    Cpinv = (X[:, keep] / np.sqrt(w[keep])) @ X[:, keep].T
    F = B1 @ Cpinv
    U, S, _ = np.linalg.svd(F, full_matrices=False)
    U = sign_fix(U[:, :k])
    return U, (S ** 2)[:k]


def eig_sym(A, k, l, its, omega, A_range=None):
    """Rayleigh-Ritz eigenpairs of a general self-adjoint A.

    Q from the self-adjoint core loop of Section 5, B2 = Q* A Q (symmetrized)
    = W diag(lambda) W*, U = Q W; the k eigenvalues largest in magnitude
    (signed, ordered by |lambda| descending), each eigenvector signed so that
    its largest-magnitude entry is positive.  Returns (U n x k, lambda k).
    """
    A = np.asarray(A, dtype=np.float64)
    Q = range_psd(A if A_range is None else A_range, l, its, omega)
    B2 = Q.T @ (A @ Q)
    B2 = 0.5 * (B2 + B2.T)
    lam, W = np.linalg.eigh(B2)
    order = np.argsort(-np.abs(lam), kind="stable")[:k]
    U = sign_fix(Q @ W[:, order])
    return U, lam[order]
