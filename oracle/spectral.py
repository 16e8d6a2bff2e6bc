"""Spectral-norm error of a low-rank approximation (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 4 takes the spectral norm ||A - U Sigma V*|| as the measure of
accuracy and estimates it with the power method from a random start
(Kuczynski and Wozniakowski, Theorem 4.1(a): within a factor of two with
overwhelming probability).

Readings of the paper taken here:
  * a block of b start vectors is used (subspace iteration on E* E), drawn
    from Philox stream 1 with the same Gaussian map as Omega;
  * each iteration is X <- orth(E* (E X)), where orth returns the Q factor of
    the QR decomposition whose R has a positive diagonal (unique, so any QR
    algorithm gives the same X up to rounding);
  * the estimate is the largest singular value of E X for the final
    orthonormal X, which never exceeds ||E||;
  * for a PSD approximation V = U; with centering, E = A_c - U Sigma V*.

Pins (tests/test_oracle_spectral.py): equality with the exact norm from a
full SVD when the iteration has converged; the lower-bound property; the
factor-of-two property on the paper's spectra; E = 0 for an exact
factorization.
"""

import numpy as np
import scipy.sparse as sps


def residual(A, U, S, V=None, center=False):
    """E = A (or A_c) - U diag(S) V^T as a dense float64 matrix."""
    A = np.asarray(A, dtype=np.float64)
    if center:
        A = A - A.mean(axis=0, keepdims=True)
    U = np.asarray(U, dtype=np.float64)
    V = U if V is None else np.asarray(V, dtype=np.float64)
    return A - (U * np.asarray(S, dtype=np.float64)) @ V.T


def spectral_err_exact(A, U, S, V=None, center=False):
    """||E||_2 from a full SVD of the residual."""
    return float(np.linalg.norm(residual(A, U, S, V, center), ord=2))


def orth_pos(X):
    """Q of X = Q R with diag(R) > 0."""
    Q, R = np.linalg.qr(np.asarray(X, dtype=np.float64), mode="reduced")
    d = np.sign(np.diag(R))
    d[d == 0] = 1.0
    return Q * d


def spectral_err_power(A, U, S, V, X0, iters, center=False):
    """Randomized block power estimate of ||A - U diag(S) V^T||_2.

    E is applied without being formed: E x = A x - U (S (V^T x)) and
    E^T y = A^T y - V (S (U^T y)) (with A replaced by A_c when centering).
    A may be a scipy.sparse matrix (then without centering).
    X0 is the n x b start block.
    """
    if sps.issparse(A):
        if center:
            raise ValueError("sparse A: no centering")
        A = sps.csr_matrix(A, dtype=np.float64)
    else:
        A = np.asarray(A, dtype=np.float64)
        if center:
            A = A - A.mean(axis=0, keepdims=True)
    U = np.asarray(U, dtype=np.float64)
    V = U if V is None else np.asarray(V, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)

    def E(X):
        return A @ X - U @ (S[:, None] * (V.T @ X))

    def Et(Y):
        return A.T @ Y - V @ (S[:, None] * (U.T @ Y))

    X = orth_pos(X0)
    for _ in range(iters):
        X = orth_pos(Et(E(X)))
    Y = E(X)
    G = Y.T @ Y
    return float(np.sqrt(max(np.linalg.eigvalsh(G)[-1], 0.0)))
