"""Pins for the oracle's randomized SVD (Sections 2, 5, 6 and 7 of the paper).

Each check is fixed by the mathematics or by the paper, not by the oracle:
brute force against numpy.linalg.svd, a closed form for the centered
spectrum, interlacing and Eckart-Young bounds, and span invariance of the
renormalizations.
"""

import numpy as np
import pytest

from oracle import philox, rsvd, spectral
from synth import dense


def _proj_diff(U1, U2):
    return np.linalg.norm(U1 @ U1.T - U2 @ U2.T, 2)


@pytest.mark.parametrize("m,n,its", [(60, 40, 0), (40, 60, 1), (50, 50, 2), (80, 30, 3)])
def test_full_width_sketch_is_exact_svd(m, n, its):
    # l = min(m, n): the sketch spans the whole range, so the result is the
    # exact truncated SVD.
    rng = np.random.default_rng(m * n + its)
    A = rng.standard_normal((m, n))
    l = min(m, n)
    k = l - 3
    U, S, V = rsvd.rsvd(A, k, l, its, philox.omega(9, n, l))
    U0, S0, V0t = np.linalg.svd(A)
    np.testing.assert_allclose(S, S0[:k], rtol=1e-11, atol=0)
    assert _proj_diff(U, U0[:, :k]) < 1e-9
    assert _proj_diff(V, V0t[:k].T) < 1e-9
    # sign convention: largest-magnitude entry of each U column is positive
    idx = np.argmax(np.abs(U), axis=0)
    assert np.all(U[idx, np.arange(k)] > 0)
    # U diag(S) V^T is the best rank-k approximation (Eckart-Young)
    err = spectral.spectral_err_exact(A, U, S, V)
    assert abs(err - S0[k]) < 1e-10 * S0[0]


@pytest.mark.parametrize("size,k", [(30, 20), (30, 21), (100, 50)])
def test_propack_diagonal_matrices(size, k):
    # Section 6: diag(1,1,1,.999 x 17, 0, ...).  rank 20 <= l = k + 2, so the
    # randomized method must return the exact values 1, .999 and 0.
    A = dense.propack_diag(size)
    l = k + 2
    U, S, V = rsvd.rsvd(A, k, l, 2, philox.omega(size + k, size, l))
    want = np.diag(A)[:k]
    np.testing.assert_allclose(S, want, atol=1e-12)
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-12)
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-12)
    # the top-20 left singular subspace is span(e_1 .. e_20)
    r = min(k, 20)
    P = U[:, :r] @ U[:, :r].T
    E = np.zeros((size, size))
    E[np.arange(20), np.arange(20)] = 1.0
    assert np.linalg.norm(P - E, 2) < 1e-9
    assert spectral.spectral_err_exact(A, U, S, V) < 1e-12


def test_centered_pca_matches_closed_form():
    # PCA after subtracting the column means (Section 2).  With l = n the
    # result is exact, and the singular values of the centered construction
    # follow from a rank-one downdate (synth.dense.centered_spectrum).
    m, n = 300, 40
    sig = dense.spectrum_small(n)
    A, (U0, s0, V0) = dense.dense(m, n, sig, seed=4, dtype=np.float64, return_factors=True)
    A = A + 0.3  # a nonzero mean in every column
    want = np.linalg.svd(A - A.mean(axis=0), compute_uv=False)
    U, S, V = rsvd.rsvd(A, 10, n, 1, philox.omega(1, n, n), center=True)
    np.testing.assert_allclose(S, want[:10], rtol=1e-11)
    # closed form for the unshifted construction
    A2, (U2, s2, V2) = dense.dense(m, n, sig, seed=5, dtype=np.float64, return_factors=True)
    cs = dense.centered_spectrum(U2, s2)
    _, S2, _ = rsvd.rsvd(A2, 10, n, 0, philox.omega(2, n, n), center=True)
    np.testing.assert_allclose(S2, cs[:10], rtol=1e-11)
    # centering changes the answer (guards against a dropped centering step)
    _, S3, _ = rsvd.rsvd(A, 10, n, 1, philox.omega(1, n, n), center=False)
    assert abs(S3[0] - S[0]) > 1e-3


@pytest.mark.parametrize("m,n", [(200, 120), (120, 200)])
def test_lu_and_householder_renormalization_agree(m, n):
    # Every renormalization multiplies by an invertible l x l matrix, so the
    # final result depends only on the sketched span.
    k, l, its = 8, 12, 3
    sig = dense.spectrum_paper(1, k, min(m, n))
    A = dense.dense(m, n, sig, seed=7, dtype=np.float64)
    om = philox.omega(8, n, l)
    U1, S1, V1 = rsvd.rsvd(A, k, l, its, om, renorm="lu")
    U2, S2, V2 = rsvd.rsvd(A, k, l, its, om, renorm="qr")
    np.testing.assert_allclose(S1, S2, rtol=1e-10)
    np.testing.assert_allclose(U1, U2, atol=1e-8)
    np.testing.assert_allclose(V1, V2, atol=1e-8)


def test_lu_renorm_properties():
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((50, 6))
    Q = rsvd.lu_renorm(Y)
    # permuted unit lower trapezoidal with |L| <= 1, same span as Y
    assert np.max(np.abs(Q)) <= 1.0 + 1e-15
    piv = [int(np.argmax(np.abs(Q[:, j]) == 1.0)) for j in range(6)]
    assert len(set(piv)) == 6
    R = np.linalg.lstsq(Q, Y, rcond=None)[0]
    assert np.linalg.norm(Q @ R - Y) < 1e-12 * np.linalg.norm(Y)
    # zero column: a zero pivot keeps a unit vector in L
    Y[:, 2] = 0.0
    Q = rsvd.lu_renorm(Y)
    assert np.linalg.matrix_rank(Q) == 6


@pytest.mark.parametrize("which", [1, 2, 3, 4, 5, 6])
@pytest.mark.parametrize("m,n,k", [(200, 100, 10), (100, 200, 10)])
def test_paper_spectra_near_optimal(which, m, n, k):
    # Section 7: with l = k + 2 and its = 2 the error is close to the best
    # possible, sigma_{k+1}; interlacing bounds every computed value.
    r = min(m, n)
    sig = dense.spectrum_paper(which, k, r, rng=np.random.default_rng(which))
    A = dense.dense(m, n, sig, seed=100 + which, dtype=np.float64)
    s_true = np.sort(sig)[::-1]
    U, S, V = rsvd.rsvd(A, k, k + 2, 2, philox.omega(which, n, k + 2))
    err = spectral.spectral_err_exact(A, U, S, V)
    assert err >= s_true[k] * (1 - 1e-9)           # Eckart-Young
    assert err <= 1.2 * s_true[k]
    assert np.all(S <= s_true[:k] * (1 + 1e-10) + 1e-15)   # Cauchy interlacing
    np.testing.assert_allclose(U.T @ U, np.eye(k), atol=1e-12)
    np.testing.assert_allclose(V.T @ V, np.eye(k), atol=1e-12)


def test_power_iterations_matter():
    # Section 7, rank-4 approximation of a noisy n x n Gaussian with mean
    # sqrt(30/n) and signs flipped where i*j is odd: its = 0 is much worse
    # than its = 2, and the best error is about half the norm.
    n, k = 400, 4
    rng = np.random.default_rng(11)
    A = rng.standard_normal((n, n)) + np.sqrt(30.0 / n)
    i = np.arange(1, n + 1)
    A[np.outer(i, i) % 2 == 1] *= -1.0
    s = np.linalg.svd(A, compute_uv=False)
    errs = {}
    for its in (0, 2):
        U, S, V = rsvd.rsvd(A, k, k + 2, its, philox.omega(12, n, k + 2))
        errs[its] = spectral.spectral_err_exact(A, U, S, V) / s[k]
    assert 0.35 < s[k] / s[0] < 0.65
    assert errs[2] < 1.1
    assert errs[0] > errs[2] * 1.2


def test_argument_checks():
    A = np.ones((5, 4))
    with pytest.raises(ValueError):
        rsvd.rsvd(A, 3, 2, 1, np.ones((4, 2)))
    with pytest.raises(ValueError):
        rsvd.rsvd(A, 2, 5, 1, np.ones((4, 5)))


def test_range_matrix_enters_only_through_its_span():
    # A_range = c A has the span of A at every step, so the result equals the
    # plain one; a perturbed A_range changes only the range finder
    rng = np.random.default_rng(31)
    A = dense.dense(300, 120, dense.spectrum_small(120), seed=31)
    om = philox.omega(5, 120, 14)
    U0, S0, V0 = rsvd.rsvd(A, 10, 14, 2, om)
    U1, S1, V1 = rsvd.rsvd(A, 10, 14, 2, om, A_range=3.0 * A.astype(np.float64))
    np.testing.assert_allclose(S1, S0, rtol=1e-12)
    np.testing.assert_allclose(np.abs(U1.T @ U0), np.eye(10), atol=1e-9)
    Ap = A + 1e-9 * rng.standard_normal(A.shape)
    U2, S2, V2 = rsvd.rsvd(A, 10, 14, 2, om, A_range=Ap, center=True)
    U3, S3, V3 = rsvd.rsvd(A, 10, 14, 2, om, center=True)
    np.testing.assert_allclose(S2, S3, rtol=1e-6)
    # the Rayleigh-Ritz values are those of Q* A for the float A: interlacing holds
    Ad = A.astype(np.float64)
    s_true = np.linalg.svd(Ad - Ad.mean(axis=0), compute_uv=False)
    assert np.all(S2 <= s_true[:10] * (1 + 1e-12))


def test_sparse_input_equals_dense_definition():
    import scipy.sparse as sps
    from synth import sparse
    m, n = 400, 250
    rp, ci, va = sparse.random_rows(m, n, 8, seed=12)
    A = sparse.to_scipy(m, n, rp, ci, va)
    om = philox.omega(3, n, 16)
    U0, S0, V0 = rsvd.rsvd(A.toarray(), 10, 16, 3, om)
    U1, S1, V1 = rsvd.rsvd(A, 10, 16, 3, om)
    np.testing.assert_allclose(S1, S0, rtol=1e-12)
    np.testing.assert_allclose(U1, U0, atol=1e-9)
    est0 = spectral.spectral_err_power(A.toarray(), U0, S0, V0, philox.omega(1, n, 4, stream=1), 5)
    est1 = spectral.spectral_err_power(A, U1, S1, V1, philox.omega(1, n, 4, stream=1), 5)
    assert est1 == pytest.approx(est0, rel=1e-10)
    with pytest.raises(ValueError):
        rsvd.rsvd(A, 10, 16, 3, om, center=True)
    assert sps.issparse(A)


# ---- renormalizing only after every second application (Section 5) ----------


@pytest.mark.parametrize("m,n,its", [(60, 40, 1), (40, 60, 2), (80, 30, 3)])
def test_fused_full_width_sketch_is_exact_svd(m, n, its):
    # l = min(m, n): whatever the renormalization schedule, the sketch spans
    # the whole range and the result is the exact truncated SVD
    rng = np.random.default_rng(m + n + its)
    A = rng.standard_normal((m, n))
    l = min(m, n)
    k = l - 3
    U, S, V = rsvd.rsvd(A, k, l, its, philox.omega(4, n, l), fused=True)
    U0, S0, V0t = np.linalg.svd(A)
    np.testing.assert_allclose(S, S0[:k], rtol=1e-11)
    assert _proj_diff(U, U0[:, :k]) < 1e-9
    assert _proj_diff(V, V0t[:k].T) < 1e-9


@pytest.mark.parametrize("center", [False, True])
@pytest.mark.parametrize("its", [1, 2, 3])
@pytest.mark.parametrize("m,n", [(300, 120), (120, 300)])
def test_fused_spans_the_same_krylov_range(m, n, its, center):
    # A (A* A)^its Omega = (A A*)^its A Omega: in exact arithmetic the fused
    # schedule sketches the same range as renormalizing after every
    # application, so on a moderately graded spectrum (where float64 loses
    # nothing by squaring) the results agree with the standard path's, for
    # centered A too (a centering dropped from either product of A* A would
    # change the range)
    k, l = 8, 12
    sig = dense.spectrum_small(min(m, n))
    A = dense.dense(m, n, sig, seed=41, dtype=np.float64) + 0.05
    om = philox.omega(6, n, l)
    for renorm in ("lu", "qr"):
        U0, S0, V0 = rsvd.rsvd(A, k, l, its, om, center=center, renorm=renorm)
        U1, S1, V1 = rsvd.rsvd(A, k, l, its, om, center=center, renorm=renorm, fused=True)
        np.testing.assert_allclose(S1, S0, rtol=1e-9)
        np.testing.assert_allclose(U1, U0, atol=1e-7)
        np.testing.assert_allclose(V1, V0, atol=1e-7)
    # its = 0 is the plain sketch, identical either way
    a = rsvd.rsvd(A, k, l, 0, om, center=center)
    b = rsvd.rsvd(A, k, l, 0, om, center=center, fused=True)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


def test_fused_schedule_costs_accuracy_on_a_wide_spectrum():
    # Section 5 says the fused schedule gives up some accuracy.  Singular
    # values 1, 0.1, ..., 1e-9 over a flat tail at 1e-10: after A* A the
    # tenth direction sits at 1e-18 of the first, below float64's rounding of
    # the product, so the unrenormalized product loses it, while
    # renormalizing after every application keeps it (ratios of 1e-9 at most).
    m, n, r, k, l = 200, 150, 10, 10, 12
    sig = np.full(n, 1e-10)
    sig[:r] = 10.0 ** (-np.arange(r))
    A = dense.dense(m, n, sig, seed=17, dtype=np.float64)
    om = philox.omega(7, n, l)
    U0, S0, V0 = rsvd.rsvd(A, k, l, 2, om)
    U1, S1, V1 = rsvd.rsvd(A, k, l, 2, om, fused=True)
    assert spectral.spectral_err_exact(A, U0, S0, V0) < 1.01 * sig[k]
    np.testing.assert_allclose(S0, sig[:k], rtol=1e-6)
    assert spectral.spectral_err_exact(A, U1, S1, V1) > 3.0 * sig[k]
    assert abs(S1[-1] - sig[k - 1]) > 0.05 * sig[k - 1]
    # the leading values are still right
    np.testing.assert_allclose(S1[:5], sig[:5], rtol=1e-8)
