"""The seeded input generators produce the spectra they claim."""

import numpy as np
import pytest

from synth import dense


@pytest.mark.parametrize("m,n", [(120, 50), (50, 120)])
def test_dense_spectrum(m, n):
    sig = dense.spectrum_small(min(m, n))
    A = dense.dense(m, n, sig, seed=1)
    assert A.dtype == np.float32
    s = np.linalg.svd(A.astype(np.float64), compute_uv=False)
    np.testing.assert_allclose(s, sig, atol=1e-6)
    A2 = dense.dense(m, n, sig, seed=1)
    np.testing.assert_array_equal(A, A2)


def test_spectra_shapes_and_paper_properties():
    k, r = 10, 100
    for w in (2, 3, 4, 5):
        s = dense.spectrum_paper(w, k, r)
        assert s[0] == pytest.approx(1.0) and s[k] == pytest.approx(1e-5)
        assert np.all(np.diff(s) <= 1e-18)
    assert np.all(dense.spectrum_paper(4, k, r)[k + 1:] == 0)
    t = dense.spectrum_tall(4000)
    assert t[49] == pytest.approx(1 / 50) and t[50] == pytest.approx(1e-3)
    sm = dense.spectrum_small(500)
    assert sm[9] == pytest.approx(0.1) and sm[10] == pytest.approx(1e-2)


def test_centered_spectrum_closed_form():
    m, n = 400, 30
    sig = dense.spectrum_tall(n)
    A, (U, s, V) = dense.dense(m, n, sig, seed=2, dtype=np.float64, return_factors=True)
    want = np.linalg.svd(A - A.mean(axis=0), compute_uv=False)
    np.testing.assert_allclose(dense.centered_spectrum(U, s), want, rtol=1e-10, atol=1e-14)


def test_psd_symmetric():
    lam = dense.spectrum_exp(50)
    A = dense.psd(50, lam, seed=3)
    np.testing.assert_array_equal(A, A.T)
    w = np.linalg.eigvalsh(A.astype(np.float64))[::-1]
    np.testing.assert_allclose(w, lam, atol=1e-6)


def test_torch_construction_on_cpu():
    torch = pytest.importorskip("torch")
    m, n = 300, 40
    sig = dense.spectrum_tall(n)
    A, s, cs = dense.dense_torch(m, n, sig, seed=5, device="cpu", center_spectrum=True)
    A64 = A.double().numpy()
    np.testing.assert_allclose(np.linalg.svd(A64, compute_uv=False), sig, atol=1e-6)
    want = np.linalg.svd(A64 - A64.mean(axis=0), compute_uv=False)
    np.testing.assert_allclose(cs, want, atol=1e-6)


def test_sparse_rows_and_transpose():
    import scipy.sparse as sp
    from synth import sparse
    m, n, r = 500, 300, 10
    rp, ci, va = sparse.random_rows(m, n, r, seed=4)
    assert rp.dtype == np.int32 and ci.dtype == np.int32 and va.dtype == np.float32
    np.testing.assert_array_equal(rp, np.arange(m + 1) * r)
    cols = ci.reshape(m, r)
    assert np.all(np.diff(cols, axis=1) > 0)          # distinct, ascending
    assert cols.min() >= 0 and cols.max() < n
    A = sparse.to_scipy(m, n, rp, ci, va)
    cp, ri, vt = sparse.transpose(m, n, rp, ci, va)
    At = sp.csr_matrix((vt, ri, cp), shape=(n, m))
    assert (At - A.T).nnz == 0 or np.abs((At - A.T).toarray()).max() == 0
    # the row scale i^-1/2 on N(0,1) values: row norms shrink like sqrt(10 / i)
    norms = np.sqrt(np.asarray(A.multiply(A).sum(axis=1)).ravel())
    assert norms[:50].mean() > 3 * norms[-50:].mean()
