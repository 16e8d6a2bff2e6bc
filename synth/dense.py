"""Dense test matrices with known singular values.

Construction (the paper's Section 7): A = U Sigma V^T where U and V come from
orthonormalizing i.i.d. N(0,1) vectors (Gram-Schmidt, or equivalently the Q
factor of a QR decomposition whose R has a positive diagonal), and Sigma holds
the prescribed singular values.  Only the thin factors are formed
(U is m x r, V is n x r with r = min(m, n)).

Host generation uses NumPy's PCG64 in float64; device generation (for the
large workloads) uses torch's generator on the device and CholeskyQR2 in
float64, which yields the same positive-diagonal QR factor up to rounding.
Either way A is rounded once to float32, and that float32 matrix is what both
the library and the oracle see.
"""

import numpy as np

# --------------------------------------------------------------------------
# spectra
# --------------------------------------------------------------------------


def spectrum_small(r):
    """sigma_j = 1/j for j <= 10, then 1e-2 * exp(-(j - 11)/50)   (1000 x 500 workload)."""
    j = np.arange(1, r + 1, dtype=np.float64)
    return np.where(j <= 10, 1.0 / j, 1e-2 * np.exp(-(j - 11) / 50.0))


def spectrum_tall(r):
    """sigma_j = 1/j for j <= 50, then 1e-3 * exp(-(j - 51)/200)  (100000 x 4000 and
    200000 x 8000 workloads)."""
    j = np.arange(1, r + 1, dtype=np.float64)
    return np.where(j <= 50, 1.0 / j, 1e-3 * np.exp(-(j - 51) / 200.0))


def spectrum_power(r, p=1.5):
    """sigma_j = j^-p (dense half of the batched workload)."""
    return np.arange(1, r + 1, dtype=np.float64) ** (-p)


def spectrum_exp(r, scale=10.0):
    """lambda_j = exp(-j/scale) (PSD half of the batched workload)."""
    return np.exp(-np.arange(1, r + 1, dtype=np.float64) / scale)


def spectrum_paper(which, k, r, rng=None):
    """The six spectra of the paper's dense tests (Section 7), S1 .. S6.

    S2-S5 have ||A|| = 1 and sigma_{k+1} = 1e-5; S4 is rank k+1; S6 is the
    absolute values of i.i.d. N(0,1) draws (needs ``rng``), sorted descending.
    """
    j = np.arange(1, r + 1, dtype=np.float64)
    if which == 1:
        return 1.0 / j
    if which == 2:
        s = np.where(j == 1, 1.0, 2e-5)
        return np.where(j <= k, s, 1e-5 * (k + 1) / j)
    if which == 3:
        return np.where(j <= k, 10.0 ** (-5.0 * (j - 1) / (k - 1)), 1e-5 * (k + 1) / j)
    if which == 4:
        s = np.where(j <= k, 10.0 ** (-5.0 * (j - 1) / (k - 1)), 0.0)
        return np.where(j == k + 1, 1e-5, s)
    if which == 5:
        return np.where(j <= k, 1e-5 + (1 - 1e-5) * (k - j) / (k - 1),
                        1e-5 * np.sqrt((k + 1) / j))
    if which == 6:
        if rng is None:
            raise ValueError("S6 needs an rng")
        return np.sort(np.abs(rng.standard_normal(r)))[::-1].copy()
    raise ValueError(which)


def propack_diag(size, rank_ones=3, rank_999=17):
    """diag(1, 1, 1, .999 x 17, 0, ...): the matrices of the paper's Section 6."""
    d = np.zeros(size)
    d[:rank_ones] = 1.0
    d[rank_ones:rank_ones + rank_999] = 0.999
    return np.diag(d)


# --------------------------------------------------------------------------
# host (NumPy) construction
# --------------------------------------------------------------------------


def haar(m, r, rng):
    """m x r matrix with orthonormal columns: Q of a Gaussian with diag(R) > 0."""
    G = rng.standard_normal((m, r))
    Q, R = np.linalg.qr(G, mode="reduced")
    return Q * np.sign(np.diag(R))


def dense(m, n, sigma, seed, dtype=np.float32, return_factors=False):
    """A = U diag(sigma) V^T, rounded to ``dtype``.

    sigma has length min(m, n).  Returns A (and (U, sigma, V) in float64 if
    ``return_factors``).
    """
    r = min(m, n)
    sigma = np.asarray(sigma, dtype=np.float64)
    if sigma.shape != (r,):
        raise ValueError("sigma must have length min(m, n)")
    rng = np.random.default_rng(seed)
    U = haar(m, r, rng)
    V = haar(n, r, rng)
    A = ((U * sigma) @ V.T).astype(dtype)
    if return_factors:
        return A, (U, sigma, V)
    return A


def psd(n, lam, seed, dtype=np.float32):
    """Symmetric PSD A = V diag(lam) V^T, exactly symmetric after rounding."""
    lam = np.asarray(lam, dtype=np.float64)
    rng = np.random.default_rng(seed)
    V = haar(n, n, rng)
    A = (V * lam) @ V.T
    A = 0.5 * (A + A.T)
    return A.astype(dtype)


def centered_spectrum(U, sigma):
    """Exact singular values of (I - 1 1^T/m) U diag(sigma) V^T.

    With P = I - 1 1^T/m (a projector), A_c^T A_c = V (Sigma^2 - w w^T) V^T
    where w = Sigma U^T 1 / sqrt(m): a rank-one downdate of Sigma^2.
    Returns the singular values in descending order.
    """
    U = np.asarray(U, dtype=np.float64)
    m = U.shape[0]
    w = sigma * U.sum(axis=0) / np.sqrt(m)
    M = np.diag(sigma ** 2) - np.outer(w, w)
    ev = np.linalg.eigvalsh(M)[::-1]
    return np.sqrt(np.maximum(ev, 0.0))


# --------------------------------------------------------------------------
# device (torch) construction for the large workloads
# --------------------------------------------------------------------------


def _cholqr2_torch(G, chunk=16384):
    """Q of G = Q R with diag(R) > 0, by Cholesky QR twice (G well conditioned)."""
    import torch
    for _ in range(2):
        R = torch.linalg.cholesky(G.T @ G, upper=True)
        if R.shape[0] > 4096:
            # the device triangular solve's workspace allocation fails at
            # this order; the r x r inverse is cheap on the host
            Rh = R.cpu()
            Rinv = torch.linalg.solve_triangular(Rh, torch.eye(R.shape[0], dtype=G.dtype),
                                                 upper=True).to(G.device)
        else:
            eye = torch.eye(R.shape[0], device=G.device, dtype=G.dtype)
            Rinv = torch.linalg.solve_triangular(R, eye, upper=True)
        for i in range(0, G.shape[0], chunk):
            G[i:i + chunk] = G[i:i + chunk] @ Rinv
    return G


def dense_torch(m, n, sigma, seed, device, center_spectrum=False):
    """Device construction of A = U diag(sigma) V^T in float64, returned as float32.

    U and V are the positive-diagonal Q factors of Gaussian matrices drawn
    with torch's device generator (seeded), computed by CholeskyQR2 in
    float64.  Returns (A float32 tensor on ``device``, sigma float64 numpy,
    centered singular values or None).
    """
    import torch
    r = min(m, n)
    sig = torch.as_tensor(np.asarray(sigma, dtype=np.float64), device=device)
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    V = _cholqr2_torch(torch.randn(n, r, generator=gen, device=device, dtype=torch.float64))
    U = _cholqr2_torch(torch.randn(m, r, generator=gen, device=device, dtype=torch.float64))
    csig = None
    if center_spectrum:
        # the r x r eigenproblem runs on the host (NumPy), not the device
        w = (sig * U.sum(dim=0) / np.sqrt(m)).cpu().numpy()
        s = np.asarray(sigma, dtype=np.float64)
        ev = np.linalg.eigvalsh(np.diag(s * s) - np.outer(w, w))[::-1]
        csig = np.sqrt(np.maximum(ev, 0.0))
    U.mul_(sig)
    A = torch.empty(m, n, device=device, dtype=torch.float32)
    step = 16384
    for i in range(0, m, step):
        A[i:i + step] = (U[i:i + step] @ V.T).to(torch.float32)
    del U, V
    return A, np.asarray(sigma, dtype=np.float64), csig


def psd_torch(n, lam, seed, device):
    """Device construction of the symmetric PSD A = V diag(lam) V^T (Haar V: the
    Householder QR of a square Gaussian in float64, columns signed so that
    diag(R) > 0), returned as float32, exactly symmetric."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    G = torch.randn(n, n, generator=gen, device=device, dtype=torch.float64)
    V, R = torch.linalg.qr(G)
    d = torch.sign(torch.diagonal(R))
    d[d == 0] = 1.0
    V = V * d
    lam = torch.as_tensor(np.asarray(lam, dtype=np.float64), device=device)
    A = (V * lam) @ V.T
    A = 0.5 * (A + A.T)
    return A.to(torch.float32)


def batch_params(count_dense=256, count_psd=256, seed=5000):
    """Shapes and ranks of the batched workload: dense problems with
    m ~ logU[256, 8192], n ~ logU[64, 2048], sigma_j = j^-1.5; PSD problems with
    n ~ logU[128, 4096], lambda_j = exp(-j/10); k ~ U{5..40}, l = k + 5, its = 2.
    Problem p is built with seed 10000 + p and solved with seed 20000 + p."""
    rng = np.random.default_rng(seed)
    out = []
    for p in range(count_dense + count_psd):
        k = int(rng.integers(5, 41))
        if p < count_dense:
            m = int(np.exp(rng.uniform(np.log(256), np.log(8192))))
            n = int(np.exp(rng.uniform(np.log(64), np.log(2048))))
            out.append(dict(kind="svd", m=m, n=max(n, k + 5), k=k, l=k + 5, its=2,
                            seed_A=10000 + p, seed=20000 + p))
        else:
            n = int(np.exp(rng.uniform(np.log(128), np.log(4096))))
            out.append(dict(kind="psd", m=n, n=n, k=k, l=k + 5, its=2, seed_A=10000 + p,
                            seed=20000 + p))
    return out


# --------------------------------------------------------------------------
# the rank-4 experiment of the paper's Section 7
# --------------------------------------------------------------------------


def noisy_gaussian(n, seed, dtype=np.float32):
    """n x n matrix of i.i.d. N(sqrt(30/n), 1) entries with the sign of entry
    (i, j) flipped when i*j is odd (1-based i, j), as in the paper's Section 7:
    two singular values about twice as large as the rest."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) + np.sqrt(30.0 / n)
    odd = (np.arange(1, n + 1) % 2 == 1)
    A[np.ix_(odd, odd)] *= -1.0
    return A.astype(dtype)


def noisy_gaussian_torch(n, seed, device, chunk=4096):
    """The same law on the device (torch's generator, float32, built in row
    blocks): for n up to 10^5 (40 GB)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    A = torch.empty(n, n, device=device, dtype=torch.float32)
    mu = float(np.sqrt(30.0 / n))
    sgn_col = torch.ones(n, device=device, dtype=torch.float32)
    sgn_col[0::2] = -1.0  # 1-based odd columns
    for i in range(0, n, chunk):
        r = min(chunk, n - i)
        blk = torch.randn(r, n, generator=gen, device=device, dtype=torch.float32) + mu
        rows_odd = torch.arange(i, i + r, device=device) % 2 == 0  # 1-based odd rows
        blk[rows_odd] *= sgn_col
        A[i:i + r] = blk
    return A
