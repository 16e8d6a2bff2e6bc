"""Parity of the precision form at its full size: 200000 x 8000 (sigma_j = 1/j
for j <= 50, then 1e-3 exp(-(j - 51)/200)), k = 100, l = 120, its = 3.

The float32 A is built on the device; its bfloat16 copy and its E4M3 copy
with per-column scales (rpca_quantize) feed the range finder, the float32 A
the Rayleigh-Ritz product.  The FP64 oracle runs the same algorithm on the
host with the same Gaussian test matrix and the same low-precision products
(the stored values times the operand rounded to bfloat16,
``oracle.precision.LowPrecisionA``), and the float32 A for B = Q* A.  The
two then differ only by float32 accumulation and renormalization rounding,
as the float32 path does:
  * bfloat16: singular values within 1e-4 relative of the oracle's, the
    unconverged tail (sigma_k / sigma_{l+1} = 1.16) included;
    ||A - U S V^T||_2 (exact, float64) within 1.1 sigma_{k+1}
    (sigma_{k+1} = 1e-3 e^-(50/200) exactly: A is not centered);
  * E4M3: the converged singular values (sigma_j = 1/j, j <= 50) within 1e-4
    of the oracle's.  The tail is parity unpinned: E4M3's 2^-4 rounding puts
    a noise floor of about 1.4 sigma_{k+1} under A's tail, the Ritz values
    there are 15-60% below the exact sigma_j and move with float32-level
    differences of the sketch.  They must obey Cauchy interlacing against the
    float32 A (sigma~_j <= sigma_j + u ||A||_F) and stay within 5% of
    the oracle's own distance below sigma_j; no error bound is claimed;
  * U and V orthonormal.
"""

import numpy as np
import pytest
import torch

from bench import exact_residual_norm
from oracle import philox, precision, rsvd
from synth import dense

pytestmark = pytest.mark.gpu

M, N, K, L, ITS, SEED, A_SEED = 200000, 8000, 100, 120, 3, 2003, 1003


@pytest.fixture(scope="module")
def workload(gpu_lib):
    sig = dense.spectrum_tall(N)
    A, _, _ = dense.dense_torch(M, N, sig, seed=A_SEED, device="cuda")
    torch.cuda.synchronize()
    return dict(ctx=gpu_lib.Context(), lib=gpu_lib, A=A, Ah=A.cpu().numpy(), sig=sig,
                om=philox.omega(SEED, N, L))


def _orth_err(X):
    X = X.astype(np.float64)
    return np.linalg.norm(X.T @ X - np.eye(X.shape[1]), 2)


@pytest.mark.parametrize("kind", ["bf16", "fp8"])
def test_fullsize_lowp(workload, kind):
    w = workload
    ctx = w["ctx"]
    q, s = ctx.quantize(w["A"], kind)
    mat = w["lib"].dense(q, col_scale=s, A_f32=w["A"])
    U, S, V = ctx.svd(q, K, L, ITS, SEED, sync=True, mat=mat)
    Sh = S.cpu().numpy()
    if kind == "bf16":
        op = precision.LowPrecisionA(
            precision.from_bf16_bits(q.view(torch.int16).cpu().numpy().view(np.uint16)))
    else:
        op = precision.LowPrecisionA(precision.e4m3_decode(q.view(torch.uint8).cpu().numpy()),
                                     s.cpu().numpy())
    _, S0, _ = rsvd.rsvd(w["Ah"], K, L, ITS, w["om"], A_range=op)
    del op
    rel = np.abs(Sh - S0) / S0
    lead = w["sig"][:K] > 1e-2  # sigma_j = 1/j, j <= 50: well separated, converged
    print("%s: max rel sigma diff %.2e (j <= 50), %.2e (tail; worst j = %s)"
          % (kind, rel[lead].max(), rel[~lead].max(), np.argsort(rel)[-3:] + 1), flush=True)
    np.testing.assert_allclose(Sh[lead], S0[lead], rtol=1e-4)
    if kind == "bf16":
        np.testing.assert_allclose(Sh, S0, rtol=1e-4)
    else:
        sig = w["sig"][:K]
        assert np.all(Sh <= sig + 1e-7)  # interlacing; u ||A||_F < 8e-8 covers the rounding of A
        gap = sig - S0
        band = np.abs(Sh - S0)[~lead] / gap[~lead]
        print("fp8 tail: |gpu - oracle| / (sigma_j - oracle) max %.3g" % band.max(), flush=True)
        assert np.all(np.abs(Sh - S0)[~lead] <= 0.05 * gap[~lead] + 1e-4 * S0[~lead])
    assert _orth_err(U.cpu().numpy()) < 1e-4
    assert _orth_err(V.cpu().numpy()) < 1e-4
    err = exact_residual_norm(w["A"], U, S, V)
    print("%s: err / sigma_{k+1} = %.5f (exact)" % (kind, err / w["sig"][K]), flush=True)
    assert err >= w["sig"][K] * (1 - 1e-4)  # Eckart-Young, less the float32 rounding of A
    if kind == "bf16":
        assert err <= 1.1 * w["sig"][K]
