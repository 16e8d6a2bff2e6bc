"""rpca_svd_noalloc (working memory from a static device array, no allocation)
against rpca_svd: the same kernels in the same configuration, so the results
are bit-identical; two calls in a row, the second on a smaller problem (the
array keeps the first call's contents), a sparse problem, and a problem too
large for the array (RPCA_ERR_NO_MEMORY before any launch, outputs untouched).
Called through the C ABI with ctypes."""

import ctypes

import numpy as np
import pytest
import torch

from synth import dense

pytestmark = pytest.mark.gpu

DETERMINISTIC, CENTER, SYNC = 4, 1, 2


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _call(rp, ctx, fn, A, k, l, its, seed, flags, mat=None):
    m, n = A.shape if mat is None else (mat.m, mat.n)
    mat = rp.dense(A) if mat is None else mat
    U = torch.full((m, k), -3.0, device="cuda")
    S = torch.full((k,), -3.0, device="cuda", dtype=torch.float64)
    V = torch.full((n, k), -3.0, device="cuda")
    st = getattr(ctx.lib, fn)(ctx.h, ctypes.byref(mat), k, l, its, seed, flags, _ptr(U), k,
                              _ptr(S), _ptr(V), k)
    torch.cuda.synchronize()
    return st, U, S, V


@pytest.mark.parametrize("center", [False, True])
def test_noalloc_matches_svd(gpu_lib, center):
    ctx = gpu_lib.Context()
    flags = DETERMINISTIC | SYNC | (CENTER if center else 0)
    cases = [(20000, 1000, 50, 60, 2, 11), (3000, 700, 10, 12, 1, 12)]  # then a smaller one
    for m, n, k, l, its, seed in cases:
        A = torch.from_numpy(dense.dense(m, n, dense.spectrum_tall(n), seed=m + n)).cuda()
        s0, U0, S0, V0 = _call(gpu_lib, ctx, "rpca_svd", A, k, l, its, seed, flags)
        s1, U1, S1, V1 = _call(gpu_lib, ctx, "rpca_svd_noalloc", A, k, l, its, seed, flags)
        assert s0 == 0 and s1 == 0, ctx.lib.rpca_last_error(ctx.h)
        assert torch.equal(S0, S1) and torch.equal(U0, U1) and torch.equal(V0, V1)
    ctx.close()


def test_noalloc_sparse_and_too_large(gpu_lib):
    from synth import sparse
    ctx = gpu_lib.Context()
    m, n = 30000, 20000
    rptr, ci, va = sparse.random_rows(m, n, 10, 5)
    cptr, ri, vt = sparse.transpose(m, n, rptr, ci, va)
    S = gpu_lib.csr(m, n, *[torch.from_numpy(a).cuda() for a in (rptr, ci, va, cptr, ri, vt)])
    r0 = _call(gpu_lib, ctx, "rpca_svd", None, 10, 16, 2, 3, DETERMINISTIC | SYNC, mat=S.mat)
    r1 = _call(gpu_lib, ctx, "rpca_svd_noalloc", None, 10, 16, 2, 3, DETERMINISTIC | SYNC,
               mat=S.mat)
    assert r0[0] == 0 and r1[0] == 0
    assert all(torch.equal(a, b) for a, b in zip(r0[1:], r1[1:]))
    # 1,000,000 x 64 at l = 64 needs far more than 64 MiB
    A = torch.zeros(1000000, 64, device="cuda")
    st, U, Sv, V = _call(gpu_lib, ctx, "rpca_svd_noalloc", A, 8, 64, 1, 1, SYNC)
    assert st == 3  # RPCA_ERR_NO_MEMORY
    assert b"static scratch" in ctx.lib.rpca_last_error(ctx.h)
    assert bool((Sv == -3.0).all()) and bool((U == -3.0).all())
    ctx.close()
