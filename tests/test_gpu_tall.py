"""Y = A X in the tall form (8 waves of 64 rows, 64-byte row segments per
stage, equal tiles per workgroup), and the partials of A^T Q in the wide form
(8 waves of 64 columns, 512-column tiles) for the low-precision copies, on
the GPU through the C ABI.

  * For the float32, bfloat16 and E4M3 copies of A, the tall form gives the
    same Y bit for bit as the 4-wave form. Both accumulate the K16 steps in
    the same order; each form is forced through a loaded tune table.
  * The float32 products are within the split-product bound of the float64
    product.
  * Shapes:
    - one and two tiles per workgroup;
    - tiles of a few rows (small m with the tall form forced);
    - n with a partial last stage;
    - n of one or two stages, so that the copies of the next tile are issued
      before the current tile is consumed;
    - lp = 32, 64 and 128.
  * The wide form of A^T Q, forced through a loaded tune table like the
    128-column form: for the bfloat16 and E4M3 copies within (m + 3) 2^-24
    (|A8^T| |Q'|) s_j of the float64 product of the same rounded operands (Q'
    the operand rounded to bfloat16, s_j the E4M3 column scale), for float32
    A within the split-product bound (2^-15 + m 2^-24)(|A^T| |Q|), on ragged
    row splits and a last tile of 16 columns.
"""

import numpy as np
import pytest
import torch

from oracle import precision

pytestmark = pytest.mark.gpu

DT = {"f32": 0, "bf16": 1, "fp8": 2}


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    return gpu_lib.Context()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _lp(l):
    return 32 if l <= 32 else 64 if l <= 64 else 128


def _class(m, n, l, dtype):
    return "%d %d %d %d" % ((m - 1).bit_length(), (n - 1).bit_length(), _lp(l), dtype)


def _forced(ctx, tmp_path, m, n, l, dtype, waves, run):
    path = tmp_path / ("ax%d.txt" % waves)
    ring = 3 if waves == 4 else 0
    path.write_text("# forced\n%s %d %d 0 0 0\n" % (_class(m, n, l, dtype), waves, ring))
    ctx.tune_clear()
    ctx.tune_load(str(path))
    try:
        return run()
    finally:
        ctx.tune_clear()


# 70001 rows: one tile of 274 rows per workgroup (256 CUs); 150001 rows: two
# tiles of 293; n = 1028 leaves the float32 form a last stage with one valid
# chunk; n = 32 and 16 are one or two stages; 1000, 777 and 33 rows force the
# tall form onto tiles of 32, 25 and 17 rows.
SHAPES = [(70001, 1028, 120), (70001, 400, 60), (150001, 208, 30), (150001, 32, 60),
          (150001, 16, 120), (1000, 512, 12), (777, 320, 60), (33, 48, 30)]


# the low-precision copies need rows of whole 16-byte chunks (n % 16 == 0 covers both)
CASES = [(kind,) + sh for sh in SHAPES for kind in ("f32", "bf16", "fp8")
         if kind == "f32" or sh[1] % 16 == 0]


@pytest.mark.parametrize("kind,m,n,l", CASES)
def test_tall_equals_four_wave_form(ctx, gpu_lib, tmp_path, kind, m, n, l):
    rng = np.random.default_rng(m + 3 * n + l)
    A = rng.standard_normal((m, n)).astype(np.float32)
    X = rng.standard_normal((n, l)).astype(np.float32)
    dA, dX = _dev(A), _dev(X)
    if kind == "f32":
        mat = None
        src = dA
    else:
        q, s = ctx.quantize(dA, kind)
        mat = gpu_lib.dense(q, col_scale=s, A_f32=dA)
        src = q
    run = lambda: ctx.matmul(src, dX, mat=mat)  # noqa: E731
    Yt = _forced(ctx, tmp_path, m, n, l, DT[kind], 16, run)
    Y4 = _forced(ctx, tmp_path, m, n, l, DT[kind], 4, run)
    assert torch.equal(Yt, Y4)
    if kind == "f32":
        # the split-bfloat16 product bound against the float64 product
        A64 = A.astype(np.float64)
        ref = A64 @ X.astype(np.float64)
        bound = (2.0 ** -15 + n * 2.0 ** -24) * (np.abs(A64) @ np.abs(X)) + 1e-30
        assert np.all(np.abs(Yt.cpu().numpy() - ref) <= bound)



def _forced_atx(ctx, tmp_path, m, n, l, dtype, waves, run):
    path = tmp_path / ("atx%d.txt" % waves)
    path.write_text("# forced\n%s 0 0 %d 0 0\n" % (_class(m, n, l, dtype), waves))
    ctx.tune_clear()
    ctx.tune_load(str(path))
    try:
        return run()
    finally:
        ctx.tune_clear()


@pytest.mark.parametrize("kind", ["f32", "bf16", "fp8"])
@pytest.mark.parametrize("m,n,l", [(5000, 528, 30), (70001, 1040, 120), (40, 512, 60),
                                   (12345, 2048, 64)])
def test_wide_atx_within_bound(ctx, gpu_lib, tmp_path, kind, m, n, l):
    rng = np.random.default_rng(m + n + l)
    A = rng.standard_normal((m, n)).astype(np.float32)
    Q = rng.standard_normal((m, l)).astype(np.float32)
    dA, dQ = _dev(A), _dev(Q)
    if kind == "f32":
        # the split-bfloat16 product bound against the float64 product
        A64 = A.astype(np.float64)
        want = A64.T @ Q.astype(np.float64)
        bound = (2.0 ** -15 + m * 2.0 ** -24) * (np.abs(A64.T) @ np.abs(Q)) + 1e-30
        run = lambda: ctx.matmul(dA, dQ, trans=True).cpu().numpy()  # noqa: E731
        for waves in (16, 4):
            Z = _forced_atx(ctx, tmp_path, m, n, l, 0, waves, run)
            assert np.all(np.abs(Z - want) <= bound), waves
        return
    q, s = ctx.quantize(dA, kind)
    mat = gpu_lib.dense(q, col_scale=s, A_f32=dA)
    if kind == "bf16":
        A8 = precision.from_bf16_bits(q.view(torch.int16).cpu().numpy().view(np.uint16))
        sh = np.ones(n)
    else:
        A8 = precision.e4m3_decode(q.view(torch.uint8).cpu().numpy())
        sh = s.cpu().numpy().astype(np.float64)
    Qb = precision.to_bf16(Q)
    want = (A8.T @ Qb) * sh[:, None]
    bound = (m + 3) * 2.0 ** -24 * (np.abs(A8.T) @ np.abs(Qb)) * sh[:, None] + 1e-30
    run = lambda: ctx.matmul(q, dQ, trans=True, mat=mat).cpu().numpy()  # noqa: E731
    for waves in (16, 4):
        Z = _forced_atx(ctx, tmp_path, m, n, l, DT[kind], waves, run)
        assert np.all(np.abs(Z - want) <= bound), waves
