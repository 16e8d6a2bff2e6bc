"""Python binding of librpca, an MI355X (gfx950) implementation of the
randomized PCA of Szlam, Kluger and Tygert (ACM TOMS 2014, arXiv:1412.3510).

The binding only marshals arguments: every step runs in the HIP kernels of
``librpca.so`` (built by ``paper_1412_3510_amd.build``).  PyTorch provides the
device memory and the stream.  There is no fallback: if the library is
missing, ``load()`` raises.

    import torch, paper_1412_3510_amd as rp
    ctx = rp.Context()
    U, S, V = ctx.svd(A, k=50, l=60, its=2, seed=1, center=True)
"""

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librpca.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "rpca.h")

F32, BF16, FP8_E4M3 = 0, 1, 2
DENSE_ROWMAJOR, SPARSE_CSR = 0, 1
CENTER, SYNC, DETERMINISTIC, RENORM_ORTH, RENORM_LU, OMEGA_UNIFORM = 1, 2, 4, 8, 16, 32
NYSTROM_SQRT = 64
FUSED_ATA = 128
_STAB = {"shift": 0, None: 0, "sqrt": NYSTROM_SQRT}
_OMEGA = {"gaussian": 0, None: 0, "uniform": OMEGA_UNIFORM}
# renormalization between applications: "chol" (one Cholesky QR pass, the
# default), "lu" (pivoted LU, the paper's choice), "orth" (Cholesky QR twice)
_RENORM = {"chol": 0, None: 0, "lu": RENORM_LU, "orth": RENORM_ORTH}

STATUS = {
    0: "RPCA_OK",
    1: "RPCA_ERR_INVALID_ARG",
    2: "RPCA_ERR_UNSUPPORTED",
    3: "RPCA_ERR_NO_MEMORY",
    4: "RPCA_ERR_HIP",
    5: "RPCA_ERR_NOT_PSD",
    6: "RPCA_ERR_NUMERICAL",
}


class RpcaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class Matrix(ctypes.Structure):
    _fields_ = [
        ("format", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("m", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("data", ctypes.c_void_p),
        ("ld", ctypes.c_int64),
        ("col_scale", ctypes.c_void_p),
        ("data_f32", ctypes.c_void_p),
        ("ld_f32", ctypes.c_int64),
        ("nnz", ctypes.c_int64),
        ("row_ptr", ctypes.c_void_p),
        ("col_idx", ctypes.c_void_p),
        ("val", ctypes.c_void_p),
        ("col_ptr", ctypes.c_void_p),
        ("row_idx", ctypes.c_void_p),
        ("val_t", ctypes.c_void_p),
    ]


class Problem(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("l", ctypes.c_int32),
        ("its", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("flags", ctypes.c_uint32),
        ("reserved", ctypes.c_int32),
        ("A", ctypes.c_void_p),
        ("U", ctypes.c_void_p),
        ("ldu", ctypes.c_int64),
        ("S", ctypes.c_void_p),
        ("V", ctypes.c_void_p),
        ("ldv", ctypes.c_int64),
    ]


class Stats(ctypes.Structure):
    _fields_ = [
        ("calls", ctypes.c_int64),
        ("a_passes", ctypes.c_int64),
        ("timed_launches", ctypes.c_int64),
        ("ms_ax", ctypes.c_double),
        ("ms_atx", ctypes.c_double),
        ("n_ax", ctypes.c_int64),
        ("n_atx", ctypes.c_int64),
        ("bytes_ax", ctypes.c_double),
        ("bytes_atx", ctypes.c_double),
        ("shift_retries", ctypes.c_int64),
        ("ms_ax_lp", ctypes.c_double),
        ("ms_atx_lp", ctypes.c_double),
        ("n_ax_lp", ctypes.c_int64),
        ("n_atx_lp", ctypes.c_int64),
        ("bytes_ax_lp", ctypes.c_double),
        ("bytes_atx_lp", ctypes.c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class TuneResult(ctypes.Structure):
    _fields_ = [
        ("ax_waves", ctypes.c_int32),
        ("ax_ring", ctypes.c_int32),
        ("atx_waves", ctypes.c_int32),
        ("atx_ring", ctypes.c_int32),
        ("lu_rows", ctypes.c_int32),
        ("candidates", ctypes.c_int32),
        ("ms_ax", ctypes.c_double),
        ("ms_atx", ctypes.c_double),
        ("ms_lu", ctypes.c_double),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_lib = None
P, I32, I64, U32, U64, D = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                            ctypes.c_uint64, ctypes.c_double)

_SIGS = {
    "rpca_create": [ctypes.POINTER(P), P],
    "rpca_destroy": [P],
    "rpca_set_stream": [P, P],
    "rpca_set_workspace_limit": [P, ctypes.c_size_t],
    "rpca_workspace_size": [P, ctypes.POINTER(Matrix), I32, I32, ctypes.POINTER(ctypes.c_size_t)],
    "rpca_svd": [P, ctypes.POINTER(Matrix), I32, I32, I32, U64, ctypes.c_uint, P, I64, P, P, I64],
    "rpca_svd_noalloc": [P, ctypes.POINTER(Matrix), I32, I32, I32, U64, ctypes.c_uint, P, I64, P,
                         P, I64],
    "rpca_eig_psd": [P, ctypes.POINTER(Matrix), I32, I32, I32, U64, ctypes.c_uint, P, I64, P],
    "rpca_eig_sym": [P, ctypes.POINTER(Matrix), I32, I32, I32, U64, ctypes.c_uint, P, I64, P],
    "rpca_spectral_err": [P, ctypes.POINTER(Matrix), I32, P, I64, P, P, I64, I32, U64,
                          ctypes.c_uint, ctypes.POINTER(D)],
    "rpca_gaussian": [P, U64, U32, I64, I64, P, I64, P],
    "rpca_uniform": [P, U64, U32, I64, I64, P, I64],
    "rpca_quantize": [P, P, I64, I64, I64, I32, P, I64, P],
    "rpca_svd_batched": [P, I32, P, ctypes.c_uint],
    "rpca_op_matmul": [P, ctypes.POINTER(Matrix), I32, I32, P, I64, P, I64, ctypes.c_uint],
    "rpca_op_renorm": [P, I32, I64, I32, P, I64, P, P],
    "rpca_op_small_svd": [P, I32, P, P, P, P],
    "rpca_set_timing": [P, I32],
    "rpca_get_stats": [P, ctypes.POINTER(Stats)],
    "rpca_reset_stats": [P],
    "rpca_set_batch_streams": [P, I32],
    "rpca_set_batch_mode": [P, I32],
    "rpca_set_batch_split": [P, I32, I32, I32],
    "rpca_batch_status": [P, I32, ctypes.POINTER(I32)],
    "rpca_sync": [P],
    "rpca_set_nystrom_retries": [P, I32],
    "rpca_tune": [P, ctypes.POINTER(Matrix), I32, I32, ctypes.POINTER(TuneResult)],
    "rpca_tune_save": [P, ctypes.c_char_p],
    "rpca_tune_load": [P, ctypes.c_char_p],
    "rpca_tune_clear": [P],
    "rpca_tune_count": [P, ctypes.POINTER(I32)],
}


def header_symbols():
    """Names of the functions declared in include/rpca.h."""
    with open(HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(rpca_\w+)\s*\(", text, re.M)))


def load():
    """Load librpca.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("librpca.so is not built: run `python -m paper_1412_3510_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.rpca_status_str.argtypes = [ctypes.c_int]
    lib.rpca_status_str.restype = ctypes.c_char_p
    lib.rpca_last_error.argtypes = [P]
    lib.rpca_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t, dtype, dim, name):
    """Check a device operand: dtype, rank, on the GPU, unit stride along its last axis."""
    if (t.dtype != dtype or t.dim() != dim or not t.is_cuda
            or (t.numel() > 0 and t.stride(-1) != 1)):
        raise ValueError("%s must be a %d-D %s CUDA tensor with unit last stride" % (name, dim, dtype))


def dense(A, dtype=None, col_scale=None, A_f32=None):
    """rpca_matrix for a row-major 2-D CUDA tensor (float32, bfloat16 or float8_e4m3fn)."""
    import torch
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError("A must be a 2-D row-major tensor")
    if not A.is_cuda:
        raise ValueError("A must live on the GPU")
    code = {torch.float32: F32, torch.bfloat16: BF16}.get(A.dtype)
    if code is None and hasattr(torch, "float8_e4m3fn") and A.dtype == torch.float8_e4m3fn:
        code = FP8_E4M3
    if code is None:
        raise ValueError("unsupported dtype %s" % A.dtype)
    mat = Matrix()
    mat.format = DENSE_ROWMAJOR
    mat.dtype = code if dtype is None else dtype
    mat.m, mat.n = A.shape
    mat.data = A.data_ptr()
    mat.ld = A.stride(0)
    mat.col_scale = col_scale.data_ptr() if col_scale is not None else None
    if A_f32 is not None:
        mat.data_f32 = A_f32.data_ptr()
        mat.ld_f32 = A_f32.stride(0)
    return mat


class SparseMatrix:
    """A sparse A for the library: CSR arrays of A and, for products with A^T,
    CSC arrays (the CSR of A^T), all int32 / float32 (or bfloat16) CUDA tensors.
    Keeps the tensors alive while the matrix is used."""

    def __init__(self, m, n, row_ptr, col_idx, val, col_ptr=None, row_idx=None, val_t=None):
        import torch
        self.shape = (int(m), int(n))
        self._keep = [row_ptr, col_idx, val, col_ptr, row_idx, val_t]
        for name, t, dt in (("row_ptr", row_ptr, torch.int32), ("col_idx", col_idx, torch.int32),
                            ("col_ptr", col_ptr, torch.int32), ("row_idx", row_idx, torch.int32)):
            if t is not None and (t.dtype != dt or not t.is_cuda or not t.is_contiguous()):
                raise ValueError("%s must be a contiguous int32 CUDA tensor" % name)
        if row_ptr.numel() != m + 1 or (col_ptr is not None and col_ptr.numel() != n + 1):
            raise ValueError("row_ptr needs m + 1 entries, col_ptr n + 1")
        code = {torch.float32: F32, torch.bfloat16: BF16}.get(val.dtype)
        if code is None or (val_t is not None and val_t.dtype != val.dtype):
            raise ValueError("values must be float32 or bfloat16 (both copies alike)")
        mat = Matrix()
        mat.format = SPARSE_CSR
        mat.dtype = code
        mat.m, mat.n = self.shape
        mat.nnz = val.numel()
        mat.row_ptr = row_ptr.data_ptr()
        mat.col_idx = col_idx.data_ptr()
        mat.val = val.data_ptr()
        if col_ptr is not None:
            mat.col_ptr = col_ptr.data_ptr()
            mat.row_idx = row_idx.data_ptr()
            mat.val_t = val_t.data_ptr()
        self.mat = mat


def csr(m, n, row_ptr, col_idx, val, col_ptr=None, row_idx=None, val_t=None):
    """SparseMatrix from CUDA tensors (CSR of A, optionally CSC of A)."""
    return SparseMatrix(m, n, row_ptr, col_idx, val, col_ptr, row_idx, val_t)


def _as_mat(A, mat):
    """(rpca_matrix, m, n) for a dense tensor or a SparseMatrix."""
    if isinstance(A, SparseMatrix):
        return A.mat, A.shape[0], A.shape[1]
    m, n = A.shape
    return (dense(A) if mat is None else mat), m, n


class Context:
    """A library context bound to a torch CUDA stream (the current one by default)."""

    def __init__(self, stream=None):
        import torch
        self.lib = load()
        self._torch = torch
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        self._check(self.lib.rpca_create(ctypes.byref(h), ctypes.c_void_p(stream.cuda_stream)))
        self.h = h
        self._keep = []

    def close(self):
        if getattr(self, "h", None):
            self.lib.rpca_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_stream(self, stream):
        """Order later calls on ``stream`` (a torch CUDA stream); synchronizes the old one."""
        self._check(self.lib.rpca_set_stream(self.h, ctypes.c_void_p(stream.cuda_stream)))
        self.stream = stream

    def _check(self, st):
        if st != 0:
            msg = self.lib.rpca_last_error(self.h).decode() if getattr(self, "h", None) else ""
            raise RpcaError(st, msg)

    # ---- solvers -------------------------------------------------------
    def svd(self, A, k, l=None, its=2, seed=0, center=False, sync=False, out=None, mat=None,
            renorm="chol", deterministic=False, omega="gaussian", fused=False):
        """U (m x k), S (k, float64), V (n x k) with U diag(S) V^T ~ A (or A - 1 c).

        omega: the test matrix's law, "gaussian" or "uniform" (on (-1, 1)).

        fused: renormalize only after every second application, so that each
        power step is Z = A^T (A Z) (Section 5's optional acceleration).

        renorm: the renormalization between applications -- "chol" (one
        Cholesky QR pass, default), "lu" (pivoted LU, the paper's choice) or
        "orth" (Cholesky QR twice).  sync: wait for the device and raise
        on device-side failures (RpcaError with RPCA_ERR_NUMERICAL for
        non-finite values)."""
        torch = self._torch
        mat, m, n = _as_mat(A, mat)
        l = k + 2 if l is None else l
        if out is None:
            U = torch.empty(m, k, device="cuda", dtype=torch.float32)
            S = torch.empty(k, device="cuda", dtype=torch.float64)
            V = torch.empty(n, k, device="cuda", dtype=torch.float32)
        else:
            U, S, V = out
        flags = (CENTER if center else 0) | (SYNC if sync else 0) | _RENORM[renorm]
        flags |= (DETERMINISTIC if deterministic else 0) | _OMEGA[omega]
        flags |= FUSED_ATA if fused else 0
        self._check(self.lib.rpca_svd(self.h, ctypes.byref(mat), k, l, its, seed, flags,
                                      _ptr(U), U.stride(0), _ptr(S), _ptr(V), V.stride(0)))
        return U, S, V

    def eig_psd(self, A, k, l=None, its=2, seed=0, sync=False, mat=None, renorm="chol",
                deterministic=False, omega="gaussian", stabilize="shift"):
        """U (n x k), lambda (k, float64) with U diag(lambda) U^T ~ A (PSD A).

        stabilize: "shift" (shifted Cholesky factor) or "sqrt" (self-adjoint
        square root with a regularized pseudoinverse).  sync: wait for the
        device and raise RpcaError(RPCA_ERR_NOT_PSD) when the shifted Cholesky
        factor was never found (else that surfaces at the next synchronizing
        call, see ``sync``)."""
        torch = self._torch
        mat, n, _ = _as_mat(A, mat)
        l = k + 2 if l is None else l
        U = torch.empty(n, k, device="cuda", dtype=torch.float32)
        lam = torch.empty(k, device="cuda", dtype=torch.float64)
        flags = (SYNC if sync else 0) | _RENORM[renorm] | _STAB[stabilize]
        flags |= (DETERMINISTIC if deterministic else 0) | _OMEGA[omega]
        self._check(self.lib.rpca_eig_psd(self.h, ctypes.byref(mat), k, l, its, seed, flags,
                                          _ptr(U), U.stride(0), _ptr(lam)))
        return U, lam

    def eig_sym(self, A, k, l=None, its=2, seed=0, sync=False, mat=None, renorm="chol",
                deterministic=False, omega="gaussian"):
        """U (n x k), lambda (k, float64, signed, by |lambda| descending) with
        U diag(lambda) U^T ~ A for a general symmetric A."""
        torch = self._torch
        mat, n, _ = _as_mat(A, mat)
        l = k + 2 if l is None else l
        U = torch.empty(n, k, device="cuda", dtype=torch.float32)
        lam = torch.empty(k, device="cuda", dtype=torch.float64)
        flags = (SYNC if sync else 0) | _RENORM[renorm] | _OMEGA[omega]
        flags |= DETERMINISTIC if deterministic else 0
        self._check(self.lib.rpca_eig_sym(self.h, ctypes.byref(mat), k, l, its, seed, flags,
                                          _ptr(U), U.stride(0), _ptr(lam)))
        return U, lam

    def spectral_err(self, A, U, S, V=None, iters=20, seed=0, center=False, mat=None):
        """Power-method estimate of ||A - U diag(S) V^T||_2 (V None: A - U diag(S) U^T)."""
        torch = self._torch
        _need(U, torch.float32, 2, "U")
        _need(S, torch.float64, 1, "S")
        if V is not None:
            _need(V, torch.float32, 2, "V")
        mat, _, _ = _as_mat(A, mat)
        out = ctypes.c_double()
        k = U.shape[1]
        self._check(self.lib.rpca_spectral_err(
            self.h, ctypes.byref(mat), k, _ptr(U), max(U.stride(0), k), _ptr(S), _ptr(V),
            max(V.stride(0), k) if V is not None else 0, iters, seed, CENTER if center else 0,
            ctypes.byref(out)))
        return out.value

    def quantize(self, A, dtype):
        """Low-precision copy of a float32 CUDA matrix: ``"bf16"`` -> (bfloat16 tensor, None),
        ``"fp8"`` -> (float8_e4m3fn tensor, float32 column scales)."""
        torch = self._torch
        _need(A, torch.float32, 2, "A")
        m, n = A.shape
        if dtype == "bf16":
            out = torch.empty(m, n, device=A.device, dtype=torch.bfloat16)
            scale = None
            code = BF16
        elif dtype == "fp8":
            out = torch.empty(m, n, device=A.device, dtype=torch.float8_e4m3fn)
            scale = torch.empty(n, device=A.device, dtype=torch.float32)
            code = FP8_E4M3
        else:
            raise ValueError("dtype must be 'bf16' or 'fp8'")
        self._check(self.lib.rpca_quantize(self.h, _ptr(A), m, n, A.stride(0), code, _ptr(out),
                                           out.stride(0), _ptr(scale)))
        return out, scale

    def svd_batched(self, problems, sync=False, deterministic=False):
        """Solve many independent problems in one call.

        ``problems``: list of dicts with keys A (dense tensor or SparseMatrix),
        k, and optionally l, its, seed, center, kind ("svd" or "psd"), renorm,
        mat (a prepared rpca_matrix).  Returns a list of (U, S, V) for "svd"
        and (U, lambda) for "psd"."""
        torch = self._torch
        arr = (Problem * len(problems))()
        outs, mats = [], []
        for i, pr in enumerate(problems):
            mat, m, n = _as_mat(pr["A"], pr.get("mat"))
            mats.append(mat)
            k = int(pr["k"])
            l = int(pr.get("l") or k + 2)
            psd = pr.get("kind", "svd") == "psd"
            U = torch.empty(m, k, device="cuda", dtype=torch.float32)
            S = torch.empty(k, device="cuda", dtype=torch.float64)
            V = None if psd else torch.empty(n, k, device="cuda", dtype=torch.float32)
            q = arr[i]
            q.kind = 1 if psd else 0
            q.k, q.l, q.its = k, l, int(pr.get("its", 2))
            q.seed = int(pr.get("seed", 0))
            q.flags = ((CENTER if pr.get("center") else 0) | _RENORM[pr.get("renorm")]
                       | _OMEGA[pr.get("omega")] | _STAB[pr.get("stabilize")]
                       | (FUSED_ATA if pr.get("fused") else 0))
            q.A = ctypes.cast(ctypes.pointer(mat), ctypes.c_void_p)
            q.U, q.ldu = U.data_ptr(), U.stride(0)
            q.S = S.data_ptr()
            if V is not None:
                q.V, q.ldv = V.data_ptr(), V.stride(0)
            outs.append((U, S) if psd else (U, S, V))
        self._batch_keep = (arr, mats, problems)
        flags = (SYNC if sync else 0) | (DETERMINISTIC if deterministic else 0)
        self._check(self.lib.rpca_svd_batched(self.h, len(problems), ctypes.cast(arr, P), flags))
        return outs

    def batch_status(self, count):
        """Per-problem status codes (0 ok, 5 not PSD, 6 non-finite) of the last batch."""
        out = (I32 * count)()
        self._check(self.lib.rpca_batch_status(self.h, count, out))
        return list(out)

    def sync(self):
        """Wait for the device; raise RpcaError for device-side failures since the last sync."""
        self._check(self.lib.rpca_sync(self.h))

    def set_nystrom_retries(self, retries):
        self._check(self.lib.rpca_set_nystrom_retries(self.h, retries))

    # ---- single steps --------------------------------------------------
    def gaussian(self, seed, n, l, stream=0, words=False):
        torch = self._torch
        out = torch.zeros(n, l, device="cuda", dtype=torch.float32)
        w = None
        if words:
            w = torch.zeros(((n * l + 3) // 4) * 4, device="cuda", dtype=torch.int32)
        self._check(self.lib.rpca_gaussian(self.h, seed, stream, n, l, _ptr(out), out.stride(0),
                                           _ptr(w)))
        return (out, w) if words else out

    def uniform(self, seed, n, l, stream=0):
        """The uniform test matrix (n x l) of the ``omega="uniform"`` option."""
        torch = self._torch
        out = torch.zeros(n, l, device="cuda", dtype=torch.float32)
        self._check(self.lib.rpca_uniform(self.h, seed, stream, n, l, _ptr(out), out.stride(0)))
        return out

    def matmul(self, A, X, trans=False, center=False, mat=None):
        torch = self._torch
        mat, m, n = _as_mat(A, mat)
        l = X.shape[1]
        Y = torch.empty(n if trans else m, l, device="cuda", dtype=torch.float32)
        self._check(self.lib.rpca_op_matmul(self.h, ctypes.byref(mat), 1 if trans else 0, l,
                                            _ptr(X), X.stride(0), _ptr(Y), Y.stride(0),
                                            CENTER if center else 0))
        return Y

    def renorm(self, Y, kind="lu"):
        torch = self._torch
        Y = Y.clone()
        rows, l = Y.shape
        piv = torch.empty(l, device=Y.device, dtype=torch.int32)
        R = torch.empty(l, l, device=Y.device, dtype=torch.float64)
        k = 0 if kind == "lu" else 1
        self._check(self.lib.rpca_op_renorm(self.h, k, rows, l, _ptr(Y), Y.stride(0),
                                            _ptr(piv) if k == 0 else None,
                                            _ptr(R) if k == 1 else None))
        return (Y, piv) if k == 0 else (Y, R)

    def small_svd(self, M):
        torch = self._torch
        l = M.shape[0]
        M = M.to(torch.float64).contiguous()
        s = torch.empty(l, device=M.device, dtype=torch.float64)
        W = torch.empty(l, l, device=M.device, dtype=torch.float64)
        X = torch.empty(l, l, device=M.device, dtype=torch.float64)
        self._check(self.lib.rpca_op_small_svd(self.h, l, _ptr(M), _ptr(s), _ptr(W), _ptr(X)))
        return W, s, X

    def set_batch_mode(self, mode):
        """0: persistent launch for the problems it takes (default); 1: streams only."""
        self._check(self.lib.rpca_set_batch_mode(self.h, mode))

    def set_batch_split(self, max_parts=8, min_parts=1, spin_limit=0):
        """Problems of the persistent launch: at most ``max_parts`` workgroups
        each (1: no splitting), at least ``min_parts`` for every problem that
        can be split (1: the cost model decides); ``spin_limit`` polls before
        a share stops waiting for the others (0: the default)."""
        self._check(self.lib.rpca_set_batch_split(self.h, max_parts, min_parts, spin_limit))

    def set_batch_streams(self, n):
        """Streams svd_batched spreads a batch over (default 8)."""
        self._check(self.lib.rpca_set_batch_streams(self.h, n))

    # ---- autotuner ----------------------------------------------------
    def tune(self, A, l, reps=3, mat=None):
        """Time the tile configurations on dense A with l sketch columns and keep the
        fastest for A's shape class; returns the choice and its times (ms per launch)."""
        mat, _, _ = _as_mat(A, mat)
        res = TuneResult()
        self._check(self.lib.rpca_tune(self.h, ctypes.byref(mat), l, reps, ctypes.byref(res)))
        return res.as_dict()

    def tune_save(self, path):
        self._check(self.lib.rpca_tune_save(self.h, os.fsencode(path)))

    def tune_load(self, path):
        self._check(self.lib.rpca_tune_load(self.h, os.fsencode(path)))

    def tune_clear(self):
        self._check(self.lib.rpca_tune_clear(self.h))

    def tune_count(self):
        c = I32()
        self._check(self.lib.rpca_tune_count(self.h, ctypes.byref(c)))
        return c.value

    # ---- diagnostics ---------------------------------------------------
    def set_timing(self, on=True):
        self._check(self.lib.rpca_set_timing(self.h, 1 if on else 0))

    def stats(self):
        st = Stats()
        self._check(self.lib.rpca_get_stats(self.h, ctypes.byref(st)))
        return st.as_dict()

    def reset_stats(self):
        self._check(self.lib.rpca_reset_stats(self.h))

    def set_workspace_limit(self, nbytes):
        self._check(self.lib.rpca_set_workspace_limit(self.h, nbytes))
