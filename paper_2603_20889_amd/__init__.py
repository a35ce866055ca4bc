"""qless: Q-less QR of tall, very skinny FP64 matrices on AMD MI355X (gfx950).

Thin ctypes binding over the C-ABI library ``libqless.so`` (declared in
``include/qless.h``).  Functions carry the C names; they only marshal
arguments: PyTorch provides device memory (tensors) and the current stream,
and every step of the computation runs in the library's HIP kernels.  There
is no CPU fallback -- when the library is missing, ``load()`` raises.

Method: Thies & Roehrig-Zoellner, "Implementation of QR factorization of tall
and very skinny matrices on current GPUs", arXiv 2603.20889.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqless.so")

QLESS_OK = 0
QLESS_ERR_ARG = -1
QLESS_ERR_UNSUPPORTED = -2
QLESS_ERR_WORKSPACE = -3
QLESS_ERR_HIP = -4

QLESS_METHOD_TSQR = 0
QLESS_METHOD_TSQR_UPDATE = 3
QLESS_METHOD_CHOLQR2 = 1
QLESS_METHOD_SVQB = 2
QLESS_METHOD_SHIFTED_CHOLQR3 = 4
QLESS_METHOD_Q_FROM_R = 5
QLESS_METHOD_GRAM = 6
QLESS_METHOD_CHOLQR2_DD = 7

QLESS_SVQB_R = 0
QLESS_SVQB_QZ = 1

QLESS_MAX_N = 64

EXPORTED = (
    "qless_status_string", "qless_version", "qless_workspace_bytes", "qless_tsqr_r", "qless_tsqr_r_update",
    "cholqr2_r", "shifted_cholqr3_r", "svqb", "qless_lstsq_finish", "qless_timing_enable", "qless_timing_reset",
    "qless_timing_read", "qless_batch_plan_create", "qless_batch_plan_destroy",
    "qless_batch_plan_workspace_bytes", "qless_batch_plan_tiles", "qless_batch_plan_upload",
    "qless_tsqr_r_batched", "qless_tune_set", "qless_tune_get", "qless_q_from_r", "svqb_q",
    "qless_two_phase_r", "qless_two_phase_workspace_bytes", "qless_tsqr_state_bytes", "qless_tsqr_state_init",
    "qless_tsqr_state_fold", "qless_tsqr_state_finish", "qless_wide_r", "qless_wide_workspace_bytes",
    "qless_gram", "cholqr2_dd_r", "qless_tsqr_r_noalloc", "qless_noalloc_scratch_bytes",
)


class qless_matrix_desc(ctypes.Structure):
    """Mirror of the C struct qless_matrix_desc."""
    _fields_ = [("X", ctypes.c_void_p), ("m", ctypes.c_int64), ("n", ctypes.c_int64), ("ldx", ctypes.c_int64),
                ("R", ctypes.c_void_p), ("ldr", ctypes.c_int64), ("accumulate", ctypes.c_int32)]


class QlessError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s" % (where, status_string(status)))


_lib = None


def load() -> ctypes.CDLL:
    """Load libqless.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libqless.so not found at %s; build it with "
                           "`python -m paper_2603_20889_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_double
    sz = ctypes.c_size_t
    lib.qless_status_string.argtypes = [ctypes.c_int]
    lib.qless_status_string.restype = ctypes.c_char_p
    lib.qless_version.argtypes = []
    lib.qless_version.restype = ctypes.c_char_p
    lib.qless_workspace_bytes.argtypes = [ctypes.c_int, i64, i64]
    lib.qless_workspace_bytes.restype = sz
    lib.qless_tsqr_r.argtypes = [vp, i64, i64, i64, vp, i64, vp, sz, vp]
    lib.qless_tsqr_r.restype = ctypes.c_int
    lib.qless_tsqr_r_update.argtypes = [vp, i64, i64, i64, vp, i64, vp, sz, vp]
    lib.qless_tsqr_r_update.restype = ctypes.c_int
    lib.cholqr2_r.argtypes = [vp, i64, i64, i64, vp, i64, vp, vp, sz, vp]
    lib.cholqr2_r.restype = ctypes.c_int
    lib.shifted_cholqr3_r.argtypes = [vp, i64, i64, i64, vp, i64, vp, vp, sz, vp]
    lib.shifted_cholqr3_r.restype = ctypes.c_int
    lib.svqb.argtypes = [vp, i64, i64, i64, ctypes.c_int, vp, i64, vp, dbl, vp, vp, sz, vp]
    lib.svqb.restype = ctypes.c_int
    lib.qless_q_from_r.argtypes = [vp, i64, i64, i64, vp, i64, vp, i64, vp, vp, sz, vp]
    lib.qless_q_from_r.restype = ctypes.c_int
    lib.svqb_q.argtypes = [vp, i64, i64, i64, vp, i64, vp, i64, vp, dbl, vp, vp, sz, vp]
    lib.svqb_q.restype = ctypes.c_int
    lib.qless_two_phase_workspace_bytes.argtypes = [i64, i64, i64]
    lib.qless_two_phase_workspace_bytes.restype = sz
    lib.qless_two_phase_r.argtypes = [vp, i64, i64, vp, i64, i64, i64, vp, i64, vp, i64, vp, sz, vp]
    lib.qless_two_phase_r.restype = ctypes.c_int
    lib.qless_tsqr_state_bytes.argtypes = [i64, i64]
    lib.qless_tsqr_state_bytes.restype = sz
    lib.qless_tsqr_state_init.argtypes = [vp, sz, i64, i64, vp]
    lib.qless_tsqr_state_init.restype = ctypes.c_int
    lib.qless_tsqr_state_fold.argtypes = [vp, i64, i64, vp, sz, i64, i64, vp]
    lib.qless_tsqr_state_fold.restype = ctypes.c_int
    lib.qless_tsqr_state_finish.argtypes = [vp, sz, i64, i64, vp, i64, vp]
    lib.qless_tsqr_state_finish.restype = ctypes.c_int
    lib.qless_wide_workspace_bytes.argtypes = [i64, i64, i64]
    lib.qless_wide_workspace_bytes.restype = sz
    lib.qless_wide_r.argtypes = [vp, i64, i64, i64, vp, i64, vp, i64, i64, vp, vp, sz, vp]
    lib.qless_wide_r.restype = ctypes.c_int
    lib.qless_gram.argtypes = [vp, i64, i64, i64, vp, i64, vp, vp, sz, vp]
    lib.qless_gram.restype = ctypes.c_int
    lib.cholqr2_dd_r.argtypes = [vp, i64, i64, i64, vp, i64, vp, vp, sz, vp]
    lib.cholqr2_dd_r.restype = ctypes.c_int
    lib.qless_lstsq_finish.argtypes = [vp, i64, i64, vp, vp, vp, vp]
    lib.qless_lstsq_finish.restype = ctypes.c_int
    lib.qless_batch_plan_create.argtypes = [ctypes.POINTER(qless_matrix_desc), i32, i64, i32,
                                            ctypes.POINTER(ctypes.c_void_p)]
    lib.qless_batch_plan_create.restype = ctypes.c_int
    lib.qless_batch_plan_destroy.argtypes = [vp]
    lib.qless_batch_plan_destroy.restype = None
    lib.qless_batch_plan_workspace_bytes.argtypes = [vp]
    lib.qless_batch_plan_workspace_bytes.restype = sz
    lib.qless_batch_plan_tiles.argtypes = [vp]
    lib.qless_batch_plan_tiles.restype = i64
    lib.qless_batch_plan_upload.argtypes = [vp, vp, sz, vp]
    lib.qless_batch_plan_upload.restype = ctypes.c_int
    lib.qless_tsqr_r_batched.argtypes = [vp, vp, sz, vp]
    lib.qless_tsqr_r_batched.restype = ctypes.c_int
    lib.qless_tune_set.argtypes = [i64, i32, i32, i32]
    lib.qless_tune_set.restype = ctypes.c_int
    lib.qless_tune_get.argtypes = [i64, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    lib.qless_tune_get.restype = ctypes.c_int
    lib.qless_tsqr_r_noalloc.argtypes = [vp, i64, i64, i64, vp, i64, vp]
    lib.qless_tsqr_r_noalloc.restype = ctypes.c_int
    lib.qless_noalloc_scratch_bytes.argtypes = []
    lib.qless_noalloc_scratch_bytes.restype = sz
    lib.qless_timing_enable.argtypes = [ctypes.c_int]
    lib.qless_timing_enable.restype = ctypes.c_int
    lib.qless_timing_reset.argtypes = []
    lib.qless_timing_reset.restype = ctypes.c_int
    lib.qless_timing_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
    lib.qless_timing_read.restype = ctypes.c_int
    _ = i32
    _lib = lib
    return lib


def status_string(status: int) -> str:
    try:
        return load().qless_status_string(int(status)).decode()
    except RuntimeError:
        return "status %d" % status


def version() -> str:
    return load().qless_version().decode()


def _check(status: int, where: str) -> None:
    if status != QLESS_OK:
        raise QlessError(status, where)


# ------------------------------------------------------------ marshalling

def _matrix(X, name="X"):
    import torch
    if not isinstance(X, torch.Tensor) or X.dtype != torch.float64 or X.dim() != 2:
        raise TypeError("%s must be a 2-D torch.float64 tensor" % name)
    if X.device.type != "cuda":
        raise TypeError("%s must live on a GPU (got %s)" % (name, X.device))
    m, n = X.shape
    # rows must be contiguous and must not overlap (an expanded or
    # transposed view would make the kernels read past the allocation)
    if m > 0 and (X.stride(1) != 1 or (m > 1 and X.stride(0) < n)):
        X = X.contiguous()
    ldx = X.stride(0) if m > 1 else n
    return X, int(m), int(n), int(max(ldx, n))


def _out(T, rows: int, cols: int, device, name: str, dtype=None):
    """Check a caller-supplied output tensor before any launch: the dtype
    (float64 unless given), X's device, at least rows x cols (a vector when
    rows == 0), unit stride along a row and non-overlapping rows."""
    import torch
    dtype = dtype or torch.float64
    if not isinstance(T, torch.Tensor) or T.dtype != dtype:
        raise TypeError("%s must be a torch.%s tensor" % (name, str(dtype).replace("torch.", "")))
    if T.device != device:
        raise ValueError("%s must live on %s (got %s)" % (name, device, T.device))
    if rows == 0:
        if T.dim() != 1 or T.numel() < cols or (cols > 1 and T.stride(0) != 1):
            raise ValueError("%s must be a contiguous vector of at least %d elements" % (name, cols))
        return T
    if T.dim() != 2 or T.shape[0] < rows or T.shape[1] < cols:
        raise ValueError("%s must be at least %d x %d (got %s)" % (name, rows, cols, tuple(T.shape)))
    if T.stride(1) != 1 or (T.shape[0] > 1 and T.stride(0) < cols):
        raise ValueError("%s must have unit column stride and rows at least %d apart" % (name, cols))
    return T


def _work_arg(work, device):
    """Caller-supplied workspace: a device tensor; returns its size in bytes."""
    import torch
    if not isinstance(work, torch.Tensor) or work.device != device or not work.is_contiguous():
        raise ValueError("work must be a contiguous tensor on %s" % device)
    return work.numel() * work.element_size()


def _stream(device):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _workspace(method: int, m: int, n: int, device):
    import torch
    nbytes = int(load().qless_workspace_bytes(method, m, n))
    if nbytes == 0:
        return None, 0
    # torch's caching allocator returns 512-byte-aligned blocks
    return torch.empty(nbytes, dtype=torch.uint8, device=device), nbytes


def qless_workspace_bytes(method: int, m: int, n: int) -> int:
    return int(load().qless_workspace_bytes(int(method), int(m), int(n)))


def qless_tsqr_r(X, R=None, work=None):
    """R (n x n, diag >= 0) of the GPU float64 matrix X by Q-less TSQR."""
    import torch
    X, m, n, ldx = _matrix(X)
    dev = X.device
    with torch.cuda.device(dev):
        if R is None:
            R = torch.empty((n, n), dtype=torch.float64, device=dev)
        else:
            _out(R, n, n, dev, "R")
        if work is None:
            work, wb = _workspace(QLESS_METHOD_TSQR, m, n, dev)
        else:
            wb = _work_arg(work, dev)
        st = load().qless_tsqr_r(ctypes.c_void_p(X.data_ptr() if m else 0), m, n, ldx,
                                 ctypes.c_void_p(R.data_ptr()), R.stride(0),
                                 ctypes.c_void_p(work.data_ptr() if work is not None else 0), wb,
                                 _stream(dev))
    _check(st, "qless_tsqr_r")
    return R


def qless_tsqr_r_update(X, R, work=None):
    """Running R: R <- R([R; X]) in place (diag >= 0), for chunks of rows."""
    import torch
    X, m, n, ldx = _matrix(X)
    dev = X.device
    _out(R, n, n, dev, "R")
    with torch.cuda.device(dev):
        if work is None:
            work, wb = _workspace(QLESS_METHOD_TSQR_UPDATE, m, n, dev)
        else:
            wb = _work_arg(work, dev)
        st = load().qless_tsqr_r_update(ctypes.c_void_p(X.data_ptr() if m else 0), m, n, ldx,
                                        ctypes.c_void_p(R.data_ptr()), R.stride(0),
                                        ctypes.c_void_p(work.data_ptr()), wb, _stream(dev))
    _check(st, "qless_tsqr_r_update")
    return R


def cholqr2_r(X, R=None, info=None, work=None):
    """Q-less CholQR2 (Alg. 1).  Returns (R, info) with info a 1-element int32
    device tensor (0 ok; j or n+j on Cholesky breakdown)."""
    import torch
    X, m, n, ldx = _matrix(X)
    dev = X.device
    with torch.cuda.device(dev):
        if R is None:
            R = torch.empty((n, n), dtype=torch.float64, device=dev)
        else:
            _out(R, n, n, dev, "R")
        if info is None:
            info = torch.empty(1, dtype=torch.int32, device=dev)
        else:
            _out(info, 0, 1, dev, "info", torch.int32)
        if work is None:
            work, wb = _workspace(QLESS_METHOD_CHOLQR2, m, n, dev)
        else:
            wb = _work_arg(work, dev)
        st = load().cholqr2_r(ctypes.c_void_p(X.data_ptr() if m else 0), m, n, ldx,
                              ctypes.c_void_p(R.data_ptr()), R.stride(0), ctypes.c_void_p(info.data_ptr()),
                              ctypes.c_void_p(work.data_ptr() if work is not None else 0), wb, _stream(dev))
    _check(st, "cholqr2_r")
    return R, info


def qless_gram(X, double_double: bool = False, C=None, C_lo=None, work=None):
    """C = X^T X on the device (tsmttsm); with double_double, accumulated in
    twice the working precision: returns (C_hi, C_lo), else (C, None)."""
    import torch
    X, m, n, ldx = _matrix(X)
    dev = X.device
    with torch.cuda.device(dev):
        if C is None:
            C = torch.empty((n, n), dtype=torch.float64, device=dev)
        else:
            _out(C, n, n, dev, "C")
        if double_double:
            if C_lo is None:
                C_lo = torch.empty((n, n), dtype=torch.float64, device=dev)
            else:
                _out(C_lo, n, n, dev, "C_lo")
                if C_lo.stride(0) != C.stride(0):
                    raise ValueError("C and C_lo must have the same row stride")
        else:
            C_lo = None
        if work is None:
            work, wb = _workspace(QLESS_METHOD_GRAM, m, n, dev)
        else:
            wb = _work_arg(work, dev)
        st = load().qless_gram(ctypes.c_void_p(X.data_ptr() if m else 0), m, n, ldx, ctypes.c_void_p(C.data_ptr()),
                               C.stride(0), ctypes.c_void_p(C_lo.data_ptr() if C_lo is not None else 0),
                               ctypes.c_void_p(work.data_ptr()), wb, _stream(dev))
    _check(st, "qless_gram")
    return C, C_lo


def cholqr2_dd_r(X, R=None, info=None, work=None):
    """Cholesky-QR2 with the first Gram matrix and Cholesky in
    double-double.  Returns (R, info)."""
    import torch
    X, m, n, ldx = _matrix(X)
    dev = X.device
    with torch.cuda.device(dev):
        if R is None:
            R = torch.empty((n, n), dtype=torch.float64, device=dev)
        else:
            _out(R, n, n, dev, "R")
        if info is None:
            info = torch.empty(1, dtype=torch.int32, device=dev)
        else:
            _out(info, 0, 1, dev, "info", torch.int32)
        if work is None:
            work, wb = _workspace(QLESS_METHOD_CHOLQR2_DD, m, n, dev)
        else:
            wb = _work_arg(work, dev)
        st = load().cholqr2_dd_r(ctypes.c_void_p(X.data_ptr() if m else 0), m, n, ldx,
                                 ctypes.c_void_p(R.data_ptr()), R.stride(0), ctypes.c_void_p(info.data_ptr()),
                                 ctypes.c_void_p(work.data_ptr()), wb, _stream(dev))
    _check(st, "cholqr2_dd_r")
    return R, info


def shifted_cholqr3_r(X, R=None, info=None, work=None):
    """Q-less shifted CholQR3.  Returns (R, info) with info a 1-element int32
    device tensor (0 ok; j, n+j or 2n+j on Cholesky breakdown)."""
    import torch
    X, m, n, ldx = _matrix(X)
    dev = X.device
    with torch.cuda.device(dev):
        if R is None:
            R = torch.empty((n, n), dtype=torch.float64, device=dev)
        else:
            _out(R, n, n, dev, "R")
        if info is None:
            info = torch.empty(1, dtype=torch.int32, device=dev)
        else:
            _out(info, 0, 1, dev, "info", torch.int32)
        if work is None:
            work, wb = _workspace(QLESS_METHOD_SHIFTED_CHOLQR3, m, n, dev)
        else:
            wb = _work_arg(work, dev)
        st = load().shifted_cholqr3_r(ctypes.c_void_p(X.data_ptr() if m else 0), m, n, ldx,
                                      ctypes.c_void_p(R.data_ptr()), R.stride(0), ctypes.c_void_p(info.data_ptr()),
                                      ctypes.c_void_p(work.data_ptr() if work is not None else 0), wb, _stream(dev))
    _check(st, "shifted_cholqr3_r")
    return R, info


def svqb(X, out: int = QLESS_SVQB_R, trunc_tol: float = 0.0, Z=None, sigma=None, info=None, work=None):
    """Q-less SVQB2.  Returns (Z_or_R, sigma, info)."""
    import torch
    X, m, n, ldx = _matrix(X)
    dev = X.device
    with torch.cuda.device(dev):
        if Z is None:
            Z = torch.empty((n, n), dtype=torch.float64, device=dev)
        else:
            _out(Z, n, n, dev, "Z")
        if sigma is None:
            sigma = torch.empty(n, dtype=torch.float64, device=dev)
        else:
            _out(sigma, 0, n, dev, "sigma")
        if info is None:
            info = torch.empty(1, dtype=torch.int32, device=dev)
        else:
            _out(info, 0, 1, dev, "info", torch.int32)
        if work is None:
            work, wb = _workspace(QLESS_METHOD_SVQB, m, n, dev)
        else:
            wb = _work_arg(work, dev)
        st = load().svqb(ctypes.c_void_p(X.data_ptr() if m else 0), m, n, ldx, int(out),
                         ctypes.c_void_p(Z.data_ptr()), Z.stride(0), ctypes.c_void_p(sigma.data_ptr()),
                         float(trunc_tol), ctypes.c_void_p(info.data_ptr()),
                         ctypes.c_void_p(work.data_ptr() if work is not None else 0), wb, _stream(dev))
    _check(st, "svqb")
    return Z, sigma, info


def qless_q_from_r(X, R, Q=None, info=None, work=None):
    """Explicit Q = X R^{-1} (m x n) from X and an upper-triangular R, one
    streaming pass (Sec. 1).  Returns (Q, info): info = j when R_jj == 0
    (Q is NaN then)."""
    import torch
    X, m, n, ldx = _matrix(X)
    dev = X.device
    R, _, nr, ldr = _matrix(R, "R")
    if R.shape[0] != n or nr != n or R.device != dev:
        raise ValueError("R must be an n x n matrix on X's device")
    with torch.cuda.device(dev):
        if Q is None:
            Q = torch.empty((m, n), dtype=torch.float64, device=dev)
        else:
            _out(Q, m, n, dev, "Q")
        if info is None:
            info = torch.empty(1, dtype=torch.int32, device=dev)
        else:
            _out(info, 0, 1, dev, "info", torch.int32)
        if work is None:
            work, wb = _workspace(QLESS_METHOD_Q_FROM_R, m, n, dev)
        else:
            wb = _work_arg(work, dev)
        st = load().qless_q_from_r(ctypes.c_void_p(X.data_ptr() if m else 0), m, n, ldx,
                                   ctypes.c_void_p(R.data_ptr()), ldr,
                                   ctypes.c_void_p(Q.data_ptr() if m else 0), Q.stride(0) if m > 1 else n,
                                   ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(work.data_ptr()), wb,
                                   _stream(dev))
    _check(st, "qless_q_from_r")
    return Q, info


def svqb_q(X, Q=None, Z=None, sigma=None, info=None, trunc_tol: float = 0.0, work=None):
    """SVQB2 with the explicit Q: X = Q Z, Q = X D1 D2.  Returns
    (Q, Z, sigma, info)."""
    import torch
    X, m, n, ldx = _matrix(X)
    dev = X.device
    with torch.cuda.device(dev):
        if Q is None:
            Q = torch.empty((m, n), dtype=torch.float64, device=dev)
        else:
            _out(Q, m, n, dev, "Q")
        if Z is None:
            Z = torch.empty((n, n), dtype=torch.float64, device=dev)
        else:
            _out(Z, n, n, dev, "Z")
        if sigma is None:
            sigma = torch.empty(n, dtype=torch.float64, device=dev)
        else:
            _out(sigma, 0, n, dev, "sigma")
        if info is None:
            info = torch.empty(1, dtype=torch.int32, device=dev)
        else:
            _out(info, 0, 1, dev, "info", torch.int32)
        if work is None:
            work, wb = _workspace(QLESS_METHOD_SVQB, m, n, dev)
        else:
            wb = _work_arg(work, dev)
        st = load().svqb_q(ctypes.c_void_p(X.data_ptr() if m else 0), m, n, ldx,
                           ctypes.c_void_p(Q.data_ptr() if m else 0), Q.stride(0) if m > 1 else n,
                           ctypes.c_void_p(Z.data_ptr()), Z.stride(0), ctypes.c_void_p(sigma.data_ptr()),
                           float(trunc_tol), ctypes.c_void_p(info.data_ptr()),
                           ctypes.c_void_p(work.data_ptr() if work is not None else 0), wb, _stream(dev))
    _check(st, "svqb_q")
    return Q, Z, sigma, info


# Leading dimensions from which qless_two_phase_r gets compact copies (a
# panel of the fold spans at most 2048 rows, addressed with 32-bit offsets).
TWO_PHASE_LD_COPY = 1 << 17


def qless_two_phase_r(Y, X, B=None, R=None, work=None):
    """Two-phase orthogonalisation in one pass (Sec. 2): B = Y^T X (p x n) and
    R = R((I - Y Y^T) X) (n x n) for Y with orthonormal columns."""
    import torch
    X, m, n, ldx = _matrix(X)
    dev = X.device
    Y, my, p, ldy = _matrix(Y, "Y")
    if my != m or Y.device != dev:
        raise ValueError("Y must have X's rows and live on X's device")
    # a leading dimension this large is outside what the kernel addresses
    # (QLESS_ERR_UNSUPPORTED): pass compact copies instead
    if ldx >= TWO_PHASE_LD_COPY:
        X, ldx = X.contiguous(), n
    if ldy >= TWO_PHASE_LD_COPY:
        Y, ldy = Y.contiguous(), p
    with torch.cuda.device(dev):
        if B is None:
            B = torch.empty((p, n), dtype=torch.float64, device=dev)
        elif p > 0:
            _out(B, p, n, dev, "B")
        if R is None:
            R = torch.empty((n, n), dtype=torch.float64, device=dev)
        else:
            _out(R, n, n, dev, "R")
        nbytes = int(load().qless_two_phase_workspace_bytes(m, p, n))
        if work is None:
            work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
            wb = work.numel()
        else:
            wb = _work_arg(work, dev)
        st = load().qless_two_phase_r(ctypes.c_void_p(Y.data_ptr() if p and m else 0), p, ldy,
                                      ctypes.c_void_p(X.data_ptr() if m else 0), m, n, ldx,
                                      ctypes.c_void_p(B.data_ptr() if p else 0), B.stride(0) if p > 1 else n,
                                      ctypes.c_void_p(R.data_ptr()), R.stride(0),
                                      ctypes.c_void_p(work.data_ptr()), wb, _stream(dev))
    _check(st, "qless_two_phase_r")
    return B, R


def qless_wide_r(X, panel: int = 64, R=None, Q=None, info=None, work=None):
    """R and the explicit Q of X for any n (m >= n), by BCGS2 over column
    panels of the Q-less TSQR (for n beyond 64).  Returns (R, Q, info)."""
    import torch
    X, m, n, ldx = _matrix(X)
    dev = X.device
    with torch.cuda.device(dev):
        if R is None:
            R = torch.empty((n, n), dtype=torch.float64, device=dev)
        else:
            _out(R, n, n, dev, "R")
        if Q is None:
            Q = torch.empty((m, n), dtype=torch.float64, device=dev)
        else:
            _out(Q, m, n, dev, "Q")
        if info is None:
            info = torch.empty(1, dtype=torch.int32, device=dev)
        else:
            _out(info, 0, 1, dev, "info", torch.int32)
        nbytes = int(load().qless_wide_workspace_bytes(m, n, int(panel)))
        if work is None:
            work = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
            wb = work.numel()
        else:
            wb = _work_arg(work, dev)
        st = load().qless_wide_r(ctypes.c_void_p(X.data_ptr()), m, n, ldx, ctypes.c_void_p(R.data_ptr()), R.stride(0),
                                 ctypes.c_void_p(Q.data_ptr()), Q.stride(0) if m > 1 else n, int(panel),
                                 ctypes.c_void_p(info.data_ptr()), ctypes.c_void_p(work.data_ptr()), wb, _stream(dev))
    _check(st, "qless_wide_r")
    return R, Q, info


def qless_lstsq_finish(Rt, x=None, resid=None, info=None):
    """x and |rho| from R([A b]) on the device (back substitution)."""
    import torch
    Rt, k, k2, ldr = _matrix(Rt, "Rt")
    if k != k2 or k < 2:
        raise ValueError("Rt must be a square (n+1) x (n+1) matrix with n >= 1 (got %d x %d)" % (k, k2))
    n = k - 1
    dev = Rt.device
    with torch.cuda.device(dev):
        if x is None:
            x = torch.empty(n, dtype=torch.float64, device=dev)
        else:
            _out(x, 0, n, dev, "x")
        if resid is None:
            resid = torch.empty(1, dtype=torch.float64, device=dev)
        else:
            _out(resid, 0, 1, dev, "resid")
        if info is None:
            info = torch.empty(1, dtype=torch.int32, device=dev)
        else:
            _out(info, 0, 1, dev, "info", torch.int32)
        st = load().qless_lstsq_finish(ctypes.c_void_p(Rt.data_ptr()), n, ldr, ctypes.c_void_p(x.data_ptr()),
                                       ctypes.c_void_p(resid.data_ptr()), ctypes.c_void_p(info.data_ptr()),
                                       _stream(dev))
    _check(st, "qless_lstsq_finish")
    return x, resid, info


# ------------------------------------------------------ running factorisation

class TsqrState:
    """Running Q-less TSQR of an m_total x n matrix whose rows arrive in
    chunks: the stage-1 triangles stay on the device between ``fold`` calls
    and ``finish`` runs the tree once (qless_tsqr_state_*).  Every call is
    enqueued on ``stream`` (default: the current stream at construction)."""

    def __init__(self, m_total: int, n: int, device, stream=None):
        import torch
        self.m_total, self.n, self.device = int(m_total), int(n), torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.nbytes = int(load().qless_tsqr_state_bytes(self.m_total, self.n))
        if self.nbytes == 0:
            raise ValueError("invalid running-state sizes m_total=%d n=%d" % (m_total, n))
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device=self.device)
        self.init()

    def _s(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def init(self):
        _check(load().qless_tsqr_state_init(ctypes.c_void_p(self.buf.data_ptr()), self.nbytes, self.m_total,
                                            self.n, self._s()), "qless_tsqr_state_init")

    def fold(self, X):
        X, m, n, ldx = _matrix(X)
        if n != self.n or X.device != self.device:
            raise ValueError("chunk must have %d columns and live on %s" % (self.n, self.device))
        _check(load().qless_tsqr_state_fold(ctypes.c_void_p(X.data_ptr() if m else 0), m, ldx,
                                            ctypes.c_void_p(self.buf.data_ptr()), self.nbytes, self.m_total,
                                            self.n, self._s()), "qless_tsqr_state_fold")

    def finish(self, R=None):
        import torch
        if R is None:
            with torch.cuda.stream(self.stream):
                R = torch.empty((self.n, self.n), dtype=torch.float64, device=self.device)
        else:
            _out(R, self.n, self.n, self.device, "R")
        _check(load().qless_tsqr_state_finish(ctypes.c_void_p(self.buf.data_ptr()), self.nbytes, self.m_total,
                                              self.n, ctypes.c_void_p(R.data_ptr()), R.stride(0), self._s()),
               "qless_tsqr_state_finish")
        return R


# ----------------------------------------------------------------- batched

class BatchPlan:
    """A batched Q-less TSQR over a fixed set of device matrices.

    ``Xs``: list of 2-D float64 GPU tensors (row-major rows, any m >= 0,
    1 <= n <= 64).  ``Rs``: optional list of n x n output tensors (allocated
    otherwise).  ``accumulate``: optional list of bools -- where true, the
    current content of that R is stacked in (R <- R([R; X])).  The plan and
    its device workspace are built once; ``run()`` enqueues the single
    persistent launch on the current stream and may be captured in a graph.
    """

    def __init__(self, Xs, Rs=None, accumulate=None, tile_bytes: int = 0, waves_per_cu: int = 0):
        import torch
        if not Xs:
            raise ValueError("empty batch")
        self.device = Xs[0].device
        self.Xs, self.Rs = [], []
        descs = (qless_matrix_desc * len(Xs))()
        for i, X in enumerate(Xs):
            X, m, n, ldx = _matrix(X)
            if X.device != self.device:
                raise ValueError("all matrices must be on one device")
            R = _out(Rs[i], n, n, self.device, "Rs[%d]" % i) if Rs is not None else \
                torch.zeros((n, n), dtype=torch.float64, device=self.device)
            self.Xs.append(X)
            self.Rs.append(R)
            descs[i] = qless_matrix_desc(X.data_ptr() if m else 0, m, n, ldx, R.data_ptr(), R.stride(0),
                                         1 if (accumulate is not None and accumulate[i]) else 0)
        lib = load()
        self._lib = lib
        self._plan = ctypes.c_void_p(0)
        with torch.cuda.device(self.device):
            _check(lib.qless_batch_plan_create(descs, len(Xs), int(tile_bytes), int(waves_per_cu),
                                               ctypes.byref(self._plan)), "qless_batch_plan_create")
            self.work_bytes = int(lib.qless_batch_plan_workspace_bytes(self._plan))
            self.work = torch.empty(self.work_bytes, dtype=torch.uint8, device=self.device)
            _check(lib.qless_batch_plan_upload(self._plan, ctypes.c_void_p(self.work.data_ptr()), self.work_bytes,
                                               _stream(self.device)), "qless_batch_plan_upload")
        self.tiles = int(lib.qless_batch_plan_tiles(self._plan))

    def run(self):
        import torch
        with torch.cuda.device(self.device):
            _check(self._lib.qless_tsqr_r_batched(self._plan, ctypes.c_void_p(self.work.data_ptr()),
                                                  self.work_bytes, _stream(self.device)), "qless_tsqr_r_batched")
        return self.Rs

    def close(self):
        if getattr(self, "_plan", None) is not None and self._plan.value:
            self._lib.qless_batch_plan_destroy(self._plan)
            self._plan = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def qless_tsqr_r_batched(Xs, **kw):
    """R of every matrix of the list ``Xs``: one persistent stage-1 launch plus
    one launch per tree level."""
    plan = BatchPlan(Xs, **kw)
    Rs = plan.run()
    import torch
    torch.cuda.current_stream(plan.device).synchronize()
    plan.close()
    return Rs


# ---------------------------------------------------------------- tuning

def qless_tune_set(n: int, waves_per_cu: int = 0, fan_in: int = 0, rows_per_lane: int = 0) -> None:
    _check(load().qless_tune_set(int(n), int(waves_per_cu), int(fan_in), int(rows_per_lane)), "qless_tune_set")


def qless_tune_get(n: int) -> dict:
    w, f, r = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().qless_tune_get(int(n), ctypes.byref(w), ctypes.byref(f), ctypes.byref(r)), "qless_tune_get")
    return {"waves_per_cu": w.value, "fan_in": f.value, "rows_per_lane": r.value}


# ------------------------------------------------------------------ timing

def timing_enable(on: bool = True) -> None:
    _check(load().qless_timing_enable(1 if on else 0), "qless_timing_enable")


def timing_reset() -> None:
    _check(load().qless_timing_reset(), "qless_timing_reset")


def timing_read(kernel: str) -> tuple[float, int]:
    ms = ctypes.c_double(0.0)
    cnt = ctypes.c_int64(0)
    _check(load().qless_timing_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(cnt)), "qless_timing_read")
    return ms.value, cnt.value
