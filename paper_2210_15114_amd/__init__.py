"""Implicit distance-matrix matrix-vector products on MI355X (gfx950).

Thin Python binding over the C ABI in ``include/dm.h`` (``libdm.so``).  It
only marshals arguments: tensors are caller-owned device memory allocated by
PyTorch, streams are PyTorch's current stream, and every step of the
computation runs in the library's HIP kernels.  There is no fallback: if the
library is missing or no GPU is present, calls raise.

    import torch, paper_2210_15114_amd as dm
    h = dm.prepare(X_cuda, dm.L1)          # Algorithm 1 (sort every coordinate)
    Y = h.matvec(Z_cuda)                    # A Z for b = Z.shape[1] right-hand sides
    h.sync()                                # raises on a sticky device-side error
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdm.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "dm.h")

L1 = 1
L2SQ = 2
TV = 3
L3 = 4
L5 = 5
L4 = 6
L6 = 7
KL = 8
CE = 9
MAHA2 = 10
BILINEAR = 11
MATRIX_METRICS = (MAHA2, BILINEAR)
F32, F64, I32, I64 = 1, 2, 3, 4

OK = 0
ERR_ARG, ERR_NONFINITE, ERR_OVERFLOW, ERR_NOMEM, ERR_DEVICE, ERR_DTYPE, ERR_STATE = -1, -2, -3, -4, -5, -6, -7

_lib = None


class Dataset(ctypes.Structure):
    """dm_dataset: one point set of a multi-dataset handle."""
    _fields_ = [("X", ctypes.c_void_p), ("n", ctypes.c_int64), ("d", ctypes.c_int32),
                ("metric", ctypes.c_int32), ("dtype", ctypes.c_int32)]


class DMError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__("%s: %s (%d)" % (where, status_string(status), status))


def lib():
    """The loaded libdm.so (ctypes).  Raises ImportError when it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libdm.so is not built; run `python -m paper_2210_15114_amd.build` "
                          "(or __graft_entry__.build())")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    L.dm_status_string.argtypes = [i32]
    L.dm_status_string.restype = ctypes.c_char_p
    L.dm_workspace_size.argtypes = [i64, i32, i32, i32, ctypes.POINTER(sz)]
    L.dm_workspace_size.restype = i32
    L.dm_prepare.argtypes = [P, i64, i32, i32, i32, P, sz, P, ctypes.POINTER(P)]
    L.dm_prepare.restype = i32
    L.dm_prepare_matrix.argtypes = [P, i64, i32, i32, i32, P, P, sz, P, ctypes.POINTER(P)]
    L.dm_prepare_matrix.restype = i32
    L.dm_matvec.argtypes = [P, P, i32, i32, P, P]
    L.dm_matvec.restype = i32
    L.dm_matvec_static.argtypes = [P, P, i32, i32, P, P]
    L.dm_matvec_static.restype = i32
    L.dm_reserve.argtypes = [P, i32]
    L.dm_reserve.restype = i32
    L.dm_sync.argtypes = [P]
    L.dm_sync.restype = i32
    L.dm_info.argtypes = [P, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.dm_info.restype = i32
    L.dm_copy_sorted.argtypes = [P, P, P, P, P]
    L.dm_copy_sorted.restype = i32
    L.dm_int_bound_ok.argtypes = [ctypes.c_double, ctypes.c_double]
    L.dm_int_bound_ok.restype = ctypes.c_int
    L.dm_free.argtypes = [P]
    L.dm_free.restype = None
    L.dm_profile_enable.argtypes = [P, i32]
    L.dm_profile_enable.restype = i32
    L.dm_profile_read.argtypes = [P, i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64)]
    L.dm_profile_read.restype = i32
    L.dm_copy_probe.argtypes = [P, P, sz, P]
    L.dm_copy_probe.restype = i32
    L.dm_gather_probe.argtypes = [P, P, P, i64, i32, P]
    L.dm_gather_probe.restype = i32
    L.dm_workspace_size_multi.argtypes = [ctypes.POINTER(Dataset), i32, ctypes.POINTER(sz)]
    L.dm_workspace_size_multi.restype = i32
    L.dm_prepare_multi.argtypes = [ctypes.POINTER(Dataset), i32, P, sz, P, ctypes.POINTER(P)]
    L.dm_prepare_multi.restype = i32
    L.dm_matvec_multi.argtypes = [P, ctypes.POINTER(P), i32, ctypes.POINTER(P), P]
    L.dm_matvec_multi.restype = i32
    L.dm_multi_variant_count.argtypes = []
    L.dm_multi_variant_count.restype = i32
    L.dm_tune_multi.argtypes = [P, ctypes.POINTER(P), i32, ctypes.POINTER(P), i32, P, ctypes.POINTER(i32),
                                ctypes.POINTER(ctypes.c_double)]
    L.dm_tune_multi.restype = i32
    L.dm_set_variant_multi.argtypes = [P, i32, i32]
    L.dm_set_variant_multi.restype = i32
    L.dm_get_variant_multi.argtypes = [P, i32, ctypes.POINTER(i32)]
    L.dm_get_variant_multi.restype = i32
    L.dm_multi_count.argtypes = [P, ctypes.POINTER(i32)]
    L.dm_multi_count.restype = i32
    L.dm_variant_count.argtypes = []
    L.dm_variant_count.restype = i32
    L.dm_tune.argtypes = [P, i32, i32, i32, P, ctypes.POINTER(i32), ctypes.POINTER(ctypes.c_double)]
    L.dm_tune.restype = i32
    L.dm_set_variant.argtypes = [P, i32, i32, i32]
    L.dm_set_variant.restype = i32
    L.dm_get_variant.argtypes = [P, i32, i32, ctypes.POINTER(i32)]
    L.dm_get_variant.restype = i32
    L.dm_lowrank.argtypes = [P, i32, i32, i32, P, P, P, P, ctypes.POINTER(i32)]
    L.dm_lowrank.restype = i32
    L.dm_embed_l2.argtypes = [P, i64, i32, i32, P, i32, P, P]
    L.dm_embed_l2.restype = i32
    _lib = L
    return L


def header_functions() -> list:
    """Names of the functions include/dm.h declares."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dm_[a-z0-9_]+)\s*\(", text)))


def status_string(status: int) -> str:
    return lib().dm_status_string(int(status)).decode()


def _check(st: int, where: str):
    if st != OK:
        raise DMError(st, where)


def workspace_size(n: int, d: int, metric: int, dtype: int) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().dm_workspace_size(n, d, metric, dtype, ctypes.byref(out)), "dm_workspace_size")
    return out.value


def int_bound_ok(sum_ranges: float, z_l1: float) -> bool:
    return bool(lib().dm_int_bound_ok(float(sum_ranges), float(z_l1)))


K_L1_PASS, K_TOTALS, K_L2, K_SORTFREE = 0, 1, 2, 3


def copy_probe(dst, src, stream=None):
    """Streaming device copy of src into dst (same byte size), for bandwidth calibration."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes:
        raise ValueError("size mismatch")
    _check(lib().dm_copy_probe(_dev_ptr(dst, "dst"), _dev_ptr(src, "src"), nbytes, _stream_ptr(stream)),
           "dm_copy_probe")


def gather_probe(perm, Z, Out, stream=None):
    """Out[perm[r]] += Z[perm[r]] for every r (perm: int32 device tensor of
    point indices; Z, Out: n x b float32 device tensors): the random-row
    accesses of a coordinate pass without its scan."""
    n, b = Z.shape
    if tuple(Out.shape) != (n, b) or perm.numel() != n:
        raise ValueError("shape mismatch")
    _check(lib().dm_gather_probe(_dev_ptr(perm, "perm"), _dev_ptr(Z, "Z"), _dev_ptr(Out, "Out"), n, b,
                                 _stream_ptr(stream)), "dm_gather_probe")


def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    m = {torch.float32: F32, torch.float64: F64, torch.int32: I32, torch.int64: I64}
    if t not in m:
        raise TypeError("unsupported dtype %s" % t)
    return m[t]


def _stream_ptr(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, name):
    if not t.is_cuda:
        raise ValueError("%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return ctypes.c_void_p(t.data_ptr())


class Handle:
    """A prepared point set (one dataset).  Owns its workspace tensor."""

    def __init__(self, ptr, workspace, n, d, metric, dtype):
        self._ptr = ptr
        self._ws = workspace
        self.n, self.d, self.metric, self.dtype = n, d, metric, dtype

    @property
    def is_int(self) -> bool:
        return self.dtype in (I32, I64)

    def matvec(self, Z, out=None, stream=None):
        """Out = A Z (Z: n x b or n device tensor; float32, or int32/int64 for integer data)."""
        torch = _torch()
        squeeze = Z.dim() == 1
        Zm = Z.unsqueeze(1) if squeeze else Z
        if Zm.dim() != 2 or Zm.shape[0] != self.n:
            raise ValueError("Z must be n x b")
        b = Zm.shape[1]
        odt = torch.int64 if self.is_int else torch.float32
        if out is None:
            out = torch.empty((self.n, b), dtype=odt, device=Zm.device)
        elif out.shape != (self.n, b) and not (squeeze and out.shape == (self.n,)):
            raise ValueError("out has the wrong shape")
        st = lib().dm_matvec(self._ptr, _dev_ptr(Zm, "Z"), _dtype_code(Zm.dtype), b, _dev_ptr(out, "out"),
                             _stream_ptr(stream))
        _check(st, "dm_matvec")
        return out.view(self.n) if squeeze and out.dim() == 2 else out

    def matvec_static(self, Z, out, stream=None):
        """Out = A Z through dm_matvec_static (scratch in the library's static
        device array; allocates nothing).  out must be given (n x b)."""
        squeeze = Z.dim() == 1
        Zm = Z.unsqueeze(1) if squeeze else Z
        if Zm.dim() != 2 or Zm.shape[0] != self.n:
            raise ValueError("Z must be n x b")
        b = Zm.shape[1]
        if out.numel() != self.n * b:
            raise ValueError("out has the wrong shape")
        st = lib().dm_matvec_static(self._ptr, _dev_ptr(Zm, "Z"), _dtype_code(Zm.dtype), b, _dev_ptr(out, "out"),
                                    _stream_ptr(stream))
        _check(st, "dm_matvec_static")
        return out

    def reserve(self, b: int):
        _check(lib().dm_reserve(self._ptr, b), "dm_reserve")

    def _zcode(self, z_dtype):
        torch = _torch()
        if z_dtype is None:
            z_dtype = torch.int32 if self.is_int else torch.float32
        return _dtype_code(z_dtype)

    def tune(self, b: int, z_dtype=None, reps: int = 6, stream=None):
        """Time the l1 pass tile variants for b columns; keep the fastest.

        Returns (chosen variant, list of mean pass times in ms)."""
        nv = lib().dm_variant_count()
        ms = (ctypes.c_double * nv)()
        chosen = ctypes.c_int32(-1)
        _check(lib().dm_tune(self._ptr, b, self._zcode(z_dtype), reps, _stream_ptr(stream), ctypes.byref(chosen),
                             ms), "dm_tune")
        return chosen.value, list(ms)

    def set_variant(self, b: int, variant: int, z_dtype=None):
        _check(lib().dm_set_variant(self._ptr, b, self._zcode(z_dtype), variant), "dm_set_variant")

    def get_variant(self, b: int, z_dtype=None) -> int:
        v = ctypes.c_int32(-1)
        _check(lib().dm_get_variant(self._ptr, b, self._zcode(z_dtype), ctypes.byref(v)), "dm_get_variant")
        return v.value

    def sync(self):
        _check(lib().dm_sync(self._ptr), "dm_sync")

    def lowrank(self, rank: int, omega, iters: int = 8, stream=None):
        """Rank-`rank` approximation A ~ U diag(lam) U^T by block Krylov iteration.

        omega: n x block float64 device tensor (the start block).  Returns
        (U: n x rank float64, lam: rank float64, Jacobi sweeps used)."""
        torch = _torch()
        if omega.dim() != 2 or omega.shape[0] != self.n or omega.dtype != torch.float64:
            raise ValueError("omega must be an n x block float64 tensor")
        U = torch.empty((self.n, rank), dtype=torch.float64, device=omega.device)
        lam = torch.empty(rank, dtype=torch.float64, device=omega.device)
        sw = ctypes.c_int32(0)
        _check(lib().dm_lowrank(self._ptr, rank, omega.shape[1], iters, _dev_ptr(omega, "omega"), _dev_ptr(U, "U"),
                                _dev_ptr(lam, "lam"), _stream_ptr(stream), ctypes.byref(sw)), "dm_lowrank")
        return U, lam, sw.value

    def sorted(self, stream=None):
        """(perm, rank, xs), each d x n on the device (l1 handles)."""
        torch = _torch()
        dev = self._ws.device
        perm = torch.empty((self.d, self.n), dtype=torch.int32, device=dev)
        rank = torch.empty((self.d, self.n), dtype=torch.int32, device=dev)
        xs = torch.empty((self.d, self.n), dtype=torch.int32 if self.is_int else torch.float32, device=dev)
        st = lib().dm_copy_sorted(self._ptr, _dev_ptr(perm, "perm"), _dev_ptr(rank, "rank"), _dev_ptr(xs, "xs"),
                                  _stream_ptr(stream))
        _check(st, "dm_copy_sorted")
        return perm, rank, xs

    def profile(self, on: bool = True):
        _check(lib().dm_profile_enable(self._ptr, 1 if on else 0), "dm_profile_enable")

    def profile_read(self, kernel_class: int):
        """(total device ms, launches) of one kernel class since profiling was switched on."""
        ms = ctypes.c_double(0.0)
        cnt = ctypes.c_int64(0)
        _check(lib().dm_profile_read(self._ptr, kernel_class, ctypes.byref(ms), ctypes.byref(cnt)),
               "dm_profile_read")
        return ms.value, cnt.value

    def free(self):
        if self._ptr:
            lib().dm_free(self._ptr)
            self._ptr = None
            self._ws = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def embed_l2(X, G, stream=None):
    """Embedded points X' (n x k float32) = (1 / (beta k)) X G^T, beta = sqrt(2/pi).

    X: n x d device tensor; G: k x d float64 device tensor of iid N(0,1).  The
    l1 distance matrix of X' approximates the l2 distance matrix of X."""
    torch = _torch()
    if X.dim() != 2 or G.dim() != 2 or G.shape[1] != X.shape[1] or G.dtype != torch.float64:
        raise ValueError("X must be n x d and G a k x d float64 tensor")
    n, d = X.shape
    k = G.shape[0]
    out = torch.empty((n, k), dtype=torch.float32, device=X.device)
    _check(lib().dm_embed_l2(_dev_ptr(X, "X"), n, d, _dtype_code(X.dtype), _dev_ptr(G, "G"), k, _dev_ptr(out, "out"),
                             _stream_ptr(stream)), "dm_embed_l2")
    return out


def prepare_l2_approx(X, G, stream=None) -> "Handle":
    """Handle whose queries approximate products with the l2 distance matrix of
    X: the l1 path on the embedded points embed_l2(X, G)."""
    Xe = embed_l2(X, G, stream)
    h = prepare(Xe, L1, stream)
    return h


def prepare(X, metric: int = L1, stream=None, M=None) -> Handle:
    """Prepare a point set X (n x d device tensor: float32/float64/int32/int64).

    M: the d x d matrix of MAHA2 and BILINEAR (host array-like, copied as
    float64 row-major); must be None for the other metrics."""
    torch = _torch()
    if X.dim() != 2:
        raise ValueError("X must be n x d")
    n, d = X.shape
    code = _dtype_code(X.dtype)
    ws_bytes = workspace_size(n, d, metric, code)
    ws = torch.empty(ws_bytes + 256, dtype=torch.uint8, device=X.device)
    off = (-ws.data_ptr()) % 256
    wsv = ws[off:off + ws_bytes]
    h = ctypes.c_void_p(None)
    if M is None:
        st = lib().dm_prepare(_dev_ptr(X, "X"), n, d, metric, code, ctypes.c_void_p(wsv.data_ptr()), ws_bytes,
                              _stream_ptr(stream), ctypes.byref(h))
        _check(st, "dm_prepare")
    else:
        import numpy as np
        Mh = np.ascontiguousarray(np.asarray(M, dtype=np.float64))
        if Mh.shape != (d, d):
            raise ValueError("M must be d x d")
        st = lib().dm_prepare_matrix(_dev_ptr(X, "X"), n, d, metric, code, Mh.ctypes.data_as(ctypes.c_void_p),
                                     ctypes.c_void_p(wsv.data_ptr()), ws_bytes, _stream_ptr(stream), ctypes.byref(h))
        _check(st, "dm_prepare_matrix")
    return Handle(h, ws, n, d, metric, code)


class MultiHandle:
    """Many prepared point sets answered together (one captured graph per b)."""

    def __init__(self, ptr, workspace, shapes, dtypes):
        self._ptr = ptr
        self._ws = workspace
        self.shapes = shapes          # [(n, d)]
        self.dtypes = dtypes          # dtype codes

    def _ptrs(self, Zs, outs):
        torch = _torch()
        if len(Zs) != len(self.shapes):
            raise ValueError("one Z per dataset")
        b = Zs[0].shape[1]
        if outs is None:
            outs = [torch.empty((n, b), dtype=torch.int64 if t in (I32, I64) else torch.float32, device=Z.device)
                    for (n, _), t, Z in zip(self.shapes, self.dtypes, Zs)]
        zp = (ctypes.c_void_p * len(Zs))()
        op = (ctypes.c_void_p * len(Zs))()
        for i, (Z, O, (n, _), t) in enumerate(zip(Zs, outs, self.shapes, self.dtypes)):
            if Z.dim() != 2 or Z.shape != (n, b):
                raise ValueError("Z[%d] must be n x b" % i)
            want = torch.int32 if t in (I32, I64) else torch.float32
            if Z.dtype != want:
                raise DMError(ERR_DTYPE, "dm_matvec_multi")
            zp[i] = _dev_ptr(Z, "Z").value
            op[i] = _dev_ptr(O, "out").value
        self._keep = (Zs, outs)       # the graph reads these pointers when it runs
        return b, zp, op, outs

    def matvec(self, Zs, outs=None, stream=None):
        """Outs[s] = A_s Zs[s] for every dataset (same b for all)."""
        b, zp, op, outs = self._ptrs(Zs, outs)
        _check(lib().dm_matvec_multi(self._ptr, zp, b, op, _stream_ptr(stream)), "dm_matvec_multi")
        return outs

    def tune(self, Zs, outs=None, reps: int = 3, stream=None):
        """Time every tile variant of the query on these right-hand sides and
        keep the fastest; returns (variant, [ms per query per variant], outs)."""
        b, zp, op, outs = self._ptrs(Zs, outs)
        nv = lib().dm_multi_variant_count()
        ch = ctypes.c_int32(0)
        ms = (ctypes.c_double * nv)()
        _check(lib().dm_tune_multi(self._ptr, zp, b, op, reps, _stream_ptr(stream), ctypes.byref(ch), ms),
               "dm_tune_multi")
        return ch.value, list(ms), outs

    def set_variant(self, b: int, variant: int):
        _check(lib().dm_set_variant_multi(self._ptr, b, variant), "dm_set_variant_multi")

    def get_variant(self, b: int) -> int:
        v = ctypes.c_int32(0)
        _check(lib().dm_get_variant_multi(self._ptr, b, ctypes.byref(v)), "dm_get_variant_multi")
        return v.value

    def sync(self):
        _check(lib().dm_sync(self._ptr), "dm_sync")

    def free(self):
        if self._ptr:
            lib().dm_free(self._ptr)
            self._ptr = None
            self._ws = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def prepare_multi(Xs, stream=None) -> MultiHandle:
    """Prepare many point sets (list of n_s x d_s device tensors) for l1 queries."""
    torch = _torch()
    arr = (Dataset * len(Xs))()
    shapes, codes = [], []
    for i, X in enumerate(Xs):
        if X.dim() != 2:
            raise ValueError("X[%d] must be n x d" % i)
        code = _dtype_code(X.dtype)
        arr[i] = Dataset(_dev_ptr(X, "X").value, X.shape[0], X.shape[1], L1, code)
        shapes.append((X.shape[0], X.shape[1]))
        codes.append(code)
    nbytes = ctypes.c_size_t(0)
    _check(lib().dm_workspace_size_multi(arr, len(Xs), ctypes.byref(nbytes)), "dm_workspace_size_multi")
    ws = torch.empty(nbytes.value + 256, dtype=torch.uint8, device=Xs[0].device)
    off = (-ws.data_ptr()) % 256
    h = ctypes.c_void_p(None)
    _check(lib().dm_prepare_multi(arr, len(Xs), ctypes.c_void_p(ws.data_ptr() + off), nbytes.value,
                                  _stream_ptr(stream), ctypes.byref(h)), "dm_prepare_multi")
    return MultiHandle(h, ws, shapes, codes)
