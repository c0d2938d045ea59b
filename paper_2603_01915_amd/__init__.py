"""dtANS-compressed sparse matrix-vector multiplication on AMD MI355X (gfx950).

Python front end of libdtans: argument marshalling around the C ABI of
``include/dtans.h``.  Encoding runs in the library's C++ host code and every
multiplication in its HIP kernels; PyTorch only provides device memory and
the current HIP stream.  Importing works without a GPU; calls that launch
kernels need one, and everything fails loudly if ``libdtans.so`` is missing.

    A = Matrix.from_csr(row_ptr, col, vals, n)   # encode once (host)
    y = A.spmv(x)                                # y = A x, decoded on the fly
    Y = A.spmm(X)                                # k right-hand sides
    dX = A.spmm_t(dY)                            # A^T dY by decode-and-scatter
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

from . import _lib
from ._lib import (DtansError, EncodeOpts, Info, LAYOUT_AUTO, LAYOUT_NNZ, LAYOUT_ROW, STAGE_AUTO,
                   STAGE_DIRECT, STAGE_RING)

__all__ = ["Matrix", "CsrBaseline", "RocsparseBaseline", "Batch", "DtansError", "autotune", "autotune_candidates", "version",
           "LAYOUT_AUTO", "LAYOUT_ROW", "LAYOUT_NNZ", "STAGE_AUTO", "STAGE_DIRECT", "STAGE_RING"]

_LAYOUTS = {"auto": LAYOUT_AUTO, "row": LAYOUT_ROW, "nnz": LAYOUT_NNZ,
            LAYOUT_AUTO: LAYOUT_AUTO, LAYOUT_ROW: LAYOUT_ROW, LAYOUT_NNZ: LAYOUT_NNZ}


def version() -> str:
    return _lib.load().dtans_version().decode()


def _np(a, dtype=None) -> np.ndarray:
    if hasattr(a, "detach"):  # torch tensor on the host
        a = a.detach().cpu().numpy()
    return np.ascontiguousarray(a, dtype=dtype)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _dtype_code(vals: np.ndarray) -> int:
    if vals.dtype == np.float64:
        return _lib.F64
    if vals.dtype == np.float32:
        return _lib.F32
    raise TypeError("values must be float32 or float64, got %s" % vals.dtype)


def _torch():
    import torch

    return torch


def _stream(stream) -> int:
    if stream is None:
        return _torch().cuda.current_stream().cuda_stream
    return int(getattr(stream, "cuda_stream", stream))


def _dev(t, dtype, name: str, dims: int):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) tensor" % name)
    if t.dtype != dtype:
        raise TypeError("%s must be %s, got %s" % (name, dtype, t.dtype))
    if t.dim() != dims:
        raise ValueError("%s must have %d dimension(s)" % (name, dims))
    if dims == 1 and t.stride(0) != 1:
        raise ValueError("%s must be contiguous" % name)
    if dims == 2 and t.size(1) > 0 and t.stride(1) != 1:
        raise ValueError("%s must be row-major with unit column stride" % name)
    return t


def _ld(t) -> int:
    return max(int(t.stride(0)), int(t.size(1)), 1)


def _encode_opts(L, layout, lane_nnz, waves_per_wg, wg_per_cu, sort_rows, seed, stream_stage, max_mult,
                 first_delta_column, escape_in_stream=False, sort_window=0) -> EncodeOpts:
    o = EncodeOpts()
    L.dtans_default_opts(ctypes.byref(o))
    o.layout = _LAYOUTS[layout]
    o.lane_nnz = lane_nnz
    o.waves_per_wg = waves_per_wg
    o.wg_per_cu = wg_per_cu
    o.sort_rows = int(bool(sort_rows))
    o.perm_seed = seed
    o.stream_stage = stream_stage
    o.max_mult = max_mult
    o.first_delta_column = int(bool(first_delta_column))
    o.escape_in_stream = int(bool(escape_in_stream))
    o.sort_window = int(sort_window)
    return o


def symmetric_split(row_ptr, col, vals):
    """The strictly upper triangle (CSR arrays) and the diagonal (duplicates
    summed) of a square CSR matrix, for ``Matrix.spmv_sym``.  The lower
    triangle is not read: the matrix is taken to be symmetric.  Host-side
    preprocessing for the encoder."""
    rp = _np(row_ptr, np.int64)
    ci = _np(col, np.int64)
    v = _np(vals)
    m = len(rp) - 1
    rows = np.repeat(np.arange(m, dtype=np.int64), np.diff(rp))
    up = ci > rows
    diag = np.zeros(m, dtype=v.dtype)
    on = ci == rows
    np.add.at(diag, rows[on], v[on])
    rpu = np.zeros(m + 1, np.int64)
    np.cumsum(np.bincount(rows[up], minlength=m), out=rpu[1:])
    return rpu.astype(np.int32), ci[up].astype(np.int32), v[up], diag


class Matrix:
    """A CSR matrix encoded in CSR-dtANS (host container + device copy)."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)
        self._L = _lib.load()
        self._reserved = 0  # right-hand sides the device scratch is sized for
        inf = self.info()
        self.shape = (inf["m"], inf["n"])
        self.nnz = inf["nnz"]
        self.is_f64 = inf["dtype"] == _lib.F64

    # --------------------------------------------------------- construction
    @classmethod
    def from_csr(cls, row_ptr, col, vals, n: int, layout="auto", lane_nnz: int = 0,
                 waves_per_wg: int = 0, wg_per_cu: int = 0, sort_rows: bool = False,
                 seed: int = 1, stream_stage: int = 0, max_mult: int = 0,
                 first_delta_column: bool = False, gpu_encode: bool = False,
                 escape_in_stream: bool = False, sort_window: int = 0, stream=None) -> "Matrix":
        """Encode host CSR arrays.  ``gpu_encode`` runs every pass over the
        nonzeros (keys, histograms, symbols, words, escapes) on the current
        GPU; the container is the same as the host encoder's.
        ``escape_in_stream`` puts the raw bits of escaped symbols into the
        word stream instead of separate regions (host encoder only).
        ``sort_window`` (row layout, a multiple of 64) encodes the rows sorted
        by descending length within windows of that many rows (a SELL-C-sigma
        base); products and ``decode_csr`` keep the original row order."""
        L = _lib.load()
        rp = _np(row_ptr, np.int32)
        ci = _np(col, np.int32)
        v = _np(vals)
        if v.dtype not in (np.float32, np.float64):
            v = v.astype(np.float64)
        m, nnz = len(rp) - 1, len(ci)
        o = _encode_opts(L, layout, lane_nnz, waves_per_wg, wg_per_cu, sort_rows, seed, stream_stage,
                         max_mult, first_delta_column, escape_in_stream, sort_window)
        h = ctypes.c_void_p()
        if gpu_encode:
            _lib.check(L.dtans_encode_csr_gpu(m, n, nnz, _ptr(rp), _ptr(ci), _ptr(v), _dtype_code(v),
                                              ctypes.byref(o), _stream(stream), ctypes.byref(h)))
        else:
            _lib.check(L.dtans_encode_csr(m, n, nnz, _ptr(rp), _ptr(ci), _ptr(v), _dtype_code(v),
                                          ctypes.byref(o), ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def from_csr_device(cls, row_ptr, col, vals, n: int, layout="auto", lane_nnz: int = 0,
                        waves_per_wg: int = 0, wg_per_cu: int = 0, seed: int = 1, stream_stage: int = 0,
                        max_mult: int = 0, first_delta_column: bool = False, escape_in_stream: bool = False,
                        sort_window: int = 0, stream=None) -> "Matrix":
        """Encode CSR arrays already in device memory: contiguous 1-D CUDA
        tensors, row_ptr and col int32, vals float32 or float64.  The passes
        over the nonzeros run on the GPU (on `stream`, default the current
        one); the container is the same as the host encoder's."""
        torch = _torch()
        for t, name in ((row_ptr, "row_ptr"), (col, "col"), (vals, "vals")):
            if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dim() != 1 or not t.is_contiguous():
                raise TypeError("%s must be a contiguous 1-D CUDA tensor" % name)
        if row_ptr.dtype != torch.int32 or col.dtype != torch.int32:
            raise TypeError("row_ptr and col must be int32")
        if vals.dtype not in (torch.float32, torch.float64):
            raise TypeError("vals must be float32 or float64")
        if col.numel() != vals.numel() or row_ptr.numel() < 1:
            raise ValueError("col and vals must have nnz entries, row_ptr m + 1")
        L = _lib.load()
        o = _encode_opts(L, layout, lane_nnz, waves_per_wg, wg_per_cu, False, seed, stream_stage, max_mult,
                         first_delta_column, escape_in_stream, sort_window)
        code = _lib.F64 if vals.dtype == torch.float64 else _lib.F32
        h = ctypes.c_void_p()
        _lib.check(L.dtans_encode_csr_device(row_ptr.numel() - 1, n, col.numel(), row_ptr.data_ptr(),
                                             col.data_ptr(), vals.data_ptr(), code, ctypes.byref(o),
                                             _stream(stream), ctypes.byref(h)))
        return cls(h.value)

    @classmethod
    def load(cls, path: str) -> "Matrix":
        L = _lib.load()
        h = ctypes.c_void_p()
        _lib.check(L.dtans_load(str(path).encode(), ctypes.byref(h)))
        return cls(h.value)

    def save(self, path: str) -> None:
        _lib.check(self._L.dtans_save(self._h, str(path).encode()))

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.dtans_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- queries
    def info(self) -> dict:
        inf = Info()
        _lib.check(self._L.dtans_matrix_info(self._h, ctypes.byref(inf)))
        return inf.as_dict()

    @property
    def torch_dtype(self):
        torch = _torch()
        return torch.float64 if self.is_f64 else torch.float32

    def set_launch(self, waves_per_wg: int = 0, wg_per_cu: int = 0, stream_stage: int = 0) -> None:
        _lib.check(self._L.dtans_set_launch(self._h, waves_per_wg, wg_per_cu, stream_stage))

    def to_device(self, stream=None) -> "Matrix":
        """Upload to the current device (waits for the copies) and reserve the
        scratch of one right-hand side."""
        _lib.check(self._L.dtans_to_device(self._h, ctypes.c_void_p(_stream(stream))))
        self._reserved = max(self._reserved, 1)
        return self

    def reserve(self, k: int, stream=None) -> "Matrix":
        """Upload if needed and size the device scratch for products with up to
        k right-hand sides (the C product calls themselves never allocate)."""
        _lib.check(self._L.dtans_reserve(self._h, int(k), ctypes.c_void_p(_stream(stream))))
        self._reserved = max(self._reserved, int(k))
        return self

    def _ready(self, k: int, stream) -> None:
        # the binding's convenience: upload / grow the scratch on first use
        if k > self._reserved:
            self.reserve(k, stream)

    # ---------------------------------------------------------- multiplies
    def spmv(self, x, y=None, alpha: float = 1.0, beta: float = 0.0, stream=None):
        """y = alpha * A x + beta * y (device tensors)."""
        torch = _torch()
        m, n = self.shape
        _dev(x, self.torch_dtype, "x", 1)
        if x.numel() != n:
            raise ValueError("x has %d entries, expected %d" % (x.numel(), n))
        if y is None:
            y = torch.empty(m, dtype=self.torch_dtype, device=x.device)
            beta = 0.0
        _dev(y, self.torch_dtype, "y", 1)
        if y.numel() != m:
            raise ValueError("y has %d entries, expected %d" % (y.numel(), m))
        self._ready(1, stream)
        _lib.check(self._L.dtans_spmv(self._h, x.data_ptr(), y.data_ptr(), alpha, beta,
                                      ctypes.c_void_p(_stream(stream))))
        return y

    def spmv_sym(self, x, diag=None, y=None, alpha: float = 1.0, beta: float = 0.0, stream=None):
        """y = alpha * (S x + S^T x + diag .* x) + beta * y, where this matrix
        holds the strict triangle S of a symmetric matrix (see
        ``symmetric_split``) and diag its diagonal (device tensor or None)."""
        torch = _torch()
        m, n = self.shape
        if m != n:
            raise ValueError("the triangle of a symmetric matrix must be square")
        _dev(x, self.torch_dtype, "x", 1)
        if x.numel() != n:
            raise ValueError("x has %d entries, expected %d" % (x.numel(), n))
        if diag is not None:
            _dev(diag, self.torch_dtype, "diag", 1)
            if diag.numel() != n:
                raise ValueError("diag has %d entries, expected %d" % (diag.numel(), n))
        if y is None:
            y = torch.empty(m, dtype=self.torch_dtype, device=x.device)
            beta = 0.0
        _dev(y, self.torch_dtype, "y", 1)
        if y.numel() != m:
            raise ValueError("y has %d entries, expected %d" % (y.numel(), m))
        self._ready(1, stream)
        _lib.check(self._L.dtans_spmv_sym(self._h, None if diag is None else diag.data_ptr(), x.data_ptr(),
                                          y.data_ptr(), alpha, beta, ctypes.c_void_p(_stream(stream))))
        return y

    def spmm(self, X, Y=None, alpha: float = 1.0, beta: float = 0.0, stream=None):
        """Y = alpha * A X + beta * Y with X [n, k] and Y [m, k] row-major."""
        torch = _torch()
        m, n = self.shape
        _dev(X, self.torch_dtype, "X", 2)
        if X.size(0) != n:
            raise ValueError("X has %d rows, expected %d" % (X.size(0), n))
        k = X.size(1)
        if Y is None:
            Y = torch.empty((m, k), dtype=self.torch_dtype, device=X.device)
            beta = 0.0
        _dev(Y, self.torch_dtype, "Y", 2)
        if tuple(Y.shape) != (m, k):
            raise ValueError("Y must be [%d, %d]" % (m, k))
        if k == 0:
            return Y
        self._ready(k, stream)
        _lib.check(self._L.dtans_spmm(self._h, k, X.data_ptr(), _ld(X), Y.data_ptr(), _ld(Y),
                                      alpha, beta, ctypes.c_void_p(_stream(stream))))
        return Y

    def spmm_noalloc(self, X, Y, alpha: float = 1.0, beta: float = 0.0, stream=None):
        """Y = alpha * A X + beta * Y through dtans_spmm_noalloc: no device
        allocation (the library's per-device scratch array instead of the
        handle's).  X [n, k] and Y [m, k] row-major, both given by the
        caller; the matrix must already be on the device (``to_device``)."""
        m, n = self.shape
        _dev(X, self.torch_dtype, "X", 2)
        if X.size(0) != n:
            raise ValueError("X has %d rows, expected %d" % (X.size(0), n))
        k = X.size(1)
        _dev(Y, self.torch_dtype, "Y", 2)
        if tuple(Y.shape) != (m, k):
            raise ValueError("Y must be [%d, %d]" % (m, k))
        if k == 0:
            return Y
        _lib.check(self._L.dtans_spmm_noalloc(self._h, k, X.data_ptr(), _ld(X), Y.data_ptr(), _ld(Y),
                                              alpha, beta, ctypes.c_void_p(_stream(stream))))
        return Y

    def spmm_t(self, dY, dX=None, alpha: float = 1.0, beta: float = 0.0, stream=None):
        """dX = alpha * A^T dY + beta * dX with dY [m, k] and dX [n, k]."""
        torch = _torch()
        m, n = self.shape
        _dev(dY, self.torch_dtype, "dY", 2)
        if dY.size(0) != m:
            raise ValueError("dY has %d rows, expected %d" % (dY.size(0), m))
        k = dY.size(1)
        if dX is None:
            dX = torch.empty((n, k), dtype=self.torch_dtype, device=dY.device)
            beta = 0.0
        _dev(dX, self.torch_dtype, "dX", 2)
        if tuple(dX.shape) != (n, k):
            raise ValueError("dX must be [%d, %d]" % (n, k))
        if k == 0:
            return dX
        self._ready(1, stream)
        _lib.check(self._L.dtans_spmm_t(self._h, k, dY.data_ptr(), _ld(dY), dX.data_ptr(),
                                        _ld(dX), alpha, beta, ctypes.c_void_p(_stream(stream))))
        return dX

    def decode_csr(self, device=None, stream=None):
        """Decode to CSR on the GPU: (row_ptr int32, col int32, vals) tensors."""
        torch = _torch()
        m, _ = self.shape
        dev = device or torch.device("cuda", torch.cuda.current_device())
        rp = torch.empty(m + 1, dtype=torch.int32, device=dev)
        ci = torch.empty(max(self.nnz, 1), dtype=torch.int32, device=dev)
        v = torch.empty(max(self.nnz, 1), dtype=self.torch_dtype, device=dev)
        self._ready(1, stream)
        _lib.check(self._L.dtans_decode_csr(self._h, rp.data_ptr(), ci.data_ptr(), v.data_ptr(),
                                            ctypes.c_void_p(_stream(stream))))
        return rp, ci[:self.nnz], v[:self.nnz]


class _CsrProducts:
    """Shape and dtype checks shared by the uncompressed baselines (the C ABI
    cannot check the sizes of device buffers)."""

    _spmv_fn = _spmm_fn = None

    def spmv(self, x, y=None, alpha: float = 1.0, beta: float = 0.0, stream=None):
        torch = _torch()
        dt = torch.float64 if self.is_f64 else torch.float32
        m, n = self.shape
        _dev(x, dt, "x", 1)
        if x.numel() != n:
            raise ValueError("x has %d entries, expected %d" % (x.numel(), n))
        if y is None:
            y = torch.empty(m, dtype=dt, device=x.device)
            beta = 0.0
        _dev(y, dt, "y", 1)
        if y.numel() != m:
            raise ValueError("y has %d entries, expected %d" % (y.numel(), m))
        _lib.check(getattr(self._L, self._spmv_fn)(self._h, x.data_ptr(), y.data_ptr(), alpha, beta,
                                                    ctypes.c_void_p(_stream(stream))))
        return y

    def spmm(self, X, Y=None, alpha: float = 1.0, beta: float = 0.0, stream=None):
        torch = _torch()
        dt = torch.float64 if self.is_f64 else torch.float32
        m, n = self.shape
        _dev(X, dt, "X", 2)
        if X.size(0) != n:
            raise ValueError("X has %d rows, expected %d" % (X.size(0), n))
        k = X.size(1)
        if Y is None:
            Y = torch.empty((m, k), dtype=dt, device=X.device)
            beta = 0.0
        _dev(Y, dt, "Y", 2)
        if tuple(Y.shape) != (m, k):
            raise ValueError("Y must be [%d, %d]" % (m, k))
        if k == 0:
            return Y
        _lib.check(getattr(self._L, self._spmm_fn)(self._h, k, X.data_ptr(), _ld(X), Y.data_ptr(), _ld(Y),
                                                    alpha, beta, ctypes.c_void_p(_stream(stream))))
        return Y

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class CsrBaseline(_CsrProducts):
    """Plain (uncompressed) CSR SpMV/SpMM on the same GPU, for comparison."""

    _spmv_fn, _spmm_fn = "dtans_csr_spmv", "dtans_csr_spmm"

    def __init__(self, row_ptr, col, vals, n: int, variant: int = 0):
        self._L = _lib.load()
        rp = _np(row_ptr, np.int32)
        ci = _np(col, np.int32)
        v = _np(vals)
        self.shape = (len(rp) - 1, n)
        self.nnz = len(ci)
        self.is_f64 = v.dtype == np.float64
        h = ctypes.c_void_p()
        _lib.check(self._L.dtans_csr_create(len(rp) - 1, n, len(ci), _ptr(rp), _ptr(ci), _ptr(v),
                                            _dtype_code(v), variant, ctypes.byref(h)))
        self._h = h

    @property
    def bytes(self) -> int:
        return int(self._L.dtans_csr_bytes(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.dtans_csr_destroy(self._h)
            self._h = ctypes.c_void_p()


class RocsparseBaseline(_CsrProducts):
    """The platform's sparse library (rocSPARSE) on the same CSR arrays, as
    context for the plain CSR kernels; bytes as for CsrBaseline."""

    _spmv_fn, _spmm_fn = "dtans_rocsparse_spmv", "dtans_rocsparse_spmm"

    def __init__(self, row_ptr, col, vals, n: int):
        self._L = _lib.load()
        rp = _np(row_ptr, np.int32)
        ci = _np(col, np.int32)
        v = _np(vals)
        self.shape = (len(rp) - 1, n)
        self.nnz = len(ci)
        self.is_f64 = v.dtype == np.float64
        h = ctypes.c_void_p()
        _lib.check(self._L.dtans_rocsparse_create(len(rp) - 1, n, len(ci), _ptr(rp), _ptr(ci), _ptr(v),
                                                  _dtype_code(v), ctypes.byref(h)))
        self._h = h

    @property
    def bytes(self) -> int:
        m, _ = self.shape
        return 4 * (m + 1) + self.nnz * (4 + (8 if self.is_f64 else 4))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.dtans_rocsparse_destroy(self._h)
            self._h = ctypes.c_void_p()


class Batch:
    """Several encoded matrices multiplied in one persistent launch."""

    def __init__(self, matrices: Sequence[Matrix]):
        self._L = _lib.load()
        self.matrices = list(matrices)
        arr = (ctypes.c_void_p * len(self.matrices))(*[m._h.value for m in self.matrices])
        h = ctypes.c_void_p()
        _lib.check(self._L.dtans_batch_create(len(self.matrices), arr, ctypes.byref(h)))
        self._h = h

    def spmv(self, xs, ys=None, alpha: float = 1.0, beta: float = 0.0, stream=None):
        torch = _torch()
        if ys is None:
            ys = [torch.empty(m.shape[0], dtype=m.torch_dtype, device=x.device)
                  for m, x in zip(self.matrices, xs)]
            beta = 0.0
        for m, x, y in zip(self.matrices, xs, ys):
            _dev(x, m.torch_dtype, "x", 1)
            _dev(y, m.torch_dtype, "y", 1)
            if x.numel() != m.shape[1] or y.numel() != m.shape[0]:
                raise ValueError("vector sizes do not match the matrices")
        cnt = len(self.matrices)
        xa = (ctypes.c_void_p * cnt)(*[x.data_ptr() for x in xs])
        ya = (ctypes.c_void_p * cnt)(*[y.data_ptr() for y in ys])
        _lib.check(self._L.dtans_batch_spmv(self._h, xa, ya, alpha, beta,
                                            ctypes.c_void_p(_stream(stream))))
        return ys

    def spmm(self, Xs, Ys=None, alpha: float = 1.0, beta: float = 0.0, stream=None):
        """Y_i = alpha * A_i X_i + beta * Y_i with X_i [n_i, k], Y_i [m_i, k]
        contiguous (the same k for every matrix)."""
        torch = _torch()
        if len(Xs) != len(self.matrices):
            raise ValueError("one X per matrix")
        k = Xs[0].size(1) if Xs and Xs[0].dim() == 2 else 0
        if Ys is None:
            Ys = [torch.empty((m.shape[0], k), dtype=m.torch_dtype, device=X.device)
                  for m, X in zip(self.matrices, Xs)]
            beta = 0.0
        for m, X, Y in zip(self.matrices, Xs, Ys):
            _dev(X, m.torch_dtype, "X", 2)
            _dev(Y, m.torch_dtype, "Y", 2)
            if tuple(X.shape) != (m.shape[1], k) or tuple(Y.shape) != (m.shape[0], k):
                raise ValueError("X_i must be [n_i, k] and Y_i [m_i, k] with one k")
            if X.stride(0) != k or Y.stride(0) != k:
                raise ValueError("X_i and Y_i must be contiguous")
        if k == 0:
            return Ys
        cnt = len(self.matrices)
        xa = (ctypes.c_void_p * cnt)(*[X.data_ptr() for X in Xs])
        ya = (ctypes.c_void_p * cnt)(*[Y.data_ptr() for Y in Ys])
        _lib.check(self._L.dtans_batch_spmm(self._h, k, xa, ya, alpha, beta,
                                            ctypes.c_void_p(_stream(stream))))
        return Ys

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self._L.dtans_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _tune_opts(layout, lane_nnz, waves_per_wg, wg_per_cu, stream_stage=0, sort_rows=False,
               perm_seed=1):
    o = EncodeOpts()
    _lib.load().dtans_default_opts(ctypes.byref(o))
    o.layout = _LAYOUTS[layout]
    o.lane_nnz = lane_nnz
    o.waves_per_wg = waves_per_wg
    o.wg_per_cu = wg_per_cu
    o.stream_stage = stream_stage
    o.sort_rows = int(bool(sort_rows))
    o.perm_seed = perm_seed
    return o


def _opts_dict(o) -> dict:
    return {"layout": o.layout, "lane_nnz": o.lane_nnz, "waves_per_wg": o.waves_per_wg,
            "wg_per_cu": o.wg_per_cu, "stream_stage": o.stream_stage}


def autotune_candidates(row_ptr, nnz: int, dtype=np.float64, k: int = 1, layout="auto",
                        lane_nnz: int = 0, waves_per_wg: int = 0, wg_per_cu: int = 0,
                        stream_stage: int = 0):
    """The options ``autotune`` would time, in its order (host only)."""
    L = _lib.load()
    rp = _np(row_ptr, np.int32)
    o = _tune_opts(layout, lane_nnz, waves_per_wg, wg_per_cu, stream_stage)
    code = _lib.F64 if np.dtype(dtype) == np.float64 else _lib.F32
    cnt = L.dtans_autotune_candidates(len(rp) - 1, nnz, _ptr(rp), code, k, ctypes.byref(o), None, 0)
    if cnt < 0:
        raise DtansError(_lib.EINVAL, L.dtans_last_error().decode())
    out = (EncodeOpts * max(cnt, 1))()
    L.dtans_autotune_candidates(len(rp) - 1, nnz, _ptr(rp), code, k, ctypes.byref(o), out, cnt)
    return [_opts_dict(out[i]) for i in range(cnt)]


def autotune(row_ptr, col, vals, n: int, k: int = 1, budget_s: float = 20.0,
             layout="auto", lane_nnz: int = 0, waves_per_wg: int = 0, wg_per_cu: int = 0,
             stream_stage: int = 0, cache: str | None = None):
    """Search layout, nonzeros per lane and launch shape on the current GPU.
    Returns (options dict for ``Matrix.from_csr``, best milliseconds per
    multiplication).  ``cache``: optional text file of earlier results."""
    L = _lib.load()
    rp = _np(row_ptr, np.int32)
    ci = _np(col, np.int32)
    v = _np(vals)
    if v.dtype not in (np.float32, np.float64):
        v = v.astype(np.float64)
    o = _tune_opts(layout, lane_nnz, waves_per_wg, wg_per_cu, stream_stage)
    best = ctypes.c_double()
    _lib.check(L.dtans_autotune(len(rp) - 1, n, len(ci), _ptr(rp), _ptr(ci), _ptr(v),
                                _dtype_code(v), k, budget_s,
                                None if cache is None else os.fsencode(cache),
                                ctypes.byref(o), ctypes.byref(best)))
    return _opts_dict(o), best.value
