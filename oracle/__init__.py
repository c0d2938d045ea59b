"""Oracle for CSR-dtANS SpMV: a plain, slow CPU implementation.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The product
(``paper_2603_01915_amd``) never imports it, and it never imports the product.

Contents:
  * ``liboracle.so`` (built from ``dtans_oracle.c`` with gcc): FP64 CSR SpMV,
    A^T x, multi-vector SpMM, (|A||x|) and a reference CSR-dtANS codec;
  * ``toy``: a generic big-integer tANS/dtANS codec pinned to the paper's
    worked examples;
  * ``container``: a Python reader/writer of the container format and a
    big-integer whole-matrix codec for tiny matrices.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "dtans_oracle.c")
_lib = None

ERRORS = {0: "ok", 1: "invalid argument", 2: "i/o error", 3: "corrupt container", 4: "out of memory"}


class OracleError(RuntimeError):
    pass


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (plain -O2, no vectorisation flags;
    OpenMP only splits the rows of the two products over threads)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-Wall", "-shared", "-fPIC", "-fopenmp",
                               "-o", tmp, _SRC])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_SO)
        P, I64, D = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        L.oracle_set_threads.argtypes = [ctypes.c_int]
        L.oracle_set_threads(1)
        L.oracle_csr_spmv_f64.argtypes = [I64, P, P, P, P, P, D, D]
        L.oracle_csr_absmv_f64.argtypes = [I64, P, P, P, P, P]
        L.oracle_csr_spmtv_f64.argtypes = [I64, I64, P, P, P, P, P, D, D]
        L.oracle_csr_spmm_f64.argtypes = [I64, I64, P, P, P, P, I64, P, I64, D, D]
        L.oracle_encode.argtypes = [ctypes.c_char_p, I64, I64, I64, P, P, P, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int]
        L.oracle_encode.restype = ctypes.c_int
        L.oracle_decode.argtypes = [ctypes.c_char_p, P, P, P]
        L.oracle_decode.restype = ctypes.c_int
        L.oracle_read_header.argtypes = [ctypes.c_char_p, P]
        L.oracle_read_header.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(row_ptr, col, val):
    return (np.ascontiguousarray(row_ptr, np.int32), np.ascontiguousarray(col, np.int32),
            np.ascontiguousarray(val, np.float64))


def set_threads(t: int) -> None:
    """Threads the SpMV / SpMM products split their rows over (default 1)."""
    lib().oracle_set_threads(int(t))


def spmv(row_ptr, col, val, x, y=None, alpha=1.0, beta=0.0):
    """y = alpha*A*x + beta*y in FP64 (inputs of any float type are widened
    exactly to FP64 first)."""
    rp, ci, v = _csr(row_ptr, col, val)
    m = len(rp) - 1
    x = np.ascontiguousarray(x, np.float64)
    out = np.zeros(m) if y is None else np.array(y, np.float64, copy=True)
    lib().oracle_csr_spmv_f64(m, _p(rp), _p(ci), _p(v), _p(x), _p(out), alpha, beta)
    return out


def absmv(row_ptr, col, val, x):
    rp, ci, v = _csr(row_ptr, col, val)
    m = len(rp) - 1
    x = np.ascontiguousarray(x, np.float64)
    out = np.zeros(m)
    lib().oracle_csr_absmv_f64(m, _p(rp), _p(ci), _p(v), _p(x), _p(out))
    return out


def spmtv(row_ptr, col, val, n, x, y=None, alpha=1.0, beta=0.0):
    rp, ci, v = _csr(row_ptr, col, val)
    m = len(rp) - 1
    x = np.ascontiguousarray(x, np.float64)
    out = np.zeros(n) if y is None else np.array(y, np.float64, copy=True)
    lib().oracle_csr_spmtv_f64(m, n, _p(rp), _p(ci), _p(v), _p(x), _p(out), alpha, beta)
    return out


def spmm(row_ptr, col, val, X, Y=None, alpha=1.0, beta=0.0):
    rp, ci, v = _csr(row_ptr, col, val)
    m = len(rp) - 1
    X = np.ascontiguousarray(X, np.float64)
    k = X.shape[1]
    out = np.zeros((m, k)) if Y is None else np.array(Y, np.float64, copy=True)
    lib().oracle_csr_spmm_f64(m, k, _p(rp), _p(ci), _p(v), _p(X), k, _p(out), k, alpha, beta)
    return out


def encode(path: str, m: int, n: int, row_ptr, col, vals, layout: int = 1, lane_nnz: int = 0,
           seed: int = 1, first_mode: int = 0, esc_mode: int = 0, sigma: int = 0) -> None:
    """Write a CSR-dtANS container with the reference encoder.  first_mode 0:
    the first delta of a row is its column (the paper's form); 1: column -
    row + 2^29 modulo 2^32 (the library's default).  esc_mode 0: escaped
    symbols in separate regions per wave; 1: in the word stream, after the
    words read before the step that decodes them (Sec. IV-F).  sigma (row
    layout, a multiple of 64): rows sorted by descending length within
    windows of sigma rows before encoding, the order stored (a SELL-C-sigma
    base, Sec. VII); decoding restores the original order."""
    rp = np.ascontiguousarray(row_ptr, np.int32)
    ci = np.ascontiguousarray(col, np.int32)
    vals = np.ascontiguousarray(vals)
    dtype = {np.dtype(np.float32): 1, np.dtype(np.float64): 2}[vals.dtype]
    rc = lib().oracle_encode(path.encode(), m, n, int(rp[-1]), _p(rp), _p(ci), _p(vals), dtype,
                             layout, lane_nnz, seed, first_mode, esc_mode, sigma)
    if rc:
        raise OracleError("oracle_encode: " + ERRORS.get(rc, str(rc)))


def read_header(path: str) -> dict:
    out = np.zeros(16, np.int64)
    rc = lib().oracle_read_header(path.encode(), _p(out))
    if rc:
        raise OracleError("oracle_read_header: " + ERRORS.get(rc, str(rc)))
    keys = ["dtype", "layout", "lane_nnz", "m", "n", "nnz", "num_lanes", "num_waves", "n_words",
            "n_esc_delta", "n_esc_value", "seed", "file_bytes", "first_mode", "esc_mode", "sigma"]
    return dict(zip(keys, (int(v) for v in out)))


def decode(path: str):
    """Decode a container to (row_ptr, col, vals) with the reference decoder."""
    h = read_header(path)
    rp = np.zeros(h["m"] + 1, np.int32)
    ci = np.zeros(max(h["nnz"], 1), np.int32)
    vals = np.zeros(max(h["nnz"], 1), np.float64 if h["dtype"] == 2 else np.float32)
    rc = lib().oracle_decode(path.encode(), _p(rp), _p(ci), _p(vals))
    if rc:
        raise OracleError("oracle_decode: " + ERRORS.get(rc, str(rc)))
    return rp, ci[:h["nnz"]], vals[:h["nnz"]]
