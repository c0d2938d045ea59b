"""ctypes binding of libdtans.so (argument marshalling only).

Every computation happens in the library's C++ host code or its HIP kernels;
this module only loads the shared library, declares the C signatures of
``include/dtans.h`` and converts status codes into exceptions.  It fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdtans.so")

OK, EINVAL, EUNSORTED, ERANGE, ENOMEM, EHIP, ECORRUPT, EUNSUPPORTED, EIO = range(9)
F32, F64 = 1, 2
LAYOUT_AUTO, LAYOUT_ROW, LAYOUT_NNZ = 0, 1, 2
STAGE_AUTO, STAGE_DIRECT, STAGE_RING = 0, 1, 2

_NAMES = {EINVAL: "EINVAL", EUNSORTED: "EUNSORTED", ERANGE: "ERANGE", ENOMEM: "ENOMEM",
          EHIP: "EHIP", ECORRUPT: "ECORRUPT", EUNSUPPORTED: "EUNSUPPORTED", EIO: "EIO"}


class DtansError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (_NAMES.get(status, str(status)), message))
        self.status = status


class EncodeOpts(ctypes.Structure):
    _fields_ = [("layout", ctypes.c_int32), ("lane_nnz", ctypes.c_int32),
                ("waves_per_wg", ctypes.c_int32), ("wg_per_cu", ctypes.c_int32),
                ("sort_rows", ctypes.c_int32), ("stream_stage", ctypes.c_int32),
                ("max_mult", ctypes.c_int32), ("first_delta_column", ctypes.c_int32),
                ("escape_in_stream", ctypes.c_int32), ("sort_window", ctypes.c_int32),
                ("reserved0", ctypes.c_int32), ("perm_seed", ctypes.c_uint64)]


class Info(ctypes.Structure):
    _fields_ = [("m", ctypes.c_int64), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("dtype", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("lane_nnz", ctypes.c_int32), ("waves_per_wg", ctypes.c_int32),
                ("num_lanes", ctypes.c_int64), ("num_waves", ctypes.c_int64),
                ("words", ctypes.c_int64), ("esc_delta", ctypes.c_int64),
                ("esc_value", ctypes.c_int64), ("table_bytes", ctypes.c_int64),
                ("stream_bytes", ctypes.c_int64), ("index_bytes", ctypes.c_int64),
                ("total_bytes", ctypes.c_int64), ("csr_bytes", ctypes.c_int64),
                ("coo_bytes", ctypes.c_int64), ("sell_bytes", ctypes.c_int64),
                ("delta_symbols", ctypes.c_int32), ("value_symbols", ctypes.c_int32),
                ("delta_entropy", ctypes.c_double), ("value_entropy", ctypes.c_double),
                ("delta_cross_entropy", ctypes.c_double),
                ("value_cross_entropy", ctypes.c_double), ("bits_per_nnz", ctypes.c_double),
                ("stream_stage", ctypes.c_int32), ("direct_table", ctypes.c_int32),
                ("first_delta_column", ctypes.c_int32), ("escape_in_stream", ctypes.c_int32),
                ("sort_window", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


# name -> (restype, argtypes); the order and types mirror include/dtans.h
_P, _I32, _I64, _D, _S = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_char_p
_PP = ctypes.POINTER(ctypes.c_void_p)
SIGNATURES = {
    "dtans_version": (ctypes.c_char_p, []),
    "dtans_last_error": (ctypes.c_char_p, []),
    "dtans_default_opts": (None, [ctypes.POINTER(EncodeOpts)]),
    "dtans_encode_csr": (_I32, [_I64, _I64, _I64, _P, _P, _P, ctypes.c_int, ctypes.POINTER(EncodeOpts), _PP]),
    "dtans_encode_csr_gpu": (_I32, [_I64, _I64, _I64, _P, _P, _P, ctypes.c_int, ctypes.POINTER(EncodeOpts), _P,
                                  _PP]),
    "dtans_encode_csr_device": (_I32, [_I64, _I64, _I64, _P, _P, _P, ctypes.c_int, ctypes.POINTER(EncodeOpts),
                                       _P, _PP]),
    "dtans_save": (_I32, [_P, _S]),
    "dtans_load": (_I32, [_S, _PP]),
    "dtans_to_device": (_I32, [_P, _P]),
    "dtans_reserve": (_I32, [_P, _I32, _P]),
    "dtans_matrix_info": (_I32, [_P, ctypes.POINTER(Info)]),
    "dtans_set_launch": (_I32, [_P, _I32, _I32, _I32]),
    "dtans_spmv": (_I32, [_P, _P, _P, _D, _D, _P]),
    "dtans_spmm": (_I32, [_P, _I32, _P, _I64, _P, _I64, _D, _D, _P]),
    "dtans_spmm_noalloc": (_I32, [_P, _I32, _P, _I64, _P, _I64, _D, _D, _P]),
    "dtans_spmv_sym": (_I32, [_P, _P, _P, _P, _D, _D, _P]),
    "dtans_spmm_t": (_I32, [_P, _I32, _P, _I64, _P, _I64, _D, _D, _P]),
    "dtans_decode_csr": (_I32, [_P, _P, _P, _P, _P]),
    "dtans_batch_create": (_I32, [_I32, _PP, _PP]),
    "dtans_batch_spmv": (_I32, [_P, _PP, _PP, _D, _D, _P]),
    "dtans_batch_spmm": (_I32, [_P, _I32, _PP, _PP, _D, _D, _P]),
    "dtans_batch_destroy": (None, [_P]),
    "dtans_csr_create": (_I32, [_I64, _I64, _I64, _P, _P, _P, ctypes.c_int, _I32, _PP]),
    "dtans_csr_spmv": (_I32, [_P, _P, _P, _D, _D, _P]),
    "dtans_csr_spmm": (_I32, [_P, _I32, _P, _I64, _P, _I64, _D, _D, _P]),
    "dtans_csr_bytes": (_I64, [_P]),
    "dtans_csr_destroy": (None, [_P]),
    "dtans_rocsparse_create": (_I32, [_I64, _I64, _I64, _P, _P, _P, ctypes.c_int, _PP]),
    "dtans_rocsparse_spmv": (_I32, [_P, _P, _P, _D, _D, _P]),
    "dtans_rocsparse_spmm": (_I32, [_P, _I32, _P, _I64, _P, _I64, _D, _D, _P]),
    "dtans_rocsparse_destroy": (None, [_P]),
    "dtans_autotune_candidates": (_I32, [_I64, _I64, _P, ctypes.c_int, _I32,
                                         ctypes.POINTER(EncodeOpts), ctypes.POINTER(EncodeOpts),
                                         _I32]),
    "dtans_autotune": (_I32, [_I64, _I64, _I64, _P, _P, _P, ctypes.c_int, _I32, _D,
                              ctypes.c_char_p, ctypes.POINTER(EncodeOpts),
                              ctypes.POINTER(ctypes.c_double)]),
    "dtans_destroy": (None, [_P]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load libdtans.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libdtans.so is not built (%s); run __graft_entry__.build() or "
                          "python paper_2603_01915_amd/build.py" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != OK:
        raise DtansError(status, load().dtans_last_error().decode(errors="replace"))
