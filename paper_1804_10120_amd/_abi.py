"""ctypes view of ``include/tl.h`` and the loader of ``libtl.so``.

The library is loaded on first use.  If it is missing the call raises: there
is no fallback implementation anywhere in this package.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libtl.so")

TL_OK, TL_ERR_NULL, TL_ERR_SIZE, TL_ERR_ALIAS, TL_ERR_ALIGN, TL_ERR_HIP, TL_ERR_INVALID = range(7)
TL_TUNE_NT = 1
TL_TUNE_XCD = 2
TL_TUNE_PTR64 = 4
TL_BW_READ = 1
TL_BW_WRITE = 2
TL_BW_READ_BLOCKS = 2048
EXPRS = ("assign1", "assign2", "assign3", "add1", "add2", "add3", "mult1", "mult2", "mult3",
         "contract1", "contract2", "contract3", "kij")
TWIN_SHAPES = ((1, 1), (6, 6), (24, 18), (30, 9), (16, 6), (43, 6), (40, 43))
ABI_VERSION = 4
TL_NOALLOC_MAX_DOMAINS = 1024
TL_NOALLOC_MAX_TILES = 262144


class CField(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("ld", ctypes.c_int64)]


class Field(ctypes.Structure):
    _fields_ = [("ptr", ctypes.c_void_p), ("ld", ctypes.c_int64)]


class Tune(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("ppt", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("grid_mult", ctypes.c_int32), ("lanes", ctypes.c_int32)]


class Domain(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("g", CField), ("dg", CField), ("beta", CField),
                ("dbeta", CField), ("K", CField), ("alpha", CField), ("dtg", Field)]


class DomainBwd(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("g", CField), ("dg", CField), ("beta", CField),
                ("K", CField), ("alpha", CField), ("w", CField), ("g_bar", Field),
                ("dg_bar", Field), ("beta_bar", Field), ("dbeta_bar", Field), ("K_bar", Field),
                ("alpha_bar", Field)]


class KernelAttr(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("ppt", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("vgprs", ctypes.c_int32), ("agprs", ctypes.c_int32), ("sgprs", ctypes.c_int32),
                ("scratch_bytes", ctypes.c_int32), ("waves_per_simd", ctypes.c_int32),
                ("max_waves_per_simd", ctypes.c_int32), ("max_threads", ctypes.c_int32)]


class TLError(RuntimeError):
    """A tl_* call returned a status other than TL_OK."""

    def __init__(self, status, message):
        self.status = status
        super().__init__(message)


_C, _F, _T, _S = CField, Field, ctypes.POINTER(Tune), ctypes.c_void_p
_I64 = ctypes.c_int64
SIGNATURES = {
    "tl_sym_inverse": [_I64, _C, _F, _S, _T],
    "tl_christoffel": [_I64, _C, _C, _F, _S, _T],
    "tl_cov_deriv": [_I64, _C, _C, _C, _F, _S, _T],
    "tl_dtg": [_I64, _C, _C, _C, _F, _S, _T],
    "tl_dtg_chain": [_I64, _C, _C, _C, _C, _C, _C, _F, _S, _T],
    "tl_dtg_chain_bwd": [_I64, _C, _C, _C, _C, _C, _C, _F, _F, _F, _F, _F, _F, _S, _T],
    "tl_dtg_chain_fwd_bwd": [_I64, _C, _C, _C, _C, _C, _C, _C, _F, _F, _F, _F, _F, _F, _F, _S,
                             _T],
    "tl_batch_plan_create": [ctypes.POINTER(Domain), ctypes.c_int32, _T, ctypes.POINTER(ctypes.c_void_p)],
    "tl_batch_plan_bwd_create": [ctypes.POINTER(DomainBwd), ctypes.c_int32, _T,
                                 ctypes.POINTER(ctypes.c_void_p)],
    "tl_batch_run_noalloc": [ctypes.POINTER(Domain), ctypes.c_int32, _T, _S],
    "tl_batch_plan_launch": [ctypes.c_void_p, _S],
    "tl_batch_plan_launch_direct": [ctypes.c_void_p, _S],
    "tl_batch_plan_info": [ctypes.c_void_p, ctypes.POINTER(_I64), ctypes.POINTER(_I64),
                           ctypes.POINTER(_I64)],
    "tl_batch_plan_destroy": [ctypes.c_void_p],
    "tl_bw_copy": [_I64, ctypes.c_void_p, ctypes.c_void_p, _S],
    "tl_bw_stream": [_I64, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, _S],
    "tl_bw_twin": [_I64, ctypes.c_int32, _C, ctypes.c_int32, _F, _S, _T],
    "tl_expr": [ctypes.c_int32, _I64, ctypes.POINTER(CField), ctypes.c_int32, _F, _S, _T],
    "tl_expr_shape": [ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
    "tl_kernel_info": [ctypes.c_char_p, _T, ctypes.POINTER(KernelAttr)],
    "tl_status_string": [ctypes.c_int],
    "tl_last_error": [],
    "tl_abi_version": [],
}
RESTYPES = {"tl_status_string": ctypes.c_char_p, "tl_last_error": ctypes.c_char_p,
            "tl_abi_version": ctypes.c_int}

_lib = None


def lib():
    """The loaded ``libtl.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_1804_10120_amd.build` "
                "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in SIGNATURES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = RESTYPES.get(name, ctypes.c_int)
        v = L.tl_abi_version()
        if v != ABI_VERSION:
            raise RuntimeError(f"libtl.so ABI version {v}, expected {ABI_VERSION}")
        _lib = L
    return _lib


def check(status):
    """Raise TLError for a status other than TL_OK."""
    if status != TL_OK:
        L = lib()
        raise TLError(status, f"{L.tl_status_string(status).decode()}: "
                              f"{L.tl_last_error().decode()}")
