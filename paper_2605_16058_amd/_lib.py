"""ctypes binding of libtsvdm.so: the C ABI of include/tsvdm.h, same names.

Argument marshalling only.  The library is built in-tree by
``python -m paper_2605_16058_amd.build``; importing this module without the
built library raises, so nothing can silently fall back to another path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_size_t, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtsvdm.so")

F64, F32, BF16, BF16X3 = 0, 1, 2, 3
TILE_AUTO, TILE_64x64, TILE_128x32, TILE_256x16 = 0, 1, 2, 3
# largest min(m, p) of the Gram form and of its in-LDS Jacobi
# (TSVDM_GRAM_MAX_R, TSVDM_GRAM_LDS_MAX_R); placements of its Jacobi
GRAM_MAX_R = 1024
GRAM_LDS_MAX_R = 128
GRAM_JACOBI = {"auto": 0, "rounds": 1, "lds": 2}
STATUS = {
    0: "OK", -1: "E_ARG", -2: "E_SHAPE", -3: "E_NOT_ORTHO", -4: "E_WORKSPACE",
    -5: "E_NOCONV", -6: "E_NONFINITE", -7: "E_HIP", -8: "E_UNSUPPORTED", -9: "E_CAPACITY",
}

_P = c_void_p
_SIGS = {
    "tsvdm_version": (c_int, []),
    "tsvdm_last_error": (ctypes.c_char_p, []),
    "tsvdm_check_transform": (c_int, [_P, c_int64, c_double, POINTER(c_double)]),
    "tsvdm_transform_workspace_size": (c_int, [c_int64, POINTER(c_size_t)]),
    "tsvdm_transform": (c_int, [_P, c_int, _P, c_int, c_int64, c_int64, c_int64, _P, c_int,
                                c_double, c_int, c_int, _P, c_size_t, _P]),
    "tsvdm_transform_mode": (c_int, [_P, c_int, _P, c_int, c_int32, _P, c_int32, _P, c_int,
                                     c_double, c_int, c_int, _P, c_size_t, _P]),
    "tsvdm_transform_dct": (c_int, [_P, c_int, _P, c_int, c_int32, _P, c_int32, c_int, c_int, _P]),
    "tsvdm_lowrank": (c_int, [_P, _P, c_int, c_int64, c_int64, c_int64, _P, _P, c_int64, _P, _P]),
    "tsvdm_slice_svd_workspace_size": (c_int, [c_int64, c_int64, c_int64, c_int, POINTER(c_size_t)]),
    "tsvdm_slice_svd": (c_int, [_P, c_int, c_int64, c_int64, c_int64, _P, _P, _P, c_int, c_int,
                                c_double, c_int, _P, c_size_t, _P]),
    "tsvdm_slice_svd_subset": (c_int, [_P, c_int, c_int64, c_int64, c_int64, _P, _P, _P, _P, c_int,
                                       c_int, c_double, c_int, _P, c_size_t, _P]),
    "tsvdm_slice_svd_precond_workspace_size": (c_int, [c_int64, c_int64, c_int64, c_int, POINTER(c_size_t)]),
    "tsvdm_slice_svd_precond": (c_int, [_P, c_int, c_int64, c_int64, c_int64, _P, _P, _P, _P, c_int, c_int,
                                        c_double, c_int, _P, c_size_t, _P]),
    "tsvdm_slice_svd_gram_workspace_size": (c_int, [c_int64, c_int64, c_int64, POINTER(c_size_t)]),
    "tsvdm_slice_svd_gram": (c_int, [_P, c_int64, c_int64, c_int64, _P, _P, _P, _P, c_int, c_int, c_double,
                                     c_int, c_int, _P, c_size_t, _P]),
    "tsvdm_pack_gram": (c_int, [_P, _P, _P, _P, c_int64, c_int64, c_int64, _P, _P, c_int64, _P, _P, _P, _P,
                                _P, c_size_t, _P]),
    "tsvdm_slice_energy": (c_int, [_P, c_int, c_int64, c_int64, c_int64, _P, _P]),
    "tsvdm_certify_lump": (c_int, [_P, _P, _P, c_int64, c_int64, _P]),
    "tsvdm_certify_check": (c_int, [_P, _P, _P, _P, c_int64, c_int, _P, _P]),
    "tsvdm_truncate_rank": (c_int, [c_int64, c_int64, c_int64, _P, _P, _P]),
    "tsvdm_truncate_tol_workspace_size": (c_int, [c_int64, c_int64, POINTER(c_size_t)]),
    "tsvdm_truncate_tol": (c_int, [_P, c_int64, c_int64, c_double, _P, _P, _P, _P, c_size_t, _P]),
    "tsvdm_truncate_tol_noalloc": (c_int, [_P, c_int64, c_int64, c_double, _P, _P, _P, _P]),
    "tsvdm_pack_workspace_size": (c_int, [c_int64, c_int64, c_int64, POINTER(c_size_t)]),
    "tsvdm_pack": (c_int, [_P, _P, _P, c_int, c_int64, c_int64, c_int64, _P, _P, c_int64, _P, _P,
                           _P, _P, _P, c_size_t, _P]),
    "tsvdm_reconstruct_workspace_size": (c_int, [c_int64, c_int64, c_int64, c_int, POINTER(c_size_t)]),
    "tsvdm_reconstruct": (c_int, [_P, _P, c_int, c_int64, c_int64, c_int64, _P, _P, c_int64, _P,
                                  c_double, _P, c_int, c_int, c_int, _P, c_size_t, _P]),
    "tsvdm_error_workspace_size": (c_int, [c_int64, POINTER(c_size_t)]),
    "tsvdm_error": (c_int, [_P, c_int, _P, c_int, c_int64, _P, _P, c_size_t, _P]),
    "tsvdm_backward_workspace_size": (c_int, [c_int64, c_int64, c_int64, c_int, POINTER(c_size_t)]),
    "tsvdm_backward": (c_int, [_P, c_int, c_int64, c_int64, c_int64, _P, c_int64, c_double, _P, _P,
                               _P, _P, _P, c_size_t, _P]),
    "tsvdm_batch_plan_create": (c_int, [_P, c_int32, c_int, c_int, c_int, c_int, c_int, _P, _P]),
    "tsvdm_batch_run": (c_int, [_P, _P, c_size_t, c_int, c_int, _P, _P]),
    "tsvdm_batch_plan_destroy": (c_int, [_P]),
    "tsvdm_stats_enable": (c_int, [c_int]),
    "tsvdm_stats_reset": (c_int, []),
    "tsvdm_stats_get": (c_int, [_P, _P, _P, _P, _P, _P, _P]),
}


class BatchItem(ctypes.Structure):
    """tsvdm_batch_item of include/tsvdm.h."""
    _fields_ = [
        ("m", c_int64), ("p", c_int64), ("n", c_int64),
        ("A", c_void_p), ("M", c_void_p), ("inv_scale", c_double),
        ("mode", c_int32), ("block", c_int32), ("k", c_int64), ("eps", c_double),
        ("rho", c_void_p), ("offsets", c_void_p), ("stats", c_void_p),
        ("U_pk", c_void_p), ("G_pk", c_void_p), ("S_pk", c_void_p), ("capacity", c_int64),
        ("A_rec", c_void_p), ("err", c_void_p), ("ttm_tile", c_int32), ("reserved", c_int32),
    ]


class TsvdmError(RuntimeError):
    def __init__(self, fn: str, code: int, msg: str):
        super().__init__(f"{fn} failed with {STATUS.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load libtsvdm.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with 'python -m paper_2605_16058_amd.build' "
            "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def last_error() -> str:
    return load().tsvdm_last_error().decode()


def call(name: str, *args) -> int:
    """Call an entry point; raise TsvdmError on a negative status."""
    lib = load()
    rc = getattr(lib, name)(*args)
    if rc != 0:
        raise TsvdmError(name, rc, last_error())
    return rc


def workspace_size(name: str, *args) -> int:
    out = c_size_t(0)
    call(name, *args, ctypes.byref(out))
    return int(out.value)


def exported_names():
    return list(_SIGS)
