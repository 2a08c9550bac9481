"""ctypes view of the C ABI in include/psf.h (argument marshalling only).

The shared library ``libpsf.so`` is built in-tree by ``build_lib.py``.  There
is no fallback: if it is missing or fails to load, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpsf.so")

PSF_OK = 0
PSF_EINVAL = -1
PSF_EGEOM = -2
PSF_ERANGE = -3
PSF_ESIZE = -4
PSF_EHIP = -5
PSF_EOVERFLOW = -6
PSF_EUNSUPPORTED = -7
PSF_ECAPACITY = -8

PSF_OPT_TABLE_GRAD = 1
PSF_OPT_STAGE_CSR = 2
PSF_OPT_WS_CLEAN = 4
PSF_OPT_CLASS_ORDER = 8
PSF_OPT_OSEM = 16
PSF_OPT_DETERMINISTIC = 32

PSF_FP32 = 0
PSF_BF16 = 1
PSF_BF16X2 = 2


class psf_geometry(C.Structure):
    _fields_ = [("n_blocks", C.c_int32), ("n_cryst_t", C.c_int32), ("n_cryst_z", C.c_int32),
                ("n_block_rings", C.c_int32), ("pitch_t", C.c_double), ("pitch_z", C.c_double),
                ("depth", C.c_double), ("radius_face", C.c_double), ("gap_z", C.c_double), ("mu", C.c_double),
                ("phi0", C.c_double)]


class psf_image(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("pad", C.c_int32),
                ("dx", C.c_double), ("dy", C.c_double), ("dz", C.c_double),
                ("cx", C.c_double), ("cy", C.c_double), ("cz", C.c_double)]


class psf_table(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("n_sub", C.c_int32), ("step_deg", C.c_double), ("data", C.c_void_p)]


class psf_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("homog_k", C.c_int32), ("threshold", C.c_double),
                ("vox_begin", C.c_int64), ("vox_end", C.c_int64), ("accumulate", C.c_int32), ("flags", C.c_int32),
                ("top_n", C.c_int32), ("reserved", C.c_int32)]


class psf_csr(C.Structure):
    _fields_ = [("n_rows", C.c_int64), ("nnz", C.c_int64), ("row_ptr", C.c_void_p), ("col", C.c_void_p),
                ("val", C.c_void_p)]


# every symbol include/psf.h declares, with (restype, argtypes)
_P = C.c_void_p
_H = C.c_void_p
SIGNATURES = {
    "psf_create": (C.c_int, [C.POINTER(psf_geometry), C.POINTER(psf_image), C.c_int32, C.POINTER(C.c_void_p)]),
    "psf_destroy": (None, [_H]),
    "psf_sizes": (C.c_int, [_H, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]),
    "psf_build_table": (C.c_int, [_H, C.c_int32, C.c_int32, C.c_double, _P, _P]),
    "psf_build_table_mc": (C.c_int, [_H, C.c_int32, C.c_int32, C.c_double, C.c_int64, C.c_uint64, C.c_int32, _P, _P,
                                     _P]),
    "psf_build_table_host": (C.c_int, [C.POINTER(psf_geometry), C.c_int32, C.c_int32, C.c_int32, C.c_double, _P]),
    "psf_workspace_size": (C.c_int, [_H, C.POINTER(psf_table), C.POINTER(psf_opts), C.c_int32, C.c_int64,
                                     C.POINTER(C.c_size_t)]),
    "build_psf_sysmat": (C.c_int, [_H, C.POINTER(psf_table), C.POINTER(psf_opts), _P, C.c_size_t,
                                   C.POINTER(psf_csr), _P]),
    "project_fwd": (C.c_int, [_H, C.POINTER(psf_table), C.POINTER(psf_opts), _P, C.c_int32, _P, C.c_int64, _P, _P,
                              C.c_size_t, _P]),
    "project_fwd_noalloc": (C.c_int, [_H, C.POINTER(psf_table), C.POINTER(psf_opts), _P, C.c_int32, _P, C.c_int64,
                                      _P, _P]),
    "project_adj": (C.c_int, [_H, C.POINTER(psf_table), C.POINTER(psf_opts), _P, C.c_int32, _P, C.c_int64, _P, _P,
                              _P, _P, C.c_size_t, _P]),
    "psf_sensitivity": (C.c_int, [_H, C.POINTER(psf_table), C.POINTER(psf_opts), _P, _P, C.c_size_t, _P]),
    "psf_lm_osem_update": (C.c_int, [_H, C.POINTER(psf_table), C.POINTER(psf_opts), _P, C.c_int64, C.c_float, _P,
                                     C.c_int32, _P, _P, _P, C.c_size_t, _P]),
    "psf_voxel_order": (C.c_int, [_H, _P]),
    "psf_osem_update": (C.c_int, [_H, C.POINTER(psf_table), C.POINTER(psf_opts), _P, C.c_int32, C.c_int32, _P, _P,
                                  _P, _P, C.c_size_t, _P]),
    "psf_subset_sensitivity": (C.c_int, [_H, C.POINTER(psf_table), C.POINTER(psf_opts), C.c_int32, C.c_int32, _P, _P,
                                         C.c_size_t, _P]),
    "psf_check": (C.c_int, [_H, _P, _P]),
    "psf_profile": (C.c_int, [_H, C.c_int32, C.c_void_p, C.c_void_p]),
    "psf_status_string": (C.c_char_p, [C.c_int]),
    "psf_last_hip_error": (C.c_int, []),
}

_lib = None
_lock = threading.Lock()


def load() -> C.CDLL:
    """Load libpsf.so (raises if it is not built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"libpsf.so is not built ({LIB_PATH}); run __graft_entry__.build()")
            L = C.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(L, name)
                fn.restype = res
                fn.argtypes = args
            _lib = L
    return _lib


class PsfError(RuntimeError):
    def __init__(self, code: int, where: str):
        L = load()
        msg = L.psf_status_string(code).decode()
        extra = f" (hip error {L.psf_last_hip_error()})" if code == PSF_EHIP else ""
        super().__init__(f"{where}: {msg}{extra} [{code}]")
        self.code = code


def check(code: int, where: str):
    if code != PSF_OK:
        raise PsfError(code, where)
