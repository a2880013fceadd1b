"""ctypes loader of libsptrsv.so and the C ABI signatures (include/sptrsv.h).

The library is loaded from this package directory only; if it is missing the
import fails with instructions to build it (no fallback path exists).
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsptrsv.so")

STATUS = {
    0: "SPTRSV_OK", -1: "SPTRSV_ERR_INVALID_ARG", -2: "SPTRSV_ERR_BAD_ROWPTR",
    -3: "SPTRSV_ERR_BAD_COLIDX", -4: "SPTRSV_ERR_NOT_TRIANGULAR", -5: "SPTRSV_ERR_DUPLICATE",
    -6: "SPTRSV_ERR_MISSING_DIAG", -7: "SPTRSV_ERR_ZERO_PIVOT", -8: "SPTRSV_ERR_HIP",
    -9: "SPTRSV_ERR_OOM", -10: "SPTRSV_ERR_TIMEOUT", -11: "SPTRSV_ERR_NOT_SUPPORTED",
    -12: "SPTRSV_ERR_BUSY", -13: "SPTRSV_ERR_TOO_LARGE", -14: "SPTRSV_ERR_NOT_RESIDENT",
}


class SpTRSVError(RuntimeError):
    def __init__(self, status):
        self.status = status
        msg = lib.sptrsv_status_string(status).decode()
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, msg))


def check(status):
    if status != 0:
        raise SpTRSVError(status)
    return status


if not os.path.exists(LIB_PATH):
    raise ImportError("libsptrsv.so is not built; run `python -m paper_1710_04985_amd.build` "
                      "(or __graft_entry__.build())")

lib = ctypes.CDLL(LIB_PATH)

_v, _i32, _i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
_pi32 = ctypes.POINTER(ctypes.c_int32)
_pi64 = ctypes.POINTER(ctypes.c_int64)
_pv = ctypes.POINTER(ctypes.c_void_p)
_int = ctypes.c_int

SIGNATURES = {
    "sptrsv_analyze": (_int, [_i32, _i32, _v, _v, _v, _int, _int, _int, _v, _pv]),
    "sptrsv_analyze_ex": (_int, [_i32, _i32, _v, _v, _v, _int, _int, _int, _int, _v, _pv]),
    "sptrsv_tune_multi": (_int, [_v, _i32, _i32, _v, _v, _v]),
    "sptrsv_probe_hop": (_int, [_int, _i32, ctypes.POINTER(ctypes.c_double)]),
    "sptrsv_get_setup": (_int, [_v, _pi32, ctypes.POINTER(ctypes.c_double)]),
    "sptrsv_analyze_batched": (_int, [_i32, _pi32, _pi32, _v, _v, _v, _int, _int, _int, _v, _pv]),
    "sptrsv_analyze_batched_ex": (_int, [_i32, _pi32, _pi32, _v, _v, _v, _int, _int, _int, _int,
                                         _v, _pv]),
    "sptrsv_update_values": (_int, [_v, _v, _v]),
    "sptrsv_update_values_batched": (_int, [_v, _v, _v]),
    "sptrsv_solve": (_int, [_v, _v, _v, _v]),
    "sptrsv_solve_transpose": (_int, [_v, _v, _v, _v]),
    "sptrsv_solve_noalloc": (_int, [_v, _v, _v, _v]),
    "sptrsv_prepare_transpose": (_int, [_v, _v]),
    "sptrsv_solve_multi": (_int, [_v, _i32, _i32, _v, _v, _int, _v]),
    "sptrsv_grad_vals": (_int, [_v, _v, _v, _v, _v, _v, _v]),
    "sptrsv_set_option": (_int, [_v, _int, _i64]),
    "sptrsv_get_option": (_int, [_v, _int, _pi64]),
    "sptrsv_tune": (_int, [_v, _v, _v, _v]),
    "sptrsv_get_info": (_int, [_v, _pi32, _pi64, _pi32, _pi32, _pi32]),
    "sptrsv_get_schedule": (_int, [_v, _pi32, _pi32, _pi32, _pi32, _pi32, _pi32, _pi32, _pi32]),
    "sptrsv_get_xp_stride": (_int, [_v, _pi32]),
    "sptrsv_export_analysis": (_int, [_v, _int, _pi32, _pi32, _pi32, _pi32]),
    "sptrsv_get_status": (_int, [_v]),
    "sptrsv_kernel_time": (_int, [_v, ctypes.POINTER(ctypes.c_double), _pi64, _int]),
    "sptrsv_status_string": (ctypes.c_char_p, [_int]),
    "sptrsv_destroy": (_int, [_v]),
    "sptrsv_graph_capture": (_int, [_v, _v, _v, _int, _v, _pv]),
    "sptrsv_graph_launch": (_int, [_v, _v]),
    "sptrsv_graph_destroy": (_int, [_v]),
    "sptrsv_analyze_host": (_int, [_i32, _i32, _pi32, _pi32, _int, _int, _pi32, _pi32, _pi32,
                                   _pi32, _pi32]),
}

for _name, (_res, _args) in SIGNATURES.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args
