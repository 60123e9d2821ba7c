"""ctypes view of libflashviterbi.so (the C ABI declared in include/flashviterbi.h).

Marshalling only: every decoding step runs in the HIP library.  Importing this
module fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libflashviterbi.so")

FV_OK, FV_E_INVALID_ARG, FV_E_UNSUPPORTED, FV_E_WORKSPACE, FV_E_DEVICE, FV_E_INFEASIBLE = 0, -1, -2, -3, -4, -5
FV_W_BEAM_FALLBACK = 1
FV_DENSE, FV_CSR = 0, 1
FV_FLAG_WIDE_ROWS, FV_FLAG_LOCAL_ROWS, FV_FLAG_VALIDATE, FV_FLAG_NO_LEAVES = 1, 2, 4, 8
FV_FLAG_RELATIVE_INIT = 16
FV_FLAG_STEP_ITEMS, FV_FLAG_STEP_TILES, FV_FLAG_ENGINE = 32, 64, 128
FV_VANILLA, FV_FLASH, FV_BEAM = 0, 1, 2
FV_EMIT_TABLE, FV_EMIT_GAUSS2D = 0, 1
METHODS = {"vanilla": FV_VANILLA, "flash": FV_FLASH, "beam": FV_BEAM}


class FvTrans(C.Structure):
    _fields_ = [("kind", C.c_int32), ("K", C.c_int32), ("log_a", C.c_void_p),
                ("row_ptr", C.c_void_p), ("col", C.c_void_p), ("val", C.c_void_p),
                ("nnz", C.c_int64)]


class FvSeq(C.Structure):
    _fields_ = [("model", C.c_int32), ("T", C.c_int32), ("log_b", C.c_void_p),
                ("ld", C.c_int64), ("path", C.c_void_p), ("score", C.c_void_p)]


class FvEmission(C.Structure):
    _fields_ = [("kind", C.c_int32), ("state_xy", C.c_void_p), ("c2", C.c_double), ("c0", C.c_double)]


class FvError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


_lib = None

# exported symbol -> (restype, argtypes)
_i32, _i64, _u32, _sz, _vp, _f = C.c_int32, C.c_int64, C.c_uint32, C.c_size_t, C.c_void_p, C.c_float
_P = C.POINTER
SIGNATURES = {
    "fv_workspace_size": (_i32, [_i32, _P(FvTrans), _i32, _vp, _vp, _i32, _i32, _i32, _P(_sz)]),
    "fv_decode_vanilla": (_i32, [_P(FvTrans), _vp, _vp, _i64, _i32, _vp, _vp, _vp, _u32, _vp, _sz, _vp]),
    "fv_decode_flash": (_i32, [_P(FvTrans), _vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp, _u32, _vp, _sz, _vp]),
    "fv_decode_flash_noalloc": (_i32, [_P(FvTrans), _vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp, _u32, _vp]),
    "fv_decode_beam": (_i32, [_P(FvTrans), _vp, _vp, _i64, _i32, _i32, _i32, _vp, _vp, _vp, _u32, _vp, _sz, _vp]),
    "fv_decode_batch": (_i32, [_P(FvTrans), _vp, _i32, _vp, _vp, _vp, _i32, _i32, _i32, _i32, _vp, _u32, _vp, _sz, _vp]),
    "fv_decode_batch_emit": (_i32, [_P(FvTrans), _P(FvEmission), _vp, _i32, _vp, _vp, _vp, _i32, _i32, _i32, _i32,
                                    _vp, _u32, _vp, _sz, _vp]),
    "fv_viterbi_backward": (_i32, [_i32, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _vp, _sz, _vp]),
    "fv_backward_workspace_size": (_i32, [_i32, _i32, _i32, _P(_sz)]),
    "fv_rescore": (_i32, [_P(FvTrans), _vp, _vp, _i32, _vp, _vp]),
    "fv_gather_emissions": (_i32, [_i32, _i32, _vp, _vp, _i32, _vp, _i64, _vp]),
    "fv_profile_engine": (_i32, [_i32]),
    "fv_profile_engine_ms": (_i32, [_P(_f)]),
    "fv_debug_engine_limits": (_i32, [_i64, _i64]),
    "fv_debug_engine_trace": (_i32, [_vp, _i32]),
    "fv_status_str": (C.c_char_p, [_i32]),
    "fv_last_error": (C.c_char_p, []),
    "fv_abi_version": (_i32, []),
}


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2510_19301_amd.build.build()")
        h = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(h, name)
            fn.restype = res
            fn.argtypes = args
        _lib = h
    return _lib


def check(status: int, where: str) -> int:
    if status < 0:
        l = lib()
        msg = l.fv_last_error().decode(errors="replace") or l.fv_status_str(status).decode()
        raise FvError(status, where, msg)
    return status
