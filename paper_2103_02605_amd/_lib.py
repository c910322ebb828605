"""ctypes declarations of libfcirc's C-ABI (include/fcirc.h).

Loading fails loudly when the shared library has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfcirc.so")

FCIRC_ZP_998244353 = 0
FCIRC_ZP_469762049 = 1
FCIRC_ZP_167772161 = 2
FCIRC_C64 = 3
FCIRC_R32 = 4
FCIRC_GFP2 = 5

STATUS = {0: "OK", 1: "EINVAL", 2: "ESIZE", 3: "ENOROOT", 4: "ERANGE", 5: "ENOMEM", 6: "EDEVICE", 7: "ESCHED", 8: "ENOPLAN"}


class fcirc_item(C.Structure):
    _fields_ = [("a_off", C.c_uint64), ("x_off", C.c_uint64), ("y_off", C.c_uint64),
                ("log2n", C.c_uint32), ("reserved", C.c_uint32)]


# name -> (restype, argtypes); every symbol declared in include/fcirc.h
SIGNATURES = {
    "fcirc_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int]),
    "fcirc_destroy": (None, [C.c_void_p]),
    "fcirc_strerror": (C.c_char_p, [C.c_int]),
    "fcirc_matvec": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_int,
                               C.c_void_p]),
    "fcirc_matvec_noalloc": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p,
                                       C.c_int, C.c_void_p]),
    "fcirc_matvec_many": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32,
                                    C.c_void_p, C.c_int, C.c_void_p]),
    "fcirc_matvec_any": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_int,
                                   C.c_void_p]),
    "fcirc_toeplitz_matvec": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64,
                                        C.c_int, C.c_void_p]),
    "fcirc_polymul_i64": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.c_void_p,
                                    C.c_void_p]),
    "fcirc_bigint_mul": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.c_void_p,
                                   C.c_void_p]),
    "fcirc_fermat_matvec": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32,
                                      C.c_uint32, C.c_void_p]),
    "fcirc_bigint_mul_fermat": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint64, C.c_void_p,
                                          C.c_void_p]),
    "fcirc_matvec_batched": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(fcirc_item),
                                       C.c_uint32, C.c_void_p, C.c_int, C.c_void_p]),
    "fcirc_set_batch_schedule": (C.c_int, [C.c_void_p, C.c_int, C.c_uint64, C.c_int, C.c_int]),
    "fcirc_get_batch_schedule": (C.c_int, [C.c_void_p, C.c_int, C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_int)]),
    "fcirc_matvec_fwd_shared": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_uint64, C.c_uint32,
                                          C.c_int, C.c_void_p]),
    "fcirc_matvec_backward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                        C.c_uint64, C.c_uint32, C.c_int, C.c_void_p]),
    "fcirc_check": (C.c_int, [C.c_void_p, C.c_void_p]),
    "fcirc_set_timing": (C.c_int, [C.c_void_p, C.c_int]),
    "fcirc_set_checks": (C.c_int, [C.c_void_p, C.c_int]),
    "fcirc_save_schedules": (C.c_int, [C.c_void_p, C.c_char_p]),
    "fcirc_load_schedules": (C.c_int, [C.c_void_p, C.c_char_p]),
    "fcirc_stage_times": (C.c_int, [C.c_void_p, C.POINTER(C.c_char_p), C.POINTER(C.c_uint64),
                                    C.POINTER(C.c_double), C.c_int]),
    "fcirc_tune": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int, C.c_void_p]),
    "fcirc_set_split": (C.c_int, [C.c_void_p, C.c_int]),
    "fcirc_get_split": (C.c_int, [C.c_void_p, C.c_uint64, C.c_int]),
    "fcirc_set_schedule": (C.c_int, [C.c_void_p, C.c_int, C.c_uint64, C.c_int, C.c_int, C.c_int]),
    "fcirc_get_schedule": (C.c_int, [C.c_void_p, C.c_int, C.c_uint64, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                     C.POINTER(C.c_int)]),
}

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2103_02605_amd.build` "
                               "(the package has no CPU fallback)")
        handle = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


class FcircError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().fcirc_strerror(code).decode()
        super().__init__(f"{where}: {STATUS.get(code, code)} ({msg})")
        self.code = code
        self.status = STATUS.get(code, str(code))


def check(code: int, where: str) -> None:
    if code != 0:
        raise FcircError(code, where)
