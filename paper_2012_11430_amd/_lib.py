"""ctypes loader of libprony.so (the C ABI declared in include/prony.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels. The module raises if the built library is missing; there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

# PRONY_LIB selects another build of the same library (the host-sanitizer build of
# build.py --sanitize); by default the in-tree libprony.so
LIB_PATH = os.environ.get("PRONY_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)), "libprony.so")

PRONY_OK = 0
PRONY_EINVAL = 1
PRONY_ENOTSUP = 2
PRONY_EHIP = 3
PRONY_ENOMEM = 4
PRONY_ECAPTURE = 5
PRONY_ENODEV = 6
STATUS_NAMES = {0: "PRONY_OK", 1: "PRONY_EINVAL", 2: "PRONY_ENOTSUP", 3: "PRONY_EHIP",
                4: "PRONY_ENOMEM", 5: "PRONY_ECAPTURE", 6: "PRONY_ENODEV"}

PRONY_FP64 = 0
PRONY_FP32 = 1
PRONY_BF16X3 = 2
PRONY_WITH_S0 = 1
PRONY_TUNE_BATCHED = 1
PRONY_TUNE_BUCKET = 2
PRONY_SCHEDULE_QUEUE = 0
PRONY_SCHEDULE_CLASSES = 1

class InstanceDesc(ctypes.Structure):
    """prony_instance_t."""
    _fields_ = [("d", ctypes.c_int), ("n", ctypes.c_int), ("m", ctypes.c_int),
                ("f", ctypes.c_void_p), ("U", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
                ("V", ctypes.c_void_p), ("S", ctypes.c_void_p)]


_c_int = ctypes.c_int
_c_i64 = ctypes.c_int64
_ptr = ctypes.c_void_p

# name -> (argtypes, restype); every entry point declared in include/prony.h
SIGNATURES = {
    "prony_create": ([ctypes.POINTER(_ptr), _c_int], _c_int),
    "prony_destroy": ([_ptr], _c_int),
    "prony_set_stream": ([_ptr, _ptr], _c_int),
    "prony_synchronize": ([_ptr], _c_int),
    "prony_last_error": ([_ptr], ctypes.c_char_p),
    "prony_reserve": ([_ptr, _c_int, _c_int, _c_int], _c_int),
    "prony_samples": ([_ptr, _c_int, _c_int, _c_int, _ptr, _ptr, _ptr, _ptr], _c_int),
    "prony_build_T": ([_ptr, _c_int, _c_int, _c_int, _ptr, _ptr, _c_i64], _c_int),
    "prony_build_S": ([_ptr, _c_int, _c_int, _c_int, _ptr, _ptr, _c_i64, _c_i64, _ptr, _ptr, _c_i64, _c_i64,
                       _c_int, ctypes.c_uint, _ptr], _c_int),
    "prony_build_S_noalloc": ([_ptr, _c_int, _c_int, _c_int, _ptr, _ptr, _c_i64, _c_i64, _ptr, _ptr, _c_i64,
                               _c_i64, _c_int, ctypes.c_uint, _ptr], _c_int),
    "prony_factors_create": ([_ptr, _c_int, _c_int, _c_int, _ptr, _c_i64, _c_i64, _ptr, _ptr, _c_i64, _c_i64,
                              _c_int, ctypes.c_uint, ctypes.POINTER(_ptr)], _c_int),
    "prony_build_S_factors": ([_ptr, _ptr, _ptr, _ptr], _c_int),
    "prony_factors_info": ([_ptr, ctypes.POINTER(_c_int), ctypes.POINTER(_c_int), ctypes.POINTER(_c_int),
                            ctypes.POINTER(_c_int), ctypes.POINTER(ctypes.c_uint)], _c_int),
    "prony_factors_destroy": ([_ptr], _c_int),
    "prony_coeffs": ([_ptr, _c_int, _c_int, _c_int, _ptr, _ptr, _ptr, _ptr, _ptr], _c_int),
    "prony_profile_enable": ([_ptr, ctypes.c_char_p], _c_int),
    "prony_tune_set": ([_ptr, _c_int, _c_int, _c_int, _c_int, ctypes.c_uint, _c_int], _c_int),
    "prony_build_S_adjoint": ([_ptr, _c_int, _c_int, _c_int, _ptr, _c_i64, _c_i64, _ptr, _ptr, _c_i64, _c_i64,
                               _ptr, _c_int, _ptr], _c_int),
    "prony_batch_create": ([_ptr, _c_int, ctypes.POINTER(InstanceDesc), _c_int, ctypes.POINTER(_ptr)], _c_int),
    "prony_batch_destroy": ([_ptr], _c_int),
    "prony_batch_set_schedule": ([_ptr, _c_int], _c_int),
    "prony_tune_get": ([_ptr, _c_int, _c_int, _c_int, _c_int, ctypes.c_uint, ctypes.POINTER(_c_int)], _c_int),
    "prony_tune_set_tile": ([_ptr, _c_int, _c_int, _c_int, _c_int, ctypes.c_uint, _c_int, _c_int], _c_int),
    "prony_tune_get_tile": ([_ptr, _c_int, _c_int, _c_int, _c_int, ctypes.c_uint, ctypes.POINTER(_c_int),
                             ctypes.POINTER(_c_int)], _c_int),
    "prony_autotune_device": ([_ptr, ctypes.c_char_p, ctypes.c_char_p], _c_int),
    "prony_build_S_plan": ([_ptr, _c_int, _c_int, _c_int, _c_int, ctypes.c_uint, ctypes.POINTER(_c_int),
                            ctypes.POINTER(_c_int), ctypes.POINTER(_c_int), ctypes.POINTER(ctypes.c_size_t)], _c_int),
    "prony_autotune": ([_ptr, ctypes.c_char_p], _c_int),
    "prony_build_S_batched": ([_ptr, _ptr], _c_int),
    "prony_build_S_adjoint_batched": ([_ptr, _ptr, _ptr, _ptr], _c_int),
    "prony_toeplitz_mm": ([_ptr, _c_int, _c_int, _c_int, _ptr, _c_int, _ptr, _c_i64, _c_int, _ptr, _c_i64], _c_int),
    "prony_graph_capture": ([_ptr, _ptr, ctypes.POINTER(_ptr)], _c_int),
    "prony_graph_launch": ([_ptr, _ptr], _c_int),
    "prony_graph_destroy": ([_ptr], _c_int),
    "prony_profile_read": ([_ptr, ctypes.POINTER(_c_int), ctypes.POINTER(ctypes.c_double)], _c_int),
}


class PronyError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load libprony.so once; raise ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2012_11430_amd/build.py "
                          "(or __graft_entry__.build()) before using the HIP path")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (argtypes, restype) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = argtypes
        fn.restype = restype
    _lib = lib
    return lib
