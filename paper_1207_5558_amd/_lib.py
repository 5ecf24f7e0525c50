"""ctypes binding of libslsht.so (C ABI in include/slsht.h).

Argument marshalling only: every step of the transform runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libslsht.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "slsht.h")

SLSHT_OK, SLSHT_EINVAL, SLSHT_ENOMEM, SLSHT_EDEVICE = 0, -1, -2, -3
SLSHT_EBUSY, SLSHT_ENOTFOUND, SLSHT_ETOOBIG = -4, -5, -6
SLSHT_FP64, SLSHT_FP32_MIXED = 0, 1
SLSHT_OUT_FULL, SLSHT_OUT_ENERGY = 0, 1
SLSHT_REAL_PAIR = 1
REQ_QUEUED, REQ_RUNNING, REQ_DONE, REQ_FAILED = 0, 1, 2, 3
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDEVICE", -4: "EBUSY",
                -5: "ENOTFOUND", -6: "ETOOBIG"}


class Desc(ctypes.Structure):
    _fields_ = [("L_f", ctypes.c_int32), ("L_h", ctypes.c_int32),
                ("l_lo", ctypes.c_int32), ("l_hi", ctypes.c_int32),
                ("n_phi", ctypes.c_int32), ("n_theta", ctypes.c_int32),
                ("n_omega", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("output_mode", ctypes.c_int32), ("flags", ctypes.c_uint32),
                ("theta_lo", ctypes.c_int32), ("theta_hi", ctypes.c_int32),
                ("n_az", ctypes.c_int32)]


class SlshtError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"slsht error {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_lib = None

_P = ctypes.c_void_p
_SZ = ctypes.POINTER(ctypes.c_size_t)
_SIGNATURES = {
    "slsht_last_error": ([], ctypes.c_char_p),
    "slsht_validate": ([ctypes.POINTER(Desc)], ctypes.c_int),
    "slsht_footprint": ([ctypes.POINTER(Desc), _SZ, _SZ, _SZ], ctypes.c_int),
    "slsht_coupling_size": ([ctypes.POINTER(Desc)], ctypes.c_int64),
    "slsht_plan": ([ctypes.POINTER(Desc), ctypes.c_int, ctypes.POINTER(_P)], ctypes.c_int),
    "slsht_plan_destroy": ([_P], ctypes.c_int),
    "slsht_plan_desc": ([_P, ctypes.POINTER(Desc)], ctypes.c_int),
    "slsht_forward": ([_P, _P, _P, _P, _P], ctypes.c_int),
    "slsht_forward_noalloc": ([_P, _P, _P, _P, _P], ctypes.c_int),
    "slsht_forward_windows": ([_P, _P, _P, ctypes.c_int, _P, _P], ctypes.c_int),
    "slsht_factored_workspace": ([ctypes.POINTER(Desc)], ctypes.c_int64),
    "slsht_forward_factored": ([_P, _P, _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "slsht_forward_batch": ([ctypes.c_int, _P, _P, _P, _P, _P], ctypes.c_int),
    "slsht_synthesize_factored": ([_P, _P, _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "slsht_wigner_delta": ([ctypes.c_int, ctypes.c_int, _P, _P], ctypes.c_int),
    "slsht_modulated_workspace": ([ctypes.POINTER(Desc)], ctypes.c_int64),
    "slsht_coupling_modulated": ([_P, _P, _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "slsht_slepian_window": ([ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int, _P,
                              ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
    "slsht_coupling": ([_P, _P, _P, _P], ctypes.c_int),
    "slsht_synthesize": ([_P, _P, _P, _P, _P], ctypes.c_int),
    "slsht_inverse": ([_P, _P, _P, _P, _P], ctypes.c_int),
    "slsht_server_create": ([ctypes.c_int, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(_P)],
                            ctypes.c_int),
    "slsht_server_destroy": ([_P], ctypes.c_int),
    "slsht_submit": ([_P, ctypes.POINTER(Desc), _P, _P, ctypes.POINTER(ctypes.c_uint64)],
                     ctypes.c_int),
    "slsht_poll": ([_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_P), _SZ,
                    ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
    "slsht_wait": ([_P, ctypes.c_uint64, ctypes.c_int], ctypes.c_int),
    "slsht_release": ([_P, ctypes.c_uint64], ctypes.c_int),
    "slsht_request_times": ([_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double),
                             ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
                            ctypes.c_int),
    "slsht_server_clock": ([_P], ctypes.c_double),
    "slsht_server_stats": ([_P, _SZ, _SZ, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)],
                           ctypes.c_int),
}


def declared_functions() -> list[str]:
    """Names of the functions declared in include/slsht.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(slsht_\w+)\s*\(", text)))


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; "
                f"g.build()'` (hipcc, gfx950)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGNATURES.items():
            fn = getattr(handle, name)
            fn.argtypes = args
            fn.restype = res
        _lib = handle
    return _lib


def check(status: int) -> int:
    if status != SLSHT_OK:
        msg = lib().slsht_last_error()
        raise SlshtError(status, msg.decode() if msg else "")
    return status


def last_error() -> str:
    msg = lib().slsht_last_error()
    return msg.decode() if msg else ""
