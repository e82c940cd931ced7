"""ctypes binding of libtfft.so (the C ABI in include/tfft.h).

Argument marshalling only: every step of the transform runs in the HIP
kernels of the library.  Importing fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtfft.so")
TUNING_PATH = os.path.join(_HERE, "tuning", "mi355x.json")

TFFT_OK = 0
TFFT_EINVAL = -1
TFFT_EUNSUPPORTED = -2
TFFT_EALIGN = -3
TFFT_EHIP = -4
TFFT_ENOMEM = -5
TFFT_ECAPTURE = -6
TFFT_ENOTPREPARED = -7
TFFT_ESCRATCH = -8
NOALLOC_SCRATCH_BYTES = 64 << 20

FORWARD = -1
INVERSE = +1
FP32 = 0
FP64 = 1
FT_OFF = 0
FT_DETECT = 1
FT_CORRECT = 2
FT_THREAD = 3

# exported symbols and their signatures, as declared in include/tfft.h
_LL = ctypes.c_longlong
_VP = ctypes.c_void_p
_I = ctypes.c_int
_D = ctypes.c_double
SIGNATURES = {
    "tfft_c2c": ([_VP, _VP, _LL, _LL, _I, _I, _I, _D, _VP, _VP], _I),
    "tfft_c2c_noalloc": ([_VP, _VP, _LL, _LL, _I, _I, _I, _D, _VP, _VP], _I),
    "tfft_c2c_offline": ([_VP, _VP, _LL, _LL, _I, _I, _D, _VP, _VP], _I),
    "tfft_c2c_ragged": ([_VP, _VP, _VP, _I, _I, _I, _I, _VP, _VP], _I),
    "tfft_prepare": ([_LL, _LL, _I, _I, _VP], _I),
    "tfft_ragged_supported": ([_LL, _I], _I),
    "tfft_ragged_plan_create": ([ctypes.POINTER(_VP), ctypes.POINTER(_LL), _LL, _I], _I),
    "tfft_ragged_plan_destroy": ([_VP], _I),
    "tfft_ragged_plan_info": ([_VP, ctypes.POINTER(_LL), _I], _I),
    "tfft_ragged_set_schedule": ([_LL, _LL, _I], _I),
    "tfft_ragged_test_wait": ([ctypes.c_uint, ctypes.c_uint], _I),
    "tfft_supported": ([_LL, _I], _I),
    "tfft_inject_arm": ([_LL, _LL, _I, _I, _I], _I),
    "tfft_inject_arm_desc": ([_VP], _I),
    "tfft_route_info": ([_LL, _I, _I, ctypes.POINTER(_LL), _I], _I),
    "tfft_inject_disarm": ([], _I),
    "tfft_set_tuning": ([_LL, _I, _I, _D], _I),
    "tfft_set_granularity": ([_LL, _I, _I], _I),
    "tfft_get_tuning": ([_LL, _I, ctypes.POINTER(_I), ctypes.POINTER(_D)], _I),
    "tfft_calibration": ([_I], _I),
    "tfft_profile": ([_I], _I),
    "tfft_profile_read": ([ctypes.c_char_p, _LL], _I),
    "tfft_profile_only": ([_I, _I, _I, _I, _I], _I),
    "tfft_c2c_stepwise": ([_VP, _VP, _LL, _LL, _I, _I, _VP], _I),
    "tfft_set_chunk": ([_LL, _I, _LL], _I),
    "tfft_routes": ([_LL, _I, _I, ctypes.POINTER(_LL), _I], _I),
    "tfft_set_route": ([_LL, _I, _LL], _I),
    "tfft_get_route": ([_LL, _I, _I, ctypes.POINTER(_LL)], _I),
    "tfft_load_tuning": ([ctypes.c_char_p], _I),
    "tfft_strerror": ([_I], ctypes.c_char_p),
    "tfft_last_hip_error": ([], _I),
}


class InjectDesc(ctypes.Structure):
    """tfft_inject_desc of include/tfft.h."""
    _fields_ = [("signal", _LL), ("element", _LL), ("part", _I), ("bit", _I),
                ("precision", _I), ("pass_", _I), ("stage", _I), ("two", _I), ("signal2", _LL)]


class TfftError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {strerror(status)} (status {status}, hip error {last_hip_error()})")


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    # the autotuner's table for this GPU, read by the host runtime
    if os.environ.get("TFFT_TUNING", "") != "off" and os.path.exists(TUNING_PATH):
        n = lib.tfft_load_tuning(TUNING_PATH.encode())
        if n < 0:
            raise TfftError(n, f"tfft_load_tuning({TUNING_PATH})")
    _lib = lib
    return lib


def strerror(status: int) -> str:
    return load().tfft_strerror(status).decode()


def last_hip_error() -> int:
    return load().tfft_last_hip_error()


def check(status: int, what: str) -> None:
    if status != TFFT_OK:
        raise TfftError(status, what)


def profile_read() -> list:
    """Per-kernel launch statistics recorded since tfft_profile(1) (see tfft.h)."""
    lib = load()
    n = lib.tfft_profile_read(None, 0)
    buf = ctypes.create_string_buffer(max(1, n))
    rc = lib.tfft_profile_read(buf, len(buf))
    if rc < 0:
        raise TfftError(rc, "tfft_profile_read")
    rows = []
    for line in buf.value.decode().splitlines():
        prec, kind, ns, ft, n_l, ms, nbytes, var, e, width = line.split()
        rows.append({"precision": prec, "kind": kind, "Ns": int(ns), "ft": int(ft),
                     "launches": int(n_l), "total_ms": float(ms), "bytes": float(nbytes),
                     "variant": int(var), "E": int(e), "width": int(width)})
    return rows
