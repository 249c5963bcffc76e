"""Signatures of the batched (multi-mesh persistent launch) and surrogate
(BF16 MFMA MLP) entry points of libpmutdg.so."""
import ctypes

_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)

SIGS = {}


def declare(L):
    for name, args in SIGS.items():
        f = getattr(L, name, None)
        if f is None:
            continue
        f.argtypes = args
        f.restype = ctypes.c_int
