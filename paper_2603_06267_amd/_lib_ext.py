"""Signatures of the batched (multi-mesh persistent launch) and surrogate
(BF16 MFMA MLP) entry points of libpmutdg.so."""
import ctypes

_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
_fp = ctypes.POINTER(ctypes.c_float)

_sp = ctypes.POINTER(ctypes.c_size_t)

SIGS = {
    "pmdg_batch_create": [ctypes.c_int, ctypes.POINTER(_vp), ctypes.POINTER(_vp)],
    "pmdg_batch_workspace_size": [_vp, _sp],
    "pmdg_batch_bind": [_vp, _vp, ctypes.c_size_t, _vp],
    "pmdg_batch_set_option": [_vp, ctypes.c_int, ctypes.c_long],
    "pmdg_batch_step": [_vp, ctypes.c_int, _vp],
}


def declare(L):
    for name, args in SIGS.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    L.pmdg_batch_destroy.argtypes = [_vp]
    L.pmdg_batch_destroy.restype = None


def symbols():
    return list(SIGS) + ["pmdg_batch_destroy"]
