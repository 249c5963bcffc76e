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
    "pmdg_mlp_create": [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_vp)],
    "pmdg_mlp_num_params": [_vp, ctypes.POINTER(ctypes.c_long)],
    "pmdg_mlp_workspace_size": [_vp, ctypes.c_int, _sp],
    "pmdg_mlp_bind": [_vp, _vp, ctypes.c_size_t, _vp],
    "pmdg_mlp_set_io_map": [_vp, ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                            _fp, _fp, ctypes.c_int, ctypes.c_float, _vp],
    "pmdg_mlp_set_io_factors": [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                _fp, _fp, _vp],
    "pmdg_mlp_set_params": [_vp, _fp, _vp],
    "pmdg_mlp_get_params": [_vp, _fp, _vp],
    "pmdg_mlp_get_grads": [_vp, _fp, _vp],
    "pmdg_mlp_forward": [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp],
    "pmdg_mlp_backward": [_vp, _vp, ctypes.c_int, _vp, _vp, _vp],
    "pmdg_mlp_adam": [_vp, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _vp],
    "pmdg_mlp_train_step": [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_float, ctypes.c_float,
                            ctypes.c_float, ctypes.c_float, _vp, _vp, _vp],
    "pmdg_mlp_pair_combine": [_vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp, _vp],
    "pmdg_mlp_fit_linear_workspace": [_vp, ctypes.c_int, ctypes.c_int, _sp],
    "pmdg_mlp_fit_linear": [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                            ctypes.c_float, _vp, ctypes.c_size_t, _vp],
    "pmdg_mlp_set_target_scale": [_vp, _vp, _vp, _vp, ctypes.c_int, ctypes.c_int, _vp, ctypes.c_size_t, _vp],
    "pmdg_mlp_out_scale": [_vp, _fp],
    "pmdg_mlp_row_errors": [_vp, _vp, _vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp, _vp],
    "pmdg_mlp_scatter_rows": [_vp, _vp, ctypes.c_int, ctypes.c_int, _vp, _vp],
}


def declare(L):
    for name, args in SIGS.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    for name in ("pmdg_batch_destroy", "pmdg_mlp_destroy"):
        getattr(L, name).argtypes = [_vp]
        getattr(L, name).restype = None


def symbols():
    return list(SIGS) + ["pmdg_batch_destroy", "pmdg_mlp_destroy"]
