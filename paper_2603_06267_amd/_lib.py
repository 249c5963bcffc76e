"""ctypes binding of libpmutdg.so (include/pmutdg.h): argument marshalling only.

The shared library is built in-tree by `paper_2603_06267_amd.build`.  There is
no fallback: if the library is missing, loading raises.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpmutdg.so")

PMDG_OK = 0
PMDG_EINVAL = -1
PMDG_ENOMEM = -2
PMDG_EHIP = -3
PMDG_EUNSTABLE = -4
PMDG_ESTATE = -5

OPT_GRAPH = 1
OPT_TILE_ROWS = 2
OPT_TILE_ZCHUNK = 3
OPT_GRAPH_CHUNK = 4
OPT_TIMING = 5
OPT_TILE_ROWS_SECONDARY = 6
OPT_TILE_ZCHUNK_SECONDARY = 7
OPT_TILE_WAVES = 8
OPT_TIME_BLOCK = 9
OPT_OVERLAP = 10
OPT_TIME_BLOCK_SECONDARY = 11
OPT_PREFETCH = 12
OPT_RESIDENT = 13

ERRNAMES = {PMDG_EINVAL: "EINVAL", PMDG_ENOMEM: "ENOMEM", PMDG_EHIP: "EHIP",
            PMDG_EUNSTABLE: "EUNSTABLE", PMDG_ESTATE: "ESTATE"}


class PmdgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Brick(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double * 3), ("x1", ctypes.c_double * 3), ("ne", ctypes.c_int * 3),
                ("order", ctypes.c_int), ("c", ctypes.c_double), ("rho", ctypes.c_double)]


class Problem(ctypes.Structure):
    _fields_ = [("ndom", ctypes.c_int), ("dom", Brick * 2), ("cfl", ctypes.c_double), ("dt", ctypes.c_double),
                ("penalty_alpha", ctypes.c_double), ("precision", ctypes.c_int), ("n_scenarios", ctypes.c_int),
                ("trace_capacity", ctypes.c_int)]


_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_lib = None

# name: (argtypes)
_SIGS = {
    "pmdg_create": [ctypes.POINTER(Problem), ctypes.POINTER(_vp)],
    "pmdg_set_pmuts": [_vp, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp, _dp, _dp],
    "pmdg_pmut_face_nodes": [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _dp],
    "pmdg_set_pmut_shape": [_vp, ctypes.c_int, _dp],
    "pmdg_set_drive": [_vp, _dp, _dp, _dp, ctypes.c_double, ctypes.c_int],
    "pmdg_set_rx": [_vp, ctypes.c_double, ctypes.c_double],
    "pmdg_set_absorbing": [_vp, ctypes.c_int, ctypes.c_int],
    "pmdg_set_pml": [_vp, ctypes.c_int, _dp, ctypes.c_double],
    "pmdg_set_vertices": [_vp, ctypes.c_int, _dp],
    "pmdg_match_faces": [ctypes.c_int, ctypes.c_int, _vp, _vp, ctypes.c_int, _vp, _vp, ctypes.c_double,
                         ctypes.c_double, _vp, _vp, _vp, _vp],
    "pmdg_set_receivers": [_vp, ctypes.c_int, _dp],
    "pmdg_workspace_size": [_vp, ctypes.POINTER(ctypes.c_size_t)],
    "pmdg_bind": [_vp, _vp, ctypes.c_size_t, _vp],
    "pmdg_bind_static": [_vp, _vp],
    "pmdg_restart": [_vp, _vp],
    "pmdg_get_dt": [_vp, _dp],
    "pmdg_lambda_max": [_vp, _dp],
    "pmdg_step": [_vp, ctypes.c_int, _vp],
    "pmdg_steps_done": [_vp, ctypes.POINTER(ctypes.c_long)],
    "pmdg_resident": [_vp, ctypes.POINTER(ctypes.c_int)],
    "pmdg_read_traces": [_vp, _dp, _vp],
    "pmdg_read_traces_device": [_vp, _vp, ctypes.c_int, _vp],
    "pmdg_read_modal": [_vp, ctypes.c_int, _dp, _dp, _dp, _vp],
    "pmdg_num_nodes": [_vp, ctypes.POINTER(ctypes.c_long)],
    "pmdg_get_state": [_vp, ctypes.c_int, _dp, _dp, _vp],
    "pmdg_set_state": [_vp, ctypes.c_int, _dp, _dp, _dp, _dp, _dp, ctypes.c_long, _vp],
    "pmdg_node_coords": [_vp, _dp],
    "pmdg_status_flags": [_vp, ctypes.POINTER(ctypes.c_int), _vp],
    "pmdg_set_option": [_vp, ctypes.c_int, ctypes.c_long],
    "pmdg_kernel_times": [_vp, _dp],
}


def lib():
    """Loads libpmutdg.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime with the same SONAME as ROCm's;
        # loading torch first makes libpmutdg bind to that one runtime, so
        # torch streams, allocations and synchronisation cover our kernels.
        import torch  # noqa: F401
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2603_06267_amd.build.build()")
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGS.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.pmdg_destroy.argtypes = [_vp]
        L.pmdg_destroy.restype = None
        L.pmdg_last_error.argtypes = []
        L.pmdg_last_error.restype = ctypes.c_char_p
        _extra(L)
        _lib = L
    return _lib


def _extra(L):
    """Declares the optional entry points of the batched and surrogate forms
    when the library exports them."""
    from . import _lib_ext
    _lib_ext.declare(L)


def check(code):
    if code != PMDG_OK:
        raise PmdgError(code, lib().pmdg_last_error().decode(errors="replace"))
    return code


def declared_symbols():
    from . import _lib_ext
    return list(_SIGS) + ["pmdg_destroy", "pmdg_last_error"] + _lib_ext.symbols()
