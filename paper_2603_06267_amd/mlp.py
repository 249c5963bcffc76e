"""Binding of the surrogate network entry points (pmdg_mlp_* in
include/pmutdg.h): argument marshalling only.  Device buffers are torch
tensors (plumbing); every arithmetic step runs in the library's kernels."""
import ctypes

import numpy as np

from ._lib import check, lib
from .solver import _stream_ptr


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class MLP:
    """widths = [n_0, ..., n_L]; max_batch rows per call (multiple of 8)."""

    def __init__(self, widths, max_batch=1024, device="cuda", stream=None):
        import torch
        self.L = lib()
        self.widths = [int(w) for w in widths]
        arr = (ctypes.c_int * len(self.widths))(*self.widths)
        h = ctypes.c_void_p()
        check(self.L.pmdg_mlp_create(len(self.widths) - 1, arr, ctypes.byref(h)))
        self.h = h
        n = ctypes.c_size_t()
        check(self.L.pmdg_mlp_workspace_size(self.h, int(max_batch), ctypes.byref(n)))
        self.max_batch = int(max_batch)
        self.device = device
        self.ws = torch.empty(n.value + 256, dtype=torch.uint8, device=device)
        ptr = (self.ws.data_ptr() + 255) // 256 * 256
        check(self.L.pmdg_mlp_bind(self.h, ctypes.c_void_p(ptr), n.value, _stream_ptr(stream)))
        npar = ctypes.c_long()
        check(self.L.pmdg_mlp_num_params(self.h, ctypes.byref(npar)))
        self.n_params = npar.value

    # ---- parameters -------------------------------------------------------
    def init_params(self, rng):
        """He initialisation W ~ N(0, 2 / n_in), b = 0 (FP32 host vector)."""
        parts = []
        for n_in, n_out in zip(self.widths[:-1], self.widths[1:]):
            parts.append((rng.standard_normal((n_out, n_in)) * np.sqrt(2.0 / n_in)).ravel())
            parts.append(np.zeros(n_out))
        vec = np.concatenate(parts).astype(np.float32)
        self.set_params(vec)
        return vec

    def set_params(self, vec, stream=None):
        v = np.ascontiguousarray(vec, dtype=np.float32)
        assert v.size == self.n_params
        check(self.L.pmdg_mlp_set_params(self.h, v.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                         _stream_ptr(stream)))

    def get_params(self, stream=None):
        v = np.empty(self.n_params, dtype=np.float32)
        check(self.L.pmdg_mlp_get_params(self.h, v.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                         _stream_ptr(stream)))
        return v

    def get_grads(self, stream=None):
        v = np.empty(self.n_params, dtype=np.float32)
        check(self.L.pmdg_mlp_get_grads(self.h, v.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                        _stream_ptr(stream)))
        return v

    def set_io_map(self, n_u, columns, out_scale=1.0, amp_col=-1, stream=None):
        """columns: one (src, op, shift, scale) per network input, op 0 affine
        ((u - shift) * scale), 1 cos(scale u + shift), 2 sin(scale u + shift),
        or (src, op, shift, scale, src2, op2, shift2, scale2) for the product
        of two such factors (src2 = -1: the first alone)."""
        cols = list(columns)
        src = np.ascontiguousarray([c[0] for c in cols], dtype=np.int32)
        op = np.ascontiguousarray([c[1] for c in cols], dtype=np.int32)
        sh = np.ascontiguousarray([c[2] for c in cols], dtype=np.float32)
        sc = np.ascontiguousarray([c[3] for c in cols], dtype=np.float32)
        ip, fp = ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_float)
        check(self.L.pmdg_mlp_set_io_map(self.h, int(n_u), len(cols), src.ctypes.data_as(ip), op.ctypes.data_as(ip),
                                         sh.ctypes.data_as(fp), sc.ctypes.data_as(fp), int(amp_col),
                                         float(out_scale), _stream_ptr(stream)))
        self.n_u = int(n_u)
        if any(len(c) > 4 for c in cols):
            c2 = [tuple(c[4:8]) if len(c) > 4 else (-1, 0, 0.0, 1.0) for c in cols]
            s2 = np.ascontiguousarray([c[0] for c in c2], dtype=np.int32)
            o2 = np.ascontiguousarray([c[1] for c in c2], dtype=np.int32)
            h2 = np.ascontiguousarray([c[2] for c in c2], dtype=np.float32)
            k2 = np.ascontiguousarray([c[3] for c in c2], dtype=np.float32)
            check(self.L.pmdg_mlp_set_io_factors(self.h, len(cols), s2.ctypes.data_as(ip), o2.ctypes.data_as(ip),
                                                 h2.ctypes.data_as(fp), k2.ctypes.data_as(fp), _stream_ptr(stream)))

    # ---- compute ----------------------------------------------------------
    def forward(self, u, y=None, idx=None, B=None, stream=None):
        """u: device FP32 [nrows, n_0]; returns y (device FP32 [B, n_L]).
        With y=False the normalised output stays inside (training)."""
        import torch
        B = int(B if B is not None else (idx.shape[0] if idx is not None else u.shape[0]))
        if y is None:
            y = torch.empty((B, self.widths[-1]), dtype=torch.float32, device=u.device)
        yp = None if y is False else _ptr(y)
        check(self.L.pmdg_mlp_forward(self.h, _ptr(u), _ptr(idx), int(u.shape[0]), B, yp, _stream_ptr(stream)))
        return None if y is False else y

    def backward(self, t, B, rowerr=None, rownorm=None, stream=None):
        check(self.L.pmdg_mlp_backward(self.h, _ptr(t), int(B), _ptr(rowerr), _ptr(rownorm), _stream_ptr(stream)))

    def adam(self, lr, b1=0.9, b2=0.999, eps=1e-8, stream=None):
        check(self.L.pmdg_mlp_adam(self.h, float(lr), float(b1), float(b2), float(eps), _stream_ptr(stream)))

    def train_step(self, u, t, idx, lr, b1=0.9, b2=0.999, eps=1e-8, rowerr=None, rownorm=None, stream=None):
        B = int(idx.shape[0]) if idx is not None else int(u.shape[0])
        check(self.L.pmdg_mlp_train_step(self.h, _ptr(u), _ptr(t), _ptr(idx), int(u.shape[0]), B, float(lr),
                                         float(b1), float(b2), float(eps), _ptr(rowerr), _ptr(rownorm),
                                         _stream_ptr(stream)))

    def fit_linear(self, u, t, idx, n, npairs, rank, ridge=0.0, stream=None):
        """Least-squares fit of the whole network on rows idx[:n] of (u, t)
        (pmdg_mlp_fit_linear); the fit workspace is a temporary torch buffer."""
        import torch
        nb = ctypes.c_size_t()
        check(self.L.pmdg_mlp_fit_linear_workspace(self.h, int(n), int(rank), ctypes.byref(nb)))
        work = torch.empty(nb.value + 256, dtype=torch.uint8, device=u.device)
        ptr = (work.data_ptr() + 255) // 256 * 256
        check(self.L.pmdg_mlp_fit_linear(self.h, _ptr(u), _ptr(t), _ptr(idx), int(u.shape[0]), int(n), int(npairs),
                                         int(rank), float(ridge), ctypes.c_void_p(ptr), nb.value,
                                         _stream_ptr(stream)))
        del work

    def set_target_scale(self, u, t, idx, n, stream=None):
        """out_scale = RMS of t / a over rows idx[:n] (pmdg_mlp_set_target_scale)."""
        import torch
        work = torch.empty(int(n), dtype=torch.float64, device=u.device)
        check(self.L.pmdg_mlp_set_target_scale(self.h, _ptr(u), _ptr(t), _ptr(idx), int(u.shape[0]), int(n),
                                               _ptr(work), 8 * int(n), _stream_ptr(stream)))

    @property
    def out_scale(self):
        v = ctypes.c_float()
        check(self.L.pmdg_mlp_out_scale(self.h, ctypes.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "h", None):
            self.L.pmdg_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pair_combine(a, b, mean=None, spread=None, stream=None):
    """mean = (a + b) / 2 and per-row |a - b| / |mean| (device FP32)."""
    import torch
    B, n = a.shape
    mean = torch.empty_like(a) if mean is None else mean
    spread = torch.empty(B, dtype=torch.float32, device=a.device) if spread is None else spread
    check(lib().pmdg_mlp_pair_combine(_ptr(a), _ptr(b), int(B), int(n), _ptr(mean), _ptr(spread),
                                      _stream_ptr(stream)))
    return mean, spread


def columns_from_kinds(kind, shift, scale):
    """Embedding columns for per-feature kinds: 0 affine, 1 angle (cos, sin)."""
    cols = []
    for c, k in enumerate(kind):
        if k == 0:
            cols.append((c, 0, float(shift[c]), float(scale[c])))
        else:
            cols += [(c, 1, 0.0, 1.0), (c, 2, 0.0, 1.0)]
    return cols


def row_errors(y, t, idx=None, stream=None):
    """err[r] = ||y_r - t[idx[r]]|| / ||t[idx[r]]|| on the device."""
    import torch
    B, n = y.shape
    err = torch.empty(B, dtype=torch.float32, device=y.device)
    check(lib().pmdg_mlp_row_errors(_ptr(y), _ptr(t), _ptr(idx), int(t.shape[0]), int(B), int(n), _ptr(err),
                                    _stream_ptr(stream)))
    return err


def scatter_rows(src, rows, dst, stream=None):
    """dst[rows[i]] = src[i] on the device (rows: device int32)."""
    nr, n = src.shape
    check(lib().pmdg_mlp_scatter_rows(_ptr(src), _ptr(rows), int(nr), int(n), _ptr(dst), _stream_ptr(stream)))
