"""Face matching on the non-conforming interface (Sec. 5, Algorithm 3) on
the GPU: a thin binding of pmdg_match_faces (argument marshalling only).

layer_hexes() gathers the corner coordinates of one element layer of a
vertex grid, the input the matcher takes."""
import ctypes

import numpy as np

from ._lib import check, lib
from .solver import _stream_ptr


def layer_hexes(V, ne, ez):
    """Corners [n, 8, 3] (corner c = cx + 2 cy + 4 cz) of element layer ez
    of the vertex grid V [(ne0+1)(ne1+1)(ne2+1), 3] (x fastest), elements
    ordered ex + ne0 ey."""
    V = np.asarray(V, dtype=np.float64)
    nx, ny = ne[0] + 1, ne[1] + 1
    ex, ey = np.meshgrid(np.arange(ne[0]), np.arange(ne[1]), indexing="xy")
    ex, ey = ex.ravel(), ey.ravel()
    out = np.empty((ex.size, 8, 3))
    for c in range(8):
        i, j, k = ex + (c & 1), ey + ((c >> 1) & 1), ez + ((c >> 2) & 1)
        out[:, c] = V[i + nx * (j + ny * k)]
    return out


def match_faces(nq, fine_hex, fine_face, coarse_hex, coarse_face, tol=1e-6, eps=1e-9, device="cuda",
                stream=None):
    """Runs pmdg_match_faces on device copies of the inputs; returns device
    tensors (elem [nf nq^2] int32, xi [nf nq^2, 3] float64, unmatched [1]
    int32), valid once `stream` has reached the call."""
    import torch
    fh = torch.as_tensor(np.ascontiguousarray(fine_hex, dtype=np.float64).reshape(-1, 24), device=device)
    ch = torch.as_tensor(np.ascontiguousarray(coarse_hex, dtype=np.float64).reshape(-1, 24), device=device)
    ff = torch.as_tensor(np.ascontiguousarray(fine_face, dtype=np.int32).reshape(-1), device=device)
    cf = torch.as_tensor(np.ascontiguousarray(coarse_face, dtype=np.int32).reshape(-1), device=device)
    nf, nc = fh.shape[0], ch.shape[0]
    npts = nf * nq * nq
    elem = torch.empty(max(npts, 1), dtype=torch.int32, device=device)
    xi = torch.empty((max(npts, 1), 3), dtype=torch.float64, device=device)
    un = torch.empty(1, dtype=torch.int32, device=device)
    vp = ctypes.c_void_p
    check(lib().pmdg_match_faces(int(nq), nf, vp(fh.data_ptr()), vp(ff.data_ptr()), nc, vp(ch.data_ptr()),
                                 vp(cf.data_ptr()), float(tol), float(eps), vp(elem.data_ptr()),
                                 vp(xi.data_ptr()), vp(un.data_ptr()), _stream_ptr(stream)))
    # the inputs must outlive the kernels: keep them with the outputs
    match_faces._keep = (fh, ch, ff, cf)
    return elem[:npts], xi[:npts], un
