"""ctypes wrapper of the FP64 CPU oracle (oracle/pmdg_ref.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline leg use this module; the product package never imports it.  It takes
plain dictionaries and NumPy arrays (the seeded workload description) and
shares no code with the HIP library.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_dp = ctypes.POINTER(ctypes.c_double)
_lp = ctypes.POINTER(ctypes.c_long)


def _d(a):
    return a.ctypes.data_as(_dp)


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        src = os.path.join(_build.HERE, "pmdg_ref.c")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(src):
            _build.build()
        L = ctypes.CDLL(path)
        vp = ctypes.c_void_p
        L.pmdg_ref_create.restype = vp
        L.pmdg_ref_create.argtypes = [ctypes.c_int, _dp, ctypes.c_double, ctypes.c_double]
        L.pmdg_ref_destroy.argtypes = [vp]
        L.pmdg_ref_num_nodes.restype = ctypes.c_long
        L.pmdg_ref_num_nodes.argtypes = [vp]
        L.pmdg_ref_dom_nodes.restype = ctypes.c_long
        L.pmdg_ref_dom_nodes.argtypes = [vp, ctypes.c_int]
        L.pmdg_ref_gamma.restype = ctypes.c_double
        L.pmdg_ref_gamma.argtypes = [vp]
        L.pmdg_ref_set_literal.argtypes = [vp, ctypes.c_int]
        L.pmdg_ref_set_absorbing_literal.argtypes = [vp, ctypes.c_int]
        L.pmdg_ref_set_sample_gain.argtypes = [vp, ctypes.c_double]
        L.pmdg_ref_set_dt.argtypes = [vp, ctypes.c_double]
        L.pmdg_ref_cfl_dt.restype = ctypes.c_double
        L.pmdg_ref_cfl_dt.argtypes = [vp, ctypes.c_double]
        L.pmdg_ref_coords.argtypes = [vp, _dp]
        L.pmdg_ref_mass.argtypes = [vp, _dp]
        L.pmdg_ref_apply_K.argtypes = [vp, _dp, _dp, ctypes.c_int]
        L.pmdg_ref_lambda_max.restype = ctypes.c_double
        L.pmdg_ref_lambda_max.argtypes = [vp, ctypes.c_int, ctypes.c_uint]
        L.pmdg_ref_set_pmuts.restype = ctypes.c_int
        L.pmdg_ref_set_pmuts.argtypes = [vp, ctypes.c_int, _dp, _dp, ctypes.c_int, _dp, _dp, _dp]
        L.pmdg_ref_pmut_nodes.restype = ctypes.c_int
        L.pmdg_ref_pmut_nodes.argtypes = [vp, ctypes.c_int, _dp]
        L.pmdg_ref_set_shape.restype = ctypes.c_int
        L.pmdg_ref_set_shape.argtypes = [vp, ctypes.c_int, _dp]
        L.pmdg_ref_coupling.restype = ctypes.c_int
        L.pmdg_ref_coupling.argtypes = [vp, ctypes.c_int, ctypes.c_int, _lp, _dp]
        L.pmdg_ref_set_drive.argtypes = [vp, _dp, _dp, ctypes.c_double, ctypes.c_double, ctypes.c_int]
        L.pmdg_ref_set_rx.argtypes = [vp, ctypes.c_double, ctypes.c_double]
        L.pmdg_ref_window.restype = ctypes.c_double
        L.pmdg_ref_window.argtypes = [ctypes.c_double, ctypes.c_double]
        L.pmdg_ref_drive.restype = ctypes.c_double
        L.pmdg_ref_drive.argtypes = [ctypes.c_double] * 4 + [ctypes.c_int, ctypes.c_double]
        L.pmdg_ref_set_receivers.restype = ctypes.c_int
        L.pmdg_ref_set_receivers.argtypes = [vp, ctypes.c_int, _dp]
        L.pmdg_ref_sample_receivers.argtypes = [vp, _dp, _dp]
        L.pmdg_ref_set_state.argtypes = [vp, _dp, _dp, _dp, _dp, _dp, _dp, ctypes.c_long]
        L.pmdg_ref_get_state.argtypes = [vp, _dp, _dp, _dp, _dp, _dp, _dp, _lp]
        L.pmdg_ref_step.argtypes = [vp, ctypes.c_int, _dp]
        L.pmdg_ref_gll.restype = ctypes.c_int
        L.pmdg_ref_gll.argtypes = [ctypes.c_int, _dp, _dp]
        L.pmdg_ref_gl.restype = ctypes.c_int
        L.pmdg_ref_gl.argtypes = [ctypes.c_int, _dp, _dp]
        L.pmdg_ref_dmat.restype = ctypes.c_int
        L.pmdg_ref_dmat.argtypes = [ctypes.c_int, _dp]
        L.pmdg_ref_lagrange.argtypes = [ctypes.c_int, _dp, ctypes.c_double, _dp, _dp]
        L.pmdg_ref_element_apply.argtypes = [ctypes.c_int, _dp, ctypes.c_double, _dp, _dp]
        L.pmdg_ref_num_threads.restype = ctypes.c_int
        L.pmdg_ref_set_threads.argtypes = [ctypes.c_int]
        L.pmdg_ref_set_vertices.restype = ctypes.c_int
        L.pmdg_ref_set_vertices.argtypes = [vp, ctypes.c_int, _dp]
        L.pmdg_ref_hex_apply.argtypes = [ctypes.c_int, _dp, ctypes.c_double, _dp, _dp]
        _ip = ctypes.POINTER(ctypes.c_int)
        L.pmdg_ref_match_faces.restype = ctypes.c_int
        L.pmdg_ref_match_faces.argtypes = [ctypes.c_int, ctypes.c_int, _dp, _ip, ctypes.c_int, _dp, _ip,
                                           ctypes.c_double, ctypes.c_double, _ip, _dp]
        L.pmdg_ref_interface_points.restype = ctypes.c_long
        L.pmdg_ref_interface_points.argtypes = [vp, _ip, _dp]
        L.pmdg_ref_set_absorbing.argtypes = [vp, ctypes.c_int, ctypes.c_int]
        L.pmdg_ref_absorbing.argtypes = [vp, _dp]
        L.pmdg_ref_set_pml.restype = ctypes.c_int
        L.pmdg_ref_set_pml.argtypes = [vp, ctypes.c_int, _dp, ctypes.c_double]
        L.pmdg_ref_pml_profile.argtypes = [vp, ctypes.c_int, ctypes.c_int, _dp]
        _lib = L
    return _lib


# ---------------------------------------------------------------- helpers

def gll(N):
    x = np.zeros(N + 1); w = np.zeros(N + 1)
    if lib().pmdg_ref_gll(N, _d(x), _d(w)):
        raise ValueError("order out of range")
    return x, w


def gl(n):
    x = np.zeros(n); w = np.zeros(n)
    if lib().pmdg_ref_gl(n, _d(x), _d(w)):
        raise ValueError("point count out of range")
    return x, w


def dmat(N):
    D = np.zeros((N + 1, N + 1))
    lib().pmdg_ref_dmat(N, _d(D))
    return D


def lagrange(nodes, t):
    nodes = np.ascontiguousarray(nodes, dtype=np.float64)
    n = len(nodes) - 1
    v = np.zeros(n + 1); d = np.zeros(n + 1)
    lib().pmdg_ref_lagrange(n, _d(nodes), float(t), _d(v), _d(d))
    return v, d


def element_apply(N, h, c, u):
    h = np.ascontiguousarray(h, dtype=np.float64)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    r = np.zeros_like(u)
    lib().pmdg_ref_element_apply(N, _d(h), float(c), _d(u), _d(r))
    return r


def window(t, Td):
    return lib().pmdg_ref_window(float(t), float(Td))


def drive(A, theta, f, ncyc, envelope, t):
    return lib().pmdg_ref_drive(float(A), float(theta), float(f), float(ncyc), int(envelope), float(t))


def num_threads():
    return lib().pmdg_ref_num_threads()


def set_threads(n):
    """Thread count of the oracle's loops from here on."""
    lib().pmdg_ref_set_threads(int(n))


def hex_apply(N, V8, c, u):
    """K_e u on one trilinear hexahedron with vertices V8 [8 x 3] (corner
    c = cx + 2 cy + 4 cz), u [(N+1)^3] with the first index fastest."""
    V8 = np.ascontiguousarray(V8, dtype=np.float64).reshape(24)
    u = np.ascontiguousarray(u, dtype=np.float64).reshape(-1)
    r = np.zeros_like(u)
    lib().pmdg_ref_hex_apply(int(N), _d(V8), float(c), _d(u), _d(r))
    return r


def match_faces(nq, fine_hex, fine_face, coarse_hex, coarse_face, tol=1e-6, eps=1e-9):
    """Face matching of Sec. 5, Algorithm 3 (see pmdg_ref_match_faces):
    returns (elem [nf*nq*nq], xi [nf*nq*nq, 3], unmatched count)."""
    fh = np.ascontiguousarray(fine_hex, dtype=np.float64).reshape(-1, 24)
    ch = np.ascontiguousarray(coarse_hex, dtype=np.float64).reshape(-1, 24)
    ff = np.ascontiguousarray(fine_face, dtype=np.int32).reshape(-1)
    cf = np.ascontiguousarray(coarse_face, dtype=np.int32).reshape(-1)
    nf, nc = len(fh), len(ch)
    assert len(ff) == nf and len(cf) == nc
    elem = np.zeros(max(nf * nq * nq, 1), dtype=np.int32)
    xi = np.zeros((max(nf * nq * nq, 1), 3))
    _ip = ctypes.POINTER(ctypes.c_int)
    n = lib().pmdg_ref_match_faces(int(nq), nf, _d(fh), ff.ctypes.data_as(_ip), nc, _d(ch),
                                   cf.ctypes.data_as(_ip), float(tol), float(eps),
                                   elem.ctypes.data_as(_ip), _d(xi))
    if n < 0:
        raise ValueError("oracle: bad face-matching arguments")
    m = nf * nq * nq
    return elem[:m], xi[:m], n


def dom_params(dom):
    """12 doubles {x0[3], h[3], ne[3], N, c, rho} from a brick description."""
    x0 = np.asarray(dom["x0"], dtype=np.float64)
    x1 = np.asarray(dom["x1"], dtype=np.float64)
    ne = np.asarray(dom["ne"], dtype=np.float64)
    h = (x1 - x0) / ne
    return np.concatenate([x0, h, ne, [dom["N"], dom["c"], dom["rho"]]])


class RefSolver:
    """One scenario of the coupled problem on the CPU, FP64."""

    def __init__(self, domains, alpha=2.0, cfl=0.3, dt=None):
        prm = np.ascontiguousarray(np.concatenate([dom_params(d) for d in domains]))
        self.L = lib()
        self.h = self.L.pmdg_ref_create(len(domains), _d(prm), 1.0, float(alpha))
        if not self.h:
            raise ValueError("oracle: invalid mesh description")
        self.ndom = len(domains)
        self.domains = [dict(d) for d in domains]
        self.n = self.L.pmdg_ref_num_nodes(self.h)
        self._cfl = None if dt is not None else float(cfl)
        self.dt = float(dt) if dt is not None else self.L.pmdg_ref_cfl_dt(self.h, float(cfl))
        self.L.pmdg_ref_set_dt(self.h, self.dt)
        self.Np = 0
        self.Nm = 0
        self.R = 0

    def __del__(self):
        try:
            if self.h:
                self.L.pmdg_ref_destroy(self.h)
                self.h = None
        except Exception:
            pass

    # ---- mesh / operators
    def dom_nodes(self, d):
        return self.L.pmdg_ref_dom_nodes(self.h, d)

    def coords(self):
        x = np.zeros((self.n, 3))
        self.L.pmdg_ref_coords(self.h, _d(x))
        return x

    def set_vertices(self, dom, V):
        """Trilinear hexahedra: vertex coordinates [(ne0+1)(ne1+1)(ne2+1), 3]
        of the single domain, x fastest.  A CFL-chosen time step is chosen
        again from the shortest element edge."""
        d = self.domains[dom]
        nv = int(np.prod(np.asarray(d["ne"]) + 1))
        V = np.ascontiguousarray(V, dtype=np.float64).reshape(nv, 3)
        r = self.L.pmdg_ref_set_vertices(self.h, int(dom), _d(V))
        if r == -2:
            raise ValueError("oracle: an element's Jacobian is not positive")
        if r:
            raise ValueError("oracle: trilinear hexahedra need a single domain without absorbing faces or layers")
        self.domains[dom]["_mapped"] = True
        if self._cfl is not None:
            self.dt = self.L.pmdg_ref_cfl_dt(self.h, self._cfl)
            self.L.pmdg_ref_set_dt(self.h, self.dt)

    def interface_points(self):
        """(coarse element (ex, ey) [npts, 2], reference (xi, eta) [npts, 2])
        of every fine-face Gauss-Legendre point, ordered (fine face, eta, xi)."""
        _ip = ctypes.POINTER(ctypes.c_int)
        n = self.L.pmdg_ref_interface_points(self.h, None, None)
        ce = np.zeros((max(n, 1), 2), dtype=np.int32)
        xi = np.zeros((max(n, 1), 2))
        self.L.pmdg_ref_interface_points(self.h, ce.ctypes.data_as(_ip), _d(xi))
        return ce[:n], xi[:n]

    def set_absorbing(self, dom, faces):
        """First-order absorbing condition on the outer faces of domain dom
        given by the bitmask faces (bit 2a: low end of axis a, 2a + 1: high
        end)."""
        if self.domains[dom].get("_mapped"):
            raise ValueError("oracle: absorbing faces on trilinear hexahedra are not built")
        self.L.pmdg_ref_set_absorbing(self.h, int(dom), int(faces))

    def set_pml(self, dom, ell, R=1e-4):
        """Perfectly matched layer inside domain dom: thickness ell[2a] at the
        low end and ell[2a + 1] at the high end of axis a (0: none),
        reflection coefficient R."""
        ell = np.ascontiguousarray(ell, dtype=np.float64).reshape(6)
        if self.L.pmdg_ref_set_pml(self.h, int(dom), _d(ell), float(R)):
            raise ValueError("oracle: bad layer description")

    def pml_profile(self, dom, axis):
        """zeta of the given axis at that axis's node coordinates of domain dom."""
        d = self.domains[dom]
        out = np.zeros(d["N"] * d["ne"][axis] + 1)
        self.L.pmdg_ref_pml_profile(self.h, int(dom), int(axis), _d(out))
        return out

    def absorbing(self):
        out = np.zeros(self.n)
        self.L.pmdg_ref_absorbing(self.h, _d(out))
        return out

    def mass(self):
        m = np.zeros(self.n)
        self.L.pmdg_ref_mass(self.h, _d(m))
        return m

    def apply_K(self, p, which=3):
        p = np.ascontiguousarray(p, dtype=np.float64)
        out = np.zeros(self.n)
        self.L.pmdg_ref_apply_K(self.h, _d(p), _d(out), which)
        return out

    def dense_K(self, which=3):
        K = np.zeros((self.n, self.n))
        e = np.zeros(self.n)
        for j in range(self.n):
            e[:] = 0.0
            e[j] = 1.0
            K[:, j] = self.apply_K(e, which)
        return K

    def gamma(self):
        return self.L.pmdg_ref_gamma(self.h)

    def lambda_max(self, iters=200, seed=1):
        return self.L.pmdg_ref_lambda_max(self.h, iters, seed)

    def set_literal(self, on):
        self.L.pmdg_ref_set_literal(self.h, 1 if on else 0)

    def set_absorbing_literal(self, on):
        """Test switch: absorbing damping on the predicted velocity alone,
        M pdd = f - K p - C pdot* (the acoustic solve as printed)."""
        self.L.pmdg_ref_set_absorbing_literal(self.h, 1 if on else 0)

    def set_sample_gain(self, g):
        self.L.pmdg_ref_set_sample_gain(self.h, float(g))

    # ---- PMUTs
    def set_pmuts(self, centers, radius, omega, zeta, eta):
        centers = np.ascontiguousarray(centers, dtype=np.float64).reshape(-1, 2)
        radius = np.ascontiguousarray(radius, dtype=np.float64).reshape(-1)
        omega = np.ascontiguousarray(omega, dtype=np.float64)
        self.Np, self.Nm = omega.shape
        zeta = np.ascontiguousarray(zeta, dtype=np.float64).reshape(self.Np, self.Nm)
        eta = np.ascontiguousarray(eta, dtype=np.float64).reshape(self.Np, self.Nm)
        self.L.pmdg_ref_set_pmuts(self.h, self.Np, _d(centers), _d(radius), self.Nm,
                                  _d(omega), _d(zeta), _d(eta))

    def pmut_nodes(self, k):
        n = self.L.pmdg_ref_pmut_nodes(self.h, k, _dp())
        xyz = np.zeros((max(n, 1), 3))
        self.L.pmdg_ref_pmut_nodes(self.h, k, _d(xyz))
        return xyz[:n]

    def set_shape(self, k, shape):
        shape = np.ascontiguousarray(shape, dtype=np.float64)
        self.L.pmdg_ref_set_shape(self.h, k, _d(shape))

    def coupling(self, k, m):
        n = self.L.pmdg_ref_pmut_nodes(self.h, k, _dp())
        node = np.zeros(max(n, 1), dtype=np.int64); val = np.zeros(max(n, 1))
        self.L.pmdg_ref_coupling(self.h, k, m, node.ctypes.data_as(_lp), _d(val))
        return node[:n], val[:n]

    def set_drive(self, amp, phase, freq, ncyc, envelope=0):
        amp = np.ascontiguousarray(amp, dtype=np.float64).reshape(-1)
        phase = np.ascontiguousarray(phase, dtype=np.float64).reshape(-1)
        self.L.pmdg_ref_set_drive(self.h, _d(amp), _d(phase), float(freq), float(ncyc), int(envelope))

    def set_rx(self, t_switch, cap):
        self.L.pmdg_ref_set_rx(self.h, float(t_switch), float(cap))

    # ---- receivers
    def set_receivers(self, xyz):
        xyz = np.ascontiguousarray(xyz, dtype=np.float64).reshape(-1, 3)
        self.R = xyz.shape[0]
        if self.L.pmdg_ref_set_receivers(self.h, self.R, _d(xyz)):
            raise ValueError("oracle: receiver outside the mesh")

    def sample(self, p):
        p = np.ascontiguousarray(p, dtype=np.float64)
        out = np.zeros(self.R)
        self.L.pmdg_ref_sample_receivers(self.h, _d(p), _d(out))
        return out

    # ---- state and stepping
    def set_state(self, p=None, pd=None, pdd=None, q=None, qd=None, qdd=None, nstep=0):
        def arr(a):
            return _dp() if a is None else _d(np.ascontiguousarray(a, dtype=np.float64))
        keep = [np.ascontiguousarray(a, dtype=np.float64) if a is not None else None
                for a in (p, pd, pdd, q, qd, qdd)]
        ptrs = [_dp() if a is None else _d(a) for a in keep]
        self.L.pmdg_ref_set_state(self.h, *ptrs, int(nstep))
        del arr

    def get_state(self):
        nm = max(self.Np * self.Nm, 1)
        p, pd, pdd = np.zeros(self.n), np.zeros(self.n), np.zeros(self.n)
        q, qd, qdd = np.zeros(nm), np.zeros(nm), np.zeros(nm)
        ns = ctypes.c_long(0)
        self.L.pmdg_ref_get_state(self.h, _d(p), _d(pd), _d(pdd), _d(q), _d(qd), _d(qdd), ctypes.byref(ns))
        k = self.Np * self.Nm
        return dict(p=p, pd=pd, pdd=pdd, q=q[:k], qd=qd[:k], qdd=qdd[:k], nstep=ns.value)

    def step(self, nsteps):
        tr = np.zeros((max(self.R, 1), nsteps))
        self.L.pmdg_ref_step(self.h, int(nsteps), _d(tr))
        return tr[: self.R]


def from_workload(wl, scenario=0, shape_fn=None):
    """Builds an oracle solver for one scenario of a workload description.

    shape_fn(k, xyz) -> [Nm x n] mode-shape samples at the given face nodes
    (the workload's own mode-shape generator)."""
    s = RefSolver(wl["domains"], alpha=wl.get("alpha", 2.0), cfl=wl.get("cfl", 0.3))
    for d, dom in enumerate(wl["domains"]):
        if dom.get("vertices") is not None:
            s.set_vertices(d, dom["vertices"])
    for d, dom in enumerate(wl["domains"]):
        if dom.get("absorbing", 0):
            s.set_absorbing(d, dom["absorbing"])
        if dom.get("pml"):
            s.set_pml(d, dom["pml"]["ell"], dom["pml"].get("R", 1e-4))
    pm = wl.get("pmuts")
    if pm is not None and len(pm["radius"]):
        s.set_pmuts(pm["centers"], pm["radius"], pm["omega"], pm["zeta"], pm["eta"])
        for k in range(s.Np):
            xyz = s.pmut_nodes(k)
            s.set_shape(k, shape_fn(k, xyz))
        dr = wl["drive"]
        s.set_drive(np.asarray(dr["amp"])[scenario], np.asarray(dr["phase"])[scenario],
                    np.asarray(dr["freq"]).reshape(-1)[scenario], dr["ncyc"], dr.get("envelope", 0))
        if "rx" in wl:
            s.set_rx(wl["rx"]["t_switch"], wl["rx"]["cap"])
    s.set_receivers(wl["receivers"])
    return s
