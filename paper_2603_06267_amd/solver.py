"""Python face of libpmutdg: a thin wrapper around the C ABI.

PyTorch provides the device workspace (one uint8 tensor) and the stream; all
per-step work runs in the library's HIP kernels.  Every method marshals its
arguments and calls exactly one (or a few) C entry points.
"""
import ctypes

import numpy as np

from . import _lib
from ._lib import check, lib

_dp = ctypes.POINTER(ctypes.c_double)


def _d(a):
    return a.ctypes.data_as(_dp)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _stream_ptr(stream):
    if stream is None:
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if hasattr(stream, "cuda_stream"):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def problem_struct(domains, cfl=0.3, dt=0.0, alpha=2.0, precision=32, n_scenarios=1, trace_capacity=1):
    pr = _lib.Problem()
    pr.ndom = len(domains)
    for i, d in enumerate(domains):
        b = pr.dom[i]
        for a in range(3):
            b.x0[a] = d["x0"][a]
            b.x1[a] = d["x1"][a]
            b.ne[a] = d["ne"][a]
        b.order = d["N"]
        b.c = d["c"]
        b.rho = d["rho"]
    pr.cfl = cfl
    pr.dt = dt
    pr.penalty_alpha = alpha
    pr.precision = precision
    pr.n_scenarios = n_scenarios
    pr.trace_capacity = trace_capacity
    return pr


class Solver:
    """One mesh (one or two bricks), S drive scenarios, on one GPU."""

    def __init__(self, domains, cfl=0.3, dt=0.0, alpha=2.0, precision=32, n_scenarios=1, trace_capacity=1,
                 device="cuda"):
        self.L = lib()
        pr = problem_struct(domains, cfl, dt, alpha, precision, n_scenarios, trace_capacity)
        h = ctypes.c_void_p()
        check(self.L.pmdg_create(ctypes.byref(pr), ctypes.byref(h)))
        self.h = h
        self.S = n_scenarios
        self.precision = precision
        self.device = device
        self.ws = None
        self.R = 0
        self.Np = 0
        self.Nm = 0

    def close(self):
        if getattr(self, "h", None):
            if getattr(self, "ws", None) is not None:
                # work enqueued on any stream may still read the workspace
                import torch
                torch.cuda.synchronize(self.ws.device)
            self.L.pmdg_destroy(self.h)
            self.h = None
        self.ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- setup
    @property
    def dt(self):
        v = ctypes.c_double()
        check(self.L.pmdg_get_dt(self.h, ctypes.byref(v)))
        return v.value

    def lambda_max(self):
        v = ctypes.c_double()
        check(self.L.pmdg_lambda_max(self.h, ctypes.byref(v)))
        return v.value

    def num_nodes(self):
        n = ctypes.c_long()
        check(self.L.pmdg_num_nodes(self.h, ctypes.byref(n)))
        return n.value

    def node_coords(self):
        xyz = np.zeros((self.num_nodes(), 3))
        check(self.L.pmdg_node_coords(self.h, _d(xyz)))
        return xyz

    def set_pmuts(self, centers, radius, omega, zeta, eta):
        c = _f64(centers).reshape(-1, 2)
        r = _f64(radius).reshape(-1)
        om = _f64(omega)
        self.Np, self.Nm = om.shape
        check(self.L.pmdg_set_pmuts(self.h, self.Np, _d(c), _d(r), self.Nm, _d(om),
                                    _d(_f64(zeta).reshape(om.shape)), _d(_f64(eta).reshape(om.shape))))

    def pmut_face_nodes(self, k):
        n = ctypes.c_int()
        check(self.L.pmdg_pmut_face_nodes(self.h, k, ctypes.byref(n), _dp()))
        xyz = np.zeros((max(n.value, 1), 3))
        check(self.L.pmdg_pmut_face_nodes(self.h, k, ctypes.byref(n), _d(xyz)))
        return xyz[: n.value]

    def set_pmut_shape(self, k, shape):
        check(self.L.pmdg_set_pmut_shape(self.h, k, _d(_f64(shape))))

    def set_drive(self, amp, phase, freq, ncyc, envelope=0):
        amp = _f64(amp).reshape(-1)
        phase = _f64(phase).reshape(-1)
        freq = _f64(freq).reshape(-1)
        check(self.L.pmdg_set_drive(self.h, _d(amp), _d(phase), _d(freq), float(ncyc), int(envelope)))

    def set_rx(self, t_switch, cap):
        check(self.L.pmdg_set_rx(self.h, float(t_switch), float(cap)))

    def set_vertices(self, dom, V):
        """Trilinear hexahedra: element vertices [(ne0+1)(ne1+1)(ne2+1), 3]
        of the single brick, x fastest; before set_pmuts, set_receivers and
        bind."""
        check(self.L.pmdg_set_vertices(self.h, int(dom), _d(_f64(V).reshape(-1, 3))))

    def set_absorbing(self, dom, faces):
        """First-order absorbing condition on the outer faces of brick dom
        (6-bit mask: bit 2a low end, 2a + 1 high end of axis a); before bind."""
        check(self.L.pmdg_set_absorbing(self.h, int(dom), int(faces)))

    def set_pml(self, dom, ell, R=1e-4):
        """Perfectly matched layer inside brick dom: thickness ell[2a] at the
        low end and ell[2a + 1] at the high end of axis a; before bind."""
        check(self.L.pmdg_set_pml(self.h, int(dom), _d(_f64(ell).reshape(6)), float(R)))

    def set_receivers(self, xyz):
        xyz = _f64(xyz).reshape(-1, 3)
        self.R = xyz.shape[0]
        check(self.L.pmdg_set_receivers(self.h, self.R, _d(xyz)))

    def workspace_size(self):
        n = ctypes.c_size_t()
        check(self.L.pmdg_workspace_size(self.h, ctypes.byref(n)))
        return n.value

    def bind(self, stream=None):
        import torch
        nbytes = self.workspace_size()
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        ptr = self.ws.data_ptr()
        ptr = (ptr + 255) // 256 * 256
        check(self.L.pmdg_bind(self.h, ctypes.c_void_p(ptr), nbytes, _stream_ptr(stream)))

    def bind_static(self, stream=None):
        """Binds the library-held workspace of the current device (no device
        allocation by anyone)."""
        check(self.L.pmdg_bind_static(self.h, _stream_ptr(stream)))

    def restart(self, stream=None):
        """Back to step 0 with everything at rest, tables and drive kept
        (pmdg_restart)."""
        check(self.L.pmdg_restart(self.h, _stream_ptr(stream)))

    def set_option(self, opt, value):
        check(self.L.pmdg_set_option(self.h, int(opt), int(value)))

    # ---- stepping
    def step(self, n, stream=None):
        check(self.L.pmdg_step(self.h, int(n), _stream_ptr(stream)))

    def steps_done(self):
        n = ctypes.c_long()
        check(self.L.pmdg_steps_done(self.h, ctypes.byref(n)))
        return n.value

    def resident(self):
        """True when step() takes the LDS-resident path."""
        v = ctypes.c_int()
        check(self.L.pmdg_resident(self.h, ctypes.byref(v)))
        return bool(v.value)

    def kernel_times(self):
        t = np.zeros(3)
        check(self.L.pmdg_kernel_times(self.h, _d(t)))
        return t

    def read_traces(self, stream=None):
        n = self.steps_done()
        out = np.zeros((self.S, self.R, max(n, 1)))
        check(self.L.pmdg_read_traces(self.h, _d(out), _stream_ptr(stream)))
        return out[:, :, :n]

    def read_traces_device(self, bits=32, stream=None):
        """Traces [S, R, steps_done] as a device tensor (FP32 or FP64),
        written by the library on `stream` without a host round trip."""
        import torch
        n = self.steps_done()
        dt = torch.float32 if bits == 32 else torch.float64
        out = torch.empty((self.S, self.R, n), dtype=dt, device=self.device)
        if out.numel():
            check(self.L.pmdg_read_traces_device(self.h, ctypes.c_void_p(out.data_ptr()), bits,
                                                 _stream_ptr(stream)))
        return out

    def read_modal(self, s=0, stream=None):
        nm = max(self.Np * self.Nm, 1)
        q, qd, qdd = np.zeros(nm), np.zeros(nm), np.zeros(nm)
        check(self.L.pmdg_read_modal(self.h, s, _d(q), _d(qd), _d(qdd), _stream_ptr(stream)))
        k = self.Np * self.Nm
        return q[:k], qd[:k], qdd[:k]

    def get_state(self, s=0, stream=None):
        n = self.num_nodes()
        p, pp = np.zeros(n), np.zeros(n)
        check(self.L.pmdg_get_state(self.h, s, _d(p), _d(pp), _stream_ptr(stream)))
        return p, pp

    def set_state(self, s, p, p_prev, q=None, qd=None, qdd=None, nstep=0, stream=None):
        keep = [None if a is None else _f64(a) for a in (p, p_prev, q, qd, qdd)]
        ptrs = [_dp() if a is None else _d(a) for a in keep]
        check(self.L.pmdg_set_state(self.h, int(s), *ptrs, int(nstep), _stream_ptr(stream)))

    def nonfinite(self, stream=None):
        v = ctypes.c_int()
        check(self.L.pmdg_status_flags(self.h, ctypes.byref(v), _stream_ptr(stream)))
        return bool(v.value)


def from_workload(wl, precision=32, n_steps=None, scenarios=None, shape_fn=None, device="cuda", bind=True):
    """Builds, fills and binds a solver for a workload description.

    scenarios: indices into the workload's drive rows (default: all rows).
    bind: True binds a caller workspace (a torch tensor), "static" the
    library-held workspace, False leaves the solver unbound."""
    dr = wl.get("drive")
    if scenarios is None:
        scenarios = list(range(np.asarray(dr["amp"]).shape[0])) if dr is not None else [0]
    S = len(scenarios)
    steps = n_steps if n_steps is not None else wl["steps"]
    s = Solver(wl["domains"], cfl=wl.get("cfl", 0.3), alpha=wl.get("alpha", 2.0), precision=precision,
               n_scenarios=S, trace_capacity=max(steps, 1), device=device)
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
            s.set_pmut_shape(k, shape_fn(k, s.pmut_face_nodes(k)))
        amp = np.asarray(dr["amp"])[scenarios]
        phase = np.asarray(dr["phase"])[scenarios]
        freq = np.asarray(dr["freq"]).reshape(-1)[scenarios]
        s.set_drive(amp, phase, freq, dr["ncyc"], dr.get("envelope", 0))
        if "rx" in wl:
            s.set_rx(wl["rx"]["t_switch"], wl["rx"]["cap"])
    s.set_receivers(wl["receivers"])
    if bind == "static":
        s.bind_static()
    elif bind:
        s.bind()
    return s
