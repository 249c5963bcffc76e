"""Seeded synthetic workload descriptions shaped like the paper's PMUT arrays.

This module only *describes inputs*: brick extents, element counts, orders,
materials, PMUT disc centres and radii, modal frequencies / damping /
coupling coefficients, mode-shape samples, drive parameters and receiver
positions.  It holds none of the method's arithmetic (no quadrature, no
operators, no time stepping) and is the only code shared by the HIP path and
the CPU oracle, which both consume its plain dictionaries.

Units: millimetres, microseconds (so c = 1.5 mm/us is 1500 m/s and
frequencies are in MHz, angular frequencies in rad/us).  Pressure and modal
amplitudes are in arbitrary consistent units (the problem is linear).

Seeds: NumPy PCG64 `default_rng(20260306 + index)`.
"""
import hashlib
import json
import math

import numpy as np

SEED0 = 20260306

# Zeros of the Bessel function J0, used by the radial mode profiles.
try:
    from scipy.special import j0 as _j0, jn_zeros as _jn_zeros

    def _bessel_zeros(n):
        return _jn_zeros(0, n)
except Exception:  # pragma: no cover - scipy is part of the image
    _j0 = None

    def _bessel_zeros(n):
        raise RuntimeError("scipy.special is required for the J0 mode profiles")

C_WATER = 1.5      # mm/us
RHO = 1.0          # arbitrary density unit; kappa = rho c^2
SHAPE_SCALE = 8.0  # modal scale s_{k,m}; unit modal mass is absorbed here
ETA = 1.0          # electro-mechanical coupling coefficient


def brick(x0, x1, ne, N, c=C_WATER, rho=RHO):
    return {"x0": [float(v) for v in x0], "x1": [float(v) for v in x1],
            "ne": [int(v) for v in ne], "N": int(N), "c": float(c), "rho": float(rho)}


def brick_vertices(dom):
    """Element vertices of a brick, [(ne0+1)(ne1+1)(ne2+1), 3], x fastest."""
    x0 = np.asarray(dom["x0"], dtype=np.float64)
    x1 = np.asarray(dom["x1"], dtype=np.float64)
    ne = np.asarray(dom["ne"])
    ax = [x0[a] + (x1[a] - x0[a]) * np.arange(ne[a] + 1) / ne[a] for a in range(3)]
    Z, Y, X = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def warped_vertices(dom, amp=0.15, jitter=0.0, seed=0):
    """Brick vertices moved by a smooth seeded displacement that keeps every
    boundary face planar (the component normal to a face vanishes on it),
    plus an optional seeded jitter of the interior vertices; amp and jitter
    are in units of the element size.  The elements stay trilinear
    hexahedra filling the same brick."""
    rng = np.random.default_rng(SEED0 + 100 + seed)
    x0 = np.asarray(dom["x0"], dtype=np.float64)
    x1 = np.asarray(dom["x1"], dtype=np.float64)
    ne = np.asarray(dom["ne"])
    h = (x1 - x0) / ne
    V = brick_vertices(dom)
    u = (V - x0) / (x1 - x0)
    ph = rng.uniform(0.0, 2 * math.pi, size=(3, 2))
    W = V.copy()
    for a in range(3):
        b, c = (a + 1) % 3, (a + 2) % 3
        W[:, a] += amp * h[a] * (np.sin(math.pi * u[:, a]) * np.sin(2 * math.pi * u[:, b] + ph[a, 0])
                                 * np.sin(2 * math.pi * u[:, c] + ph[a, 1]))
    if jitter > 0:
        inner = np.all((u > 1e-12) & (u < 1 - 1e-12), axis=1)
        W[inner] += jitter * h * rng.uniform(-1.0, 1.0, size=(int(inner.sum()), 3))
    return W


def disc_conforming_vertices(dom, centres, radius, pitch, shrink=1e-9):
    """Brick vertices moved in x-y so that element edges follow each PMUT
    disc: in the square cell of side `pitch` around a disc centre (a vertex,
    with pitch / h an even number of elements), the vertex ring at
    Chebyshev distance m_d = floor(radius / h) elements lands on the circle
    of radius radius (1 - shrink), inner rings on concentric circles, and the
    rings between the circle and the cell boundary are blended linearly
    towards the unchanged cell boundary.  The same map applies at every
    height.  `shrink` keeps the ring's nodes strictly inside the disc."""
    x0 = np.asarray(dom["x0"], dtype=np.float64)
    x1 = np.asarray(dom["x1"], dtype=np.float64)
    ne = np.asarray(dom["ne"])
    h = (x1 - x0) / ne
    k = pitch / h[0]
    if abs(h[0] - h[1]) > 1e-12 * h[0] or abs(k - round(k)) > 1e-9 or int(round(k)) % 2:
        raise ValueError("the pitch must be an even number of equal x-y elements")
    half = int(round(k)) // 2
    md = int(math.floor(radius / h[0] + 1e-12))
    if not 1 <= md < half:
        raise ValueError("the disc must span at least one element ring inside its cell")
    V = brick_vertices(dom)
    out = V.copy()
    ctr = np.asarray(centres, dtype=np.float64).reshape(-1, 2)
    rc = radius * (1.0 - shrink)
    for cx, cy in ctr:
        u = np.rint((V[:, 0] - cx) / h[0])
        v = np.rint((V[:, 1] - cy) / h[1])
        m = np.maximum(np.abs(u), np.abs(v))
        sel = (m > 0) & (m < half)
        if not sel.any():
            continue
        us, vs, ms = u[sel], v[sel], m[sel]
        nrm = np.hypot(us, vs)
        pcx, pcy = rc * us / nrm, rc * vs / nrm
        t = np.where(ms <= md, 0.0, (ms - md) / (half - md))
        sc = np.where(ms <= md, ms / md, 1.0)
        out[sel, 0] = cx + (1 - t) * sc * pcx + t * us * h[0]
        out[sel, 1] = cy + (1 - t) * sc * pcy + t * vs * h[1]
    return out


def _grid_centres(nx, ny, pitch, offset):
    return np.array([[offset + pitch * i, offset + pitch * j] for j in range(ny) for i in range(nx)],
                    dtype=np.float64)


def _receivers_in(rng, dom, R):
    x0 = np.asarray(dom["x0"]); x1 = np.asarray(dom["x1"])
    u = rng.uniform(0.05, 0.95, size=(R, 3))
    return x0 + u * (x1 - x0)


def _pmut_block(centres, radius, freqs_mhz, zeta=0.01, eta=ETA, scale=SHAPE_SCALE):
    Np = centres.shape[0]
    freqs_mhz = np.asarray(freqs_mhz, dtype=np.float64).reshape(Np, -1)
    Nm = freqs_mhz.shape[1]
    return {"centers": centres, "radius": np.full(Np, float(radius)),
            "omega": 2.0 * math.pi * freqs_mhz, "zeta": np.full((Np, Nm), zeta),
            "eta": np.full((Np, Nm), eta), "scale": np.full((Np, Nm), scale)}


def mode_shapes(wl, k, xyz):
    """U_{k,m}.n at the given bottom-face points, [Nm x n]: the radial profile
    s_{k,m} J0(j_{0,m} r / a_k) inside the disc of PMUT k and zero outside."""
    pm = wl["pmuts"]
    ctr = np.asarray(pm["centers"])[k]
    a = float(np.asarray(pm["radius"])[k])
    scale = np.asarray(pm["scale"])[k]
    Nm = scale.shape[0]
    r = np.hypot(xyz[:, 0] - ctr[0], xyz[:, 1] - ctr[1])
    zeros = _bessel_zeros(Nm)
    out = np.zeros((Nm, xyz.shape[0]))
    inside = r <= a
    for m in range(Nm):
        out[m, inside] = scale[m] * _j0(zeros[m] * r[inside] / a)
    return out


def shape_fn(wl):
    return lambda k, xyz: mode_shapes(wl, k, xyz)


# ---------------------------------------------------------------- configs

def config1():
    """Single cube [0,1 mm]^3, 4^3 hexes, N = 4; one disc (r = 0.433 mm) on the
    bottom face with 3 modes (1.0 / 2.1 / 3.4 MHz, 1 % damping); 3-cycle
    2 MHz burst; 8 seeded interior receivers; 200 steps at CFL 0.3."""
    rng = np.random.default_rng(SEED0 + 1)
    dom = brick([0, 0, 0], [1, 1, 1], [4, 4, 4], 4)
    pm = _pmut_block(np.array([[0.5, 0.5]]), 0.433, [[1.0, 2.1, 3.4]])
    return {"name": "cube-4x4x4-N4-1pmut", "domains": [dom], "cfl": 0.3, "alpha": 2.0,
            "pmuts": pm,
            "drive": {"amp": np.ones((1, 1)), "phase": np.zeros((1, 1)), "freq": np.array([2.0]),
                      "ncyc": 3.0, "envelope": 0},
            "receivers": _receivers_in(rng, dom, 8), "steps": 200}


def config2():
    """Primary 16x16x4 hexes N = 4 over [0,4]x[0,4]x[0,1] mm with a 4x4 PMUT
    array (pitch 1 mm, 8 modes each, frequencies U[1.5,3] MHz) on its bottom
    face; secondary 8x8x32 hexes N = 3 over [0,4]x[0,4]x[1,17] mm through a
    2:1 nested non-conforming interface; 2.5 MHz drive with phases
    U[0,2pi); 64 receivers in the secondary; 2000 steps."""
    rng = np.random.default_rng(SEED0 + 2)
    prim = brick([0, 0, 0], [4, 4, 1], [16, 16, 4], 4)
    sec = brick([0, 0, 1], [4, 4, 17], [8, 8, 32], 3)
    ctr = _grid_centres(4, 4, 1.0, 0.5)
    freqs = rng.uniform(1.5, 3.0, size=(16, 8))
    pm = _pmut_block(ctr, 0.433, freqs)
    phase = rng.uniform(0.0, 2 * math.pi, size=(1, 16))
    rec = _receivers_in(rng, sec, 64)
    return {"name": "two-domain-16x16x4N4+8x8x32N3-16pmut", "domains": [prim, sec], "cfl": 0.3,
            "alpha": 2.0, "pmuts": pm,
            "drive": {"amp": np.ones((1, 16)), "phase": phase, "freq": np.array([2.5]),
                      "ncyc": 3.0, "envelope": 0},
            "receivers": rec, "steps": 2000}


def config3(steps=5000):
    """Large array at one-GPU scale: 32x32 = 1024 discs at 1 mm pitch, 10 modes
    each (frequencies U[2.375,2.625] MHz), primary 128x128x8 hexes N = 4 over
    [0,32]^2 x [0,2] mm, secondary 96x96x96 hexes N = 3 over
    [0,32]^2 x [2,34] mm (4:3 non-nested interface); beam steered 20 degrees
    along x by linear phase delays; 64 receivers; 5000 steps."""
    rng = np.random.default_rng(SEED0 + 3)
    prim = brick([0, 0, 0], [32, 32, 2], [128, 128, 8], 4)
    sec = brick([0, 0, 2], [32, 32, 34], [96, 96, 96], 3)
    ctr = _grid_centres(32, 32, 1.0, 0.5)
    freqs = rng.uniform(2.375, 2.625, size=(1024, 10))
    pm = _pmut_block(ctr, 0.433, freqs)
    f = 2.5
    phase = (2 * math.pi * f * ctr[:, 0] * math.sin(math.radians(20.0)) / C_WATER).reshape(1, -1)
    rec = _receivers_in(rng, sec, 64)
    return {"name": "array-1024pmut-128x128x8N4+96^3N3", "domains": [prim, sec], "cfl": 0.3,
            "alpha": 2.0, "pmuts": pm,
            "drive": {"amp": np.ones((1, 1024)), "phase": phase, "freq": np.array([f]),
                      "ncyc": 3.0, "envelope": 0},
            "receivers": rec, "steps": steps}


def batch_geometry():
    """The cube of config 1 with a 4x4 PMUT array on its bottom face: one disc
    of radius 0.108 mm per boundary element face (pitch 0.25 mm), 3 modes each
    (1.0 / 2.1 / 3.4 MHz); 64 receivers."""
    rng = np.random.default_rng(SEED0 + 4)
    dom = brick([0, 0, 0], [1, 1, 1], [4, 4, 4], 4)
    ctr = _grid_centres(4, 4, 0.25, 0.125)
    pm = _pmut_block(ctr, 0.108, np.tile([1.0, 2.1, 3.4], (16, 1)))
    rec = _receivers_in(rng, dom, 64)
    return {"name": "cube-4x4x4-N4-4x4pmut", "domains": [dom], "cfl": 0.3, "alpha": 2.0,
            "pmuts": pm, "receivers": rec, "steps": 512, "ncyc": 3.0}


def scenario_params(rng, S, Np=16):
    """Drive parameters of S scenarios: per-PMUT phases U[0,2pi), one
    frequency U[1.5,3] MHz and one amplitude U[0.5,1] per scenario."""
    phase = rng.uniform(0.0, 2 * math.pi, size=(S, Np))
    freq = rng.uniform(1.5, 3.0, size=S)
    amp = rng.uniform(0.5, 1.0, size=S)
    return phase, freq, amp


def config4():
    """Batched: 64 excitation scenarios on the batch geometry, plus 16 uneven
    single-brick meshes from 8x8x4 to 24x24x8 hexes with orders cycling 3..6
    (one centred disc each, config-1 modes, 2 MHz drive), 512 steps each."""
    rng = np.random.default_rng(SEED0 + 4 + 1000)
    base = batch_geometry()
    S = 64
    phase, freq, amp = scenario_params(rng, S)
    base = dict(base)
    base["drive"] = {"amp": np.repeat(amp[:, None], 16, axis=1), "phase": phase, "freq": freq,
                     "ncyc": 3.0, "envelope": 0}
    meshes = []
    for j in range(16):
        nxy = 8 + int(round(16 * j / 15))
        nz = 4 + j % 5
        N = 3 + j % 4
        h = 0.25
        dom = brick([0, 0, 0], [nxy * h, nxy * h, nz * h], [nxy, nxy, nz], N)
        mrng = np.random.default_rng(SEED0 + 4 + 100 + j)
        pm = _pmut_block(np.array([[0.5 * nxy * h, 0.5 * nxy * h]]), 0.433, [[1.0, 2.1, 3.4]])
        meshes.append({"name": f"brick-{nxy}x{nxy}x{nz}-N{N}", "domains": [dom], "cfl": 0.3,
                       "alpha": 2.0, "pmuts": pm,
                       "drive": {"amp": np.ones((1, 1)), "phase": np.zeros((1, 1)),
                                 "freq": np.array([2.0]), "ncyc": 3.0, "envelope": 0},
                       "receivers": _receivers_in(mrng, dom, 64), "steps": 512})
    return {"name": "batched-64scen+16meshes", "scenarios": base, "meshes": meshes}


def config5(n_runs=4096, n_holdout=512):
    """Surrogate data set: n_runs scenarios of the batch geometry (drive
    parameters as in config 4), of which the last n_holdout are held out
    (half calibration, half test).  Surrogate inputs: 16 phases, frequency,
    amplitude (18 values); outputs 64 receivers x 512 samples."""
    rng = np.random.default_rng(SEED0 + 5)
    base = batch_geometry()
    phase, freq, amp = scenario_params(rng, n_runs)
    base = dict(base)
    base["drive"] = {"amp": np.repeat(amp[:, None], 16, axis=1), "phase": phase, "freq": freq,
                     "ncyc": 3.0, "envelope": 0}
    return {"name": "surrogate-4096runs", "scenarios": base, "n_holdout": n_holdout,
            "features": np.concatenate([phase, freq[:, None], amp[:, None]], axis=1)}


def small_two_domain(nested=True, steps=60):
    """Small two-domain case used by the parity tests: several tiles and a
    ragged tail on both sides of a nested 2:1 (or non-nested 4:3) interface."""
    rng = np.random.default_rng(SEED0 + 11 + (0 if nested else 1))
    if nested:
        prim = brick([0, 0, 0], [3, 2, 0.5], [12, 8, 2], 4)
        sec = brick([0, 0, 0.5], [3, 2, 2.5], [6, 4, 4], 3)
    else:
        prim = brick([0, 0, 0], [3, 2, 0.5], [12, 8, 2], 4)
        sec = brick([0, 0, 0.5], [3, 2, 2.5], [9, 6, 6], 3)
    ctr = _grid_centres(3, 2, 1.0, 0.5)
    freqs = rng.uniform(1.5, 3.0, size=(6, 4))
    pm = _pmut_block(ctr, 0.433, freqs)
    phase = rng.uniform(0.0, 2 * math.pi, size=(1, 6))
    rec = np.concatenate([_receivers_in(rng, sec, 12), _receivers_in(rng, prim, 4)])
    return {"name": "small-two-domain-" + ("nested" if nested else "4to3"), "domains": [prim, sec],
            "cfl": 0.3, "alpha": 2.0, "pmuts": pm,
            "drive": {"amp": np.ones((1, 6)), "phase": phase, "freq": np.array([2.5]),
                      "ncyc": 3.0, "envelope": 0},
            "receivers": rec, "steps": steps}


def mapped_cube(kind="conforming", N=4, ne=(4, 4, 4), steps=400, seed=0):
    """The config-1 cube (one disc of radius 0.433 mm at the centre of the
    bottom face) meshed by trilinear hexahedra: "conforming" puts element
    edges on the disc's circle, "warped" moves the vertices by a smooth
    seeded field, "jittered" adds a seeded jitter of the interior vertices
    to that; the boundary planes stay where they are."""
    wl = config1()
    dom = brick([0, 0, 0], [1, 1, 1], list(ne), N)
    if kind == "conforming":
        V = disc_conforming_vertices(dom, np.array([[0.5, 0.5]]), 0.433, 1.0)
    elif kind == "warped":
        V = warped_vertices(dom, amp=0.2, seed=seed)
    elif kind == "jittered":
        V = warped_vertices(dom, amp=0.2, jitter=0.25, seed=seed)
    else:
        raise ValueError(kind)
    dom["vertices"] = V
    return dict(wl, name=f"cube-{kind}-{ne[0]}x{ne[1]}x{ne[2]}N{N}-1pmut", domains=[dom], steps=steps)


def mapped_array(steps=1000):
    """The large array's PMUT brick on its own, meshed so that element edges
    follow every disc: 32x32 = 1024 discs (r = 0.433 mm) at 1 mm pitch,
    10 modes each, 128x128x8 trilinear hexahedra of order N = 4 over
    [0,32]^2 x [0,2] mm (8.68M unique DOFs); the beam steered 20 degrees
    along x; 64 receivers in the brick's upper half."""
    rng = np.random.default_rng(SEED0 + 6)
    dom = brick([0, 0, 0], [32, 32, 2], [128, 128, 8], 4)
    ctr = _grid_centres(32, 32, 1.0, 0.5)
    dom["vertices"] = disc_conforming_vertices(dom, ctr, 0.433, 1.0)
    freqs = rng.uniform(2.375, 2.625, size=(1024, 10))
    pm = _pmut_block(ctr, 0.433, freqs)
    f = 2.5
    phase = (2 * math.pi * f * ctr[:, 0] * math.sin(math.radians(20.0)) / C_WATER).reshape(1, -1)
    rec = np.column_stack([rng.uniform(1.0, 31.0, size=64), rng.uniform(1.0, 31.0, size=64),
                           rng.uniform(1.0, 1.95, size=64)])
    return {"name": "array-1024pmut-conforming-128x128x8N4", "domains": [dom], "cfl": 0.3,
            "alpha": 2.0, "pmuts": pm,
            "drive": {"amp": np.ones((1, 1024)), "phase": phase, "freq": np.array([f]),
                      "ncyc": 3.0, "envelope": 0},
            "receivers": rec, "steps": steps}


CONFIGS = {1: config1, 2: config2, 3: config3}


def unique_dofs(wl):
    n = 0
    for d in wl["domains"]:
        n += int(np.prod([d["N"] * e + 1 for e in d["ne"]]))
    return n


def element_local_dofs(wl):
    n = 0
    for d in wl["domains"]:
        n += int(np.prod(d["ne"])) * (d["N"] + 1) ** 3
    return n


def workload_key(wl):
    """SHA-256 over every input array of a single-mesh workload description
    (bricks, PMUT data, drive, receivers): stored results computed from a
    workload carry it, so a changed generator is noticed."""
    h = hashlib.sha256()
    h.update(json.dumps([{k: v for k, v in d.items() if k != "vertices"} for d in wl["domains"]],
                        sort_keys=True).encode())
    for d in wl["domains"]:
        if d.get("vertices") is not None:
            h.update(np.ascontiguousarray(d["vertices"], dtype=np.float64).tobytes())
    h.update(json.dumps([wl.get("cfl"), wl.get("alpha")]).encode())
    for k in ("centers", "radius", "omega", "zeta", "eta", "scale"):
        h.update(np.ascontiguousarray(wl["pmuts"][k], dtype=np.float64).tobytes())
    dr = wl["drive"]
    for k in ("amp", "phase", "freq"):
        h.update(np.ascontiguousarray(dr[k], dtype=np.float64).tobytes())
    h.update(json.dumps([dr["ncyc"], dr.get("envelope", 0)]).encode())
    h.update(np.ascontiguousarray(wl["receivers"], dtype=np.float64).tobytes())
    return h.hexdigest()
