"""GPU parity of the trilinear-hexahedron path (pmdg_set_vertices: Sec. 3,
elements as trilinear images of the reference cube, the stiffness with its
metric terms computed per element from the corners) against the FP64 CPU
oracle on the same seeded inputs, through the C ABI.

- The config-1 cube with its disc (one PMUT, three modes) meshed so that
  element edges follow the disc, smoothly warped, and warped with jittered
  interior vertices: 400 steps, FP32 <= 1e-5 and FP64 <= 1e-10 relative L2,
  every receiver and all together; modal state too.
- Orders 1 to 8 on a jittered mesh: one step from a seeded smooth state,
  every node against the oracle's step.
- Two scenarios with different drives in one solver.
- A brick given as its vertices runs the element path and agrees with the
  brick path; graph replay equals direct launches bitwise.
"""
import sys

import numpy as np
import pytest

from oracle import ref
from paper_2603_06267_amd import solver, workloads as W

pytestmark = pytest.mark.gpu

TOL = {32: 1e-5, 64: 1e-10}


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def per_receiver_max(tg, to, floor=0.01):
    tg = np.asarray(tg).reshape(-1, tg.shape[-1])
    to = np.asarray(to).reshape(-1, to.shape[-1])
    nr = np.linalg.norm(to, axis=1)
    return float((np.linalg.norm(tg - to, axis=1) / np.maximum(nr, floor * nr.max())).max())


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("kind", ["conforming", "warped", "jittered"])
def test_mapped_cube_traces(kind, precision):
    wl = W.mapped_cube(kind, steps=400)
    _say(f"mapped cube {kind} precision={precision}")
    sf = W.shape_fn(wl)
    o = ref.from_workload(wl, shape_fn=sf)
    to = o.step(400)
    g = solver.from_workload(wl, precision=precision, n_steps=400, shape_fn=sf)
    assert abs(g.dt - o.dt) <= 1e-14 * o.dt
    g.step(400)
    tg = g.read_traces()[0]
    assert not g.nonfinite()
    err, pr = rel_l2(tg, to), per_receiver_max(tg, to)
    _say(f"  rel L2 {err:.3e}, per receiver max {pr:.3e}")
    assert np.abs(to).max() > 0
    assert err <= TOL[precision] and pr <= TOL[precision]
    q, _, _ = g.read_modal()
    assert rel_l2(q, o.get_state()["q"]) <= 10 * TOL[precision]
    # node coordinates follow the vertices
    assert np.abs(g.node_coords() - o.coords()).max() < 1e-12


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 6, 7, 8])
def test_one_step_every_node(N, precision):
    """One step from a smooth seeded state with non-zero modal
    accelerations, against the oracle's explicit update
    p^{n+1} = 2 p^n - p^{n-1} + dt^2 M^{-1} (f(qdd^n) - K p^n) at every node
    (its K, M and face coupling on the same trilinear mesh), relative to the
    largest change of p over the step."""
    dom = W.brick([0, 0, 0], [1.0, 1.0, 0.6], [3, 3, 2], N)
    dom["vertices"] = W.warped_vertices(dom, amp=0.2, jitter=0.25, seed=N)
    rec = np.random.default_rng(40 + N).uniform(0.05, 0.55, size=(6, 3))
    wl = dict(W.config1(), domains=[dom], steps=4, receivers=rec)
    _say(f"one step N={N} precision={precision}")
    sf = W.shape_fn(wl)
    g = solver.from_workload(wl, precision=precision, n_steps=4, shape_fn=sf)
    o = ref.from_workload(wl, shape_fn=sf)
    x = o.coords()
    p = np.sin(2.1 * x[:, 0] + 0.3) * np.cos(1.7 * x[:, 1]) * np.cos(2.9 * x[:, 2] - 0.2)
    pp = p - 0.05 * np.cos(1.3 * x[:, 0] - 0.4 * x[:, 1] + 2.2 * x[:, 2])
    nm = g.Np * g.Nm
    qdd = np.random.default_rng(N).standard_normal(nm)
    g.set_state(0, p, pp, np.zeros(nm), np.zeros(nm), qdd, nstep=0)
    g.step(1)
    pn, _ = g.get_state(0)
    f = np.zeros(o.n)
    kappa = dom["rho"] * dom["c"] ** 2
    for k in range(o.Np):
        for m in range(o.Nm):
            nd, val = o.coupling(k, m)
            f[nd] += -kappa * qdd[k * o.Nm + m] * val
    assert np.abs(f).max() > 0
    expect = 2 * p - pp + o.dt ** 2 * (f - o.apply_K(p)) / o.mass()
    err = np.abs(pn - expect).max() / np.abs(expect - p).max()
    _say(f"  max |diff| / max |step change| = {err:.3e}")
    assert err <= (1e-5 if precision == 32 else 1e-10)


def test_two_scenarios():
    wl = W.mapped_cube("jittered", steps=300)
    wl = dict(wl, drive=dict(wl["drive"], amp=np.array([[1.0], [0.5]]), phase=np.array([[0.0], [1.0]]),
                             freq=np.array([2.0, 2.6])))
    sf = W.shape_fn(wl)
    g = solver.from_workload(wl, precision=32, n_steps=300, shape_fn=sf)
    g.step(300)
    tg = g.read_traces()
    for sc in (0, 1):
        to = ref.from_workload(wl, scenario=sc, shape_fn=sf).step(300)
        assert rel_l2(tg[sc], to) <= TOL[32]
        assert per_receiver_max(tg[sc], to) <= TOL[32]


def test_brick_as_vertices_and_graph_replay():
    wl = W.config1()
    wl = dict(wl, steps=300)
    wv = dict(wl, domains=[dict(wl["domains"][0], vertices=W.brick_vertices(wl["domains"][0]))])
    sf = W.shape_fn(wl)
    a = solver.from_workload(wl, precision=32, shape_fn=sf)
    a.step(300)
    out = []
    for graph in (0, 1):
        g = solver.from_workload(wv, precision=32, shape_fn=sf, bind=False)
        g.set_option(1, graph)
        g.set_option(4, 37)
        g.bind()
        g.step(300)
        out.append(g.read_traces())
    assert np.array_equal(out[0], out[1])
    assert rel_l2(out[1], a.read_traces()) <= 2e-6


@pytest.mark.parametrize("precision", [32, 64])
def test_mapped_array_traces(precision):
    """The large array's PMUT brick meshed by trilinear hexahedra whose edges
    follow every disc (8.68M DOFs, 1024 PMUTs), 1,000 steps with graph
    replay as the benchmark runs it, against the oracle's stored traces
    (tests/golden/make_traces.py --config mapped)."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "configmapped_traces.npz")
    if not os.path.exists(path):
        pytest.skip("oracle traces of the trilinear PMUT brick not generated")
    z = np.load(path)
    wl = W.mapped_array(steps=int(z["steps"]))
    assert str(z["key"]) == W.workload_key(wl), "stored traces belong to another workload"
    _say(f"mapped array precision={precision}")
    g = solver.from_workload(wl, precision=precision, shape_fn=W.shape_fn(wl))
    assert abs(g.dt - float(z["dt"])) <= 1e-14 * g.dt
    g.step(wl["steps"])
    tg = g.read_traces()[0]
    to = z["traces"]
    err, pr = rel_l2(tg, to), per_receiver_max(tg, to)
    _say(f"  rel L2 {err:.3e}, per receiver max {pr:.3e}")
    assert err <= TOL[precision] and pr <= TOL[precision]
    g.close()
