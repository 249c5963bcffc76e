"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle on
the same seeded inputs.  Tolerances: relative L2 of all receiver traces
<= 1e-5 for the FP32 solver (increment-form state, FP64 ODE and traces) and
<= 1e-10 for the FP64 solver."""
import math
import sys

import numpy as np
import pytest

from oracle import ref
from paper_2603_06267_amd import solver, workloads as W

pytestmark = pytest.mark.gpu

TOL = {32: 1e-5, 64: 1e-10}


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def per_receiver_max(tg, to, floor=0.01):
    """Largest relative L2 over receivers, each receiver's error measured
    against max(its own trace norm, floor x the loudest receiver's norm)."""
    tg = np.asarray(tg).reshape(-1, tg.shape[-1])
    to = np.asarray(to).reshape(-1, to.shape[-1])
    nr = np.linalg.norm(to, axis=1)
    return float((np.linalg.norm(tg - to, axis=1) / np.maximum(nr, floor * nr.max())).max())


def check_traces(tg, to, precision, label):
    """Global and receiver-by-receiver relative L2 within the tolerance."""
    err = rel_l2(tg, to)
    pr = per_receiver_max(tg, to)
    _say(f"  {label}: rel L2 {err:.3e}, per receiver max {pr:.3e}")
    assert err <= TOL[precision]
    assert pr <= TOL[precision]
    return err


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_pair(wl, precision, steps=None, scen=0):
    steps = steps or wl["steps"]
    sf = W.shape_fn(wl)
    o = ref.from_workload(wl, scenario=scen, shape_fn=sf)
    to = o.step(steps)
    g = solver.from_workload(wl, precision=precision, n_steps=steps, scenarios=[scen], shape_fn=sf)
    g.step(steps)
    tg = g.read_traces()[0]
    assert not g.nonfinite()
    return tg, to, g, o


@pytest.mark.parametrize("precision", [32, 64])
def test_config1_cube_single_pmut(precision):
    _say(f"config1 precision={precision}")
    wl = W.config1()
    tg, to, g, o = run_pair(wl, precision)
    assert abs(g.dt - o.dt) < 1e-15 * o.dt
    assert np.abs(to).max() > 0
    check_traces(tg, to, precision, "config1")
    # modal state agrees as well
    q, qd, qdd = g.read_modal()
    st = o.get_state()
    assert rel_l2(q, st["q"]) <= 10 * TOL[precision]


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("nested", [True, False])
def test_small_two_domain(precision, nested):
    """Several tiles in x and y with ragged tails, both interface kinds
    (nested 2:1 and non-nested 4:3), receivers in both bricks."""
    _say(f"small two-domain nested={nested} precision={precision}")
    wl = W.small_two_domain(nested, steps=400)
    tg, to, g, o = run_pair(wl, precision)
    check_traces(tg, to, precision, "small two-domain")


@pytest.mark.parametrize("precision", [32, 64])
def test_config2_two_domain_array(precision):
    _say(f"config2 precision={precision} (2000 steps)")
    wl = W.config2()
    tg, to, g, o = run_pair(wl, precision)
    check_traces(tg, to, precision, "config2")


@pytest.mark.parametrize("precision", [32, 64])
def test_absorbing_faces_cube(precision):
    """First-order absorbing condition on every face of the config-1 cube
    but the PMUT face, 400 steps (the wave has crossed the cube twice):
    traces against the oracle; it cannot be switched on after bind."""
    wl = W.config1()
    wl = dict(wl, domains=[dict(wl["domains"][0], absorbing=0b101111)], steps=400)
    _say(f"absorbing cube precision={precision}")
    tg, to, g, o = run_pair(wl, precision)
    check_traces(tg, to, precision, "absorbing cube")
    with pytest.raises(Exception):
        g.set_absorbing(0, 1)


@pytest.mark.parametrize("precision", [32, 64])
def test_absorbing_faces_two_domain(precision):
    """Absorbing side walls on both bricks and an absorbing top on the
    secondary, non-nested 4:3 interface, 400 steps, against the oracle."""
    wl = W.small_two_domain(False, steps=400)
    prim, sec = wl["domains"]
    wl = dict(wl, domains=[dict(prim, absorbing=0b001111), dict(sec, absorbing=0b101111)])
    tg, to, g, o = run_pair(wl, precision)
    check_traces(tg, to, precision, f"absorbing two-domain precision={precision}")


def test_graph_replay_equals_direct_launches():
    wl = W.small_two_domain(True, steps=150)
    sf = W.shape_fn(wl)
    out = []
    for graph in (0, 1):
        g = solver.from_workload(wl, precision=32, shape_fn=sf, bind=False)
        g.set_option(1, graph)
        g.set_option(4, 37)  # odd chunk length: replays cross step parity
        g.bind()
        g.step(150)
        out.append(g.read_traces())
    assert np.array_equal(out[0], out[1])


@pytest.mark.parametrize("rows,zchunk", [(1, 0), (2, 5), (4, 3), (1, 11)])
def test_tilings_agree(rows, zchunk):
    """Every tile shape gives the same arithmetic per node (bitwise).  With
    3- and 5-plane z chunks an interface element layer spans two chunks, so
    the face kernel writes that brick's interface traces, which the
    17-plane reference's stiffness launches write themselves: both paths
    agree bitwise."""
    wl = W.small_two_domain(False, steps=80)
    sf = W.shape_fn(wl)
    ref_tr = None
    for r, z in ((1, 17), (rows, zchunk)):
        g = solver.from_workload(wl, precision=32, shape_fn=sf, bind=False)
        g.set_option(2, r)
        g.set_option(3, z)
        g.bind()
        g.step(80)
        tr = g.read_traces()
        if ref_tr is None:
            ref_tr = tr
        else:
            assert np.array_equal(tr, ref_tr)


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("depth,rows,zchunk", [(3, 2, 0), (4, 2, 5), (3, 1, 11), (4, 1, 0)])
def test_prefetch_distances_agree(precision, depth, rows, zchunk):
    """Prefetching 3 or 4 planes ahead changes only when loads are issued:
    state and traces are bitwise those of the 2-plane default, with z chunks
    shorter than, and not a multiple of, the unrolled loop."""
    wl = W.small_two_domain(False, steps=90)
    sf = W.shape_fn(wl)
    out = []
    for d in (2, depth):
        g = solver.from_workload(wl, precision=precision, shape_fn=sf, bind=False)
        g.set_option(2, rows)
        g.set_option(3, zchunk)
        g.set_option(12, d)
        g.bind()
        g.step(90)
        out.append((g.read_traces(), *g.get_state(0)))
        g.close()
    for a, b in zip(out[0], out[1]):
        assert np.array_equal(a, b)


def test_scenarios_batch_equals_single():
    """S scenarios in one launch == S separate single-scenario solvers."""
    wl = W.config4()["scenarios"]
    wl = dict(wl, steps=120)
    sf = W.shape_fn(wl)
    sc = [0, 5, 17]
    gb = solver.from_workload(wl, precision=32, scenarios=sc, shape_fn=sf)
    gb.step(120)
    tb = gb.read_traces()
    for i, s in enumerate(sc):
        g1 = solver.from_workload(wl, precision=32, scenarios=[s], shape_fn=sf)
        g1.step(120)
        assert np.array_equal(g1.read_traces()[0], tb[i])
    o = ref.from_workload(wl, scenario=17, shape_fn=sf)
    assert rel_l2(tb[2], o.step(120)) <= 1e-5


@pytest.mark.parametrize("precision", [32, 64])
def test_checkpoint_resume(precision):
    wl = W.small_two_domain(True, steps=200)
    sf = W.shape_fn(wl)
    g = solver.from_workload(wl, precision=precision, shape_fn=sf)
    g.step(200)
    full = g.read_traces()
    h = solver.from_workload(wl, precision=precision, shape_fn=sf)
    h.step(90)
    p, pp = h.get_state(0)
    q, qd, qdd = h.read_modal(0)
    k = solver.from_workload(wl, precision=precision, shape_fn=sf)
    k.set_state(0, p, pp, q, qd, qdd, nstep=90)
    k.step(110)
    tail = k.read_traces()[:, :, 90:]
    if precision == 64:
        assert np.array_equal(tail, full[:, :, 90:])
    else:
        # the increment is re-derived from p and p_prev in FP64 on the host
        assert rel_l2(tail, full[:, :, 90:]) < 1e-6


@pytest.mark.parametrize("precision", [32, 64])
def test_standing_wave(precision):
    """Rigid cube, separable discrete eigenvector as initial state:
    p^n = v cos(n theta) (closed form of the discrete scheme)."""
    from tests._indep import sem_1d
    N, ne, c = 4, 3, 1.5
    dom = W.brick([0, 0, 0], [1, 1, 1], [ne, ne, ne], N, c=c)
    g = solver.Solver([dom], precision=precision, trace_capacity=400)
    g.set_receivers([[0.3, 0.6, 0.2]])
    g.bind()
    K, M = sem_1d(N, ne, 1.0 / ne)
    Mi = 1 / np.sqrt(M)
    lam, V = np.linalg.eigh(Mi[:, None] * K * Mi[None, :])
    v1, v2 = Mi * V[:, 1], Mi * V[:, 2]
    v = np.kron(v1, np.kron(v2, v1))
    lam3 = c * c * (2 * lam[1] + lam[2])
    theta = math.acos(1 - 0.5 * g.dt ** 2 * lam3)
    g.set_state(0, v, v * math.cos(theta))
    g.step(400)
    p, _ = g.get_state(0)
    err = np.abs(p - v * math.cos(400 * theta)).max() / np.abs(v).max()
    assert err < (2e-5 if precision == 32 else 1e-11)


def _smooth_field(xyz, seed):
    rng = np.random.default_rng(seed)
    f = np.zeros(len(xyz))
    for _ in range(4):
        k = rng.uniform(0.5, 2.5, size=3)
        ph = rng.uniform(0, 2 * np.pi, size=3)
        f += np.prod(np.cos(k * xyz + ph), axis=1) * rng.uniform(0.5, 1.0)
    return f


@pytest.mark.parametrize("precision", [32, 64])
def test_config3_full_size_one_step(precision):
    """Full-size config 3 (32.8M nodes, 1024 PMUTs, 4:3 interface) in the
    launch configuration the benchmark times (automatic tile rows and z
    chunks, hipGraph replay): one step from a smooth state with non-zero
    modal accelerations, against the oracle's explicit update
    p^{n+1} = 2 p^n - p^{n-1} + dt^2 M^{-1} (f(qdd^n) - K p^n) at every node,
    relative to the largest change of p over the step."""
    _say(f"config3 one step precision={precision}")
    wl = W.config3(steps=4)
    sf = W.shape_fn(wl)
    g = solver.from_workload(wl, precision=precision, n_steps=4, shape_fn=sf)
    xyz = g.node_coords()
    p = _smooth_field(xyz, 1)
    pp = p - 0.05 * _smooth_field(xyz, 2)
    rng = np.random.default_rng(3)
    nm = g.Np * g.Nm
    qdd = rng.standard_normal(nm)
    g.set_state(0, p, pp, np.zeros(nm), np.zeros(nm), qdd, nstep=0)
    g.step(1)
    pn, _ = g.get_state(0)
    del xyz
    o = ref.from_workload(wl, shape_fn=sf)
    Kp = o.apply_K(p)
    M = o.mass()
    f = np.zeros(o.n)
    kappa = wl["domains"][0]["rho"] * wl["domains"][0]["c"] ** 2
    for k in range(o.Np):
        for m in range(o.Nm):
            nd, val = o.coupling(k, m)
            f[nd] += -kappa * qdd[k * o.Nm + m] * val
    expect = 2 * p - pp + o.dt ** 2 * (f - Kp) / M
    d = pn - expect
    scale = np.abs(expect - p).max()
    err = np.abs(d).max() / scale
    _say(f"  max |diff| / max |p^(n+1) - p^n| = {err:.3e}")
    assert err < (1e-5 if precision == 32 else 1e-10)


@pytest.mark.parametrize("case", ["cube", "nested", "4to3"])
def test_two_step_pass_matches_single_steps(case):
    """Fusing the volume update of two steps (the coupled planes completed
    after the coupling of the first) gives the single-step traces, and both
    match the oracle; odd step counts end with a single step."""
    _say(f"two-step pass: {case}")
    if case == "cube":
        wl, steps = W.config1(), 121
    else:
        wl, steps = W.small_two_domain(case == "nested", steps=121), 121
    sf = W.shape_fn(wl)
    out = {}
    # (primary, secondary) steps per pass: both single, both two-step, and
    # two-step passes for the secondary only
    modes = [(1, 1), (2, 2)] + ([(1, 2)] if case != "cube" else [])
    for tb in modes:
        for graph in (0, 1):
            g = solver.from_workload(wl, precision=32, n_steps=steps, shape_fn=sf, bind=False)
            g.set_option(9, tb[0])
            g.set_option(11, tb[1])
            g.set_option(1, graph)
            g.set_option(4, 37)
            g.bind()
            g.step(steps)
            assert not g.nonfinite()
            out[(tb, graph)] = g.read_traces()
    ref_tr = out[((1, 1), 0)]
    for k, tr in out.items():
        d = rel_l2(tr, ref_tr)
        _say(f"  steps per pass={k[0]} graph={k[1]}: rel diff to single steps {d:.2e}")
        assert d < 1e-6
    o = ref.from_workload(wl, shape_fn=sf)
    err = rel_l2(out[((2, 2), 1)][0], o.step(steps))
    _say(f"  two-step vs oracle rel L2 {err:.2e}")
    assert err <= TOL[32]


def test_two_step_checkpoint_resume():
    wl = W.small_two_domain(False, steps=100)
    sf = W.shape_fn(wl)
    g = solver.from_workload(wl, precision=32, shape_fn=sf, bind=False)
    g.set_option(9, 2)
    g.bind()
    g.step(100)
    full = g.read_traces()
    h = solver.from_workload(wl, precision=32, shape_fn=sf, bind=False)
    h.set_option(9, 2)
    h.bind()
    h.step(44)
    p, pp = h.get_state(0)
    q, qd, qdd = h.read_modal(0)
    k = solver.from_workload(wl, precision=32, shape_fn=sf, bind=False)
    k.set_option(9, 2)
    k.bind()
    k.set_state(0, p, pp, q, qd, qdd, nstep=44)
    k.step(56)
    assert rel_l2(k.read_traces()[:, :, 44:], full[:, :, 44:]) < 1e-6


@pytest.mark.parametrize("precision", [32])
def test_config3_two_step_pass_full_size(precision):
    """Full-size config 3: four steps as two two-step passes against four
    single steps from the same smooth state (every node)."""
    _say("config3 two-step pass, 4 steps")
    wl = W.config3(steps=6)
    sf = W.shape_fn(wl)
    res = []
    for tb in (1, 2):
        g = solver.from_workload(wl, precision=32, n_steps=6, shape_fn=sf, bind=False)
        g.set_option(9, tb)
        g.bind()
        xyz = g.node_coords()
        p = _smooth_field(xyz, 1)
        pp = p - 0.05 * _smooth_field(xyz, 2)
        del xyz
        rng = np.random.default_rng(3)
        nm = g.Np * g.Nm
        g.set_state(0, p, pp, np.zeros(nm), np.zeros(nm), rng.standard_normal(nm), nstep=0)
        g.step(4)
        pn, _ = g.get_state(0)
        res.append(pn)
        del g
    d = np.abs(res[1] - res[0]).max() / np.abs(res[0]).max()
    _say(f"  max |two-step - single| / max |p| = {d:.2e}")
    assert d < 1e-5


@pytest.mark.parametrize("mode", [1, 2, 3])
@pytest.mark.parametrize("graph", [0, 1])
def test_overlapped_face_work_equals_sequential(graph, mode):
    """Running the PMUT face work (mode 1), or the primary's whole chain of
    stiffness and face work (mode 2), on a side stream alongside the
    secondary's stiffness launch, or the face kernel alongside the interface
    kernels (mode 3, the face kernel reading the step counter's copy), gives
    bitwise the traces and modal state of running every kernel in
    sequence."""
    wl = W.small_two_domain(False, steps=90)
    sf = W.shape_fn(wl)
    res = []
    for ov in (0, mode):
        g = solver.from_workload(wl, precision=32, shape_fn=sf, bind=False)
        g.set_option(10, ov)
        g.set_option(1, graph)
        g.bind()
        g.step(90)
        res.append((g.read_traces(), g.read_modal(0)[2]))
    assert np.array_equal(res[0][0], res[1][0])
    assert np.array_equal(res[0][1], res[1][1])


def _pml_cube():
    wl = W.config1()
    dom = dict(wl["domains"][0], absorbing=0b111110, pml={"ell": [0.25, 0.25, 0.25, 0.25, 0.0, 0.25], "R": 1e-4})
    return dict(wl, domains=[dom], steps=400)


def _pml_two_domain():
    wl = W.small_two_domain(False, steps=400)
    prim, sec = wl["domains"]
    hp = (prim["x1"][0] - prim["x0"][0]) / prim["ne"][0]
    hs = (sec["x1"][0] - sec["x0"][0]) / sec["ne"][0]
    prim = dict(prim, absorbing=0b001111, pml={"ell": [hp, hp, hp, hp, 0.0, 0.0], "R": 1e-4})
    sec = dict(sec, absorbing=0b101111, pml={"ell": [hs, hs, hs, hs, 0.0, hs], "R": 1e-4})
    return dict(wl, domains=[prim, sec])


@pytest.mark.parametrize("precision", [32, 64])
@pytest.mark.parametrize("case", ["cube", "two-domain"])
def test_perfectly_matched_layer(precision, case):
    """Perfectly matched layers (Sec. 2, eq. full_problem) in front of
    absorbing faces: the config-1 cube with a one-element layer on every face
    but the PMUT face, and the 4:3 two-domain case with layers on the side
    walls of both bricks and the secondary's top; 400 steps, traces against
    the oracle."""
    wl = _pml_cube() if case == "cube" else _pml_two_domain()
    _say(f"matched layer {case} precision={precision}")
    tg, to, g, o = run_pair(wl, precision)
    check_traces(tg, to, precision, f"matched layer {case} precision={precision}")
    # the layer changes the result: without it (absorbing faces only) the
    # traces differ
    plain = dict(wl, domains=[{k: v for k, v in d.items() if k != "pml"} for d in wl["domains"]])
    o2 = ref.from_workload(plain, shape_fn=W.shape_fn(plain))
    assert rel_l2(o2.step(wl["steps"]), to) > 1e-3
