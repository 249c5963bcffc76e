"""GPU parity of the LDS-resident path (PMDG_OPT_RESIDENT: small single-brick
FP32 solvers run whole steps, Sec. 3.1 Algorithm 1 in its synchronised
reading, inside one launch with the pressure in LDS) against the FP64 oracle
and against the tiled path on the same seeded inputs.

- config 1 (the cube with one PMUT, 4,913 nodes): traces and modal state,
  FP32 <= 1e-5 relative L2 against the oracle, every receiver;
- the batch cube (4x4 PMUTs) with 64 drive scenarios, one workgroup each:
  every scenario against the tiled path, scenario 0 against the oracle's
  stored traces;
- the TX -> RX switch inside a run;
- a run longer than one launch (2,500 steps), and a run that switches
  between the two paths through get_state / set_state.
"""
import os
import sys

import numpy as np
import pytest

from oracle import ref
from paper_2603_06267_amd import _lib, solver, workloads as W

pytestmark = pytest.mark.gpu


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


def _run(wl, steps, resident, scenarios=None, chunks=None):
    g = solver.from_workload(wl, precision=32, n_steps=steps, scenarios=scenarios, shape_fn=W.shape_fn(wl),
                             bind=False)
    g.set_option(_lib.OPT_RESIDENT, resident)
    g.bind()
    assert g.resident() == bool(resident)
    for n in (chunks or [steps]):
        g.step(n)
    assert not g.nonfinite()
    return g


def test_config1_against_oracle_and_tiled_path():
    wl = W.config1()
    steps = 400
    _say("resident config1")
    o = ref.from_workload(wl, shape_fn=W.shape_fn(wl))
    to = o.step(steps)
    g = _run(wl, steps, 1)
    t = _run(wl, steps, 0)
    tg, tt = g.read_traces()[0], t.read_traces()[0]
    err, pr = rel_l2(tg, to), per_receiver_max(tg, to)
    _say(f"  vs oracle: rel L2 {err:.3e}, per receiver {pr:.3e}; vs tiled {rel_l2(tg, tt):.3e}")
    assert err <= 1e-5 and pr <= 1e-5
    assert rel_l2(tg, tt) <= 1e-6
    q, qd, _ = g.read_modal()
    assert rel_l2(q, o.get_state()["q"]) <= 1e-4
    p, pp = g.get_state(0)
    p2, pp2 = t.get_state(0)
    assert rel_l2(p, p2) <= 1e-6 and rel_l2(pp, pp2) <= 1e-6


def test_batch_cube_64_scenarios():
    c4 = W.config4()
    wl = c4["scenarios"]
    steps = 512
    _say("resident batch cube, 64 scenarios")
    g = _run(wl, steps, 1)
    t = _run(wl, steps, 0)
    tg, tt = g.read_traces(), t.read_traces()
    assert tg.shape[0] == 64
    worst = max(rel_l2(tg[s], tt[s]) for s in range(64))
    _say(f"  worst scenario vs tiled: {worst:.3e}")
    assert worst <= 1e-6
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "config4base_traces.npz")
    if os.path.exists(path):
        z = np.load(path)
        base = dict(wl, steps=int(z["steps"]))
        if str(z["key"]) == W.workload_key(base):
            n = min(steps, int(z["steps"]))
            assert rel_l2(tg[0][:, :n], z["traces"][:, :n]) <= 1e-5
            assert per_receiver_max(tg[0][:, :n], z["traces"][:, :n]) <= 1e-5


def test_rx_switch_inside_run():
    wl = W.config1()
    steps = 300
    o0 = ref.from_workload(wl, shape_fn=W.shape_fn(wl))
    t_sw = 120 * o0.dt
    wl_rx = dict(wl, rx={"t_switch": t_sw, "cap": 0.2})
    o = ref.from_workload(wl_rx, shape_fn=W.shape_fn(wl_rx))
    to = o.step(steps)
    g = _run(wl_rx, steps, 1)
    tg = g.read_traces()[0]
    assert rel_l2(tg, to) <= 1e-5 and per_receiver_max(tg, to) <= 1e-5


def test_long_run_and_path_switch():
    wl = W.config1()
    # longer than one launch of 2,048 steps, in uneven calls
    g = _run(wl, 2500, 1, chunks=[1, 2047, 452])
    t = _run(wl, 2500, 0)
    assert rel_l2(g.read_traces()[0], t.read_traces()[0]) <= 2e-6
    # resident steps, then the tiled path from the same state
    a = _run(wl, 300, 1, chunks=[150])
    a.set_option(_lib.OPT_RESIDENT, 0)
    assert not a.resident()
    a.step(150)
    b = _run(wl, 300, 0)
    assert rel_l2(a.read_traces()[0], b.read_traces()[0]) <= 1e-6
    pa, _ = a.get_state(0)
    pb, _ = b.get_state(0)
    assert rel_l2(pa, pb) <= 1e-6


@pytest.mark.parametrize("receivers", [0, 1])
def test_without_pmuts(receivers):
    """A brick without PMUTs (no PMUT tables at all), with and without a
    receiver: the resident path from a smooth state against the tiled path."""
    dom = W.brick([0, 0, 0], [1, 1, 1], [3, 3, 3], 4)
    out = []
    for mode in (1, 0):
        g = solver.Solver([dom], precision=32, trace_capacity=200)
        if receivers:
            g.set_receivers([[0.3, 0.6, 0.2]])
        g.set_option(_lib.OPT_RESIDENT, mode)
        g.bind()
        assert g.resident() == bool(mode)
        x = g.node_coords()
        p = np.cos(np.pi * x[:, 0]) * np.cos(2 * np.pi * x[:, 2])
        g.set_state(0, p, 0.999 * p)
        g.step(150)
        out.append((g.get_state(0)[0], g.read_traces() if receivers else None))
    assert rel_l2(out[0][0], out[1][0]) <= 1e-6
    if receivers:
        assert rel_l2(out[0][1], out[1][1]) <= 1e-6
