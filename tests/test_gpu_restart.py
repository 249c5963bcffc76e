"""pmdg_restart on the GPU: a bound solver sent back to step 0 and given a
new drive steps exactly as a solver built afresh with that drive (bitwise:
same kernels, same tables, state zeroed), on the LDS-resident path, the
tiled path with graph replay, two bricks with an interface, matched layers
and trilinear hexahedra."""
import sys

import numpy as np
import pytest

from paper_2603_06267_amd import _lib, solver, workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _drive(wl, seed):
    """Another drive of the same shape as wl's: phases, frequencies and
    amplitudes redrawn."""
    dr = wl["drive"]
    S, Np = np.asarray(dr["amp"]).shape
    rng = np.random.default_rng(seed)
    return dict(dr, amp=rng.uniform(0.5, 1.0, (S, Np)), phase=rng.uniform(0, 2 * np.pi, (S, Np)),
                freq=rng.uniform(1.5, 3.0, S))


def _build(wl, steps, resident):
    g = solver.from_workload(wl, precision=32, n_steps=steps, shape_fn=W.shape_fn(wl), bind=False)
    g.set_option(_lib.OPT_RESIDENT, resident)
    g.bind()
    return g


def _set_drive(g, dr):
    g.set_drive(np.asarray(dr["amp"]), np.asarray(dr["phase"]), np.asarray(dr["freq"]).reshape(-1), dr["ncyc"],
                dr.get("envelope", 0))


@pytest.mark.parametrize("resident", [1, 0])
def test_restart_with_new_drive_equals_fresh_solver(resident):
    """Eight batch-cube scenarios: run 150 steps of one drive, restart, set a
    second drive and run 120 steps; the traces equal those of a solver built
    with the second drive (and twice over, so a second restart is as good
    as the first)."""
    _say(f"restart resident={resident}")
    base = W.config4()["scenarios"]
    dr0 = {k: (v[:8] if hasattr(v, "__len__") and not isinstance(v, float) else v) for k, v in base["drive"].items()}
    wl = dict(base, drive=dr0)
    g = _build(wl, 200, resident)
    assert g.resident() == bool(resident)
    g.step(150)
    first = g.read_traces()
    for seed in (11, 12):
        dr = _drive(wl, seed)
        g.restart()
        assert g.steps_done() == 0
        _set_drive(g, dr)
        g.step(120)
        tr = g.read_traces()
        assert tr.shape == (8, first.shape[1], 120)
        f = _build(dict(wl, drive=dr), 200, resident)
        f.step(120)
        np.testing.assert_array_equal(tr, f.read_traces())
        assert not g.nonfinite()
        f.close()
    g.close()


def _pml_cube():
    wl = W.config1()
    dom = dict(wl["domains"][0], absorbing=0b111110, pml={"ell": [0.25, 0.25, 0.25, 0.25, 0.0, 0.25], "R": 1e-4})
    return dict(wl, domains=[dom], steps=300)


@pytest.mark.parametrize("case", ["two-domain", "pml", "mapped"])
@pytest.mark.parametrize("precision", [32, 64])
def test_restart_repeats_the_run(case, precision):
    """Same drive after a restart: the second run repeats the first bit for
    bit, so nothing of the first run (pressure levels, increments, layer
    fields, element residuals, modal states, interface traces) survives the
    restart."""
    _say(f"restart repeat case={case} precision={precision}")
    if case == "two-domain":
        wl = W.small_two_domain(False, steps=300)
    elif case == "pml":
        wl = _pml_cube()
    else:
        wl = W.mapped_cube("warped", steps=300)
    g = solver.from_workload(wl, precision=precision, n_steps=300, shape_fn=W.shape_fn(wl))
    g.step(200)
    a = g.read_traces()
    g.step(0)  # no steps: nothing changes
    assert g.steps_done() == 200
    np.testing.assert_array_equal(g.read_traces(), a)
    g.step(50)
    g.restart()
    g.step(200)
    b = g.read_traces()
    assert np.isfinite(a).all() and np.abs(a).max() > 0
    np.testing.assert_array_equal(a, b)
    g.close()


def test_surrogate_solve_reuses_restarted_solvers():
    """The surrogate's fallback solve keeps one bound solver per scenario-slot
    count and restarts it for each call: 60 rows, then 37 rows on the same
    64-slot solver, 100 rows on a 128-slot one, then 60 rows again, each
    equal bit for bit to a solver built for exactly those rows."""
    import torch
    from paper_2603_06267_amd import surrogate as SG
    _say("surrogate solve with cached solvers")
    SG.clear_solver_cache()
    rng = np.random.default_rng(5)
    F = np.concatenate([rng.uniform(0, 2 * np.pi, (100, 16)), rng.uniform(1.5, 3, (100, 1)),
                        rng.uniform(0.5, 1, (100, 1))], 1)
    base = W.batch_geometry()
    for rows in (F[:60], F[:37], F[:100], F[:60]):
        got = SG.solve(rows, steps=128).cpu().numpy()
        f = solver.from_workload(dict(base, drive=SG.drive_from_features(rows)), precision=32, n_steps=128,
                                 shape_fn=W.shape_fn(base))
        f.step(128)
        want = f.read_traces_device(32).reshape(len(rows), -1).cpu().numpy()
        f.close()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(got, want)
    assert sorted(k[2] for k in SG._SOLVERS) == [64, 128]
    SG.clear_solver_cache()
