"""Batched form on the GPU: persistent launches over many problems give the
same results as stepping each problem on its own on the tiled path
(bitwise), match the FP64 oracle, and the tile autotuner returns a valid,
cached choice.  The individual solvers are held to the tiled path: a small
single-brick solver would otherwise take the LDS-resident steps, whose PMUT
and receiver sums run in another order (compared at a tolerance in
test_gpu_resident.py)."""
import numpy as np
import pytest

from oracle import ref
from paper_2603_06267_amd import _lib, batch as B, solver, workloads as W

pytestmark = pytest.mark.gpu


def _tiled(wl, steps, sf):
    s = solver.from_workload(wl, precision=32, n_steps=steps, shape_fn=sf, bind=False)
    s.set_option(_lib.OPT_RESIDENT, 0)
    s.bind()
    return s


def _workloads(steps, nscen=8, mesh_ids=(0, 5, 10, 15)):
    c4 = W.config4()
    base = dict(c4["scenarios"], steps=steps)
    dr = base["drive"]
    base["drive"] = {k: (v[:nscen] if hasattr(v, "__len__") and not isinstance(v, float) else v)
                     for k, v in dr.items()}
    meshes = [dict(c4["meshes"][i], steps=steps) for i in mesh_ids]
    return [base] + meshes


def test_batch_equals_individual_solvers():
    steps = 100
    wls = _workloads(steps)
    sfs = [W.shape_fn(w) for w in wls]
    b = B.build_batch(wls, shape_fns=sfs, n_steps=steps)
    b.step(steps)
    for wl, sf, sb in zip(wls, sfs, b.solvers):
        s1 = _tiled(wl, steps, sf)
        s1.step(steps)
        np.testing.assert_array_equal(sb.read_traces(), s1.read_traces())


def test_batch_vs_oracle_highest_order_mesh():
    steps = 150
    wls = _workloads(steps, nscen=4, mesh_ids=(3, 15))
    sfs = [W.shape_fn(w) for w in wls]
    b = B.build_batch(wls, shape_fns=sfs, n_steps=steps)
    b.set_option(4, 29)
    b.step(steps)
    for i, sc in ((0, 3), (2, 0)):
        o = ref.from_workload(wls[i], scenario=sc, shape_fn=sfs[i])
        to = o.step(steps)
        tg = b.solvers[i].read_traces()[sc]
        err = np.linalg.norm(tg - to) / np.linalg.norm(to)
        assert err <= 1e-5, (i, sc, err)


def test_batch_with_absorbing_faces():
    """Meshes with first-order absorbing faces in a batch: bitwise the
    individual solvers, and the oracle to 1e-5."""
    steps = 120
    wls = _workloads(steps, nscen=4, mesh_ids=(2, 9))
    wls[1] = dict(wls[1], domains=[dict(wls[1]["domains"][0], absorbing=0b111111)])
    wls[2] = dict(wls[2], domains=[dict(wls[2]["domains"][0], absorbing=0b100011)])
    sfs = [W.shape_fn(w) for w in wls]
    b = B.build_batch(wls, shape_fns=sfs, n_steps=steps)
    b.step(steps)
    for wl, sf, sb in zip(wls, sfs, b.solvers):
        s1 = _tiled(wl, steps, sf)
        s1.step(steps)
        np.testing.assert_array_equal(sb.read_traces(), s1.read_traces())
    o = ref.from_workload(wls[1], scenario=0, shape_fn=sfs[1])
    to = o.step(steps)
    tg = b.solvers[1].read_traces()[0]
    assert np.linalg.norm(tg - to) / np.linalg.norm(to) <= 1e-5


def test_tuner_choice_valid_and_cached(tmp_path):
    t = B.TileTuner(path=str(tmp_path / "tiles.json"), candidates=[(1, 9), (2, 17)], steps=3)
    dom = W.config4()["meshes"][6]["domains"]
    best = t.tune(dom, S=1)
    assert best in [(1, 9), (2, 17)]
    t2 = B.TileTuner(path=str(tmp_path / "tiles.json"))
    assert t2.tune(dom, S=1) == best


def test_batch_fixes_member_tile_options():
    """A batch fixes its solvers' tiles and kernel arguments when it is
    created: tile options of a member are refused until the batch is
    destroyed; graph and timing options stay open."""
    from paper_2603_06267_amd import _lib
    steps = 20
    wls = _workloads(steps, nscen=2, mesh_ids=(1,))
    sfs = [W.shape_fn(w) for w in wls]
    b = B.build_batch(wls, shape_fns=sfs, n_steps=steps)
    s0 = b.solvers[0]
    for opt, val in ((_lib.OPT_TILE_ROWS, 2), (_lib.OPT_TILE_ZCHUNK, 5), (_lib.OPT_TILE_WAVES, 8),
                     (_lib.OPT_PREFETCH, 3), (_lib.OPT_TIME_BLOCK, 2)):
        with pytest.raises(_lib.PmdgError) as e:
            s0.set_option(opt, val)
        assert e.value.code == _lib.PMDG_ESTATE
    s0.set_option(_lib.OPT_TIMING, 0)
    b.step(steps)
    tr = s0.read_traces()
    assert np.isfinite(tr).all()
    b.close()
    s0.set_option(_lib.OPT_TILE_ROWS, 2)
