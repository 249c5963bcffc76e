"""GPU face matching (pmdg_match_faces: Sec. 5, Algorithm 3) against the
oracle's Algorithm 3 and its closed-form interface list, through the C ABI.
Coarse element indices bit-exact, reference points within 1e-12.

- The small two-domain interfaces (nested 2:1 and non-nested 4:3) as
  hexahedra: the oracle's brick interface list.
- Warped interfaces (seeded in-plane jitter on both sides): the oracle's
  Algorithm 3, every point.
- Coarse faces listed twice, first with a co-oriented face: the normal
  filter skips those.
- The large array's interface (128 x 128 fine faces against 96 x 96 coarse
  ones, 5 x 5 points per face): the oracle's brick interface list at every
  one of its 409,600 points; and the same interface warped, against the
  oracle's Algorithm 3 on a seeded sample of fine faces.
"""
import sys

import numpy as np
import pytest

from oracle import ref
from paper_2603_06267_amd import matching as M, workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _gpu(nq, fine, ff, coarse, cf, **kw):
    import torch
    e, x, u = M.match_faces(nq, fine, ff, coarse, cf, **kw)
    torch.cuda.synchronize()
    return e.cpu().numpy(), x.cpu().numpy(), int(u.cpu().numpy()[0])


def _warp(dom, seed, amp=0.25):
    rng = np.random.default_rng(1000 + seed)
    V = W.brick_vertices(dom)
    x0 = np.asarray(dom["x0"]); x1 = np.asarray(dom["x1"])
    h = (x1 - x0) / np.asarray(dom["ne"])
    side = np.any(np.abs(V[:, :2] - x0[:2]) < 1e-12, axis=1) | np.any(np.abs(V[:, :2] - x1[:2]) < 1e-12, axis=1)
    V[~side, 0] += amp * h[0] * rng.uniform(-1, 1, size=(~side).sum())
    V[~side, 1] += amp * h[1] * rng.uniform(-1, 1, size=(~side).sum())
    return V


def _sides(prim, sec, Vf=None, Vc=None):
    Vf = W.brick_vertices(prim) if Vf is None else Vf
    Vc = W.brick_vertices(sec) if Vc is None else Vc
    fine = M.layer_hexes(Vf, prim["ne"], prim["ne"][2] - 1)
    coarse = M.layer_hexes(Vc, sec["ne"], 0)
    return fine, np.full(len(fine), 5), coarse, np.full(len(coarse), 4)


def test_degenerate_face_sets():
    """No coarse faces: every point is unmatched (element -1) and counted, as
    the oracle has it; no fine faces: nothing to match and a count of 0,
    whatever the unmatched counter held before."""
    prim = W.brick([0, 0, 0], [2, 2, 1], [4, 4, 1], 2)
    sec = W.brick([0, 0, 1], [2, 2, 2], [3, 3, 1], 2)
    fine, ff, coarse, cf = _sides(prim, sec)
    e, x, u = _gpu(3, fine, ff, coarse[:0], cf[:0])
    eo, xo, uo = ref.match_faces(3, fine, ff, coarse[:0], cf[:0])
    assert u == uo == len(fine) * 9
    assert (e == -1).all() and np.array_equal(e, eo)
    e, x, u = _gpu(3, fine, ff, coarse, cf)  # leaves a count of 0 ...
    e, x, u = _gpu(3, fine[:1], ff[:1], coarse[:0], cf[:0])  # ... then 9
    assert u == 9
    e, x, u = _gpu(3, fine[:0], ff[:0], coarse, cf)
    assert u == 0 and len(e) == 0


@pytest.mark.parametrize("nested", [True, False])
def test_brick_interface_list(nested):
    wl = W.small_two_domain(nested=nested)
    prim, sec = wl["domains"]
    nq = max(prim["N"], sec["N"]) + 1
    args = _sides(prim, sec)
    e, x, u = _gpu(nq, *args)
    ce, cxi = ref.RefSolver([prim, sec]).interface_points()
    assert u == 0
    assert np.array_equal(e, ce[:, 0] + sec["ne"][0] * ce[:, 1])
    assert np.abs(x[:, :2] - cxi).max() < 1e-12 and np.abs(x[:, 2] + 1).max() < 1e-12
    eo, xo, uo = ref.match_faces(nq, *args)
    assert np.array_equal(e, eo) and np.abs(x - xo).max() < 1e-12


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_warped_interfaces(seed):
    prim = W.brick([0, 0, 0], [3, 3, 1], [8, 8, 2], 3)
    sec = W.brick([0, 0, 1], [3, 3, 4], [6, 6, 3], 3)
    args = _sides(prim, sec, _warp(prim, seed), _warp(sec, seed + 10))
    for nq in (2, 4, 7):
        e, x, u = _gpu(nq, *args)
        eo, xo, uo = ref.match_faces(nq, *args)
        assert u == uo == 0
        assert np.array_equal(e, eo)
        assert np.abs(x - xo).max() < 1e-12


def test_normal_filter_and_unmatched_points():
    prim = W.brick([0, 0, 0], [2, 2, 1], [4, 4, 1], 2)
    sec = W.brick([0, 0, 1], [2, 2, 1.3], [3, 3, 1], 2)
    fine, ff, coarse, cf = _sides(prim, sec)
    both = np.concatenate([coarse, coarse])
    faces = np.concatenate([np.full(len(coarse), 5), cf])
    e, x, u = _gpu(3, fine, ff, both, faces)
    eo, xo, uo = ref.match_faces(3, fine, ff, both, faces)
    assert u == 0 and (e >= len(coarse)).all()
    assert np.array_equal(e, eo) and np.abs(x - xo).max() < 1e-12
    # drop the coarse faces over the first fine column: those points stay
    # unmatched, and are counted
    keep = np.arange(len(coarse)) % 3 != 0
    e2, x2, u2 = _gpu(3, fine, ff, coarse[keep], cf[keep])
    eo2, xo2, uo2 = ref.match_faces(3, fine, ff, coarse[keep], cf[keep])
    assert u2 == uo2 > 0 and np.array_equal(e2, eo2)
    assert (e2 < 0).sum() == u2


def test_large_array_interface():
    """The large array's interface: 16,384 fine faces, 9,216 coarse faces,
    409,600 points."""
    wl = W.config3(steps=1)
    prim, sec = wl["domains"]
    nq = 5
    args = _sides(prim, sec)
    _say("large interface, brick hexahedra")
    e, x, u = _gpu(nq, *args)
    assert u == 0
    o = ref.RefSolver([prim, sec])
    ce, cxi = o.interface_points()
    del o
    assert np.array_equal(e, ce[:, 0] + sec["ne"][0] * ce[:, 1])
    assert np.abs(x[:, :2] - cxi).max() < 1e-12 and np.abs(x[:, 2] + 1).max() < 1e-12
    _say("large interface, warped")
    args = _sides(prim, sec, _warp(prim, 7), _warp(sec, 8))
    e, x, u = _gpu(nq, *args)
    assert u == 0
    rng = np.random.default_rng(11)
    sample = np.sort(rng.choice(len(args[0]), size=96, replace=False))
    eo, xo, uo = ref.match_faces(nq, args[0][sample], args[1][sample], args[2], args[3])
    pts = (sample[:, None] * nq * nq + np.arange(nq * nq)[None, :]).ravel()
    assert uo == 0
    assert np.array_equal(e[pts], eo) and np.abs(x[pts] - xo).max() < 1e-12


def test_radius_is_the_face_diameter():
    """A coarse interface face shaped as a thin trapezoid (one edge of 10,
    diagonals of about 5.1) and a fine face near the far end of that edge."""
    bot = np.array([[0, 0], [10, 0], [4.9, 0.1], [5.1, 0.1]])
    coarse = np.array([[*bot[c & 3], 0.0 if c < 4 else 1.0] for c in range(8)])[None]
    fx, fy = (9.80, 9.90), (0.0002, 0.0008)
    fine = np.array([[fx[c & 1], fy[(c >> 1) & 1], -1.0 if c < 4 else 0.0] for c in range(8)])[None]
    ff, cf = np.array([5]), np.array([4])
    e, x, u = _gpu(2, fine, ff, coarse, cf)
    eo, xo, uo = ref.match_faces(2, fine, ff, coarse, cf)
    assert u == uo == 0 and (e == 0).all() and np.array_equal(e, eo) and np.abs(x - xo).max() < 1e-12
