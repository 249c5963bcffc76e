"""Pins of the oracle's perfectly matched layer (Sec. 2, eq. full_problem:
p_tt + alpha p_t + beta p = div(c^2 grad p) + div Phi - gamma psi,
Phi_t = Z1 Phi + c^2 Z2 grad p + c^2 Z3 grad psi, psi_t = p, with the
damping profile zeta_i and its constant zt = (c / ell) log(1 / R)).

- The profile is the printed one at every node coordinate.
- A layer of zero thickness leaves the solver exactly as it was.
- A plane pulse crossing a layer that ends on a rigid wall comes back
  attenuated by exp(-2 int zeta / c) = R over the round trip (the design
  value of the constant); a wrong sign of the damping would amplify it, a
  wrong factor would change the attenuation.
- In a cube with a centred pulse, absorbing faces alone leave reflections
  from oblique incidence and corners that the layer removes (the paper's
  Sec. 6.3 observation), and a long run stays bounded."""
import math

import numpy as np
import pytest

from oracle import ref as R
from paper_2603_06267_amd import workloads as W


def _zeta(d, ell, c, Rc):
    """The profile of Sec. 2 at distance d into a layer of thickness ell."""
    zt = c / ell * math.log(1.0 / Rc)
    d = np.clip(d, 0.0, ell)
    return np.where(d > 0, zt * (d / ell - np.sin(2 * np.pi * d / ell) / (2 * np.pi)), 0.0)


def test_profile_is_the_printed_one():
    dom = W.brick([0, 0, 0], [2.0, 1.5, 3.0], [8, 6, 12], 4, c=1.5)
    s = R.RefSolver([dom])
    ell = [0.5, 0.25, 0.0, 0.75, 1.0, 0.5]
    Rc = 1e-4
    s.set_pml(0, ell, Rc)
    for a in range(3):
        x = np.unique(s.coords()[:, a])
        lo, hi = dom["x0"][a] + ell[2 * a], dom["x1"][a] - ell[2 * a + 1]
        expect = np.zeros_like(x)
        if ell[2 * a] > 0:
            expect = np.where(x < lo, _zeta(lo - x, ell[2 * a], 1.5, Rc), expect)
        if ell[2 * a + 1] > 0:
            expect = np.where(x > hi, _zeta(x - hi, ell[2 * a + 1], 1.5, Rc), expect)
        z = s.pml_profile(0, a)
        assert np.abs(z - expect).max() <= 1e-12 * max(1.0, np.abs(expect).max())
        # zero at the layer's inner face, the constant zt at the outer face
        if ell[2 * a + 1] > 0:
            assert abs(z[-1] - 1.5 / ell[2 * a + 1] * math.log(1 / Rc)) < 1e-12 * z[-1]
            assert z[np.argmin(np.abs(x - hi))] == 0.0
        # non-decreasing into each layer
        if ell[2 * a + 1] > 0:
            zz = z[x >= hi]
            assert (np.diff(zz) >= 0).all()


def test_zero_thickness_changes_nothing():
    wl = W.config1()
    sf = W.shape_fn(wl)
    a = R.from_workload(wl, shape_fn=sf)
    b = R.from_workload(wl, shape_fn=sf)
    b.set_pml(0, [0.0] * 6, 1e-4)
    assert np.array_equal(a.step(150), b.step(150))


def test_bad_layers_are_refused():
    s = R.RefSolver(W.config2()["domains"])
    with pytest.raises(ValueError):
        s.set_pml(0, [0, 0, 0, 0, 0, 0.25], 1e-4)   # primary top is Gamma_I
    with pytest.raises(ValueError):
        s.set_pml(1, [0, 0, 0, 0, 0.5, 0], 1e-4)    # secondary bottom is Gamma_I
    with pytest.raises(ValueError):
        s.set_pml(1, [3.0, 1.5, 0, 0, 0, 0], 1e-4)  # thicker than the brick
    with pytest.raises(ValueError):
        s.set_pml(1, [0.5] * 4 + [0, 0.5], 1.5)      # R outside (0, 1)


def _column(ell, Rc, t_end=4.0, samples=8):
    """Gaussian plane pulse travelling +z in a rigid column [0, 0.25]^2 x
    [0, 4]; a layer of thickness ell ends on the rigid top.  Largest |p|
    outside the layer at `samples` times up to t_end."""
    dom = W.brick([0, 0, 0], [0.25, 0.25, 4.0], [1, 1, 16], 4, c=1.5)
    s = R.RefSolver([dom])
    s.set_pml(0, [0, 0, 0, 0, 0, ell], Rc)
    z = s.coords()[:, 2]
    sg, z0, c = 0.25, 1.5, 1.5
    g = np.exp(-((z - z0) / sg) ** 2)
    gp = -2 * (z - z0) / sg ** 2 * g
    gpp = (4 * (z - z0) ** 2 / sg ** 4 - 2 / sg ** 2) * g
    s.set_state(p=g, pd=-c * gp, pdd=c * c * gpp)
    out = []
    for _ in range(samples):
        s.step(int(round(t_end / samples / s.dt)))
        out.append(np.abs(s.get_state()["p"][z < 4.0 - ell]).max())
    return np.array(out)


def test_round_trip_attenuation_is_R():
    """Through the layer and back, a plane wave at normal incidence is
    attenuated by exp(-(2/c) int_0^ell zeta) = exp(-zt ell / c) = R.  With
    R = 1e-2 the pulse that returns from the rigid wall behind the layer
    has 1% of its amplitude (it is back in the interior from t = 2.5 on);
    with R = 1e-4 it is below the 1e-3 level of the scheme's dispersion tail."""
    a = _column(1.0, 1e-2)
    back = a[4:].max()
    assert 0.9e-2 < back < 1.1e-2, back
    b = _column(1.0, 1e-4)
    assert b[4:].max() < 1e-3
    assert a[0] > 0.99


def _cube(mode, steps_per=None, samples=6, t_end=3.0):
    dom = W.brick([0, 0, 0], [2.0, 2.0, 2.0], [8, 8, 8], 4, c=1.5)
    s = R.RefSolver([dom])
    if mode in ("abc", "pml"):
        s.set_absorbing(0, 0b111111)
    if mode == "pml":
        s.set_pml(0, [0.5] * 6, 1e-4)
    x = s.coords()
    p0 = np.exp(-((x - 1.0) ** 2).sum(1) / 0.2 ** 2)
    s.set_state(p=p0, pd=np.zeros_like(p0), pdd=-s.apply_K(p0) / s.mass())
    inner = np.all((x > 0.5 - 1e-9) & (x < 1.5 + 1e-9), axis=1)
    n = steps_per or int(round(t_end / samples / s.dt))
    out = []
    for _ in range(samples):
        s.step(n)
        out.append(np.abs(s.get_state()["p"][inner]).max())
    return np.array(out), n


def test_layer_removes_oblique_and_corner_reflections():
    """Centred pulse in a cube: after the wavefront has reached the walls
    (t >= 1.5), absorbing faces alone leave reflections of a few 1e-3 in the
    interior (oblique incidence, edges, corners), rigid walls 0.1 and more;
    with a layer of two elements in front of the absorbing faces what is
    left is an order of magnitude smaller, and it decays."""
    rigid, _ = _cube("rigid")
    abc, _ = _cube("abc")
    pml, n = _cube("pml")
    assert rigid[2:].max() > 0.05
    assert abc[2:].max() > 2e-3
    assert pml[3:].max() < 0.1 * abc[2:].max()
    assert pml[-1] < 0.5 * pml[2]
    # a long run stays bounded and decaying
    longer, _ = _cube("pml", steps_per=4 * n)
    assert np.isfinite(longer).all() and longer[-1] < pml[-1]
