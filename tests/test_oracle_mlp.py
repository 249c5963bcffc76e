"""Pins of the FP64 MLP oracle (oracle/mlp_ref.py) against facts that do not
come from the oracle itself: central finite differences of the loss, the
normal-distribution values of GELU, the least-squares solution of a linear
layer (numpy.linalg.lstsq), and the closed-form Adam steps for a constant
gradient."""
import math

import numpy as np
import pytest

from oracle import mlp_ref as M


def test_gelu_values():
    # gelu(z) = z Phi(z): Phi(0) = 1/2, Phi(1) = 0.8413447460685429,
    # Phi(-1.959963984540054) = 0.025
    assert M.gelu(np.array(0.0)) == 0.0
    assert abs(M.gelu(np.array(1.0)) - 0.8413447460685429) < 1e-15
    z = -1.959963984540054
    assert abs(M.gelu(np.array(z)) - 0.025 * z) < 1e-15
    # Phi(z) + Phi(-z) = 1  =>  gelu(z) - gelu(-z) = z
    zz = np.linspace(-6, 6, 101)
    assert np.allclose(M.gelu(zz) - M.gelu(-zz), zz, atol=1e-14)


def test_gelu_prime_by_differences():
    z = np.linspace(-5, 5, 41)
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.abs(fd - M.gelu_prime(z)).max() < 1e-8
    assert M.gelu_prime(np.array(0.0)) == 0.5


@pytest.mark.parametrize("widths", [[3, 8, 5], [4, 6, 6, 6, 7]])
def test_gradient_finite_differences(widths):
    """Every weight and bias of a small network against central differences."""
    rng = np.random.default_rng(7)
    params = M.init_params(widths, rng)
    params = [(W, rng.standard_normal(b.shape) * 0.3) for W, b in params]
    u = rng.standard_normal((5, widths[0]))
    t = rng.standard_normal((5, widths[-1]))
    y, cache = M.forward(params, u)
    g = M.flatten(M.backward(params, cache, y, t))
    vec = M.flatten(params)
    h = 1e-6
    fd = np.empty_like(vec)
    for i in range(len(vec)):
        vp = vec.copy()
        vp[i] += h
        vm = vec.copy()
        vm[i] -= h
        lp = M.loss(M.forward(M.unflatten(vp, widths), u)[0], t)
        lm = M.loss(M.forward(M.unflatten(vm, widths), u)[0], t)
        fd[i] = (lp - lm) / (2 * h)
    assert np.abs(fd - g).max() <= 1e-7 * max(1.0, np.abs(g).max())


def test_linear_layer_gradient_vanishes_at_least_squares():
    rng = np.random.default_rng(3)
    u = rng.standard_normal((40, 6))
    t = rng.standard_normal((40, 3))
    A = np.concatenate([u, np.ones((40, 1))], axis=1)
    sol = np.linalg.lstsq(A, t, rcond=None)[0]
    params = [(sol[:6].T.copy(), sol[6].copy())]
    y, cache = M.forward(params, u)
    gW, gb = M.backward(params, cache, y, t)[0]
    assert np.abs(gW).max() < 1e-12 and np.abs(gb).max() < 1e-12
    # and away from it the gradient does not vanish
    params = [(sol[:6].T + 0.1, sol[6].copy())]
    y, cache = M.forward(params, u)
    assert np.abs(M.backward(params, cache, y, t)[0][0]).max() > 1e-3


def test_embedding():
    """Affine columns map their feature; cos / sin columns of an angle lie on
    the unit circle, recover the angle and are 2 pi periodic in it; a Fourier
    column of a scalar equals cos(scale u + shift)."""
    rng = np.random.default_rng(5)
    u = np.concatenate([rng.uniform(0, 2 * math.pi, (6, 2)), rng.uniform(1.5, 3, (6, 1))], axis=1)
    cols = [(0, 1, 0.0, 1.0), (0, 2, 0.0, 1.0), (1, 1, 0.0, 1.0), (1, 2, 0.0, 1.0), (2, 0, 2.25, 1 / 0.75),
            (2, 1, 0.5, 3.0)]
    x = M.embed(u, cols)
    assert x.shape == (6, 6)
    assert np.allclose(x[:, 0] ** 2 + x[:, 1] ** 2, 1.0, atol=1e-15)
    assert np.allclose(np.arctan2(x[:, 1], x[:, 0]) % (2 * math.pi), u[:, 0], atol=1e-13)
    assert np.allclose(x[:, 4], (u[:, 2] - 2.25) / 0.75, atol=0)
    assert np.allclose(x[:, 5], [math.cos(3.0 * v + 0.5) for v in u[:, 2]], atol=1e-15)
    u2 = u.copy()
    u2[:, :2] += 2 * math.pi
    assert np.allclose(M.embed(u2, cols)[:, :4], x[:, :4], atol=1e-13)
    assert np.array_equal(M.embed(u), u)


def test_embedding_products():
    """Two-factor columns against the angle-addition identities
    cos a cos b - sin a sin b = cos(a + b), sin a cos b + cos a sin b =
    sin(a + b), the Pythagorean identity for a factor times itself, and an
    affine factor times a cosine; src2 = -1 leaves a single factor."""
    rng = np.random.default_rng(6)
    u = np.concatenate([rng.uniform(0, 2 * math.pi, (7, 2)), rng.uniform(1.5, 3, (7, 1))], axis=1)
    cols = [(0, 1, 0.0, 1.0, 1, 1, 0.0, 1.0), (0, 2, 0.0, 1.0, 1, 2, 0.0, 1.0),
            (0, 2, 0.0, 1.0, 1, 1, 0.0, 1.0), (0, 1, 0.0, 1.0, 1, 2, 0.0, 1.0),
            (0, 1, 0.0, 1.0, 0, 1, 0.0, 1.0), (0, 2, 0.0, 1.0, 0, 2, 0.0, 1.0),
            (2, 0, 2.25, 1 / 0.75, 0, 1, 0.3, 2.0), (2, 0, 1.0, 2.0, -1, 0, 0.0, 1.0)]
    x = M.embed(u, cols)
    a, b, f = u[:, 0], u[:, 1], u[:, 2]
    assert np.allclose(x[:, 0] - x[:, 1], np.cos(a + b), atol=1e-14)
    assert np.allclose(x[:, 2] + x[:, 3], np.sin(a + b), atol=1e-14)
    assert np.allclose(x[:, 4] + x[:, 5], 1.0, atol=1e-14)
    assert np.allclose(x[:, 6], (f - 2.25) / 0.75 * np.cos(2.0 * a + 0.3), atol=1e-14)
    assert np.allclose(x[:, 7], (f - 1.0) * 2.0, atol=0)


def test_adam_constant_gradient_closed_form():
    """With a constant gradient g the bias-corrected moments are exactly g and
    g^2 at every step, so each step moves by -lr g / (|g| + eps)."""
    W = np.array([[1.0, -2.0]])
    b = np.array([0.5])
    g = (np.array([[0.3, -4.0]]), np.array([1e-3]))
    opt = M.Adam([(W, b)], lr=0.01, eps=1e-8)
    p = [(W, b)]
    for k in range(1, 6):
        p = opt.step(p, [g])
        expW = W - k * 0.01 * g[0] / (np.abs(g[0]) + 1e-8)
        expb = b - k * 0.01 * g[1] / (np.abs(g[1]) + 1e-8)
        assert np.allclose(p[0][0], expW, rtol=0, atol=1e-12)
        assert np.allclose(p[0][1], expb, rtol=0, atol=1e-12)


def test_training_reduces_loss_on_smooth_target():
    rng = np.random.default_rng(11)
    widths = [2, 32, 32, 4]
    params = M.init_params(widths, rng)
    u = rng.uniform(-1, 1, (128, 2))
    t = np.stack([np.sin(2 * u[:, 0]), np.cos(u[:, 1]), u[:, 0] * u[:, 1], u[:, 0] ** 2], axis=1)
    opt = M.Adam(params, lr=3e-3)
    first = None
    for _ in range(300):
        params, l = M.train_step(params, opt, u, t)
        first = l if first is None else first
    assert l < 0.05 * first
