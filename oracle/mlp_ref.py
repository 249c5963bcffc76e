"""FP64 NumPy oracle of the surrogate MLP (forward, mean-squared-error loss,
backward, Adam).

TEST INFRASTRUCTURE ONLY: used by tests/ to check the BF16-MFMA kernels of
the surrogate form; the product package never imports it.

The network is the plain definition of a fully connected perceptron with the
Gauss error linear unit on the hidden layers:
    z_l = x_l W_l^T + b_l,   x_{l+1} = gelu(z_l)  (l < L-1),   y = z_{L-1},
    gelu(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2,
trained on the mean squared error (1 / (B n)) sum (y - t)^2 by Adam
(Kingma and Ba, 2015, Algorithm 1: bias-corrected first and second moments).
Raw input features u pass through a fixed embedding (each network input is
one raw feature mapped affinely, (u - shift) * scale, or through cos or sin of
scale u + shift); the physical output is out_scale * a * y with a either 1 or
one raw feature the output is proportional to, and the loss compares y with
t / (out_scale * a).

Parameters are a list of (W, b) pairs with W of shape [n_out, n_in].
"""
import numpy as np
from scipy.special import erf

SQRT2 = np.sqrt(2.0)
INV_SQRT_2PI = 1.0 / np.sqrt(2.0 * np.pi)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_prime(z):
    # d/dz [z Phi(z)] = Phi(z) + z phi(z)
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * INV_SQRT_2PI * np.exp(-0.5 * z * z)


def init_params(widths, rng):
    """He-style initialisation: W ~ N(0, 2 / n_in), b = 0."""
    params = []
    for n_in, n_out in zip(widths[:-1], widths[1:]):
        W = rng.standard_normal((n_out, n_in)) * np.sqrt(2.0 / n_in)
        params.append((W, np.zeros(n_out)))
    return params


def flatten(params):
    """Pack as the library's host layout: per layer W (row-major) then b."""
    return np.concatenate([np.concatenate([W.ravel(), b]) for W, b in params])


def unflatten(vec, widths):
    params, o = [], 0
    for n_in, n_out in zip(widths[:-1], widths[1:]):
        W = vec[o:o + n_in * n_out].reshape(n_out, n_in)
        o += n_in * n_out
        b = vec[o:o + n_out]
        o += n_out
        params.append((W.copy(), b.copy()))
    return params


def _factor(v, op, shift, scale):
    if op == 0:
        return (v - shift) * scale
    if op == 1:
        return np.cos(scale * v + shift)
    return np.sin(scale * v + shift)


def embed(u, columns=None):
    """Network input x_0 from raw features u [B, n_u]; columns: one (src, op,
    shift, scale) per input, op 0 = (u_src - shift) * scale, 1 = cos(scale
    u_src + shift), 2 = sin(scale u_src + shift); or (src, op, shift, scale,
    src2, op2, shift2, scale2), the product of two such factors (src2 = -1:
    the first alone).  None: u itself."""
    u = np.asarray(u, dtype=np.float64)
    if columns is None:
        return u.copy()
    cols = []
    for c in columns:
        v = _factor(u[:, c[0]], c[1], c[2], c[3])
        if len(c) > 4 and c[4] >= 0:
            v = v * _factor(u[:, c[4]], c[5], c[6], c[7])
        cols.append(v)
    return np.stack(cols, axis=1)


def forward(params, x):
    """Returns (y, cache) with y the normalised output of network input x and
    cache the per-layer inputs x_l and pre-activations z_l."""
    x = np.asarray(x, dtype=np.float64)
    xs, zs = [], []
    L = len(params)
    for l, (W, b) in enumerate(params):
        xs.append(x)
        z = x @ W.T + b
        zs.append(z)
        x = gelu(z) if l < L - 1 else z
    return x, (xs, zs)


def loss(y, t):
    return float(np.mean((y - t) ** 2))


def backward(params, cache, y, t):
    """Gradients of loss(y, t) with respect to every W_l and b_l."""
    xs, zs = cache
    B, n = y.shape
    dz = 2.0 * (y - t) / (B * n)
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        grads[l] = (dz.T @ xs[l], dz.sum(axis=0))
        if l > 0:
            dz = (dz @ W) * gelu_prime(zs[l - 1])
    return grads


class Adam:
    """Adam with bias correction on a list of (W, b) parameters."""

    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.t = 0
        self.m = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]
        self.v = [(np.zeros_like(W), np.zeros_like(b)) for W, b in params]

    def step(self, params, grads, lr=None):
        lr = self.lr if lr is None else lr
        self.t += 1
        c1 = 1.0 - self.b1 ** self.t
        c2 = 1.0 - self.b2 ** self.t
        out = []
        for l, ((W, b), (gW, gb)) in enumerate(zip(params, grads)):
            new = []
            for j, (p, g) in enumerate(((W, gW), (b, gb))):
                m = self.b1 * self.m[l][j] + (1 - self.b1) * g
                v = self.b2 * self.v[l][j] + (1 - self.b2) * g * g
                self.m[l] = self.m[l][:j] + (m,) + self.m[l][j + 1:]
                self.v[l] = self.v[l][:j] + (v,) + self.v[l][j + 1:]
                new.append(p - lr * (m / c1) / (np.sqrt(v / c2) + self.eps))
            out.append(tuple(new))
        return out


def train_step(params, opt, x, t, out_scale=1.0, lr=None):
    """One minibatch step on network inputs x and physical targets t (out_scale
    may be a per-row column); returns (new params, loss before the step)."""
    y, cache = forward(params, x)
    tn = np.asarray(t, dtype=np.float64) / out_scale
    g = backward(params, cache, y, tn)
    return opt.step(params, g, lr), loss(y, tn)
