"""Pins of the oracle's quadrature and derivative matrix (Sec. 3: Lagrangian
GLL basis with reduced integration; Sec. 5: Gauss-Legendre points on the
finer interface face)."""
import math
import os

import numpy as np
import pytest

from oracle import ref
from tests._indep import gll_numpy

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("N", range(1, 9))
def test_gll_exactness(N):
    x, w = ref.gll(N)
    for k in range(0, 2 * N):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-13
    # GLL with N+1 points is not exact at degree 2N
    assert abs(np.dot(w, x ** (2 * N)) - 2.0 / (2 * N + 1)) > 1e-6


@pytest.mark.parametrize("N", range(1, 9))
def test_gll_matches_numpy_roots(N):
    x, w = ref.gll(N)
    xn, wn = gll_numpy(N)
    assert np.allclose(x, xn, atol=1e-14) and np.allclose(w, wn, atol=1e-14)


def test_gll_n4_closed_form():
    x, w = ref.gll(4)
    s = math.sqrt(3.0 / 7.0)
    assert np.allclose(x, [-1, -s, 0, s, 1], atol=1e-15)
    assert np.allclose(w, [1 / 10, 49 / 90, 32 / 45, 49 / 90, 1 / 10], atol=1e-15)


@pytest.mark.parametrize("n", range(1, 11))
def test_gl_exactness_and_numpy(n):
    x, w = ref.gl(n)
    for k in range(0, 2 * n):
        exact = 0.0 if k % 2 else 2.0 / (k + 1)
        assert abs(np.dot(w, x ** k) - exact) < 1e-13
    xn, wn = np.polynomial.legendre.leggauss(n)
    assert np.allclose(x, xn, atol=1e-14) and np.allclose(w, wn, atol=1e-14)


def test_gl4_positions_printed_in_matching_figure():
    """The face-matching figure (Sec. 5, fig. DG_matching) draws the 4x4
    Gauss-Legendre points of each fine face at fractions of the face edge;
    (1 + x_q) / 2 of the 4-point rule must reproduce them to the 4 digits the
    figure carries."""
    printed = np.loadtxt(os.path.join(GOLDEN, "gl4_face_fractions.txt"))
    x, _ = ref.gl(4)
    assert np.allclose((1 + x) / 2, printed, atol=6e-5)


@pytest.mark.parametrize("N", range(1, 9))
def test_dmat_differentiates_polynomials(N):
    x, w = ref.gll(N)
    D = ref.dmat(N)
    for k in range(0, N + 1):
        d = k * x ** (k - 1) if k > 0 else np.zeros_like(x)
        assert np.allclose(D @ x ** k, d, atol=1e-12)


@pytest.mark.parametrize("N", range(1, 9))
def test_dmat_summation_by_parts(N):
    x, w = ref.gll(N)
    D = ref.dmat(N)
    Q = np.diag(w) @ D
    E = np.zeros((N + 1, N + 1)); E[0, 0] = -1.0; E[N, N] = 1.0
    assert np.allclose(Q + Q.T, E, atol=1e-13)


def test_lagrange_cardinal_and_reproduction():
    x, _ = ref.gll(5)
    for i, xi in enumerate(x):
        v, _ = ref.lagrange(x, xi)
        assert np.allclose(v, np.eye(6)[i], atol=1e-14)
    t = 0.3141
    v, d = ref.lagrange(x, t)
    for k in range(6):
        assert abs(np.dot(v, x ** k) - t ** k) < 1e-13
        assert abs(np.dot(d, x ** k) - (k * t ** (k - 1) if k else 0.0)) < 1e-12
