"""Independent NumPy constructions used to pin the oracle.

Everything here is built from numpy.polynomial (Legendre roots, monomial fits,
polynomial derivatives), never from the oracle's own routines, so that a wrong
node, weight, sign or index in the oracle shows up as a mismatch.
"""
import numpy as np
from numpy.polynomial import legendre as npleg
from numpy.polynomial import polynomial as nppoly


def gll_numpy(N):
    """GLL nodes: +-1 and the roots of P_N'; weights 2/(N(N+1)P_N(x)^2)."""
    cN = np.zeros(N + 1); cN[N] = 1.0
    inner = np.sort(np.real(npleg.legroots(npleg.legder(cN)))) if N > 1 else np.array([])
    x = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (N * (N + 1) * npleg.legval(x, cN) ** 2)
    return x, w


def lagrange_polys(nodes):
    """Monomial coefficient arrays of the Lagrange polynomials through nodes."""
    n = len(nodes)
    polys = []
    for j in range(n):
        c = np.array([1.0])
        for m in range(n):
            if m != j:
                c = nppoly.polymul(c, np.array([-nodes[m], 1.0]) / (nodes[j] - nodes[m]))
        polys.append(c)
    return polys


def basis_tables(nodes, pts):
    """Values V[q, j] = l_j(pts[q]) and derivatives Dv[q, j] = l_j'(pts[q])."""
    P = lagrange_polys(nodes)
    V = np.array([[nppoly.polyval(t, p) for p in P] for t in pts])
    Dv = np.array([[nppoly.polyval(t, nppoly.polyder(p)) for p in P] for t in pts])
    return V, Dv


def sem_1d(N, ne, h):
    """Assembled 1D C0 stiffness and lumped mass on ne equal elements of size h
    with GLL collocation: K = sum_e (2/h) B^T W B, M = sum_e (h/2) W."""
    x, w = gll_numpy(N)
    _, Dv = basis_tables(x, x)
    n = N * ne + 1
    K = np.zeros((n, n)); M = np.zeros(n)
    kl = (2.0 / h) * Dv.T @ np.diag(w) @ Dv
    for e in range(ne):
        s = slice(N * e, N * e + N + 1)
        K[s, s] += kl
        M[s] += 0.5 * h * w
    return K, M
