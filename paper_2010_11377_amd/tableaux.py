"""Butcher tableaux for the GPU path, in float64 numpy.

Built independently of the test oracle (which uses 50-digit collocation):
nodes from Legendre-basis root finding refined by Newton steps, and the
coefficients as exact integrals of Lagrange polynomials evaluated by
Gauss--Legendre quadrature.

* Gauss--Legendre (order 2s): nodes = zeros of P_s(2x-1),
  ``a_ij = int_0^{c_i} l_j``, ``b_j = int_0^1 l_j``.
* Radau IIA (order 2s-1): nodes = zeros of P_s(2x-1) - P_{s-1}(2x-1).
* Lobatto IIIC (order 2s-2): nodes 0, 1 and the zeros of P'_{s-1}(2x-1);
  ``a_i1 = b_1`` and, with l~ the Lagrange basis of the last s-1 nodes,
  ``a_ij = int_0^{c_i} l~_j - b_1 l~_j(0)`` for j >= 2.
"""
import numpy as np
from numpy.polynomial import legendre as npleg


def _refine(roots, coeffs_leg):
    """Newton refinement of roots of a Legendre series in t in [-1, 1]."""
    d = npleg.legder(coeffs_leg)
    r = np.array(roots, dtype=np.float64)
    for _ in range(4):
        f = npleg.legval(r, coeffs_leg)
        fp = npleg.legval(r, d)
        step = np.where(fp != 0, f / np.where(fp == 0, 1.0, fp), 0.0)
        r = r - step
    return r


def _roots01(coeffs_leg):
    t = npleg.legroots(coeffs_leg)
    t = np.sort(np.real(t))
    t = _refine(t, coeffs_leg)
    return (t + 1.0) / 2.0


def _lagrange(nodes, j, x):
    num = np.ones_like(x)
    den = 1.0
    for m, cm in enumerate(nodes):
        if m != j:
            num = num * (x - cm)
            den *= nodes[j] - cm
    return num / den


def _integral(nodes, j, upper):
    """int_0^upper l_j(x) dx, exact for the degree len(nodes)-1 polynomial."""
    q = len(nodes)
    t, w = npleg.leggauss(max(q, 1))
    x = 0.5 * upper * (t + 1.0)
    return 0.5 * upper * float(np.sum(w * _lagrange(nodes, j, x)))


def _collocation(c):
    s = len(c)
    A = np.array([[_integral(c, j, c[i]) for j in range(s)] for i in range(s)])
    b = np.array([_integral(c, j, 1.0) for j in range(s)])
    return A, b


def gauss_legendre(s):
    coeffs = np.zeros(s + 1)
    coeffs[s] = 1.0
    c = _roots01(coeffs)
    A, b = _collocation(c)
    return A, b, c


def radau_iia(s):
    if s == 1:
        return np.array([[1.0]]), np.array([1.0]), np.array([1.0])
    coeffs = np.zeros(s + 1)
    coeffs[s] = 1.0
    coeffs[s - 1] = -1.0
    c = _roots01(coeffs)
    c[-1] = 1.0
    A, b = _collocation(c)
    return A, b, c


def lobatto_iiic(s):
    if s < 2:
        raise ValueError("Lobatto IIIC needs s >= 2")
    inner = np.array([])
    if s > 2:
        coeffs = np.zeros(s)
        coeffs[s - 1] = 1.0
        inner = _roots01(npleg.legder(coeffs))
    c = np.concatenate([[0.0], inner, [1.0]])
    b = np.array([_integral(c, j, 1.0) for j in range(s)])
    tail = c[1:]
    A = np.zeros((s, s))
    for i in range(s):
        A[i, 0] = b[0]
        for j in range(s - 1):
            A[i, j + 1] = _integral(tail, j, c[i]) - b[0] * float(_lagrange(tail, j, np.array(0.0)))
    return A, b, c


FAMILIES = {"gauss": gauss_legendre, "radau_iia": radau_iia, "lobatto_iiic": lobatto_iiic}


def tableau(family, s):
    """``(A, b, c)`` float64 for family in {"gauss", "radau_iia", "lobatto_iiic"}."""
    return FAMILIES[family](s)
