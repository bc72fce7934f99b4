"""Pins for the oracle's Butcher tableaux (Sec. 2, Table 1).

Independent facts used:
* order conditions B(p) with p the order of Table 1, and failure of B(p+1);
* the simplifying condition D(s) (GL) / D(s-1) (Radau IIA), which the
  construction does not impose;
* the stability function ``R(z) = 1 + z b^T (I - zA)^-1 1`` equals the Pade
  approximant of exp(z) of type (s,s) for GL, (s-1,s) for Radau IIA and
  (s-2,s) for Lobatto IIIC (textbook closed form, Hairer-Wanner II, IV.3);
* A-stability / L-stability as listed in Table 1;
* a few textbook coefficients (GL2, Radau IIA3 nodes, Lobatto IIIC2/3).
"""
import math
from fractions import Fraction

import mpmath as mp
import numpy as np
import pytest

from oracle.tableau import ORDER, tableau, tableau_mp

FAMILIES = ["gauss", "radau_iia", "lobatto_iiic"]
CASES = [(f, s) for f in FAMILIES for s in range(2, 8)] + [("gauss", 1), ("radau_iia", 1)]


def pade(k, j, z):
    """Pade approximant R_kj of exp(z): numerator degree k, denominator j."""
    P = sum(Fraction(math.factorial(k + j - i) * math.factorial(k),
                     math.factorial(k + j) * math.factorial(i) * math.factorial(k - i)) * z ** i
            for i in range(k + 1))
    Q = sum(Fraction(math.factorial(k + j - i) * math.factorial(j),
                     math.factorial(k + j) * math.factorial(i) * math.factorial(j - i)) * (-z) ** i
            for i in range(j + 1))
    return P / Q


def pade_type(family, s):
    return {"gauss": (s, s), "radau_iia": (s - 1, s), "lobatto_iiic": (s - 2, s)}[family]


def stability(A, b, z):
    s = A.shape[0]
    return 1.0 + z * (b @ np.linalg.solve(np.eye(s) - z * A, np.ones(s)))


@pytest.mark.parametrize("family,s", CASES)
def test_order_conditions_B(family, s):
    A, b, c = tableau(family, s)
    p = ORDER[family](s)
    for k in range(1, p + 1):
        assert abs(b @ c ** (k - 1) - 1.0 / k) < 1e-14, (family, s, k)
    # the order is exactly p: B(p+1) fails
    assert abs(b @ c ** p - 1.0 / (p + 1)) > 1e-12


@pytest.mark.parametrize("family,s", CASES)
def test_row_sums_and_weights(family, s):
    A, b, c = tableau(family, s)
    assert abs(b.sum() - 1.0) < 1e-15
    assert np.max(np.abs(A.sum(axis=1) - c)) < 1e-15


@pytest.mark.parametrize("family,s", [(f, s) for f in ["gauss", "radau_iia"] for s in range(2, 8)])
def test_condition_D(family, s):
    """D(zeta): sum_i b_i c_i^(k-1) a_ij = b_j (1 - c_j^k) / k for k <= zeta,
    zeta = s (GL) or s-1 (Radau IIA).  Not used by the construction."""
    A, b, c = tableau(family, s)
    zeta = s if family == "gauss" else s - 1
    for k in range(1, zeta + 1):
        lhs = (b * c ** (k - 1)) @ A
        rhs = b * (1.0 - c ** k) / k
        assert np.max(np.abs(lhs - rhs)) < 1e-14


@pytest.mark.parametrize("family,s", [(f, s) for f in FAMILIES for s in range(2, 8)])
def test_stability_function_is_pade(family, s):
    A, b, c = tableau(family, s)
    k, j = pade_type(family, s)
    for z in [Fraction(-1), Fraction(-7, 2), Fraction(1, 3), Fraction(-40), Fraction(5, 2)]:
        ref = float(pade(k, j, z))
        got = stability(A, b, float(z))
        assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref)), (family, s, z, got, ref)
    # complex argument: evaluate the Pade quotient in complex floating point
    for z in [-1 + 3j, -0.5 - 8j, 2j]:
        P = sum(math.factorial(k + j - i) * math.factorial(k)
                / (math.factorial(k + j) * math.factorial(i) * math.factorial(k - i)) * z ** i
                for i in range(k + 1))
        Q = sum(math.factorial(k + j - i) * math.factorial(j)
                / (math.factorial(k + j) * math.factorial(i) * math.factorial(j - i)) * (-z) ** i
                for i in range(j + 1))
        assert abs(stability(A, b, z) - P / Q) < 1e-12 * max(1.0, abs(P / Q))


def test_exact_rational_stability_values():
    """R(-1) in exact arithmetic from the 50-digit tableaux: GL2 7/19,
    Radau IIA2 4/11, Radau IIA3 39/106."""
    for family, s, frac in [("gauss", 2, Fraction(7, 19)), ("radau_iia", 2, Fraction(4, 11)),
                            ("radau_iia", 3, Fraction(39, 106))]:
        with mp.workdps(50):
            A, b, c = tableau_mp(family, s)
            Am = mp.matrix(A)
            z = mp.mpf(-1)
            x = mp.lu_solve(mp.eye(s) - z * Am, mp.matrix([1] * s))
            R = 1 + z * sum(b[i] * x[i] for i in range(s))
            assert abs(R - mp.mpf(frac.numerator) / frac.denominator) < mp.mpf(10) ** -40


@pytest.mark.parametrize("family,s", [(f, s) for f in FAMILIES for s in range(2, 8)])
def test_A_and_L_stability(family, s):
    """Table 1: GL is A-stable with |R(-inf)| = 1; Radau IIA and Lobatto
    IIIC are L-stable (R(-inf) = 0)."""
    A, b, c = tableau(family, s)
    for y in np.linspace(-50, 50, 41):
        assert abs(stability(A, b, 1j * y)) <= 1.0 + 1e-12
    for x in [-0.1, -1.0, -10.0, -1e3]:
        for y in [0.0, 2.0, -30.0]:
            assert abs(stability(A, b, x + 1j * y)) <= 1.0 + 1e-12
    # R(-inf) = 1 - b^T A^-1 1 (limit of the stability function)
    r_inf = 1.0 - b @ np.linalg.solve(A, np.ones(s))
    if family == "gauss":
        assert abs(abs(r_inf) - 1.0) < 1e-10
    else:
        assert abs(r_inf) < 1e-10


def test_textbook_coefficients():
    A, b, c = tableau("gauss", 2)
    r3 = math.sqrt(3.0)
    assert np.allclose(A, [[0.25, 0.25 - r3 / 6], [0.25 + r3 / 6, 0.25]], atol=1e-15)
    assert np.allclose(c, [0.5 - r3 / 6, 0.5 + r3 / 6], atol=1e-15)
    A, b, c = tableau("radau_iia", 3)
    r6 = math.sqrt(6.0)
    assert np.allclose(c, [(4 - r6) / 10, (4 + r6) / 10, 1.0], atol=1e-15)
    assert np.allclose(b, [(16 - r6) / 36, (16 + r6) / 36, 1.0 / 9], atol=1e-15)
    A, b, c = tableau("lobatto_iiic", 2)
    assert np.allclose(A, [[0.5, -0.5], [0.5, 0.5]], atol=1e-15)
    A, b, c = tableau("lobatto_iiic", 3)
    assert np.allclose(A, [[1 / 6, -1 / 3, 1 / 6], [1 / 6, 5 / 12, -1 / 12], [1 / 6, 2 / 3, 1 / 6]],
                       atol=1e-15)
    A, b, c = tableau("radau_iia", 1)
    assert np.allclose(A, [[1.0]]) and np.allclose(b, [1.0])   # backward Euler
    A, b, c = tableau("gauss", 1)
    assert np.allclose(A, [[0.5]]) and np.allclose(c, [0.5])   # implicit midpoint
