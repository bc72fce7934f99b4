"""Butcher tableaux ``(A, b, c)`` of the IRK families the paper lists in Table 1
(Sec. 2): Gauss--Legendre (order 2s), Radau IIA (order 2s-1) and Lobatto IIIC
(order 2s-2).  The paper prints no coefficients, so they are built here from
their textbook definitions in 50-digit arithmetic (mpmath) and rounded once to
float64.

* Gauss--Legendre: nodes are the zeros of the shifted Legendre polynomial
  ``P_s(2x-1)``; collocation, i.e. ``A`` from the simplifying condition C(s)
  and ``b`` from B(s).
* Radau IIA: nodes are the zeros of ``P_s(2x-1) - P_{s-1}(2x-1)`` (so
  ``c_s = 1``); collocation as above.
* Lobatto IIIC: nodes are ``0``, ``1`` and the zeros of ``P'_{s-1}(2x-1)``;
  ``b`` from B(s); first column ``a_{i1} = b_1`` and the other columns from
  C(s-1).

Test infrastructure only (see the package docstring).
"""
import mpmath as mp
import numpy as np

DPS = 50


def _shifted_legendre_coeffs(n):
    """Coefficients (ascending powers of x) of P_n(2x-1), exact integers."""
    return [(-1) ** (n + k) * mp.binomial(n, k) * mp.binomial(n + k, k) for k in range(n + 1)]


def _roots_ascending(coeffs_asc):
    """Real roots in [0, 1] of a polynomial given by ascending coefficients."""
    desc = list(reversed(coeffs_asc))
    while desc and desc[0] == 0:
        desc.pop(0)
    roots = mp.polyroots(desc, maxsteps=400, extraprec=400)
    for r in roots:
        if abs(mp.im(r)) > mp.mpf(10) ** (-(DPS - 10)):
            raise ArithmeticError("complex node %s" % r)
    return sorted(mp.re(r) for r in roots)


def _solve(M, rhs):
    return mp.lu_solve(mp.matrix(M), mp.matrix(rhs))


def _b_from_nodes(c):
    """Quadrature weights from B(s): sum_j b_j c_j^(k-1) = 1/k, k = 1..s."""
    s = len(c)
    V = [[c[j] ** k for j in range(s)] for k in range(s)]
    rhs = [mp.mpf(1) / (k + 1) for k in range(s)]
    x = _solve(V, rhs)
    return [x[j] for j in range(s)]


def _collocation_A(c):
    """Rows of A from C(s): sum_j a_ij c_j^(k-1) = c_i^k / k, k = 1..s."""
    s = len(c)
    V = [[c[j] ** k for j in range(s)] for k in range(s)]
    A = []
    for i in range(s):
        rhs = [c[i] ** (k + 1) / (k + 1) for k in range(s)]
        x = _solve(V, rhs)
        A.append([x[j] for j in range(s)])
    return A


def _to_np(A, b, c):
    return (np.array([[float(a) for a in row] for row in A], dtype=np.float64),
            np.array([float(x) for x in b], dtype=np.float64),
            np.array([float(x) for x in c], dtype=np.float64))


def gauss_legendre_mp(s):
    with mp.workdps(DPS):
        c = _roots_ascending(_shifted_legendre_coeffs(s))
        return _collocation_A(c), _b_from_nodes(c), c


def radau_iia_mp(s):
    with mp.workdps(DPS):
        ps = _shifted_legendre_coeffs(s)
        pm = _shifted_legendre_coeffs(s - 1) + [0]
        c = _roots_ascending([a - b for a, b in zip(ps, pm)])
        c[-1] = mp.mpf(1)  # the root at x = 1 is exact
        return _collocation_A(c), _b_from_nodes(c), c


def lobatto_iiic_mp(s):
    if s < 2:
        raise ValueError("Lobatto IIIC needs s >= 2")
    with mp.workdps(DPS):
        p = _shifted_legendre_coeffs(s - 1)
        # d/dx of P_{s-1}(2x-1), ascending coefficients
        dp = [k * p[k] for k in range(1, len(p))]
        inner = _roots_ascending(dp) if len(dp) > 1 else []
        c = [mp.mpf(0)] + inner + [mp.mpf(1)]
        b = _b_from_nodes(c)
        # row i: a_i1 = b_1; the remaining s-1 entries from C(s-1) with the
        # first column moved to the right-hand side.
        A = []
        V = [[c[j] ** k for j in range(1, s)] for k in range(s - 1)]
        for i in range(s):
            rhs = [c[i] ** (k + 1) / (k + 1) - b[0] * c[0] ** k for k in range(s - 1)]
            x = _solve(V, rhs)
            A.append([b[0]] + [x[j] for j in range(s - 1)])
        return A, b, c


_FAMILIES = {
    "gauss": gauss_legendre_mp,
    "radau_iia": radau_iia_mp,
    "lobatto_iiic": lobatto_iiic_mp,
}

ORDER = {
    "gauss": lambda s: 2 * s,
    "radau_iia": lambda s: 2 * s - 1,
    "lobatto_iiic": lambda s: 2 * s - 2,
}


def tableau_mp(family, s):
    """50-digit tableau ``(A, b, c)`` as nested lists of mpf."""
    return _FAMILIES[family](s)


def tableau(family, s):
    """float64 tableau ``(A, b, c)``: A is (s, s) row-major, b and c are (s,)."""
    return _to_np(*tableau_mp(family, s))
