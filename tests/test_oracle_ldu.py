"""Pins for the LDU factorisation and the preconditioner coefficient matrices
(Sec. 4.1, (4.3); Sec. 4.3, Tables 2-4).

Independent facts used:
* the pivots of an LDU factorisation without pivoting are ratios of leading
  principal minors, ``d_k = det(A_k) / det(A_{k-1})``;
* Sec. 4.1: the leading minors are nonsingular for GL, Lobatto IIIC and
  Radau IIA at s = 2..7, and ``(LD)^-1 A = U``, ``A (DU)^-1 = L`` have all
  eigenvalues equal to one;
* Tables 2-4 print condition numbers of the preconditioned block systems on
  FEM grids.  For ``M = I`` and symmetric K the right-preconditioned
  operator is unitarily block-diagonal over the eigenvalues lam of K with
  blocks ``(I + h lam A)(I + h lam A~)^-1``, whose limit as ``h lam -> inf``
  is ``A A~^-1``; the printed values must sit at or a little above
  ``kappa(A A~^-1)`` (left: ``kappa(A~^-1 A)``).  A swapped reading (LD vs
  DU, tril vs LD, a transposed factor) moves the limit far outside that band.
"""
import json
import os

import numpy as np
import pytest

from oracle.ldu import coefficient_matrix, ldu
from oracle.tableau import tableau

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_condition_numbers.json")


def golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("family", ["gauss", "radau_iia", "lobatto_iiic"])
@pytest.mark.parametrize("s", range(2, 8))
def test_ldu_factors(family, s):
    A, b, c = tableau(family, s)
    L, d, U = ldu(A)
    assert np.allclose(np.diag(L), 1.0) and np.allclose(np.diag(U), 1.0)
    assert np.allclose(L, np.tril(L)) and np.allclose(U, np.triu(U))
    assert np.max(np.abs(L @ np.diag(d) @ U - A)) < 1e-15
    # pivots are ratios of leading principal minors
    minors = [1.0] + [np.linalg.det(A[:k, :k]) for k in range(1, s + 1)]
    for k in range(s):
        assert abs(minors[k + 1]) > 1e-12      # Sec. 4.1: nonsingular leading minors
        assert abs(d[k] - minors[k + 1] / minors[k]) < 1e-12 * max(1.0, abs(d[k]))
    # (LD)^-1 A = U and A (DU)^-1 = L, both with unit eigenvalues
    LD = coefficient_matrix(A, "LD")
    DU = coefficient_matrix(A, "DU")
    assert np.allclose(np.linalg.solve(LD, A), U, atol=1e-13)
    assert np.allclose(A @ np.linalg.inv(DU), L, atol=1e-13)
    # unit triangular, hence every eigenvalue is one (a numerical eig of this
    # defective matrix would only be accurate to eps^(1/s))
    for Mx in (np.linalg.solve(LD, A), A @ np.linalg.inv(DU)):
        assert np.allclose(np.diag(Mx), 1.0, atol=1e-13)
        assert (np.allclose(np.tril(Mx, -1), 0.0, atol=1e-13)
                or np.allclose(np.triu(Mx, 1), 0.0, atol=1e-13))


def test_ldu_zero_pivot_raises():
    with pytest.raises(ZeroDivisionError):
        ldu(np.array([[0.0, 1.0], [1.0, 0.0]]))


def test_pivots_positive_for_configured_tableaux():
    """All pivots of the configured tableaux are positive, so every block
    I + h d_i K is an M-matrix when K is one."""
    for family, s in [("gauss", 2), ("radau_iia", 3), ("radau_iia", 5), ("gauss", 7)]:
        A, b, c = tableau(family, s)
        assert np.all(ldu(A)[1] > 0)


def _band(paper, limit, lo=1.0 - 1e-3, hi=1.2):
    ratio = paper / limit
    assert lo <= ratio <= hi, (paper, limit, ratio)


@pytest.mark.parametrize("kind", ["J", "GSL", "DU", "LD"])
def test_table2_right_limits(kind):
    t = golden()["table2_heat_right"]
    for s, paper in zip(t["s"], t[kind]):
        A, b, c = tableau("radau_iia", s)
        At = coefficient_matrix(A, kind)
        _band(paper, np.linalg.cond(A @ np.linalg.inv(At)))


def test_table3_double_glazing_limits():
    t = golden()["table3_double_glazing"]
    for i, s in enumerate(t["s"]):
        A, b, c = tableau("radau_iia", s)
        for kind in ["GSL", "LD"]:
            At = coefficient_matrix(A, kind)
            _band(t["left_" + kind][i], np.linalg.cond(np.linalg.solve(At, A)))
            _band(t["right_" + kind][i], np.linalg.cond(A @ np.linalg.inv(At)))


def test_table4_left_LD_limits():
    t = golden()["table4_left_LD"]
    for family in ["radau_iia", "lobatto_iiic"]:
        for i, s in enumerate(t[family]["s"]):
            A, b, c = tableau(family, s)
            LD = coefficient_matrix(A, "LD")
            lim = np.linalg.cond(np.linalg.solve(LD, A))
            _band(t[family]["1D"][i], lim)
            _band(t[family]["2D"][i], lim)


def test_wrong_readings_leave_the_band():
    """Swapping the LD and DU readings, or using tril(A) for LD, puts the
    limits outside the band of Table 2 for s >= 4."""
    t = golden()["table2_heat_right"]
    for s, paper_ld in zip(t["s"], t["LD"]):
        if s < 4:
            continue
        A, b, c = tableau("radau_iia", s)
        for wrong in ["DU", "GSL", "J"]:
            At = coefficient_matrix(A, wrong)
            ratio = paper_ld / np.linalg.cond(A @ np.linalg.inv(At))
            assert not (0.999 <= ratio <= 1.2)
