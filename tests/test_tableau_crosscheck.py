"""The GPU path's tableau generator (``paper_2010_11377_amd.tableaux``: numpy
Legendre roots refined by Newton steps, Lagrange integrals by Gauss
quadrature) against the oracle's (50-digit collocation, ``oracle.tableau``).

Both compute the collocation tableaux of Sec. 2 (Table 1) from their
definitions by different routes; the oracle's is pinned by the order
conditions and the Pade stability functions in ``test_oracle_tableau.py``.
Agreement to 1e-14 in every entry of (A, b, c) ties the coefficients that the
HIP library receives to those pins.
"""
import numpy as np
import pytest

from oracle.tableau import tableau as oracle_tableau
from paper_2010_11377_amd import tableaux

CASES = ([("gauss", s) for s in range(1, 9)] + [("radau_iia", s) for s in range(1, 9)]
         + [("lobatto_iiic", s) for s in range(2, 9)])


@pytest.mark.parametrize("family,s", CASES)
def test_product_tableau_equals_oracle(family, s):
    A, b, c = tableaux.tableau(family, s)
    Ao, bo, co = oracle_tableau(family, s)
    assert A.shape == Ao.shape == (s, s)
    assert np.max(np.abs(A - Ao)) <= 1e-14
    assert np.max(np.abs(b - bo)) <= 1e-14
    assert np.max(np.abs(c - co)) <= 1e-14
