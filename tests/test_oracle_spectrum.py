"""The condition-number and spectrum study of Sec. 4.3-4.4 (Tables 2-4 and
the eigenvalue figures there) on the finite-difference problems, exact
preconditioners, CPU only.

Pins of the routes themselves:
* the sine-basis block route (oracle/spectrum.py) equals the condition number
  and spectrum of the assembled dense matrices on small grids;
* the sparse-LU/Lanczos route equals the dense one on a small nonsymmetric
  (double-glazing) operator.

The study (the paper's values are for P2/P1 elements, so agreement is
approximate; the relations checked are stated per test and the computed
tables are printed):
* heat, right preconditioning, Radau IIA 2-7 at h_x = 2^-3 (Table 2): P_GSL
  has the smallest condition number for s = 2, 3, P_LD for s >= 4; P_DU the
  largest; every finite-difference value lies between 0.7 and 1.0 times the
  paper's;
* heat, left P_LD (Table 4, 2-D columns): within 20% of the paper's values
  (Radau IIA within 8%, Lobatto IIIC 11-15% below);
* double glazing eps = 0.005, h_x = 2^-4 (Table 3): left P_LD better than
  left P_GSL for every s and within 10% of the paper's values; right P_LD
  better than right P_GSL from s = 5 (the paper: from s = 4);
* eigenvalues (the figures of Sec. 4.3): for s = 3..5 every eigenvalue of the
  right-P_LD-preconditioned heat system lies closer to 1 than the farthest
  eigenvalue of P_J, P_GSL or P_DU does.
"""
import json
import os

import numpy as np
import pytest

from oracle.ldu import coefficient_matrix
from oracle.operators import double_glazing, heat_K
from oracle.spectrum import (dense_condition_number, heat_condition_number, heat_spectrum,
                             operator_condition_number)
from oracle.tableau import tableau

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden",
                                   "paper_condition_numbers.json")))
KINDS = ("J", "GSL", "DU", "LD")


def _ht(hx, p, q):
    return hx ** ((p + 1.0) / q)


@pytest.mark.parametrize("side", ["right", "left"])
@pytest.mark.parametrize("family,s", [("radau_iia", 3), ("gauss", 2), ("lobatto_iiic", 4)])
def test_block_route_equals_dense(side, family, s):
    n, h = 4, 0.07
    A, _, _ = tableau(family, s)
    K = heat_K(n)
    for kind in KINDS:
        At = coefficient_matrix(A, kind)
        a = heat_condition_number(A, At, h, n, side=side)
        d = dense_condition_number(A, At, h, K, side=side)
        assert a == pytest.approx(d, rel=1e-10), kind
    # spectrum: the union of the block eigenvalues
    At = coefficient_matrix(A, "LD")
    ev = heat_spectrum(A, At, h, n, side=side)
    F = np.kron(np.eye(s), np.eye(n * n)) + h * np.kron(A, K.toarray())
    P = np.kron(np.eye(s), np.eye(n * n)) + h * np.kron(At, K.toarray())
    X = F @ np.linalg.inv(P) if side == "right" else np.linalg.solve(P, F)
    evd = np.linalg.eigvals(X)
    # same set (nearest neighbours both ways) and same sum (multiplicities)
    dist = np.abs(ev[:, None] - evd[None, :])
    assert dist.min(axis=1).max() < 1e-8 and dist.min(axis=0).max() < 1e-8
    assert abs(ev.sum() - np.trace(X)) < 1e-10 * s * n * n


@pytest.mark.parametrize("side", ["right", "left"])
def test_operator_route_equals_dense(side):
    A, _, _ = tableau("radau_iia", 3)
    K = double_glazing(7, 0.005)[0]
    for kind in ("GSL", "LD"):
        At = coefficient_matrix(A, kind)
        d = dense_condition_number(A, At, 0.2, K, side=side)
        o = operator_condition_number(A, At, 0.2, K, side=side)
        assert o == pytest.approx(d, rel=1e-8)


def test_table2_heat_right():
    g = GOLD["table2_heat_right"]
    hx, n = 2.0 ** -3, 7
    rows = []
    for idx, s in enumerate(g["s"]):
        A, _, _ = tableau("radau_iia", s)
        h = _ht(hx, 2, 2 * s - 1)
        k = {kind: heat_condition_number(A, coefficient_matrix(A, kind), h, n) for kind in KINDS}
        rows.append((s, k))
        best = min(k, key=k.get)
        assert best == ("GSL" if s <= 3 else "LD"), (s, k)
        assert max(k, key=k.get) == "DU"
        for kind in KINDS:
            ratio = k[kind] / g[kind][idx]
            assert 0.7 <= ratio <= 1.0, (s, kind, k[kind], g[kind][idx])
    print("\nFD heat, right, h_x = 2^-3: " + "; ".join(
        "s=%d %s" % (s, " ".join("%s %.2f" % (q, v) for q, v in k.items())) for s, k in rows))


def test_table4_heat_left_ld():
    g = GOLD["table4_left_LD"]
    hx, n = 2.0 ** -3, 7
    for family, q_of in (("radau_iia", lambda s: 2 * s - 1), ("lobatto_iiic", lambda s: 2 * s - 2)):
        for idx, s in enumerate(g[family]["s"]):
            A, _, _ = tableau(family, s)
            h = _ht(hx, 2, q_of(s))
            k = heat_condition_number(A, coefficient_matrix(A, "LD"), h, n, side="left")
            assert abs(k / g[family]["2D"][idx] - 1.0) <= 0.20, (family, s, k)


def test_table3_double_glazing():
    g = GOLD["table3_double_glazing"]
    hx = 2.0 ** -4
    n = int(round(2.0 / hx)) - 1            # [-1, 1]^2 with spacing h_x
    K = double_glazing(n, 0.005)[0]
    out = []
    for idx, s in enumerate(g["s"]):
        A, _, _ = tableau("radau_iia", s)
        h = _ht(hx, 1, 2 * s - 1)
        k = {(side, kind): operator_condition_number(A, coefficient_matrix(A, kind), h, K, side)
             for side in ("left", "right") for kind in ("GSL", "LD")}
        out.append((s, k))
        assert k[("left", "LD")] < k[("left", "GSL")]
        assert abs(k[("left", "LD")] / g["left_LD"][idx] - 1.0) <= 0.10
        if s >= 5:
            assert k[("right", "LD")] < k[("right", "GSL")]
    print("\nFD double glazing: " + "; ".join(
        "s=%d %s" % (s, " ".join("%s-%s %.2f" % (a, b, v) for (a, b), v in k.items()))
        for s, k in out))


@pytest.mark.parametrize("s", [3, 4, 5])
def test_ld_clusters_eigenvalues_tightest(s):
    hx, n = 2.0 ** -3, 7
    A, _, _ = tableau("radau_iia", s)
    h = _ht(hx, 2, 2 * s - 1)
    radius = {kind: np.abs(heat_spectrum(A, coefficient_matrix(A, kind), h, n) - 1.0).max()
              for kind in KINDS}
    assert all(radius["LD"] < radius[kind] for kind in ("J", "GSL", "DU")), radius
