"""Pins for the oracle's linear-element heat operators and its steps with a
mass matrix (Sec. 3.1: M_kl = int phi_k phi_l, F_kl = int grad phi_k . grad
phi_l; Sec. 4: I_s (x) M + h A (x) K).

* On the right-triangle mesh the P1 stiffness matrix is the five-point
  Laplacian stencil (the diagonal couplings cancel): compared with the
  finite-difference K times h^2.
* u^T M u is the L2 norm squared of the piecewise-linear interpolant and
  u^T K u its H1 seminorm squared: both evaluated here triangle by triangle
  with quadrature (edge midpoints, exact for quadratics) and the gradient of
  the linear interpolant, independently of the element matrices.
* Row sums of M are the area h^2 associated with a node away from the
  boundary.
* The exact step with M: through the generalised eigenvectors K v = lam M v
  (M-orthonormal) every mode is multiplied by the stability function
  R(z) = 1 + z b^T (I - z A)^-1 1 at z = -h lam.  The oracle's sparse stage
  solve (and its eigen-decoupled route) must reproduce that.
* The GPU-side builder (stencil formula) equals the oracle's assembly.
"""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.fem import p1_heat
from oracle.operators import heat_K
from oracle.step import DirectStepper, EigenStepper
from oracle.tableau import tableau
from paper_2010_11377_amd import problems


def _interp_values(u, n):
    """Values of u on the (n+2)^2 node grid including the zero boundary."""
    U = np.zeros((n + 2, n + 2))
    U[1:-1, 1:-1] = u.reshape(n, n)
    return U                                             # indexed [j, i]


def _triangles(n):
    """Vertex (i, j) triples of every triangle of the mesh."""
    for j in range(n + 1):
        for i in range(n + 1):
            yield ((i, j), (i + 1, j), (i + 1, j + 1))
            yield ((i, j), (i + 1, j + 1), (i, j + 1))


@pytest.mark.parametrize("n", [3, 6])
def test_stiffness_is_five_point_laplacian(n):
    M, K = p1_heat(n)
    h = 1.0 / (n + 1)
    assert abs(K - h * h * heat_K(n)).max() < 1e-13


@pytest.mark.parametrize("n,length", [(5, 1.0), (4, 2.0)])
def test_quadratic_forms_match_quadrature(n, length):
    M, K = p1_heat(n, length)
    h = length / (n + 1)
    u = np.random.default_rng(7).standard_normal(n * n)
    U = _interp_values(u, n)
    l2 = 0.0
    h1 = 0.0
    for tri in _triangles(n):
        vals = np.array([U[j, i] for i, j in tri])
        area = 0.5 * h * h
        mids = [(vals[a] + vals[b]) / 2 for a, b in ((0, 1), (1, 2), (2, 0))]
        l2 += area / 3.0 * sum(m * m for m in mids)
        P = np.array([[h * i, h * j, 1.0] for i, j in tri])
        gx, gy, _ = np.linalg.solve(P, vals)             # u = gx x + gy y + c
        h1 += area * (gx * gx + gy * gy)
    assert u @ (M @ u) == pytest.approx(l2, rel=1e-12)
    assert u @ (K @ u) == pytest.approx(h1, rel=1e-12)


def test_mass_row_sums_and_pattern():
    n = 6
    M, K = p1_heat(n)
    h = 1.0 / (n + 1)
    Md = M.toarray()
    assert np.allclose(Md, Md.T)
    for j in range(1, n - 1):
        for i in range(1, n - 1):
            p = j * n + i
            assert Md[p].sum() == pytest.approx(h * h, rel=1e-13)
            assert Md[p, p] == pytest.approx(h * h / 2, rel=1e-13)
            assert np.count_nonzero(Md[p]) == 7
            assert Md[p, p + n + 1] == pytest.approx(h * h / 12, rel=1e-13)  # north-east
            assert Md[p, p + n - 1] == 0.0                                   # north-west


@pytest.mark.parametrize("family,s,h", [("gauss", 2, 0.02), ("radau_iia", 3, 0.05),
                                         ("lobatto_iiic", 3, 0.1)])
def test_step_with_mass_is_stability_function_of_generalised_modes(family, s, h):
    n = 7
    M, K = p1_heat(n)
    A, b, _ = tableau(family, s)
    lam, V = sla.eigh(K.toarray(), M.toarray())           # V^T M V = I
    z = -h * lam
    R = np.array([1.0 + zz * (b @ np.linalg.solve(np.eye(s) - zz * A, np.ones(s))) for zz in z])
    u0 = np.random.default_rng(3).standard_normal(n * n)
    expect = V @ (R * (V.T @ (M @ u0)))
    got = DirectStepper(A, b, K, h, M=M).step(u0)
    got2 = EigenStepper(A, b, K, h, M=M).step(u0)
    scale = np.linalg.norm(expect)
    assert np.linalg.norm(got - expect) / scale < 1e-12
    assert np.linalg.norm(got2 - expect) / scale < 1e-12


@pytest.mark.parametrize("n", [4, 9])
def test_gpu_side_builder_matches_assembly(n):
    import scipy.sparse as sp
    Mo, Ko = p1_heat(n)
    (mp, mi, md), (kp, ki, kd) = problems.p1_heat(n)
    N = n * n
    Mg = sp.csr_matrix((md, mi, mp), shape=(N, N))
    Kg = sp.csr_matrix((kd, ki, kp), shape=(N, N))
    assert abs(Mg - Mo).max() < 1e-15
    assert abs(Kg - Ko).max() < 1e-13
