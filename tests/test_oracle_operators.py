"""Pins for the oracle's finite-difference operators (Sec. 3.1 and Sec. 3.2).

Independent facts used:
* the 2-D sine modes are eigenvectors of the five-point Dirichlet Laplacian
  with the closed-form eigenvalues ``4/h^2 (sin^2(p pi h/2) + sin^2(q pi h/2))``;
* central differences reproduce ``-eps Lap`` exactly on quadratics; first-order
  upwind differences of ``x^2`` give ``2x - h sign(w_x)``, a closed form that
  tells upwind from downwind;
* first-order upwinding makes the double-glazing operator an M-matrix;
* the kappa operator reduces to the heat operator for kappa = 1, is symmetric
  positive definite, and is a second-order accurate approximation of
  ``-div(kappa grad u)``.
"""
import numpy as np
import scipy.sparse.linalg as spla

from oracle.operators import (double_glazing, grid_coords, heat_eigenvalues, heat_K,
                              kappa_diffusion_K)


def test_heat_sine_modes_are_eigenvectors():
    n = 13
    K = heat_K(n)
    lam = heat_eigenvalues(n)
    x, y = grid_coords(n)
    for p, q in [(1, 1), (2, 5), (13, 7), (4, 4)]:
        v = np.sin(p * np.pi * x) * np.sin(q * np.pi * y)
        assert np.allclose(K @ v, lam[q - 1, p - 1] * v, rtol=1e-12, atol=1e-9)
    assert abs(K - K.T).max() == 0.0


def test_heat_scaled_square():
    n = 7
    K2 = heat_K(n, length=2.0)
    K1 = heat_K(n)
    assert np.allclose(K2.toarray() * 4.0, K1.toarray())


def test_double_glazing_quadratic_closed_form():
    n, eps = 15, 0.005
    h = 2.0 / (n + 1)

    def quad(xb, yb):
        return xb * xb

    K, g = double_glazing(n, eps, boundary=quad)
    x, y = grid_coords(n, -1.0, 1.0)
    wx = 2.0 * y * (1.0 - x * x)
    wy = -2.0 * x * (1.0 - y * y)
    lhs = K @ (x * x) - g
    # -eps * Lap(x^2) = -2 eps; upwind x-derivative of x^2 = 2x - h sign(wx); y part 0
    rhs = -2.0 * eps + wx * (2.0 * x - h * np.sign(wx))
    assert np.allclose(lhs, rhs, atol=1e-10)
    del wy

    def linear(xb, yb):
        return 0.3 + 2.0 * xb - 1.5 * yb

    K, g = double_glazing(n, eps, boundary=linear)
    lhs = K @ linear(x, y) - g
    assert np.allclose(lhs, 2.0 * wx - 1.5 * (-2.0 * x * (1.0 - y * y)), atol=1e-10)


def test_double_glazing_m_matrix_and_source():
    n, eps = 24, 0.005
    K, g = double_glazing(n, eps)
    Kd = K.toarray()
    off = Kd - np.diag(np.diag(Kd))
    assert off.max() <= 0.0
    assert np.all(np.diag(Kd) + off.sum(axis=1) >= -1e-9)
    # the source sits on the column next to the east wall and is positive there
    G = g.reshape(n, n)
    assert np.all(G[:, -1] > 0) and np.all(G[:, :-1] == 0.0)
    # steady state lies in [0, 1] (discrete maximum principle of an M-matrix)
    u = spla.spsolve(K.tocsc(), g)
    assert u.min() > -1e-12 and u.max() < 1.0 + 1e-12


def test_kappa_reduces_to_heat_and_is_spd():
    n = 9
    K = kappa_diffusion_K(np.ones((n + 2, n + 2)))
    assert np.allclose(K.toarray(), heat_K(n).toarray(), rtol=1e-13, atol=1e-9)
    rng = np.random.default_rng(0)
    kn = np.exp(0.5 * rng.standard_normal((n + 2, n + 2)))
    K = kappa_diffusion_K(kn)
    Kd = K.toarray()
    assert np.allclose(Kd, Kd.T)
    assert np.linalg.eigvalsh(Kd).min() > 0


def test_kappa_second_order_consistency():
    """-div((1 + x + y^2) grad u) for u = sin(pi x) sin(pi y): error O(h^2)."""
    errs = []
    for n in [15, 31, 63]:
        t = np.linspace(0.0, 1.0, n + 2)
        X, Y = np.meshgrid(t, t, indexing="xy")
        kn = 1.0 + X + Y * Y
        K = kappa_diffusion_K(kn)
        x, y = grid_coords(n)
        u = np.sin(np.pi * x) * np.sin(np.pi * y)
        kap = 1.0 + x + y * y
        ux = np.pi * np.cos(np.pi * x) * np.sin(np.pi * y)
        uy = np.pi * np.sin(np.pi * x) * np.cos(np.pi * y)
        exact = -(1.0 * ux + kap * (-np.pi ** 2) * u + 2.0 * y * uy + kap * (-np.pi ** 2) * u)
        errs.append(np.max(np.abs(K @ u - exact)))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5
