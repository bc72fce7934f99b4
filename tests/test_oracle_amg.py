"""Pins for the oracle's multigrid V-cycle (the approximate block subsolve of
Sec. 4.2; the components are the reading stated in ``oracle/amg.py``).

Independent facts used:
* hand-derived Galerkin stencils of the heat operator: in 1-D, R K P is
  h^-2 (-1/2, 1, -1/2) inside and h^-2 (w + 1/2, -1/2) at a Dirichlet end,
  and R P is (1/4, 3/2, 1/4) inside and (w + 3/4, 1/4) at the end, with
  w = 2/3 the boundary interpolation weight of the finest level; the 2-D
  stencils are the tensor sums of these;
* linear interpolation reproduces the linear function that vanishes at the
  boundary, which pins the boundary weights of every level;
* the V-cycle equals a dense-matrix formulation of the same cycle, built from
  the error-propagation operators of each colour half sweep;
* with one level the cycle is the exact solve; with exact subsolves the block
  substitution equals the oracle's exact P^-1;
* the V-cycle convergence factor of the heat blocks does not grow with the
  grid (the point of multigrid) and stays small.
"""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from oracle.amg import (apply_vcycle_preconditioner, colours, ends_cycle, hierarchy, prolongation,
                        restriction, vcycle)
from oracle.ldu import coefficient_matrix
from oracle.operators import double_glazing, heat_K, kappa_diffusion_K
from oracle.precond import apply_inverse
from oracle.tableau import tableau
from paper_2010_11377_amd.workloads import gaussian_random_field


def _stencil(A, nx, i, j):
    """3 x 3 stencil of row (i, j) of A, [dy + 1][dx + 1]."""
    row = A.getrow(j * nx + i).toarray().ravel()
    st = np.zeros((3, 3))
    for dy in (-1, 0, 1):
        for dx in (-1, 0, 1):
            ii, jj = i + dx, j + dy
            if 0 <= ii < nx and 0 <= jj < A.shape[0] // nx:
                st[dy + 1, dx + 1] = row[jj * nx + ii]
    return st


def test_transfer_operators():
    nx, ny = 8, 6
    P, R = prolongation(nx, ny), restriction(nx, ny)
    assert P.shape == (48, 12) and R.shape == (12, 48)
    # R sums 2 x 2 cells
    assert np.allclose(R @ np.ones(48), 4.0)
    # P reproduces constants away from the boundary, 2/3 per boundary side
    p1 = (P @ np.ones(12)).reshape(ny, nx)
    assert np.allclose(p1[1:-1, 1:-1], 1.0)
    assert np.isclose(p1[0, 3], 2 / 3) and np.isclose(p1[0, 0], 4 / 9)
    # weights of fine node (3, 2) (odd column, even row): coarse (1, 1) 9/16,
    # (2, 1) 3/16, (1, 0) 3/16, (2, 0) 1/16
    row = P.getrow(2 * nx + 3).toarray().ravel().reshape(ny // 2, nx // 2)
    assert np.isclose(row[1, 1], 9 / 16) and np.isclose(row[1, 2], 3 / 16)
    assert np.isclose(row[0, 1], 3 / 16) and np.isclose(row[0, 2], 1 / 16)
    assert np.isclose(row.sum(), 1.0)


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_interpolation_of_boundary_linear_functions(level):
    """On level l the finest spacing is h and node i sits at distance
    d_l + i 2^l h from the boundary, d_l = (2^l + 1) h / 2.  The function
    f(x) = x (distance from the left boundary) is linear and vanishes at the
    boundary, so linear interpolation from the coarse nodes must reproduce
    it exactly at the first fine nodes (away from the right end)."""
    from oracle.amg import _interp_1d, boundary_weight
    n = 16
    d = lambda l: (2.0 ** l + 1.0) / 2.0
    fine = d(level) + np.arange(n) * 2.0 ** level
    coarse = d(level + 1) + np.arange(n // 2) * 2.0 ** (level + 1)
    P1 = _interp_1d(n, boundary_weight(level))
    assert np.allclose((P1 @ coarse)[: n // 2], fine[: n // 2], rtol=1e-14)


def test_galerkin_heat_stencils():
    n = 16
    h2 = 1.0 / (1.0 / (n + 1)) ** 2
    lev = hierarchy(heat_K(n), n, n, coarse_max=1)
    _, _, S1, K1 = lev[1][:4]
    nc = n // 2
    k_in = h2 * np.array([[-0.25, -0.5, -0.25], [-0.5, 3.0, -0.5], [-0.25, -0.5, -0.25]])
    assert np.allclose(_stencil(K1, nc, 3, 4), k_in, rtol=1e-13, atol=1e-9)
    m1 = np.array([0.25, 1.5, 0.25])
    assert np.allclose(_stencil(S1, nc, 3, 4), np.outer(m1, m1), rtol=1e-14)
    # w = 2/3: corner 2 (7/6)(17/12) = 119/36; edge (x = 0, interior y):
    # (7/6)(3/2) + (17/12)(1) = 19/6; the corner of S_1 is (17/12)^2
    assert np.isclose(K1[0, 0], 119 / 36 * h2, rtol=1e-13)
    assert np.isclose(K1[4 * nc, 4 * nc], 19 / 6 * h2, rtol=1e-13)
    assert np.isclose(K1[0, 1], -0.5 * 17 / 12 * h2 + 7 / 6 * 0.25 * h2, rtol=1e-13)
    assert np.isclose(S1[0, 0], (17 / 12) ** 2, rtol=1e-14)
    # row sums vanish inside (constants are in the kernel of the Laplacian)
    assert abs(K1.getrow(4 * nc + 3).sum()) < 1e-9 * h2
    # levels stop at coarse_max or an odd dimension
    assert [(l[0], l[1]) for l in hierarchy(heat_K(12), 12, 12, coarse_max=1)] == \
        [(12, 12), (6, 6), (3, 3)]
    assert len(hierarchy(heat_K(16), 16, 16, coarse_max=64)) == 2


def _dense_cycle(levels, tau, nu, l=0):
    """Approximate inverse of the V(nu, nu)-cycle on level l as a dense
    matrix: B = (I - S_post (I - P B_c R D) S_pre) D^-1, with the colour half
    sweep error propagators G_c = I - Pi_c diag(D)^-1 D."""
    nx, ny, S, K, P, R = levels[l]
    D = (S + tau * K).toarray()
    n = D.shape[0]
    if P is None:
        return np.linalg.inv(D)
    col = colours(nx, ny)
    G = [np.eye(n) - np.diag((col == c) / np.diag(D)) @ D for c in (0, 1)]
    pre = np.linalg.matrix_power(G[1] @ G[0], nu)
    post = np.linalg.matrix_power(G[0] @ G[1], nu)
    Bc = _dense_cycle(levels, tau, nu, l + 1)
    E = post @ (np.eye(n) - P.toarray() @ Bc @ R.toarray() @ D) @ pre
    return (np.eye(n) - E) @ np.linalg.inv(D)


@pytest.mark.parametrize("problem", ["heat", "dg", "kappa"])
@pytest.mark.parametrize("nu", [1, 2])
def test_vcycle_equals_dense_formulation(problem, nu):
    n, tau = 16, 3e-4
    if problem == "heat":
        K = heat_K(n)
    elif problem == "dg":
        K = double_glazing(n, 0.005)[0]
    else:
        K = kappa_diffusion_K(np.exp(gaussian_random_field(n + 2, seed=3)))
    levels = hierarchy(K, n, n, coarse_max=16)
    assert len(levels) == 3          # 16^2 -> 8^2 -> 4^2
    b = np.random.default_rng(8).standard_normal(n * n)
    x = vcycle(levels, tau, b, nu)
    ref = _dense_cycle(levels, tau, nu) @ b
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)


def test_one_level_is_exact_and_rectangular_grids():
    nx, ny, tau = 12, 10, 1e-3
    K = heat_K(nx, ny=ny)
    assert K.shape == (120, 120)
    b = np.random.default_rng(9).standard_normal(nx * ny)
    lev = hierarchy(K, nx, ny, coarse_max=1000)
    assert len(lev) == 1
    x = vcycle(lev, tau, b)
    ref = spla.spsolve((sp.identity(nx * ny) + tau * K).tocsc(), b)
    assert np.linalg.norm(x - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("kind", ["LD", "DU", "GSL", "J"])
def test_block_substitution_with_exact_subsolves(kind):
    n, h = 10, 2e-3
    A, _, _ = tableau("radau_iia", 3)
    K = double_glazing(n, 0.005)[0]
    At = coefficient_matrix(A, kind)
    v = np.random.default_rng(4).standard_normal((3, n * n))
    z = apply_vcycle_preconditioner(At, K, h, v, n, n, coarse_max=10 ** 6)
    ref = apply_inverse(At, K, h, v)
    assert np.linalg.norm(z - ref) <= 1e-12 * np.linalg.norm(ref)


def test_convergence_factor_is_grid_independent():
    """Stationary iteration x <- x + V(b - D x) in the Poisson limit of the
    heat blocks (tau h^-2 >> 1): the factor per cycle stays below 0.1 and
    does not grow from 32^2 to 256^2."""
    tau = 1e3
    rates = []
    for n in (32, 64, 128, 256):
        K = heat_K(n)
        D = (sp.identity(n * n) + tau * K).tocsr()
        levels = hierarchy(K, n, n, coarse_max=64)
        b = np.random.default_rng(n).standard_normal(n * n)
        x = np.zeros(n * n)
        res = [np.linalg.norm(b)]
        for _ in range(6):
            x = x + vcycle(levels, tau, b - D @ x)
            res.append(np.linalg.norm(b - D @ x))
        rates.append((res[-1] / res[2]) ** 0.25)
    assert max(rates) < 0.1
    assert rates[-1] < 1.1 * rates[0]


@pytest.mark.parametrize("kind", ["LD", "GSL"])
def test_block_substitution_with_mass_matrix(kind):
    """With a mass matrix (linear elements) and exact subsolves the block
    substitution solves P z = v for the assembled P = I (x) M + h A~ (x) K."""
    from oracle.fem import p1_heat
    from oracle.precond import assemble
    n, h = 9, 0.05
    M, K = p1_heat(n)
    A, _, _ = tableau("radau_iia", 3)
    At = coefficient_matrix(A, kind)
    v = np.random.default_rng(5).standard_normal((3, n * n))
    z = apply_vcycle_preconditioner(At, K, h, v, n, n, coarse_max=10 ** 6, M=M)
    ref = spla.spsolve(assemble(At, K, h, M), v.ravel()).reshape(3, n * n)
    assert np.linalg.norm(z - ref) <= 1e-12 * np.linalg.norm(ref)


def test_mass_matrix_convergence_factor():
    """V-cycles on M + tau K (linear elements, Galerkin hierarchy from M and
    K) contract by less than 0.1 per cycle on every grid from 32^2 to 128^2."""
    from oracle.fem import p1_heat
    for n in (32, 64, 128):
        M, K = p1_heat(n)
        lev = hierarchy(K, n, n, 64, M)
        for tau in (1e-2, 1.0):
            D = (lev[0][2] + tau * lev[0][3]).tocsr()
            e = np.random.default_rng(0).standard_normal(n * n)
            for _ in range(8):
                e2 = e - vcycle(lev, tau, D @ e)
                f = np.linalg.norm(e2) / np.linalg.norm(e)
                e = e2 / np.linalg.norm(e2)
            assert f < 0.1, (n, tau, f)


def test_constant_interpolation_is_parent_value():
    nx, ny = 6, 4
    P = prolongation(nx, ny, 0, "constant")
    xc = np.arange(1.0, 1.0 + (nx // 2) * (ny // 2))
    xf = P @ xc
    for j in range(ny):
        for i in range(nx):
            assert xf[j * nx + i] == xc[(j // 2) * (nx // 2) + i // 2]


def _m_matrix(D):
    """Non-positive off-diagonals and non-negative row sums."""
    D = sp.csr_matrix(D)
    off = D - sp.diags(D.diagonal())
    return off.data.max(initial=0.0) <= 1e-14 * D.diagonal().max() and \
        (np.asarray(D.sum(axis=1)).ravel() >= -1e-12 * D.diagonal().max()).all()


def test_constant_interpolation_keeps_m_matrices_and_converges():
    """Double glazing, eps = 0.005, tau = 1: with piecewise-constant
    interpolation every Galerkin level is an M-matrix and the V-cycle
    contracts; with linear interpolation coarse levels lose the property
    and the cycle diverges (the reason for the option)."""
    n, tau = 64, 1.0
    K = double_glazing(n, 0.005)[0]
    factors = {}
    for interp in ("constant", "linear"):
        lev = hierarchy(K, n, n, 64, interp=interp)
        mm = [_m_matrix(S + tau * Kl) for (_, _, S, Kl, _, _) in lev]
        D = (lev[0][2] + tau * lev[0][3]).tocsr()
        e = np.random.default_rng(0).standard_normal(n * n)
        for _ in range(8):
            e2 = e - vcycle(lev, tau, D @ e)
            f = np.linalg.norm(e2) / np.linalg.norm(e)
            e = e2 / np.linalg.norm(e2)
        factors[interp] = (all(mm), f)
    assert factors["constant"][0] and factors["constant"][1] < 0.75
    assert not factors["linear"][0] and factors["linear"][1] > 1.0


# ---- early end of the cycle (coarse_ratio) ---------------------------------

def _heat_ratio_closed_forms(n):
    """tau-free ratios max_p (K_l)_pp / (S_l)_pp on levels 0 and 1 of the FD
    heat hierarchy, from the closed-form stencils above: level 0 K = 4 h^-2,
    S = 1; level 1 interior K = 3 h^-2, S = 1.5^2; edge K = 19/6 h^-2,
    S = 1.5 (17/12); corner K = 119/36 h^-2, S = (17/12)^2."""
    h2 = float(n + 1) ** 2
    r0 = 4.0 * h2
    r1 = h2 * max(3.0 / 2.25, (19.0 / 6.0) / (1.5 * 17.0 / 12.0), (119.0 / 36.0) / (17.0 / 12.0) ** 2)
    return r0, r1


def test_cycle_end_rule_closed_form():
    n, tau = 16, 1e-3
    lev = hierarchy(heat_K(n), n, n, coarse_max=1)
    r0, r1 = _heat_ratio_closed_forms(n)
    (_, _, S0, K0) = lev[0][:4]
    (_, _, S1, K1) = lev[1][:4]
    for S, Kl, r in ((S0, K0, r0), (S1, K1, r1)):
        assert ends_cycle(S, Kl, tau, tau * r * (1 + 1e-9))
        assert not ends_cycle(S, Kl, tau, tau * r * (1 - 1e-9))
    assert not ends_cycle(S0, K0, tau, 0.0) and not ends_cycle(S0, K0, 0.0, 1e9)


def test_cycle_ending_on_level_1_equals_dense_formulation():
    """The cycle that ends on level 1 is the V-cycle whose level-1 coarse
    correction is zero: B_1 = (I - post_1 pre_1) D_1^-1."""
    n, tau, nu = 16, 3e-2, 2
    lev = hierarchy(heat_K(n), n, n, coarse_max=16)
    r0, r1 = _heat_ratio_closed_forms(n)
    ratio = tau * 0.5 * (r0 + r1)           # between the two levels' ratios
    b = np.random.default_rng(18).standard_normal(n * n)
    x = vcycle(lev, tau, b, nu, coarse_ratio=ratio)

    def dense(l):
        nx, ny, S, K, P, R = lev[l]
        D = (S + tau * K).toarray()
        m = D.shape[0]
        col = colours(nx, ny)
        G = [np.eye(m) - np.diag((col == c) / np.diag(D)) @ D for c in (0, 1)]
        pre = np.linalg.matrix_power(G[1] @ G[0], nu)
        post = np.linalg.matrix_power(G[0] @ G[1], nu)
        corr = np.zeros((m, m)) if l == 1 else P.toarray() @ dense(l + 1) @ R.toarray() @ D
        return (np.eye(m) - post @ (np.eye(m) - corr) @ pre) @ np.linalg.inv(D)

    ref = dense(0) @ b
    assert np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
    # and it differs from the full cycle
    assert np.linalg.norm(vcycle(lev, tau, b, nu) - x) > 1e-6 * np.linalg.norm(x)


def test_cycle_ending_on_the_finest_level_is_smoothing():
    """Ending on level 0: nu red-black sweeps (colour 0, 1) then nu (colour 1,
    0) from zero, written here as exact solves of the diagonal colour blocks."""
    n, tau, nu = 12, 1e-2, 2
    K = double_glazing(n, 0.005)[0]
    lev = hierarchy(K, n, n, coarse_max=16)
    b = np.random.default_rng(19).standard_normal(n * n)
    x = vcycle(lev, tau, b, nu, coarse_ratio=1e12)
    D = (sp.identity(n * n) + tau * K).tocsr()
    col = colours(n, n)
    y = np.zeros(n * n)
    for c in [0, 1] * nu + [1, 0] * nu:
        m = np.flatnonzero(col == c)
        o = np.flatnonzero(col != c)
        Dcc = D[m][:, m].toarray()
        y[m] = np.linalg.solve(Dcc, b[m] - D[m][:, o] @ y[o])
    assert np.linalg.norm(x - y) <= 1e-12 * np.linalg.norm(y)


def _cheb_T(k, x):
    """Chebyshev polynomial of the first kind, any real x."""
    x = np.asarray(x, dtype=np.float64)
    return np.where(np.abs(x) <= 1.0, np.cos(k * np.arccos(np.clip(x, -1.0, 1.0))),
                    np.cosh(k * np.arccosh(np.maximum(np.abs(x), 1.0))) * np.sign(x) ** k)


def _error_matrix(smooth, D):
    """Error propagation matrix of one smoother application from columns:
    with b = D x_true and x0 = 0 the error after smoothing is E x_true."""
    n = D.shape[0]
    E = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        E[:, j] = e - smooth(D @ e)
    return E


@pytest.mark.parametrize("degree", [1, 2, 3])
def test_chebyshev_smoother_error_polynomial(degree):
    """The Chebyshev smoother multiplies the error by the scaled Chebyshev
    polynomial of D^-1 A on [lam_max/10, 1.1 lam_max]: checked on the
    eigenvectors of D^-1 A of a heat block (closed form of the semi-
    iteration), and the Gershgorin bound is >= the largest eigenvalue."""
    from oracle.amg import chebyshev, gershgorin_bound
    n, tau = 6, 2e-3
    D = (sp.identity(n * n) + tau * heat_K(n)).tocsr()
    diag = D.diagonal()
    lam_max = gershgorin_bound(D, diag)
    Dd = D.toarray()
    mu = np.linalg.eigvals(np.diag(1.0 / diag) @ Dd).real
    assert lam_max >= mu.max() - 1e-12
    E = _error_matrix(lambda b: chebyshev(D, diag, b, np.zeros_like(b), degree, lam_max), D)
    a, c = lam_max / 10.0, 1.1 * lam_max
    theta, delta = 0.5 * (a + c), 0.5 * (c - a)
    # D^-1 A = S diag(mu) S^-1 with S = diag^-1/2 Q (Q orthogonal eigenvectors
    # of the symmetric diag^-1/2 A diag^-1/2)
    Dh = np.diag(diag ** -0.5)
    w, Q = np.linalg.eigh(Dh @ Dd @ Dh)
    Sm = Dh @ Q
    p = _cheb_T(degree, (theta - w) / delta) / _cheb_T(degree, theta / delta)
    ref = Sm @ np.diag(p) @ np.linalg.inv(Sm)
    assert np.max(np.abs(E - ref)) <= 1e-12


def test_jacobi_smoother_error_matrix():
    from oracle.amg import jacobi
    n, tau, omega = 6, 2e-3, 0.8
    D = (sp.identity(n * n) + tau * double_glazing(n, 0.005)[0]).tocsr()
    diag = D.diagonal()
    E = _error_matrix(lambda b: jacobi(D, diag, b, np.zeros_like(b), omega), D)
    ref = np.eye(n * n) - omega * np.diag(1.0 / diag) @ D.toarray()
    assert np.max(np.abs(E - ref)) <= 1e-14


def _dense_cycle_smoother(levels, tau, nu, G_pre, G_post, l=0):
    """Dense V-cycle with given per-level smoother error propagators."""
    nx, ny, S, K, P, R = levels[l]
    D = (S + tau * K).toarray()
    n = D.shape[0]
    if P is None:
        return np.linalg.inv(D)
    pre = np.linalg.matrix_power(G_pre(D), nu)
    post = np.linalg.matrix_power(G_post(D), nu)
    Bc = _dense_cycle_smoother(levels, tau, nu, G_pre, G_post, l + 1)
    E = post @ (np.eye(n) - P.toarray() @ Bc @ R.toarray() @ D) @ pre
    return (np.eye(n) - E) @ np.linalg.inv(D)


@pytest.mark.parametrize("smoother", ["jacobi", "chebyshev"])
def test_vcycle_other_smoothers_dense_and_symmetric(smoother):
    """V-cycles with damped Jacobi (omega 0.8) or degree-2 Chebyshev smoothing
    equal the dense formulation built from the smoothers' closed-form error
    polynomials, and on a symmetric heat block with R = P^T (the constant
    interpolation) their operator is symmetric (pre- and post-smoother are the
    same polynomial in D^-1 A)."""
    from oracle.amg import gershgorin_bound
    n, tau, nu = 16, 3e-4, 2
    levels = hierarchy(heat_K(n), n, n, coarse_max=16)

    def G(D):
        d = np.diag(D)
        M = np.diag(1.0 / d) @ D
        if smoother == "jacobi":
            return np.eye(D.shape[0]) - 0.8 * M
        lam = float(np.max(np.abs(D).sum(axis=1) / np.abs(d)))
        a, c = lam / 10.0, 1.1 * lam
        theta, delta = 0.5 * (a + c), 0.5 * (c - a)
        # T_2((theta - x)/delta) / T_2(theta/delta) as a matrix polynomial
        Y = (theta * np.eye(D.shape[0]) - M) / delta
        return (2.0 * Y @ Y - np.eye(D.shape[0])) / (2.0 * (theta / delta) ** 2 - 1.0)

    B = _dense_cycle_smoother(levels, tau, nu, G, G)
    b = np.random.default_rng(8).standard_normal(n * n)
    x = vcycle(levels, tau, b, nu, smoother=smoother)
    assert np.linalg.norm(x - B @ b) <= 1e-12 * np.linalg.norm(x)
    Bx = np.column_stack([vcycle(levels, tau, e, nu, smoother=smoother)
                          for e in np.eye(n * n)[:, :64].T])
    Bfull = B[:, :64]
    assert np.max(np.abs(Bx - Bfull)) <= 1e-12 * np.max(np.abs(Bfull))
    lev_c = hierarchy(heat_K(n), n, n, coarse_max=16, interp="constant")
    Bc = np.column_stack([vcycle(lev_c, tau, e, nu, smoother=smoother) for e in np.eye(n * n)])
    assert np.max(np.abs(Bc - Bc.T)) <= 1e-12 * np.max(np.abs(Bc))
    # red-black Gauss-Seidel (colours 0,1 before and 1,0 after) too
    Bg = np.column_stack([vcycle(lev_c, tau, e, nu) for e in np.eye(n * n)])
    assert np.max(np.abs(Bg - Bg.T)) <= 1e-12 * np.max(np.abs(Bg))
    assert gershgorin_bound(sp.csr_matrix(np.eye(3)), np.ones(3)) == 1.0
