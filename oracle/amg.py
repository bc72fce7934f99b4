"""The geometric-algebraic multigrid V-cycle used as the approximate subsolve
of the block preconditioner (Sec. 4.2), written out plainly in FP64.

The paper states only that each diagonal block ``M + h A~_ii K`` is
approximated by one algebraic multigrid V-cycle; the components below are the
reading taken for the structured finite-difference grids of Sec. 3:

* coarsening: 2 x 2 cells; coarse node (I, J) owns fine columns 2I, 2I+1 and
  rows 2J, 2J+1;
* prolongation P: linear interpolation in each direction between the
  coarse nodes (the centres of the 2 x 2 cells), tensorised in 2-D: fine
  2I takes 3/4 of coarse I and 1/4 of I-1, fine 2I+1 takes 3/4 of I and 1/4
  of I+1.  The outermost fine node has no coarse neighbour beyond it; it
  interpolates between coarse node 0 and the Dirichlet boundary value zero
  at the boundary's true position.  On the finest grid the boundary lies one
  spacing h beyond the outermost node, and each coarsening moves the
  outermost node inwards by half the fine spacing, so on level l the
  outermost node is (2^l + 1) h / 2 from the boundary and its weight is
  w_l = (2^l + 1) / (2^(l+1) + 1) (2/3, 3/5, 5/9, ...), not 3/4;
* restriction R: the sum over each 2 x 2 cell (the transpose of piecewise
  constant interpolation);
* the alternative prolongation ``interp="constant"`` is P = R^T (every fine
  node takes its coarse parent's value).  It keeps the Galerkin coarse
  operators of an M-matrix M-matrices, which the linear one does not for the
  advection-dominated double glazing at large time steps;
* coarse operators by the Galerkin product: S_{l+1} = R S_l P, K_{l+1} =
  R K_l P with S_0 = M = I, and the stage-i block on level l is
  D_{i,l} = S_l + tau_i K_l (tau_i = h A~_ii);
* levels are added while the level has more than ``coarse_max`` nodes and
  both dimensions are even; the last level is solved exactly;
* smoother: red-black (colour (i + j) mod 2) point relaxation, Jacobi within
  a colour (for five-point operators that is Gauss-Seidel), ``nu`` sweeps of
  colours 0 then 1 before the coarse correction and ``nu`` sweeps of colours
  1 then 0 after it;
* other smoothers, for the comparison with the reading above
  (``smoother=``): ``"jacobi"``, ``nu`` damped Jacobi sweeps
  x += omega D^-1 (b - A x) before and after the coarse correction;
  ``"chebyshev"``, ``nu`` applications of the degree-``cheb_degree``
  Chebyshev iteration for D^-1 A on [lam_max / 10, 1.1 lam_max], lam_max the
  Gershgorin bound of D^-1 A (symmetric positive definite blocks only);
* one V-cycle from a zero initial guess per block;
* optional early end of the cycle (``coarse_ratio`` > 0): the first level
  whose block is dominated by its mass part, tau_i max_p (K_l)_pp / (S_l)_pp
  <= coarse_ratio, runs its pre- and post-smoothing with no coarse
  correction (the levels below it are not visited).  Such a block is close
  to its mass matrix, which the smoother alone reduces well, so the coarser
  levels add little; in algebraic multigrid terms the hierarchy of that
  block stops where the operator stops being dominated by the stiffness
  part.

Parity of this reading against the paper is unpinned (the paper gives no AMG
details); the tests pin the code against closed-form Galerkin stencils, a
dense-matrix formulation of the cycle, and the exact solve when one level
remains.

Test infrastructure only (see the package docstring).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def boundary_weight(level):
    """Weight of the outermost coarse node at the outermost fine node of
    level ``level``: the ratio of their distances to the boundary."""
    return (2.0 ** level + 1.0) / (2.0 ** (level + 1) + 1.0)


def _interp_1d(n, wb):
    """Linear interpolation from n // 2 coarse nodes to n fine nodes: fine 2I
    takes 3/4 of I and 1/4 of I-1, fine 2I+1 takes 3/4 of I and 1/4 of I+1;
    a fine node whose second coarse node would lie outside the grid takes wb
    of its own coarse node (the boundary value is zero)."""
    nc = n // 2
    rows, cols, vals = [], [], []
    for i in range(n):
        I = i // 2
        nb = I - 1 if i % 2 == 0 else I + 1
        rows.append(i)
        cols.append(I)
        if 0 <= nb < nc:
            vals.append(0.75)
            rows.append(i)
            cols.append(nb)
            vals.append(0.25)
        else:
            vals.append(wb)
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, nc))


def _sum_1d(n):
    """Sum of fine nodes 2I and 2I+1 into coarse node I."""
    nc = n // 2
    rows = np.repeat(np.arange(nc), 2)
    cols = np.arange(2 * nc)
    return sp.csr_matrix((np.ones(2 * nc), (rows, cols)), shape=(nc, n))


def prolongation(nx, ny, level=0, interp="linear"):
    """P from level+1 to level, x-fastest ordering (index = y * nx + x)."""
    if interp == "constant":
        return restriction(nx, ny).T.tocsr()
    if interp != "linear":
        raise ValueError(interp)
    wb = boundary_weight(level)
    return sp.kron(_interp_1d(ny, wb), _interp_1d(nx, wb), format="csr")


def restriction(nx, ny):
    return sp.kron(_sum_1d(ny), _sum_1d(nx), format="csr")


def hierarchy(K, nx, ny, coarse_max=64, M=None, interp="linear"):
    """[(nx_l, ny_l, S_l, K_l, P_l, R_l)] with P_l, R_l the transfers between
    level l and l+1 (None on the last level); S_0 = M (the identity if None)."""
    levels = []
    S = sp.identity(nx * ny, format="csr") if M is None else sp.csr_matrix(M)
    Kl = sp.csr_matrix(K)
    while True:
        if nx * ny > coarse_max and nx % 2 == 0 and ny % 2 == 0 and nx >= 2 and ny >= 2:
            P, R = prolongation(nx, ny, len(levels), interp), restriction(nx, ny)
            levels.append((nx, ny, S, Kl, P, R))
            S = (R @ S @ P).tocsr()
            Kl = (R @ Kl @ P).tocsr()
            nx, ny = nx // 2, ny // 2
        else:
            levels.append((nx, ny, S, Kl, None, None))
            return levels


def colours(nx, ny):
    """Colour (i + j) mod 2 of every node, x-fastest."""
    j, i = np.divmod(np.arange(nx * ny), nx)
    return (i + j) % 2


def relax(D, diag, col, b, x, colour):
    """One colour half sweep: every node of that colour takes the value that
    zeroes its residual, all from the same old x (Jacobi within the colour)."""
    r = b - D @ x
    m = col == colour
    x = x.copy()
    x[m] += r[m] / diag[m]
    return x


def jacobi(D, diag, b, x, omega):
    """One damped Jacobi sweep x += omega D^-1 (b - A x)."""
    return x + omega * (b - D @ x) / diag


def gershgorin_bound(D, diag):
    """An upper bound of the spectrum of D^-1 A: the largest row sum of
    |D^-1 A|."""
    return float(np.max(np.asarray(abs(D).sum(axis=1)).ravel() / np.abs(diag)))


def chebyshev(D, diag, b, x, degree, lam_max):
    """``degree`` steps of the Chebyshev iteration for A x = b preconditioned
    by the diagonal, for spectra of D^-1 A in [a, c] = [lam_max/10,
    1.1 lam_max]: the error is multiplied by T_k((theta - D^-1 A)/delta) /
    T_k(theta/delta), theta = (a + c)/2, delta = (c - a)/2 (three-term
    recurrence of the Chebyshev semi-iteration)."""
    a, c = lam_max / 10.0, 1.1 * lam_max
    theta, delta = 0.5 * (a + c), 0.5 * (c - a)
    sigma = theta / delta
    rho = 1.0 / sigma
    r = b - D @ x
    d = (r / diag) / theta
    for _ in range(degree):
        x = x + d
        r = r - D @ d
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (r / diag)
        rho = rho_new
    return x


def ends_cycle(S, Kl, tau, coarse_ratio):
    """True if the level's block S_l + tau K_l ends the V-cycle:
    tau max_p (K_l)_pp / (S_l)_pp <= coarse_ratio (never for coarse_ratio 0
    or tau <= 0)."""
    if coarse_ratio <= 0.0 or tau <= 0.0:
        return False
    return tau * np.max(Kl.diagonal() / S.diagonal()) <= coarse_ratio


def vcycle(levels, tau, b, nu=2, level=0, coarse_ratio=0.0, smoother="rbgs", omega=0.8,
           cheb_degree=2):
    """One V(nu, nu)-cycle from x = 0 for D_l = S_l + tau K_l."""
    nx, ny, S, Kl, P, R = levels[level]
    D = (S + tau * Kl).tocsr()
    if P is None:
        return spla.spsolve(D.tocsc(), b) if D.shape[0] > 1 else b / D.toarray()[0, 0]
    diag = D.diagonal()
    col = colours(nx, ny)
    lam_max = gershgorin_bound(D, diag) if smoother == "chebyshev" else 0.0

    def smooth(x, pre):
        for _ in range(nu):
            if smoother == "rbgs":
                first, second = (0, 1) if pre else (1, 0)
                x = relax(D, diag, col, b, x, first)
                x = relax(D, diag, col, b, x, second)
            elif smoother == "jacobi":
                x = jacobi(D, diag, b, x, omega)
            elif smoother == "chebyshev":
                x = chebyshev(D, diag, b, x, cheb_degree, lam_max)
            else:
                raise ValueError(smoother)
        return x

    x = smooth(np.zeros_like(b), True)
    if not ends_cycle(S, Kl, tau, coarse_ratio):
        rc = R @ (b - D @ x)
        x = x + P @ vcycle(levels, tau, rc, nu, level + 1, coarse_ratio, smoother, omega,
                           cheb_degree)
    return smooth(x, False)


def apply_vcycle_preconditioner(Atilde, K, h, v, nx, ny, nu=2, coarse_max=64, M=None,
                                interp="linear", coarse_ratio=0.0, smoother="rbgs", omega=0.8,
                                cheb_degree=2, levels=None):
    """``z ~= P^-1 v`` by block substitution (Sec. 4.2) with one V-cycle per
    diagonal block ``M + h A~_jj K`` instead of an exact solve (M = I if
    None)."""
    At = np.asarray(Atilde, dtype=np.float64)
    s = At.shape[0]
    N = K.shape[0]
    lower = np.allclose(At, np.tril(At))
    upper = np.allclose(At, np.triu(At))
    if not (lower or upper):
        raise ValueError("A~ must be triangular")
    if levels is None:
        levels = hierarchy(K, nx, ny, coarse_max, M, interp)
    order = range(s) if lower else range(s - 1, -1, -1)
    v = np.asarray(v, dtype=np.float64).reshape(s, N)
    z = np.zeros((s, N))
    for j in order:
        rhs = v[j].copy()
        for k in range(s):
            if k != j and At[j, k] != 0.0:
                rhs -= h * At[j, k] * (K @ z[k])
        z[j] = vcycle(levels, h * At[j, j], rhs, nu, coarse_ratio=coarse_ratio,
                      smoother=smoother, omega=omega, cheb_degree=cheb_degree)
    return z
