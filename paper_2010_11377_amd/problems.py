"""Spatial operators fed to the GPU solver, as CSR arrays.

The paper's test problems (Sec. 3.1, heat equation (3.1); Sec. 3.2, double
glazing (3.3)) discretised by finite differences on the ``n x n`` interior
nodes of a square, boundary nodes eliminated, unknown ``j * n + i`` with x
fastest, ``M = I`` and ``u' = -K u + g``; the variable-coefficient diffusion
``u_t = div(kappa grad u)`` used by the adjoint; and the heat equation with
linear finite elements, where ``M u' = -K u`` with a consistent mass matrix.

Each builder returns ``(indptr, indices, data)`` with sorted columns (int32,
int32, float64) and, where the problem has boundary data, the source ``g``.
"""
import numpy as np

# neighbour order inside a row, by increasing column index: S, W, C, E, N
_OFFS = [(0, -1), (-1, 0), (0, 0), (1, 0), (0, 1)]
# seven-point pattern of linear elements on right triangles whose diagonals
# run from south-west to north-east: SW, S, W, C, E, N, NE
_OFFS7 = [(-1, -1), (0, -1), (-1, 0), (0, 0), (1, 0), (0, 1), (1, 1)]


def _assemble(n, coef, ny=None, offs=_OFFS):
    """CSR from coefficient fields coef[k] (ny x n, indexed [j, i]) for the
    neighbours in offs (sorted by column); couplings that leave the grid are
    dropped."""
    ny = n if ny is None else ny
    jj, ii = np.meshgrid(np.arange(ny), np.arange(n), indexing="ij")
    present = []
    for (dx, dy) in offs:
        present.append((ii + dx >= 0) & (ii + dx < n) & (jj + dy >= 0) & (jj + dy < ny))
    counts = np.sum(np.stack(present), axis=0).ravel()
    indptr = np.zeros(n * ny + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    nnz = int(indptr[-1])
    indices = np.empty(nnz, dtype=np.int32)
    data = np.empty(nnz, dtype=np.float64)
    pos = indptr[:-1].copy()
    row = (jj * n + ii).ravel()
    for k, (dx, dy) in enumerate(offs):
        m = present[k].ravel()
        r = row[m]
        indices[pos[m]] = (r + dy * n + dx).astype(np.int32)
        data[pos[m]] = coef[k].ravel()[m]
        pos[m] += 1
    return indptr.astype(np.int32), indices, data


def heat(n, length=1.0, ny=None):
    """Five-point ``-Laplacian``, homogeneous Dirichlet, spacing length/(n+1)
    in both directions, on n columns and ``ny`` (default n) rows."""
    ny = n if ny is None else ny
    h = length / (n + 1)
    inv = 1.0 / (h * h)
    f = np.full((ny, n), -inv)
    return _assemble(n, [f, f, np.full((ny, n), 4.0 * inv), f, f], ny)


def double_glazing(n, eps):
    """Double glazing on [-1, 1]^2 (Sec. 3.2): ``-eps Lap u + w . grad u``
    with central diffusion and first-order upwind advection, wind
    ``w = (2y(1-x^2), -2x(1-y^2))``, ``u = 1`` on the wall x = 1 and 0 on the
    others.  Returns ``(indptr, indices, data, g)``."""
    h = 2.0 / (n + 1)
    t = -1.0 + h * np.arange(1, n + 1)
    Y, X = np.meshgrid(t, t, indexing="ij")      # arrays indexed [j, i]
    wx = 2.0 * Y * (1.0 - X * X)
    wy = -2.0 * X * (1.0 - Y * Y)
    d = eps / (h * h)
    west = -d - np.maximum(wx, 0.0) / h
    east = -d + np.minimum(wx, 0.0) / h
    south = -d - np.maximum(wy, 0.0) / h
    north = -d + np.minimum(wy, 0.0) / h
    centre = 4.0 * d + (np.abs(wx) + np.abs(wy)) / h
    indptr, indices, data = _assemble(n, [south, west, centre, east, north])
    g = np.zeros((n, n))
    g[:, n - 1] = -east[:, n - 1] * 1.0      # east wall carries u = 1
    return indptr, indices, data, g.ravel()


def kappa_diffusion(kappa_nodes, length=1.0):
    """``(K u)_P = h^-2 sum_faces kappa_f (u_P - u_Q)``, ``kappa_f`` the mean of
    the two nodal values; ``kappa_nodes`` is (n+2) x (n+2) including the
    boundary nodes, indexed [j, i]."""
    kn = np.asarray(kappa_nodes, dtype=np.float64)
    n = kn.shape[0] - 2
    h = length / (n + 1)
    inv = 1.0 / (h * h)
    c = kn[1:-1, 1:-1]
    kw = 0.5 * (c + kn[1:-1, :-2])
    ke = 0.5 * (c + kn[1:-1, 2:])
    ks = 0.5 * (c + kn[:-2, 1:-1])
    kN = 0.5 * (c + kn[2:, 1:-1])
    return _assemble(n, [-ks * inv, -kw * inv, (kw + ke + ks + kN) * inv, -ke * inv, -kN * inv])


def to_dense(indptr, indices, data, n):
    """Dense matrix (tests only, small n)."""
    A = np.zeros((n, n))
    for r in range(n):
        for e in range(indptr[r], indptr[r + 1]):
            A[r, indices[e]] += data[e]
    return A


def p1_heat(n, length=1.0):
    """Heat equation with continuous piecewise-linear elements on the uniform
    triangulation of a square of side ``length`` (n x n interior nodes,
    spacing h = length/(n+1), every cell cut by its south-west to north-east
    diagonal), homogeneous Dirichlet data: returns ``(M, K)`` as CSR triples.

    On this mesh the stiffness matrix is the five-point stencil
    ``(4, -1, -1, -1, -1)`` (the couplings along the diagonals cancel) and the
    consistent mass matrix has ``h^2 / 2`` on the diagonal and ``h^2 / 12`` for
    each of the six neighbours joined by an edge (W, E, S, N, SW, NE)."""
    h = length / (n + 1)
    one = np.ones((n, n))
    K = _assemble(n, [-one, -one, 4.0 * one, -one, -one])
    e = h * h / 12.0
    M = _assemble(n, [e * one, e * one, e * one, 6.0 * e * one, e * one, e * one, e * one],
                  offs=_OFFS7)
    return M, K
