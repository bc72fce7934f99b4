"""Finite-difference spatial operators for the paper's two test problems
(Sec. 3.1 heat equation (3.1); Sec. 3.2 double-glazing advection-diffusion
(3.3)) and for a variable-coefficient diffusion ``u_t = div(kappa grad u)``.

Conventions (the paper uses FEM; these are the FD readings):

* ``n x n`` interior nodes, spacing ``h = L / (n + 1)``, boundary nodes
  eliminated (Dirichlet), unknown index ``j * n + i`` with ``x`` fastest
  (node (i, j) at ``x = x0 + (i + 1) h``, ``y = y0 + (j + 1) h``).
* ``M = I``.  The semi-discrete system is ``u' = -K u + g``, so the IRK stage
  system is ``(I + h_t A (x) K) k = 1 (x) (g - K u_n)``.

Test infrastructure only (see the package docstring).
"""
import numpy as np
import scipy.sparse as sp


def _tridiag_1d(n, h):
    """Second-difference matrix ``tridiag(-1, 2, -1) / h^2`` of size n."""
    e = np.ones(n)
    return sp.diags([-e[:-1], 2.0 * e, -e[:-1]], [-1, 0, 1], format="csr") / (h * h)


def heat_K(n, length=1.0, ny=None):
    """Five-point negative Laplacian on the n x n interior grid of a square of
    side ``length`` with homogeneous Dirichlet data: ``K = I (x) T + T (x) I``.
    With ``ny`` rows instead of n (same spacing ``length / (n + 1)``):
    ``K = I_ny (x) T_n + T_ny (x) I_n``."""
    ny = n if ny is None else ny
    h = length / (n + 1)
    return (sp.kron(sp.identity(ny), _tridiag_1d(n, h)) +
            sp.kron(_tridiag_1d(ny, h), sp.identity(n))).tocsr()


def heat_eigenvalues(n, length=1.0):
    """Eigenvalues ``lambda_pq = 4/h^2 (sin^2(p pi h'/2) + sin^2(q pi h'/2))``
    of ``heat_K`` (with ``h' = 1/(n+1)``), as an (n, n) array indexed [q, p]."""
    h = length / (n + 1)
    k = np.arange(1, n + 1)
    mu = 4.0 / (h * h) * np.sin(k * np.pi / (2.0 * (n + 1))) ** 2
    return mu[:, None] + mu[None, :]


def grid_coords(n, lo=0.0, hi=1.0):
    """Interior node coordinates (x, y), each of shape (n*n,), x fastest."""
    h = (hi - lo) / (n + 1)
    t = lo + h * np.arange(1, n + 1)
    X, Y = np.meshgrid(t, t, indexing="xy")  # X[j, i] = t[i], Y[j, i] = t[j]
    return X.ravel(), Y.ravel()


def _east_wall_hot(xb, yb):
    """Boundary data of the double-glazing problem: 1 on x = 1, else 0."""
    return np.where(np.isclose(xb, 1.0), 1.0, 0.0)


def double_glazing(n, eps, boundary=_east_wall_hot):
    """Double-glazing problem on [-1, 1]^2 (Sec. 3.2, (3.3)) discretised by
    central differences for ``-eps Lap u`` and first-order upwind differences
    for ``w . grad u`` with the recirculating wind
    ``w = (2 y (1 - x^2), -2 x (1 - y^2))``.  Dirichlet data: ``u = 1`` on the
    east wall ``x = 1``, ``u = 0`` on the other walls.

    Returns ``(K, g)`` with ``u' = -K u + g``: row P of ``K u`` is
    ``-eps (u_E + u_W + u_N + u_S - 4 u_P)/h^2 + w_x D_x u + w_y D_y u`` with
    ``D_x u = (u_P - u_W)/h`` where ``w_x > 0`` and ``(u_E - u_P)/h`` where
    ``w_x < 0`` (likewise in y); ``g`` carries the boundary values, given by
    ``boundary(x, y)`` at boundary nodes (default: the hot east wall).
    """
    h = 2.0 / (n + 1)
    x, y = grid_coords(n, -1.0, 1.0)
    wx = 2.0 * y * (1.0 - x * x)
    wy = -2.0 * x * (1.0 - y * y)
    N = n * n
    idx = np.arange(N)
    i = idx % n
    j = idx // n
    rows, cols, vals = [], [], []
    g = np.zeros(N)
    diag = np.full(N, 4.0 * eps / (h * h)) + np.abs(wx) / h + np.abs(wy) / h

    def couple(mask_in, nbr, coef, boundary_value):
        # interior neighbours go into K; boundary neighbours move to g
        rows.append(idx[mask_in])
        cols.append(nbr[mask_in])
        vals.append(coef[mask_in])
        out = ~mask_in
        g[out] -= coef[out] * boundary_value[out]

    # west neighbour: coefficient -eps/h^2 - max(wx,0)/h
    couple(i > 0, idx - 1, -eps / (h * h) - np.maximum(wx, 0.0) / h, boundary(x - h, y))
    # east neighbour: coefficient -eps/h^2 + min(wx,0)/h
    couple(i < n - 1, idx + 1, -eps / (h * h) + np.minimum(wx, 0.0) / h, boundary(x + h, y))
    # south neighbour
    couple(j > 0, idx - n, -eps / (h * h) - np.maximum(wy, 0.0) / h, boundary(x, y - h))
    # north neighbour
    couple(j < n - 1, idx + n, -eps / (h * h) + np.minimum(wy, 0.0) / h, boundary(x, y + h))
    rows.append(idx)
    cols.append(idx)
    vals.append(diag)
    K = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    K.sum_duplicates()
    K.sort_indices()
    return K, g


def kappa_face_values(kappa_nodes):
    """Face coefficients from nodal kappa on the full (n+2) x (n+2) grid
    (boundary nodes included), ``kappa_f = (kappa_P + kappa_Q) / 2``.

    Returns ``(kx, ky)``: ``kx[j, i]`` is the face between nodes (i-1, j) and
    (i, j) in full-grid indexing restricted to interior rows, shape (n, n+1);
    ``ky[j, i]`` the face between (i, j-1) and (i, j), shape (n+1, n).
    """
    kn = np.asarray(kappa_nodes, dtype=np.float64)
    kx = 0.5 * (kn[1:-1, :-1] + kn[1:-1, 1:])   # (n, n+1)
    ky = 0.5 * (kn[:-1, 1:-1] + kn[1:, 1:-1])   # (n+1, n)
    return kx, ky


def kappa_diffusion_K(kappa_nodes, length=1.0):
    """``(K u)_P = h^-2 sum_{faces f=(P,Q)} kappa_f (u_P - u_Q)`` on the n x n
    interior grid, ``u_Q = 0`` on the boundary (homogeneous Dirichlet).
    ``kappa_nodes`` has shape (n+2, n+2) (indexed [j, i]) including boundary
    nodes."""
    kx, ky = kappa_face_values(kappa_nodes)
    return face_diffusion_K(kx, ky, length)


def face_diffusion_K(kx, ky, length=1.0):
    """The same operator from its face coefficients: ``kx`` (n, n+1) and ``ky``
    (n+1, n) as returned by ``kappa_face_values``."""
    kx = np.asarray(kx, dtype=np.float64)
    ky = np.asarray(ky, dtype=np.float64)
    n = kx.shape[0]
    h = length / (n + 1)
    N = n * n
    rows, cols, vals = [], [], []
    diag = np.zeros((n, n))
    for j in range(n):
        for i in range(n):
            P = j * n + i
            kw, ke = kx[j, i], kx[j, i + 1]
            ks, kN = ky[j, i], ky[j + 1, i]
            diag[j, i] = kw + ke + ks + kN
            for (ii, jj, kf) in ((i - 1, j, kw), (i + 1, j, ke), (i, j - 1, ks), (i, j + 1, kN)):
                if 0 <= ii < n and 0 <= jj < n:
                    rows.append(P)
                    cols.append(jj * n + ii)
                    vals.append(-kf)
    rows.extend(range(N))
    cols.extend(range(N))
    vals.extend(diag.ravel())
    K = sp.csr_matrix((np.array(vals) / (h * h), (np.array(rows), np.array(cols))), shape=(N, N))
    K.sort_indices()
    return K
