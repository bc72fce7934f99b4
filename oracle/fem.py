"""Linear finite elements for the heat equation (Sec. 3.1, with piecewise
linear instead of quadratic elements): the mass matrix ``M_kl = int phi_k phi_l``
and the stiffness matrix ``F_kl = int grad phi_k . grad phi_l`` of Sec. 3.1
(F is called K here), so that the semi-discrete system is ``M u' = -K u`` and
the IRK stage system ``(I_s (x) M + h A (x) K) k = 1_s (x) (-K u_n)``.

Mesh: the square of side ``length`` with (n + 2) x (n + 2) nodes, spacing
``h = length / (n + 1)``; every cell is cut by its diagonal from the lower-left
to the upper-right corner.  Homogeneous Dirichlet data: the rows and columns of
boundary nodes are removed, the interior unknown of node (i, j) (1-based grid
position) is ``(j - 1) * n + (i - 1)``, x fastest.

The matrices are assembled element by element from the element matrices of
the two triangle shapes (every triangle is a translate of one of them):
stiffness ``|T| grad phi_a . grad phi_b`` from the gradients of the
barycentric basis, mass ``|T| / 12 (1 + delta_ab)``.

Test infrastructure only (see the package docstring).
"""
import numpy as np
import scipy.sparse as sp


def _element_matrices(verts):
    """Stiffness and mass element matrices of the triangle with vertex
    coordinates ``verts`` (3 x 2)."""
    x = np.asarray(verts, dtype=np.float64)
    B = np.array([x[1] - x[0], x[2] - x[0]]).T          # columns: edge vectors
    area = 0.5 * abs(np.linalg.det(B))
    # gradients of the basis functions phi_1, phi_2 are the rows of B^-1,
    # grad phi_0 = -(grad phi_1 + grad phi_2)
    Binv = np.linalg.inv(B)
    G = np.vstack([-(Binv[0] + Binv[1]), Binv[0], Binv[1]])
    Ke = area * (G @ G.T)
    Me = area / 12.0 * (np.ones((3, 3)) + np.eye(3))
    return Ke, Me


def p1_heat(n, length=1.0):
    """``(M, K)`` for the n x n interior nodes, as scipy CSR matrices."""
    h = length / (n + 1)
    m = n + 2                                            # nodes per direction
    # the two triangles of the cell with lower-left node (i, j):
    #   lower: (i, j), (i+1, j), (i+1, j+1);  upper: (i, j), (i+1, j+1), (i, j+1)
    shapes = [((0, 0), (1, 0), (1, 1)), ((0, 0), (1, 1), (0, 1))]
    rows, cols, kv, mv = [], [], [], []
    ci, cj = np.meshgrid(np.arange(m - 1), np.arange(m - 1), indexing="xy")
    ci, cj = ci.ravel(), cj.ravel()
    for shape in shapes:
        Ke, Me = _element_matrices([(h * a, h * b) for a, b in shape])
        nodes = [(cj + b) * m + (ci + a) for a, b in shape]  # global node ids
        for a in range(3):
            for b in range(3):
                rows.append(nodes[a])
                cols.append(nodes[b])
                kv.append(np.full(ci.size, Ke[a, b]))
                mv.append(np.full(ci.size, Me[a, b]))
    rows, cols = np.concatenate(rows), np.concatenate(cols)
    Kfull = sp.csr_matrix((np.concatenate(kv), (rows, cols)), shape=(m * m, m * m))
    Mfull = sp.csr_matrix((np.concatenate(mv), (rows, cols)), shape=(m * m, m * m))
    jj, ii = np.meshgrid(np.arange(1, n + 1), np.arange(1, n + 1), indexing="ij")
    interior = (jj * m + ii).ravel()                     # x fastest
    Kin = Kfull[interior][:, interior].tocsr()
    Min = Mfull[interior][:, interior].tocsr()
    Kin.eliminate_zeros()
    Min.eliminate_zeros()
    return Min, Kin
