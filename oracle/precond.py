"""Exact application of the block preconditioners of Sec. 4 and Sec. 4.2.

``P = I_s (x) M + h A~ (x) K`` with ``A~`` diagonal (P_J), lower triangular
(P_GSL, P_LD) or upper triangular (P_DU).  Sec. 4.2 applies ``P^-1 v`` by
substitution over the stage blocks: block j solves

    (M + h A~_jj K) w_j = v_j - sum_{k != j, A~_jk != 0} h A~_jk K w_k,

in increasing j for a lower triangular A~ (forward substitution) and in
decreasing j for an upper triangular A~ (back substitution).  Here every
subsolve is an exact sparse LU, so the result equals ``P^-1 v``; the GPU path
replaces the subsolve by one AMG V-cycle.

Test infrastructure only (see the package docstring).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def assemble(Atilde, K, h, M=None):
    """The assembled sN x sN matrix ``I_s (x) M + h A~ (x) K``."""
    s = Atilde.shape[0]
    N = K.shape[0]
    Mm = sp.identity(N, format="csr") if M is None else M
    return (sp.kron(sp.identity(s), Mm) + h * sp.kron(sp.csr_matrix(Atilde), K)).tocsc()


def apply_inverse(Atilde, K, h, v, M=None):
    """``P^-1 v`` by block substitution with exact subsolves (Sec. 4.2).

    ``v`` has shape (s, N).  ``Atilde`` must be lower or upper triangular."""
    At = np.asarray(Atilde, dtype=np.float64)
    s = At.shape[0]
    N = K.shape[0]
    Mm = sp.identity(N, format="csr") if M is None else M
    lower = np.allclose(At, np.tril(At))
    upper = np.allclose(At, np.triu(At))
    if not (lower or upper):
        raise ValueError("A~ must be triangular")
    order = range(s) if lower else range(s - 1, -1, -1)
    w = np.zeros((s, N))
    v = np.asarray(v, dtype=np.float64).reshape(s, N)
    for j in order:
        rhs = v[j].copy()
        for k in range(s):
            if k != j and At[j, k] != 0.0:
                rhs -= h * At[j, k] * (K @ w[k])
        Dj = (Mm + h * At[j, j] * K).tocsc()
        w[j] = spla.spsolve(Dj, rhs)
    return w
