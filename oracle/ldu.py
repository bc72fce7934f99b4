"""LDU factorisation of the Butcher matrix without pivoting and the
preconditioner coefficient matrices A~ of Sec. 4 and Sec. 4.1.

``A = L D U`` with L unit lower triangular, D = diag(d) and U unit upper
triangular exists without pivoting when every leading principal submatrix of A
is nonsingular (Sec. 4.1).  The preconditioner coefficient matrices are

* ``A~_J   = diag(A)``            (block Jacobi, Sec. 4, (4.2))
* ``A~_GSL = tril(A)``            (block Gauss--Seidel, Sec. 4, (4.2))
* ``A~_DU  = D U``                (Sec. 4.1, (4.3))
* ``A~_LD  = L D``                (Sec. 4.1, (4.3), the paper's method)

Test infrastructure only (see the package docstring).
"""
import numpy as np


def ldu(A):
    """Doolittle elimination without row exchanges.

    Returns ``(L, d, U)`` with ``L`` unit lower, ``d`` the pivots, ``U`` unit
    upper, so that ``L @ diag(d) @ U == A`` up to rounding.  Raises
    ``ZeroDivisionError`` on a zero pivot (a singular leading minor).
    """
    A = np.array(A, dtype=np.float64)
    s = A.shape[0]
    W = A.copy()
    L = np.eye(s)
    for k in range(s):
        if W[k, k] == 0.0:
            raise ZeroDivisionError("zero pivot at %d" % k)
        for i in range(k + 1, s):
            L[i, k] = W[i, k] / W[k, k]
            W[i, k:] -= L[i, k] * W[k, k:]
    d = np.diag(W).copy()
    U = W / d[:, None]
    return L, d, np.triu(U)


def coefficient_matrix(A, kind):
    """The preconditioner coefficient matrix A~ for ``kind`` in
    {"J", "GSL", "DU", "LD"}."""
    A = np.asarray(A, dtype=np.float64)
    if kind == "J":
        return np.diag(np.diag(A))
    if kind == "GSL":
        return np.tril(A)
    L, d, U = ldu(A)
    if kind == "DU":
        return np.diag(d) @ U
    if kind == "LD":
        return L @ np.diag(d)
    raise ValueError(kind)
