"""Condition numbers and eigenvalues of the preconditioned stage matrix for
the finite-difference heat problem (the quantities of Sec. 4.3, Tables 2-4
and the eigenvalue figures there), computed exactly through the sine basis.

With ``M = I`` and the five-point K, the orthonormal 2-D DST diagonalises K
(eigenvalues ``lam``).  ``Q = I_s (x) DST`` is orthogonal, and under it the
stage matrix ``I + h A (x) K`` and the preconditioner ``I + h A~ (x) K`` become
block diagonal with one s x s block per eigenvalue:

    right:  (I + h lam A) (I + h lam A~)^-1
    left:   (I + h lam A~)^-1 (I + h lam A)

Orthogonal similarity keeps singular values and eigenvalues, and the singular
values of a block-diagonal matrix are the union of its blocks' singular
values, so

    kappa_2 = max over blocks of sigma_max / min over blocks of sigma_min,

and the spectrum is the union of the blocks' eigenvalues.

Test infrastructure only (see the package docstring).
"""
import numpy as np

from .operators import heat_eigenvalues


def blocks(A, Atilde, h, lam, side="right"):
    """The s x s blocks of the preconditioned stage matrix, one per entry of
    ``lam``, as an array of shape (len(lam), s, s)."""
    A = np.asarray(A, dtype=np.float64)
    At = np.asarray(Atilde, dtype=np.float64)
    s = A.shape[0]
    lam = np.asarray(lam, dtype=np.float64).ravel()
    eye = np.eye(s)
    F = eye[None] + (h * lam)[:, None, None] * A[None]
    P = eye[None] + (h * lam)[:, None, None] * At[None]
    if side == "right":
        # F P^-1 = (P^-T F^T)^T
        return np.transpose(np.linalg.solve(np.transpose(P, (0, 2, 1)),
                                            np.transpose(F, (0, 2, 1))), (0, 2, 1))
    if side == "left":
        return np.linalg.solve(P, F)
    raise ValueError(side)


def heat_condition_number(A, Atilde, h, n, length=1.0, side="right"):
    """2-norm condition number of the preconditioned stage matrix of the
    five-point heat operator on the n x n interior grid."""
    B = blocks(A, Atilde, h, heat_eigenvalues(n, length), side)
    sv = np.linalg.svd(B, compute_uv=False)
    return sv[:, 0].max() / sv[:, -1].min()


def heat_spectrum(A, Atilde, h, n, length=1.0, side="right"):
    """All eigenvalues of the preconditioned stage matrix (complex array of
    length s n^2)."""
    B = blocks(A, Atilde, h, heat_eigenvalues(n, length), side)
    return np.linalg.eigvals(B).ravel()


def unpreconditioned_condition_number(A, h, n, length=1.0):
    """2-norm condition number of ``I + h A (x) K`` itself."""
    s = np.asarray(A).shape[0]
    return heat_condition_number(A, np.zeros((s, s)), h, n, length, "right")


def dense_condition_number(A, Atilde, h, K, side="right", M=None):
    """The same quantity for any (small) K and M from the assembled dense
    matrices: kappa_2 of (I (x) M + h A (x) K) P^-1 or P^-1 (I (x) M + h A (x) K)."""
    A = np.asarray(A, dtype=np.float64)
    At = np.asarray(Atilde, dtype=np.float64)
    s = A.shape[0]
    Kd = np.asarray(K.todense() if hasattr(K, "todense") else K, dtype=np.float64)
    N = Kd.shape[0]
    Md = np.eye(N) if M is None else np.asarray(M.todense() if hasattr(M, "todense") else M)
    F = np.kron(np.eye(s), Md) + h * np.kron(A, Kd)
    P = np.kron(np.eye(s), Md) + h * np.kron(At, Kd)
    X = np.linalg.solve(P.T, F.T).T if side == "right" else np.linalg.solve(P, F)
    return np.linalg.cond(X)


def operator_condition_number(A, Atilde, h, K, side="right", M=None, tol=1e-10):
    """kappa_2 = sigma_max(X) sigma_max(X^-1) for X the preconditioned stage
    matrix, from the largest singular values of X and X^-1 applied through
    sparse LU factorisations (for grids too large for dense matrices)."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as spla
    A = np.asarray(A, dtype=np.float64)
    At = np.asarray(Atilde, dtype=np.float64)
    s = A.shape[0]
    N = K.shape[0]
    Mm = sp.identity(N) if M is None else M
    F = (sp.kron(sp.identity(s), Mm) + h * sp.kron(sp.csr_matrix(A), K)).tocsc()
    P = (sp.kron(sp.identity(s), Mm) + h * sp.kron(sp.csr_matrix(At), K)).tocsc()
    Flu, Plu = spla.splu(F), spla.splu(P)
    n = s * N
    if side == "right":       # X = F P^-1, X^-1 = P F^-1
        mv = lambda x: F @ Plu.solve(x)
        rmv = lambda y: Plu.solve(F.T @ y, trans="T")
        imv = lambda x: P @ Flu.solve(x)
        irmv = lambda y: Flu.solve(P.T @ y, trans="T")
    elif side == "left":      # X = P^-1 F, X^-1 = F^-1 P
        mv = lambda x: Plu.solve(F @ x)
        rmv = lambda y: F.T @ Plu.solve(y, trans="T")
        imv = lambda x: Flu.solve(P @ x)
        irmv = lambda y: P.T @ Flu.solve(y, trans="T")
    else:
        raise ValueError(side)
    def top_singular_value(f, ft):
        # largest eigenvalue of the normal operator, by Lanczos
        op = spla.LinearOperator((n, n), matvec=lambda x: ft(f(x)), dtype=np.float64)
        lam = spla.eigsh(op, k=1, which="LM", ncv=20, tol=tol, v0=np.ones(n),
                         return_eigenvectors=False)[0]
        return np.sqrt(lam)

    return top_singular_value(mv, rmv) * top_singular_value(imv, irmv)
