"""Right-preconditioned flexible GMRES (Saad's FGMRES), written out plainly
for iteration-count studies of the block preconditioners of Sec. 4 with
approximate (multigrid) subsolves.

The paper solves the stage system with GMRES to a relative residual of 1e-8
(Sec. 5); a preconditioner that changes from one application to the next (a
multigrid cycle in reduced precision) needs the flexible variant, which keeps
the preconditioned vectors z_j and forms x = x0 + Z y.  Arnoldi with modified
Gram-Schmidt, Givens rotations for the Hessenberg least-squares problem, x0 =
0, stopping test ||r|| <= rtol ||b|| on the Givens estimate.

Test infrastructure only (see the package docstring).
"""
import numpy as np


def fgmres(matvec, precond, b, rtol=1e-8, restart=60, max_iter=400):
    """Solve A x = b.  Returns ``(x, iterations, estimate history)``; the
    history holds ||r_j|| / ||b|| after each iteration."""
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    x = np.zeros_like(b)
    if nb == 0.0:
        return x, 0, []
    hist = []
    its = 0
    while its < max_iter:
        r = b - matvec(x) if its else b.copy()
        beta = np.linalg.norm(r)
        if beta <= rtol * nb:
            break
        m = min(restart, max_iter - its)
        V = np.zeros((m + 1, b.size))
        Z = np.zeros((m, b.size))
        H = np.zeros((m + 1, m))
        cs, sn = np.zeros(m), np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            for i in range(j + 1):
                H[i, j] = V[i] @ w
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            d = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / d, H[j + 1, j] / d
            H[j, j] = d
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            k = j + 1
            its += 1
            hist.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) <= rtol * nb:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + Z[:k].T @ y
        if hist and hist[-1] <= rtol:
            break
    return x, its, hist
