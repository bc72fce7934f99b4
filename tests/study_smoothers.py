"""Smoother comparison for the multigrid subsolves of the block preconditioner
(Sec. 4.2: one V-cycle per diagonal block), by FGMRES iteration counts on the
FP64 CPU oracle.

Workload: 2-D heat, Gauss-Legendre 7 stages, h_t = 1e-3 (the 2048^2 benchmark
configuration's method and step) on n x n grids, P_LD right preconditioning,
FGMRES relative tolerance 1e-8 from k = 0, the stage system of the first step
from a smooth initial value (8 random sine modes, seed 0) and a white-noise
one (seed 1).  The multigrid is the reading of ``oracle/amg.py`` (structured
2 x 2 coarsening, linear interpolation, Galerkin levels, cycle end at
coarse_ratio 2, coarse_max 64) with the smoother varied:

* ``rbgs``: red-black Gauss-Seidel, V(2,2) (four colour half sweeps per side);
* ``jacobi``: damped Jacobi, omega = 0.8, V(1,1) and V(2,2);
* ``chebyshev``: degree-2 Chebyshev on [lam_max/10, 1.1 lam_max], one
  application per side (two operator applications, as V(2,2) Jacobi).

Run from the repository root: ``python tests/study_smoothers.py [n ...]``
(default 256 512).  It calls the oracle only.
"""
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle.amg import apply_vcycle_preconditioner, hierarchy  # noqa: E402
from oracle.krylov import fgmres  # noqa: E402
from oracle.ldu import coefficient_matrix  # noqa: E402
from oracle.operators import heat_K  # noqa: E402
from oracle.tableau import tableau  # noqa: E402
from paper_2010_11377_amd.workloads import fourier_modes, white_noise  # noqa: E402

VARIANTS = [("rbgs", 2), ("jacobi", 1), ("jacobi", 2), ("chebyshev", 1)]


def initial_values(n):
    """(name, u0): the smooth 8-mode field (seed 0) and white noise (seed 1)."""
    return [("smooth", fourier_modes(n, seed=0)), ("white noise", white_noise(n, seed=1))]


def iterations(n, smoother, nu, u0, h=1e-3, rtol=1e-8):
    A, b, c = tableau("gauss", 7)
    s = A.shape[0]
    K = heat_K(n)
    LD = coefficient_matrix(A, "LD")
    levels = hierarchy(K, n, n, coarse_max=64)

    def matvec(k):
        kk = k.reshape(s, -1)
        Kk = np.stack([K @ kk[i] for i in range(s)])
        return (kk + h * (A @ Kk)).ravel()

    def precond(v):
        return apply_vcycle_preconditioner(LD, K, h, v.reshape(s, -1), n, n, nu=nu,
                                           coarse_ratio=2.0, smoother=smoother,
                                           levels=levels).ravel()

    rhs = np.tile(-(K @ u0), s)
    _, its, _ = fgmres(matvec, precond, rhs, rtol=rtol, restart=80, max_iter=80)
    return its


def main(sizes):
    print("GL7, h_t = 1e-3, P_LD, FGMRES rtol 1e-8: iterations of the first step")
    for n in sizes:
        for name, u0 in initial_values(n):
            row = []
            for sm, nu in VARIANTS:
                t = time.time()
                its = iterations(n, sm, nu, u0)
                row.append("%s V(%d,%d) %d" % (sm, nu, nu, its))
                print("  %4d^2 %-11s %-10s V(%d,%d): %3d iterations (%.0f s)" % (
                    n, name, sm, nu, nu, its, time.time() - t), flush=True)


if __name__ == "__main__":
    main([int(a) for a in sys.argv[1:]] or [256, 512])
