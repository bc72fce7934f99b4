"""Plain FP64 CPU oracle for the IRK stage solve of Rana, Howle, Long, Meek and
Milestone, "A New Block Preconditioner for Implicit Runge--Kutta Methods for
Parabolic PDE Problems" (arXiv 2010.11377).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library, its
Python binding, the problem builders that feed it) imports, calls or links any
module in this package.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it, to check the GPU path.

The oracle computes what the method reaches, directly and slowly:

* every IRK step is ``u_{n+1} = u_n + h sum_i b_i k_i`` (Sec. 2) with ``k`` the
  exact solution of the coupled stage system ``(I_s (x) M + h A (x) K) k =
  1_s (x) (g - K u_n)`` (Sec. 3.1, block system (3.2); Sec. 4), solved by a sparse direct
  factorisation, by a 2-D sine transform (constant-coefficient heat), or by
  decoupling through the eigenvectors of ``A``;
* the preconditioners ``P = I_s (x) M + h A~ (x) K`` (Sec. 4, general form
  (4.1); P_LD and P_DU in (4.3)) are applied exactly by block forward or back substitution with
  sparse direct subsolves (Sec. 4.2);
* the discrete adjoint of the IRK step (not in the paper) is the transposed
  stage solve, checked by finite differences of the forward oracle.

Everything is float64 (complex128 where the eigen-decoupling needs it).  The
Butcher tableaux are built in 50-digit arithmetic from their collocation
definitions and rounded once.

Module map:
  tableau   -- Gauss--Legendre, Radau IIA, Lobatto IIIC tableaux (Sec. 2, Table 1)
  ldu       -- LDU factorisation of A without pivoting and the A~ matrices (Sec. 4.1)
  operators -- finite-difference K and source g for the test problems (Sec. 3)
  fem       -- linear-element M and K for the heat equation (Sec. 3.1)
  step      -- exact IRK steps (Sec. 2, Sec. 3.1)
  precond   -- exact block preconditioner application (Sec. 4.2)
  amg       -- the multigrid V-cycle subsolve as read for this path (Sec. 4.2, 5)
  adjoint   -- discrete adjoint step and gradient for kappa-diffusion
"""
