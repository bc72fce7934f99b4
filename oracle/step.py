"""Exact IRK steps: the result the preconditioned Krylov solve converges to.

One step of an s-stage IRK method for ``M u' = -K u + g`` (``M = I`` for the
finite-difference operators) is ``u_{n+1} = u_n + h sum_i b_i k_i`` (Sec. 2)
where the stage vectors solve the coupled block system of Sec. 3.1, (3.2),
written with Kronecker products in Sec. 4:

    (I_s (x) M + h A (x) K) k = 1_s (x) (g - K u_n).

Three independent routes reach the same ``u_{n+1}``:

* ``DirectStepper``  -- assemble the sN x sN matrix with ``scipy.sparse.kron``
  and factor it once with SuperLU (small and medium grids);
* ``HeatDSTStepper`` -- for the constant-coefficient heat operator the 2-D
  orthonormal DST-I diagonalises K, so every sine mode obeys its own s x s
  stage system ``(I + h lam A) k^ = 1 (g^ - lam u^)``, solved exactly;
* ``EigenStepper``   -- ``A = V Lam V^-1`` decouples the stages into s
  independent systems ``(M + h lam_m K)``, one sparse LU per eigenvalue
  (conjugate pairs share one), for large variable-coefficient grids.

Test infrastructure only (see the package docstring).
"""
import numpy as np
import scipy.fft as sfft
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .operators import heat_eigenvalues


def stage_matrix(A, K, h, M=None):
    """The block matrix ``I_s (x) M + h A (x) K`` of Sec. 4 (M = I if None)."""
    s = A.shape[0]
    N = K.shape[0]
    Mm = sp.identity(N, format="csr") if M is None else M
    return (sp.kron(sp.identity(s), Mm) + h * sp.kron(sp.csr_matrix(A), K)).tocsc()


class DirectStepper:
    """Exact step by a sparse LU of the assembled stage matrix (factored once)."""

    def __init__(self, A, b, K, h, g=None, M=None):
        self.A = np.asarray(A, dtype=np.float64)
        self.b = np.asarray(b, dtype=np.float64)
        self.s = self.A.shape[0]
        self.K = K.tocsr()
        self.N = K.shape[0]
        self.h = float(h)
        self.g = np.zeros(self.N) if g is None else np.asarray(g, dtype=np.float64)
        self.lu = spla.splu(stage_matrix(self.A, self.K, self.h, None if M is None else M.tocsr()))

    def stages(self, u):
        """Stage vectors k, shape (s, N), for the step from u."""
        f = self.g - self.K @ u
        return self.lu.solve(np.tile(f, self.s)).reshape(self.s, self.N)

    def step(self, u):
        k = self.stages(u)
        return u + self.h * (self.b @ k)

    def adjoint_stages(self, mu):
        """Solve the transposed stage system ``(I + h A (x) K)^T psi = mu``."""
        return self.lu.solve(np.ravel(mu), trans="T").reshape(self.s, self.N)


class HeatDSTStepper:
    """Exact step for ``K`` = five-point Dirichlet Laplacian on an n x n grid,
    no source.  In the orthonormal DST-I basis every mode with eigenvalue
    ``lam`` satisfies ``(I + h lam A) k^ = -lam u^ 1``, so
    ``u^_{n+1} = u^_n + h b^T k^ = G(lam) u^_n``.  G is formed once per
    (tableau, h, grid) from batched s x s solves."""

    def __init__(self, A, b, n, h, length=1.0, workers=None):
        self.n = n
        self.h = float(h)
        self.workers = workers
        A = np.asarray(A, dtype=np.float64)
        b = np.asarray(b, dtype=np.float64)
        s = A.shape[0]
        lam = heat_eigenvalues(n, length).ravel()
        G = np.empty_like(lam)
        chunk = 1 << 16
        eye = np.eye(s)
        ones = np.ones(s)
        for lo in range(0, lam.size, chunk):
            l = lam[lo:lo + chunk]
            Mb = eye[None, :, :] + (self.h * l)[:, None, None] * A[None, :, :]
            rhs = np.broadcast_to((-l)[:, None] * ones[None, :], (l.size, s))[..., None]
            kh = np.linalg.solve(Mb, rhs)[..., 0]          # k^ per unit u^
            G[lo:lo + chunk] = 1.0 + self.h * (kh @ b)
        self.G = G.reshape(n, n)

    def step(self, u):
        U = np.asarray(u, dtype=np.float64).reshape(self.n, self.n)
        Uh = sfft.dstn(U, type=1, norm="ortho", workers=self.workers)
        out = sfft.idstn(self.G * Uh, type=1, norm="ortho", workers=self.workers)
        return out.ravel()


class EigenStepper:
    """Exact step through the eigen-decomposition ``A = V diag(lam) V^-1``.

    With ``k~ = (V^-1 (x) I) k`` the stage system splits into
    ``(M + h lam_m K) k~_m = (V^-1 1)_m f`` with ``f = g - K u_n``, and
    ``u_{n+1} = u_n + h sum_m (b^T V)_m k~_m``.  Conjugate eigenvalues give
    conjugate terms, so one complex LU per pair is enough."""

    def __init__(self, A, b, K, h, g=None, M=None, permc_spec="COLAMD", workers=1):
        """``permc_spec``: SuperLU's fill-reducing column ordering (it changes
        only the rounding order of the exact solve; ``MMD_AT_PLUS_A`` halves
        the fill of a five-point grid).  ``workers``: factorisations run in
        that many threads."""
        A = np.asarray(A, dtype=np.float64)
        b = np.asarray(b, dtype=np.float64)
        self.K = K.tocsr()
        self.N = K.shape[0]
        self.h = float(h)
        self.g = np.zeros(self.N) if g is None else np.asarray(g, dtype=np.float64)
        lam, V = np.linalg.eig(A)
        w_in = np.linalg.solve(V, np.ones(A.shape[0]))     # V^-1 1
        w_out = b @ V                                       # b^T V
        Mm = sp.identity(self.N, format="csc") if M is None else sp.csc_matrix(M)
        used = np.zeros(lam.size, dtype=bool)
        blocks = []    # (matrix M + h lam K, weight, multiplicity)
        for m in range(lam.size):
            if used[m]:
                continue
            used[m] = True
            mult = 1.0
            if abs(lam[m].imag) > 1e-14 * abs(lam[m]):
                # find and consume the conjugate partner
                partner = np.argmin(np.abs(lam - np.conj(lam[m])) + used * 1e300)
                used[partner] = True
                mult = 2.0
                B = (Mm + self.h * lam[m] * self.K.astype(np.complex128)).tocsc()
            else:
                B = (Mm + self.h * lam[m].real * self.K).tocsc()
            blocks.append((B, w_in[m] * w_out[m], mult))

        def factor(B):
            return spla.splu(B, permc_spec=permc_spec)

        if workers > 1:
            from concurrent.futures import ThreadPoolExecutor
            with ThreadPoolExecutor(workers) as ex:
                lus = list(ex.map(factor, [B for B, _, _ in blocks]))
        else:
            lus = [factor(B) for B, _, _ in blocks]
        self.terms = [(lu, w, mult) for lu, (_, w, mult) in zip(lus, blocks)]

    def step(self, u):
        f = self.g - self.K @ u
        acc = np.zeros(self.N)
        for lu, w, mult in self.terms:
            if mult == 2.0:
                acc += 2.0 * np.real(w * lu.solve(f.astype(np.complex128)))
            else:
                acc += np.real(w) * lu.solve(f)
        return u + self.h * acc


def run_steps(stepper, u0, nsteps):
    u = np.array(u0, dtype=np.float64)
    for _ in range(nsteps):
        u = stepper.step(u)
    return u
