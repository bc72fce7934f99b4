"""Discrete adjoint of the IRK time stepper for ``u_t = div(kappa grad u)``
(homogeneous Dirichlet, ``M = I``, no source) and the gradient of
``J = 1/2 ||u_N - u_target||^2`` with respect to nodal ``kappa``.

The paper has no adjoint; this is the exact derivative of the discrete
stepper of Sec. 2 / Sec. 3.1 written out:

* forward:  ``Acal k = -1 (x) K u_n``,  ``u_{n+1} = u_n + h (b^T (x) I) k``,
  with ``Acal = I + h A (x) K``, stage values ``U_i = u_n + h sum_j a_ij k_j``;
* backward: ``lam_N = u_N - u_target``; for n = N-1..0 solve
  ``Acal^T psi = h (b (x) lam_{n+1})`` and set
  ``lam_n = lam_{n+1} - K^T sum_i psi_i``;
* parameters: ``K = sum_f kappa_f K_f`` over faces, so
  ``dJ/dkappa_f = - sum_n sum_i psi_i^T K_f U_i
               = - h^-2 sum_n sum_i (psi_iP - psi_iQ)(U_iP - U_iQ)``
  (boundary values of psi and U are zero), and with
  ``kappa_f = (kappa_P + kappa_Q)/2`` every face passes half of its
  gradient to each of its two nodes.

Test infrastructure only (see the package docstring).
"""
import numpy as np

from .operators import face_diffusion_K, kappa_diffusion_K
from .step import DirectStepper


def forward(A, b, kappa_nodes, h, u0, nsteps, length=1.0, K=None):
    """Run the exact stepper; returns (u_N, list of (u_n, U_n) per step).
    ``K`` given: use it instead of the operator of ``kappa_nodes``."""
    if K is None:
        K = kappa_diffusion_K(kappa_nodes, length)
    st = DirectStepper(A, b, K, h)
    A = np.asarray(A, dtype=np.float64)
    u = np.array(u0, dtype=np.float64)
    tape = []
    for _ in range(nsteps):
        k = st.stages(u)
        U = u[None, :] + h * (A @ k)
        tape.append((u.copy(), U))
        u = u + h * (np.asarray(b) @ k)
    return u, tape, st


def objective(A, b, kappa_nodes, h, u0, nsteps, u_target, length=1.0):
    uN, _, _ = forward(A, b, kappa_nodes, h, u0, nsteps, length)
    r = uN - u_target
    return 0.5 * float(r @ r)


def objective_faces(A, b, kx, ky, h, u0, nsteps, u_target, length=1.0):
    """J for an operator given by its face coefficients (``face_diffusion_K``)."""
    uN, _, _ = forward(A, b, None, h, u0, nsteps, length, K=face_diffusion_K(kx, ky, length))
    r = uN - u_target
    return 0.5 * float(r @ r)


def gradient(A, b, kappa_nodes, h, u0, nsteps, u_target, length=1.0, faces=False):
    """``(J, dJ/dkappa_nodes)``, the gradient with the shape of kappa_nodes
    ((n+2) x (n+2)).  ``faces=True`` returns ``(J, g, gx, gy)`` with the face
    gradients ``gx`` (n, n+1) and ``gy`` (n+1, n) laid out as the face
    coefficients of ``kappa_face_values``."""
    kn = np.asarray(kappa_nodes, dtype=np.float64)
    n = kn.shape[0] - 2
    hx = length / (n + 1)
    s = len(b)
    uN, tape, st = forward(A, b, kn, h, u0, nsteps, length)
    K = st.K
    r = uN - u_target
    J = 0.5 * float(r @ r)
    lam = r.copy()
    gx = np.zeros((n, n + 1))   # faces between (i-1, j) and (i, j), full-grid i
    gy = np.zeros((n + 1, n))   # faces between (i, j-1) and (i, j), full-grid j
    for (u_n, U) in reversed(tape):
        mu = h * np.outer(b, lam)
        psi = st.adjoint_stages(mu)
        for i in range(s):
            P = np.zeros((n + 2, n + 2))
            Q = np.zeros((n + 2, n + 2))
            P[1:-1, 1:-1] = psi[i].reshape(n, n)
            Q[1:-1, 1:-1] = U[i].reshape(n, n)
            dpx = P[1:-1, 1:] - P[1:-1, :-1]
            dux = Q[1:-1, 1:] - Q[1:-1, :-1]
            dpy = P[1:, 1:-1] - P[:-1, 1:-1]
            duy = Q[1:, 1:-1] - Q[:-1, 1:-1]
            gx -= dpx * dux / (hx * hx)
            gy -= dpy * duy / (hx * hx)
        lam = lam - K.T @ psi.sum(axis=0)
    g = np.zeros((n + 2, n + 2))
    g[1:-1, :-1] += 0.5 * gx
    g[1:-1, 1:] += 0.5 * gx
    g[:-1, 1:-1] += 0.5 * gy
    g[1:, 1:-1] += 0.5 * gy
    if faces:
        return J, g, gx, gy
    return J, g
