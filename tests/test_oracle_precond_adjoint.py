"""Pins for the oracle's exact block preconditioner (Sec. 4, (4.1)-(4.3);
Sec. 4.2) and its discrete adjoint.

Independent facts used:
* block substitution with exact subsolves inverts the assembled Kronecker
  matrix ``I (x) M + h A~ (x) K``;
* for ``M = I`` and symmetric K, ``A P^-1`` is similar to the block diagonal
  of ``(I + h lam A)(I + h lam A~)^-1`` over the closed-form eigenvalues lam
  of K, so its dense spectrum on a tiny grid is that union of s x s spectra;
* the transposed step recursion is the transpose of the linear step map
  (dot-product test); the adjoint gradient matches central finite
  differences of the forward oracle.
"""
import numpy as np
import scipy.sparse as sp
import pytest

from oracle import adjoint
from oracle.ldu import coefficient_matrix
from oracle.operators import double_glazing, heat_eigenvalues, heat_K, kappa_diffusion_K
from oracle.precond import apply_inverse, assemble
from oracle.step import DirectStepper, stage_matrix
from oracle.tableau import tableau
from paper_2010_11377_amd.workloads import fd_directions, fourier_modes, gaussian_random_field

import scipy.sparse.linalg as spla


@pytest.mark.parametrize("kind", ["J", "GSL", "DU", "LD"])
def test_substitution_inverts_assembled(kind):
    n, h = 8, 5e-3
    A, b, c = tableau("radau_iia", 3)
    K, g = double_glazing(n, 0.005)
    At = coefficient_matrix(A, kind)
    v = np.random.default_rng(3).standard_normal((3, n * n))
    w = apply_inverse(At, K, h, v)
    ref = spla.spsolve(assemble(At, K, h), v.ravel()).reshape(3, -1)
    assert np.linalg.norm(w - ref) <= 1e-12 * np.linalg.norm(ref)


def _sorted_eigs(z):
    z = np.asarray(z)
    return z[np.lexsort((np.round(z.imag, 9), np.round(z.real, 9)))]


@pytest.mark.parametrize("kind", ["J", "GSL", "DU", "LD"])
@pytest.mark.parametrize("family,s", [("radau_iia", 3), ("gauss", 2), ("lobatto_iiic", 3)])
def test_dense_spectrum_is_union_of_blocks(kind, family, s):
    n, h = 5, 0.05
    A, b, c = tableau(family, s)
    At = coefficient_matrix(A, kind)
    K = heat_K(n)
    Acal = stage_matrix(A, K, h).toarray()
    P = assemble(At, K, h).toarray()
    dense = np.linalg.eigvals(Acal @ np.linalg.inv(P))
    blocks = []
    for lam in heat_eigenvalues(n).ravel():
        B = (np.eye(s) + h * lam * A) @ np.linalg.inv(np.eye(s) + h * lam * At)
        blocks.extend(np.linalg.eigvals(B))
    d, bl = _sorted_eigs(dense), _sorted_eigs(np.array(blocks))
    assert np.max(np.abs(d - bl)) < 1e-6
    if kind == "LD":
        # a transposed factor gives a different spectrum
        alt = []
        for lam in heat_eigenvalues(n).ravel():
            B = (np.eye(s) + h * lam * A) @ np.linalg.inv(np.eye(s) + h * lam * At.T)
            alt.extend(np.linalg.eigvals(B))
        assert np.max(np.abs(_sorted_eigs(np.array(alt)) - d)) > 1e-3


def test_step_map_dot_product():
    n, h, s = 7, 2e-3, 3
    A, b, c = tableau("radau_iia", s)
    kn = np.exp(0.5 * np.random.default_rng(4).standard_normal((n + 2, n + 2)))
    K = kappa_diffusion_K(kn)
    st = DirectStepper(A, b, K, h)
    rng = np.random.default_rng(9)
    u, lam = rng.standard_normal(n * n), rng.standard_normal(n * n)
    Su = st.step(u)
    psi = st.adjoint_stages(h * np.outer(b, lam))
    STlam = lam - K.T @ psi.sum(axis=0)
    assert abs(Su @ lam - u @ STlam) <= 1e-13 * abs(Su @ lam) + 1e-15


def test_adjoint_gradient_matches_finite_differences():
    n, h, steps, s = 8, 2e-3, 4, 3
    A, b, c = tableau("radau_iia", s)
    gfield = gaussian_random_field(n + 2, seed=3)
    kappa = np.exp(gfield)
    u0 = fourier_modes(n, seed=2)
    u_target = adjoint.forward(A, b, np.ones((n + 2, n + 2)), h, u0, steps)[0]
    J, grad = adjoint.gradient(A, b, kappa, h, u0, steps, u_target)
    assert J > 0
    for dg in fd_directions(n + 2, count=3):
        eps = 1e-4
        Jp = adjoint.objective(A, b, kappa * np.exp(eps * dg), h, u0, steps, u_target)
        Jm = adjoint.objective(A, b, kappa * np.exp(-eps * dg), h, u0, steps, u_target)
        fd = (Jp - Jm) / (2 * eps)
        an = float(np.sum(grad * kappa * dg))
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
    # corner nodes touch no face
    assert grad[0, 0] == 0.0 and grad[-1, -1] == 0.0


def test_face_gradient_matches_finite_differences():
    """dJ/dkappa_f against central differences in random face directions
    (the operator built from its face coefficients directly), and the nodal
    gradient as the half-and-half chain of the face gradient."""
    from oracle.operators import kappa_face_values
    n, h, steps, s = 8, 2e-3, 3, 3
    A, b, c = tableau("radau_iia", s)
    kappa = np.exp(gaussian_random_field(n + 2, seed=3))
    u0 = fourier_modes(n, seed=2)
    u_target = adjoint.forward(A, b, np.ones((n + 2, n + 2)), h, u0, steps)[0]
    J, g, gx, gy = adjoint.gradient(A, b, kappa, h, u0, steps, u_target, faces=True)
    kx, ky = kappa_face_values(kappa)
    assert abs(adjoint.objective_faces(A, b, kx, ky, h, u0, steps, u_target) - J) <= 1e-14 * J
    rng = np.random.default_rng(17)
    for _ in range(3):
        dx, dy = rng.standard_normal(kx.shape), rng.standard_normal(ky.shape)
        eps = 1e-4
        Jp = adjoint.objective_faces(A, b, kx * np.exp(eps * dx), ky * np.exp(eps * dy), h, u0,
                                     steps, u_target)
        Jm = adjoint.objective_faces(A, b, kx * np.exp(-eps * dx), ky * np.exp(-eps * dy), h, u0,
                                     steps, u_target)
        fd = (Jp - Jm) / (2 * eps)
        an = float(np.sum(gx * kx * dx) + np.sum(gy * ky * dy))
        assert abs(fd - an) <= 1e-6 * abs(an), (fd, an)
    # a single face: the east face of interior node (2, 3)
    e = np.zeros_like(kx)
    e[3, 3] = 1.0
    eps = 1e-5
    fd = (adjoint.objective_faces(A, b, kx + eps * e, ky, h, u0, steps, u_target)
          - adjoint.objective_faces(A, b, kx - eps * e, ky, h, u0, steps, u_target)) / (2 * eps)
    assert abs(fd - gx[3, 3]) <= 1e-6 * abs(gx[3, 3])
    # nodal = each face's gradient split equally between its two nodes
    chain = np.zeros_like(g)
    chain[1:-1, :-1] += 0.5 * gx
    chain[1:-1, 1:] += 0.5 * gx
    chain[:-1, 1:-1] += 0.5 * gy
    chain[1:, 1:-1] += 0.5 * gy
    assert np.allclose(chain, g, rtol=0, atol=1e-15 * np.abs(g).max())


def test_fgmres_pins():
    """FGMRES: with the exact inverse as preconditioner one iteration gives the
    exact solution; unpreconditioned on an n x n system it reaches the direct
    solution in at most n iterations; its estimate equals the true residual;
    restarts still converge."""
    import scipy.sparse.linalg as spla
    from oracle.krylov import fgmres
    from oracle.operators import double_glazing
    K = double_glazing(6, 0.005)[0]
    A = (sp.identity(36) + 3e-3 * K).tocsc()
    b = np.random.default_rng(3).standard_normal(36)
    ref = spla.spsolve(A, b)
    x, its, _ = fgmres(lambda v: A @ v, lambda v: spla.spsolve(A, v), b, rtol=1e-13)
    assert its == 1 and np.linalg.norm(x - ref) <= 1e-12 * np.linalg.norm(ref)
    x, its, hist = fgmres(lambda v: A @ v, lambda v: v, b, rtol=1e-12)
    assert its <= 36 and np.linalg.norm(x - ref) <= 1e-10 * np.linalg.norm(ref)
    assert abs(np.linalg.norm(b - A @ x) / np.linalg.norm(b) - hist[-1]) <= 1e-12
    x, its, _ = fgmres(lambda v: A @ v, lambda v: v, b, rtol=1e-10, restart=5, max_iter=500)
    assert its > 5 and np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b) * 1.0001
