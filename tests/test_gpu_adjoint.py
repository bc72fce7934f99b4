"""GPU tests of the discrete adjoint IRK step and dJ/dkappa (kappa-diffusion,
u_t = div(kappa grad u), homogeneous Dirichlet, Radau IIA 3).

* dot-product test: the adjoint step is the transpose of the (linear) step
  map, <S u, lam> = <u, S^T lam>;
* parity with the CPU oracle's adjoint gradient on a small grid;
* central finite differences of J on 16 seeded directions at the 256^2,
  20-step configuration (J = 1/2 ||u_T - u_target||^2, u_target from kappa = 1,
  kappa = exp(g) with g a Gaussian random field);
* parity with the oracle's adjoint gradient (nodal and per face) at the
  configured 256^2, 20-step size;
* a backward that runs after another forward on the same solver (a different
  kappa) still uses its own forward's operator;
* an operator update (new kappa) leaves the solver bit-identical to a fresh
  setup with that kappa.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import adjoint as oracle_adjoint
from oracle.tableau import tableau as oracle_tableau
from paper_2010_11377_amd import problems, tableaux, workloads

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def make_solver(n, kn, h, dev, rtol=1e-12):
    from paper_2010_11377_amd.solver import IRKSolver
    A, b, c = tableaux.tableau("radau_iia", 3)
    return IRKSolver(A, b, c, problems.kappa_diffusion(kn), h, (n, n), rtol=rtol, device=dev)


def test_adjoint_dot_product(dev):
    say("case adjoint dot product")
    n, h = 32, 2e-3
    kn = np.exp(workloads.gaussian_random_field(n + 2, seed=3))
    S = make_solver(n, kn, h, dev)
    rng = np.random.default_rng(21)
    u = torch.tensor(rng.standard_normal(n * n), dtype=torch.float64, device=dev)
    lam = torch.tensor(rng.standard_normal(n * n), dtype=torch.float64, device=dev)
    Su = S.step(u)
    lam0, psi, U = S.adjoint_step(u, lam)
    lhs = float(torch.dot(Su, lam))
    rhs = float(torch.dot(u, lam0))
    say("  <Su,lam> %.15e  <u,S^T lam> %.15e" % (lhs, rhs))
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)
    # the stage values U_i = u + h sum_j a_ij k_j match a stage solve
    u1, k = S.step_stages(u)
    A = oracle_tableau("radau_iia", 3)[0]
    Uref = u.cpu().numpy()[None, :] + h * (A @ k.cpu().numpy())
    assert np.linalg.norm(U.cpu().numpy() - Uref) <= 1e-12 * np.linalg.norm(Uref)
    S.close()


def test_gradient_matches_oracle_adjoint(dev):
    say("case adjoint vs oracle")
    from paper_2010_11377_amd.autograd import IRKDiffusionFn
    n, h, steps = 16, 2e-3, 4
    hx = 1.0 / (n + 1)
    kn = np.exp(workloads.gaussian_random_field(n + 2, seed=3))
    u0 = workloads.fourier_modes(n, seed=2)
    Ao, bo, _ = oracle_tableau("radau_iia", 3)
    u_tgt = oracle_adjoint.forward(Ao, bo, np.ones((n + 2, n + 2)), h, u0, steps)[0]
    J_ref, g_ref = oracle_adjoint.gradient(Ao, bo, kn, h, u0, steps, u_tgt)
    S = make_solver(n, kn, h, dev)
    kt = torch.tensor(kn, dtype=torch.float64, device=dev, requires_grad=True)
    u0t = torch.tensor(u0, dtype=torch.float64, device=dev)
    uT = IRKDiffusionFn.apply(kt, u0t, S, steps, hx)
    J = 0.5 * torch.sum((uT - torch.tensor(u_tgt, device=dev)) ** 2)
    J.backward()
    g = kt.grad.cpu().numpy()
    say("  J %.6e (oracle %.6e), grad rel err %.2e" % (float(J.detach()), J_ref,
        np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)))
    assert abs(float(J.detach()) - J_ref) <= 1e-9 * J_ref
    assert np.linalg.norm(g - g_ref) <= 1e-7 * np.linalg.norm(g_ref)
    S.close()


@pytest.mark.timeout(600)
def test_gradient_matches_oracle_adjoint_256(dev):
    """The configured size: 256^2, Radau IIA 3, h_t = 2e-3, 20 steps.  J, the
    nodal gradient (autograd path) and the face gradient
    (irk_grad_diffusion_faces) against the oracle's exact adjoint."""
    say("case adjoint vs oracle 256")
    from paper_2010_11377_amd.autograd import IRKDiffusionFn
    n, h, steps = 256, 2e-3, 20
    hx = 1.0 / (n + 1)
    kn = np.exp(workloads.gaussian_random_field(n + 2, seed=3))
    u0 = workloads.fourier_modes(n, seed=2)
    Ao, bo, _ = oracle_tableau("radau_iia", 3)
    S = make_solver(n, kn, h, dev)
    u0t = torch.tensor(u0, dtype=torch.float64, device=dev)
    with torch.no_grad():
        u_tgt_t = IRKDiffusionFn.apply(torch.ones(n + 2, n + 2, dtype=torch.float64), u0t, S,
                                       steps, hx).clone()
    u_tgt_ref = oracle_adjoint.forward(Ao, bo, np.ones((n + 2, n + 2)), h, u0, steps)[0]
    tgt_err = np.linalg.norm(u_tgt_t.cpu().numpy() - u_tgt_ref) / np.linalg.norm(u_tgt_ref)
    say("  target state rel err %.2e" % tgt_err)
    assert tgt_err <= 1e-10
    # both sides use the oracle's target so that J is the same function
    u_tgt = torch.tensor(u_tgt_ref, dtype=torch.float64, device=dev)
    kt = torch.tensor(kn, dtype=torch.float64, device=dev, requires_grad=True)
    uT = IRKDiffusionFn.apply(kt, u0t, S, steps, hx)
    J = 0.5 * torch.sum((uT - u_tgt) ** 2)
    J.backward()
    g = kt.grad.cpu().numpy()
    # face gradient through the ABI, from the same checkpoints
    S.update_operator(problems.kappa_diffusion(kn))
    u = u0t
    ckpt = []
    for _ in range(steps):
        ckpt.append(u)
        u = S.step(u)
    lam = (u - u_tgt).contiguous()
    nfx, nfy = n * (n + 1), (n + 1) * n
    gface = torch.zeros(nfx + nfy, dtype=torch.float64, device=dev)
    for u_n in reversed(ckpt):
        lam, psi, U = S.adjoint_step(u_n, lam)
        S.grad_diffusion_faces(psi, U, hx, gface)
    gf = gface.cpu().numpy()
    J_ref, g_ref, gx_ref, gy_ref = oracle_adjoint.gradient(Ao, bo, kn, h, u0, steps, u_tgt_ref,
                                                           faces=True)
    e_nodes = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    gfr = np.concatenate([gx_ref.ravel(), gy_ref.ravel()])
    e_faces = np.linalg.norm(gf - gfr) / np.linalg.norm(gfr)
    say("  J %.10e (oracle %.10e)  nodal grad rel err %.2e  face grad rel err %.2e" % (
        float(J.detach()), J_ref, e_nodes, e_faces))
    assert abs(float(J.detach()) - J_ref) <= 1e-9 * J_ref
    assert e_nodes <= 1e-7
    assert e_faces <= 1e-7
    S.close()


def test_backward_after_another_forward(dev):
    """forward(kappa_1), forward(kappa_2), then backward of the first: the
    gradient is the oracle's at kappa_1 (the shared solver holds kappa_2's
    operator when the backward starts)."""
    say("case adjoint backward after another forward")
    from paper_2010_11377_amd.autograd import IRKDiffusionFn
    n, h, steps = 16, 2e-3, 4
    hx = 1.0 / (n + 1)
    k1 = np.exp(workloads.gaussian_random_field(n + 2, seed=3))
    k2 = np.exp(workloads.gaussian_random_field(n + 2, seed=4))
    u0 = workloads.fourier_modes(n, seed=2)
    Ao, bo, _ = oracle_tableau("radau_iia", 3)
    u_tgt = oracle_adjoint.forward(Ao, bo, np.ones((n + 2, n + 2)), h, u0, steps)[0]
    J_ref, g_ref = oracle_adjoint.gradient(Ao, bo, k1, h, u0, steps, u_tgt)
    S = make_solver(n, np.ones((n + 2, n + 2)), h, dev)
    u0t = torch.tensor(u0, dtype=torch.float64, device=dev)
    tgt = torch.tensor(u_tgt, device=dev)
    kt1 = torch.tensor(k1, dtype=torch.float64, device=dev, requires_grad=True)
    kt2 = torch.tensor(k2, dtype=torch.float64, device=dev, requires_grad=True)
    J1 = 0.5 * torch.sum((IRKDiffusionFn.apply(kt1, u0t, S, steps, hx) - tgt) ** 2)
    J2 = 0.5 * torch.sum((IRKDiffusionFn.apply(kt2, u0t, S, steps, hx) - tgt) ** 2)
    J1.backward()
    e1 = np.linalg.norm(kt1.grad.cpu().numpy() - g_ref) / np.linalg.norm(g_ref)
    say("  first backward rel err %.2e" % e1)
    assert e1 <= 1e-7
    J2.backward()
    g2_ref = oracle_adjoint.gradient(Ao, bo, k2, h, u0, steps, u_tgt)[1]
    e2 = np.linalg.norm(kt2.grad.cpu().numpy() - g2_ref) / np.linalg.norm(g2_ref)
    say("  second backward rel err %.2e" % e2)
    assert e2 <= 1e-7
    S.close()


def test_gradient_finite_differences_256(dev):
    """The configured case: 256^2, Radau IIA 3, h_t = 2e-3, 20 steps, 16 FD
    directions (seeds 100-115), kappa perturbed as kappa * exp(eps dg)."""
    say("case adjoint FD 256")
    from paper_2010_11377_amd.autograd import IRKDiffusionFn
    n, h, steps = 256, 2e-3, 20
    hx = 1.0 / (n + 1)
    gfield = workloads.gaussian_random_field(n + 2, seed=3)
    kn = np.exp(gfield)
    u0t = torch.tensor(workloads.fourier_modes(n, seed=2), dtype=torch.float64, device=dev)
    S = make_solver(n, np.ones((n + 2, n + 2)), h, dev)
    with torch.no_grad():
        u_tgt = IRKDiffusionFn.apply(torch.ones(n + 2, n + 2, dtype=torch.float64), u0t, S,
                                     steps, hx).clone()

    def objective(kappa):
        with torch.no_grad():
            uT = IRKDiffusionFn.apply(torch.tensor(kappa, dtype=torch.float64), u0t, S, steps, hx)
            return 0.5 * float(torch.sum((uT - u_tgt) ** 2))

    kt = torch.tensor(kn, dtype=torch.float64, requires_grad=True)
    uT = IRKDiffusionFn.apply(kt, u0t, S, steps, hx)
    J = 0.5 * torch.sum((uT - u_tgt) ** 2)
    J.backward()
    grad = kt.grad.numpy()
    say("  J = %.6e, adjoint iterations of the last step %d" % (float(J.detach()), S.last_stats.iters))
    worst, worst_fixed = 0.0, 0.0
    for idx, dg in enumerate(workloads.fd_directions(n + 2, count=16)):
        an = float(np.sum(grad * kn * dg))
        errs = {}
        for eps in (1e-3, 1e-4, 1e-5, 1e-6):
            fd = (objective(kn * np.exp(eps * dg)) - objective(kn * np.exp(-eps * dg))) / (2 * eps)
            errs[eps] = abs(fd - an) / abs(an)
        best = min(errs.values())
        say("  direction %2d  dJ = %+.10e  best rel err %.2e  at eps 1e-4 %.2e" % (
            idx, an, best, errs[1e-4]))
        worst = max(worst, best)
        worst_fixed = max(worst_fixed, errs[1e-4])
    say("  worst best-eps error %.2e, worst error at the fixed eps 1e-4 %.2e" % (worst, worst_fixed))
    assert worst <= 1e-6
    assert worst_fixed <= 1e-4
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_update_operator_equals_fresh_setup(dev, precision):
    """irk_update_operator (new kappa: stiffness and hierarchy rebuilt, buffers
    kept) leaves the solver in the state a fresh setup with that kappa has:
    forward and adjoint steps agree bit for bit."""
    from paper_2010_11377_amd.solver import IRKSolver
    say("case update operator %s" % precision)
    n, h = 96, 2e-3
    A, b, c = tableaux.tableau("radau_iia", 3)
    k1 = np.exp(workloads.gaussian_random_field(n + 2, seed=3))
    k2 = np.exp(workloads.gaussian_random_field(n + 2, seed=4))
    S = IRKSolver(A, b, c, problems.kappa_diffusion(k1), h, (n, n), precision=precision,
                  rtol=1e-11, device=dev)
    F = IRKSolver(A, b, c, problems.kappa_diffusion(k2), h, (n, n), precision=precision,
                  rtol=1e-11, device=dev)
    rng = np.random.default_rng(5)
    u = torch.tensor(rng.standard_normal(n * n), dtype=torch.float64, device=dev)
    lam = torch.tensor(rng.standard_normal(n * n), dtype=torch.float64, device=dev)
    S.step(u)  # runs with the first kappa before the update
    S.update_operator(problems.kappa_diffusion(k2))
    for _ in range(2):
        assert torch.equal(S.step(u), F.step(u))
        assert S.last_stats.iters == F.last_stats.iters
        for x, y in zip(S.adjoint_step(u, lam), F.adjoint_step(u, lam)):
            assert torch.equal(x, y)
    S.close()
    F.close()
