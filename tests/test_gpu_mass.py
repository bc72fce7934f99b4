"""GPU tests of the stage system with a mass matrix (Sec. 3.1 and Sec. 4:
``(I_s (x) M + h A (x) K) k = 1_s (x) (-K u_n)``), on the heat equation with
linear elements on right triangles (seven-point consistent mass matrix, the
five-point stiffness matrix).

* steps: FP64 and mixed solves reach the oracle's exact steps (sparse LU of
  the assembled stage matrix, or the eigen-decoupled route on larger grids);
* the Kronecker product ``(I (x) M + h A (x) K) x`` through the C ABI equals
  the oracle's assembled matrix times x;
* one preconditioner application with V-cycle subsolves equals the oracle's
  V-cycle reading with the hierarchy started from M, and with a single level
  the exact ``P^-1 v``;
* the adjoint step (transposed stage system with M^T) matches the oracle's
  transposed solve;
* iteration counts stay flat in h_x at the paper's h_t rule (printed).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.amg import apply_vcycle_preconditioner
from oracle.fem import p1_heat as oracle_p1
from oracle.ldu import coefficient_matrix
from oracle.precond import apply_inverse
from oracle.step import DirectStepper, EigenStepper, run_steps, stage_matrix
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


def solver(dev, family, s, n, h, **kw):
    from paper_2010_11377_amd.solver import IRKSolver
    A, b, c = tableaux.tableau(family, s)
    M, K = problems.p1_heat(n)
    return IRKSolver(A, b, c, K, h, (n, n), M=M, device=dev, **kw)


@pytest.mark.parametrize("family,s,n,h,steps,precision", [
    ("radau_iia", 3, 64, 2e-3, 5, "fp64"),
    ("radau_iia", 3, 64, 2e-3, 5, "mixed"),
    ("gauss", 2, 96, 5e-3, 4, "mixed"),
    ("radau_iia", 5, 256, 2e-3, 3, "fp64"),
    ("gauss", 7, 256, 1e-3, 3, "mixed"),
])
def test_mass_steps_match_oracle(dev, family, s, n, h, steps, precision):
    say("case mass steps %s s=%d n=%d h=%g %s" % (family, s, n, h, precision))
    S = solver(dev, family, s, n, h, precision=precision, rtol=1e-11)
    u0 = workloads.fourier_modes(n, seed=0)
    u = torch.tensor(u0, dtype=torch.float64, device=dev)
    its = []
    for _ in range(steps):
        u = S.step(u)
        its.append(S.last_stats.iters)
    S.close()
    Mo, Ko = oracle_p1(n)
    Ao, bo, _ = oracle_tableau(family, s)
    st = DirectStepper(Ao, bo, Ko, h, M=Mo) if n <= 96 else EigenStepper(Ao, bo, Ko, h, M=Mo)
    ref = run_steps(st, u0, steps)
    err = np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref)
    say("  iterations %s, rel err %.2e" % (its, err))
    assert err < 1e-9


def test_mass_apply_operator(dev):
    n, h = 48, 3e-3
    S = solver(dev, "radau_iia", 3, n, h)
    x = np.random.default_rng(2).standard_normal(3 * n * n)
    y = S.apply_operator(torch.tensor(x, dtype=torch.float64, device=dev)).cpu().numpy()
    S.close()
    Mo, Ko = oracle_p1(n)
    Ao, _, _ = oracle_tableau("radau_iia", 3)
    ref = stage_matrix(Ao, Ko, h, Mo) @ x
    assert np.linalg.norm(y - ref) <= 1e-14 * np.linalg.norm(ref)


@pytest.mark.parametrize("n,precision,coarse_max", [(32, "fp64", 1024), (128, "fp64", 64),
                                                    (128, "mixed", 64), (256, "mixed", 64)])
def test_mass_preconditioner_matches_oracle(dev, n, precision, coarse_max):
    say("case mass preconditioner n=%d %s coarse_max=%d" % (n, precision, coarse_max))
    h = 1e-2
    S = solver(dev, "radau_iia", 3, n, h, precision=precision, coarse_max=coarse_max)
    v = np.random.default_rng(12).standard_normal((3, n * n))
    z = S.apply_preconditioner(torch.tensor(v.ravel(), dtype=torch.float64, device=dev))
    z = z.cpu().numpy().reshape(3, n * n)
    cr = S.options.coarse_ratio
    S.close()
    Mo, Ko = oracle_p1(n)
    Ao, _, _ = oracle_tableau("radau_iia", 3)
    At = coefficient_matrix(Ao, "LD")
    if coarse_max >= n * n:
        ref = apply_inverse(At, Ko, h, v, M=Mo)
    else:
        ref = apply_vcycle_preconditioner(At, Ko, h, v, n, n, coarse_max=coarse_max, M=Mo,
                                          coarse_ratio=cr)
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    say("  rel err %.2e" % err)
    assert err < (1e-11 if precision == "fp64" else 2e-5)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_mass_adjoint_matches_oracle(dev, precision):
    """psi = (I (x) M + h A (x) K)^-T h (b (x) lam) and lam_n = lam - K^T sum psi
    against the oracle's sparse LU of the transposed stage matrix."""
    say("case mass adjoint", precision)
    n, h = 48, 5e-3
    S = solver(dev, "radau_iia", 3, n, h, precision=precision, rtol=1e-12)
    rng = np.random.default_rng(31)
    u = rng.standard_normal(n * n)
    lam = rng.standard_normal(n * n)
    ut = torch.tensor(u, dtype=torch.float64, device=dev)
    lt = torch.tensor(lam, dtype=torch.float64, device=dev)
    lam_n, psi, U = S.adjoint_step(ut, lt)
    Ao, bo, _ = oracle_tableau("radau_iia", 3)
    Mo, Ko = oracle_p1(n)
    st = DirectStepper(Ao, bo, Ko, h, M=Mo)
    psi_ref = st.adjoint_stages(h * np.outer(bo, lam))
    lam_ref = lam - Ko.T @ psi_ref.sum(axis=0)
    e_psi = np.linalg.norm(psi.cpu().numpy().ravel() - psi_ref.ravel()) / np.linalg.norm(psi_ref)
    e_lam = np.linalg.norm(lam_n.cpu().numpy() - lam_ref) / np.linalg.norm(lam_ref)
    say("  psi rel err %.2e  lam rel err %.2e" % (e_psi, e_lam))
    assert e_psi <= 1e-9 and e_lam <= 1e-9
    # the stage values come from the forward stages
    k = st.stages(u)
    Uref = u[None, :] + h * (Ao @ k)
    assert np.linalg.norm(U.cpu().numpy() - Uref) <= 1e-9 * np.linalg.norm(Uref)
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_mass_iterations_mesh_independent(dev, precision):
    counts = {}
    for n in (64, 128, 256, 512):
        hx = 1.0 / (n + 1)
        h = hx ** (3.0 / 5.0)                          # Radau IIA 3: q = 5
        S = solver(dev, "radau_iia", 3, n, h, precision=precision, rtol=1e-8)
        u = torch.tensor(workloads.fourier_modes(n, seed=0), dtype=torch.float64, device=dev)
        its = []
        for _ in range(2):
            u = S.step(u)
            its.append(S.last_stats.iters)
        S.close()
        counts[n] = max(its)
    say("case linear elements h_x independence (Radau IIA 3, P_LD, %s): %s" % (precision, counts))
    v = list(counts.values())
    assert max(v) <= 1.5 * min(v) + 1
