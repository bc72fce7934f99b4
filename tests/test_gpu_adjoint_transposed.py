"""GPU tests of the adjoint step for a non-symmetric K (the double-glazing
advection-diffusion operator, Sec. 3.2): the transposed stage system
``(I + h A^T (x) K^T) psi = h (b (x) lam)`` is solved by a second solver of
the same kind built on A^T and K^T.

* psi and lam_n = lam - K^T sum_i psi_i against the oracle's sparse LU of the
  transposed stage matrix, in both precisions of the V-cycles;
* the dot-product identity of the linear part of the step map,
  <S u, lam> = <u, S^T lam> with S u = step(u) - step(0) (the source g makes
  the step affine);
* after irk_update_operator (a different wind strength) the adjoint uses the
  new K^T: the oracle's result for the new operator.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.operators import double_glazing
from oracle.step import DirectStepper
from oracle.tableau import tableau as oracle_tableau
from paper_2010_11377_amd import problems, tableaux

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def make(n, eps, h, dev, precision="fp64", s=5):
    from paper_2010_11377_amd.solver import IRKSolver
    A, b, c = tableaux.tableau("radau_iia", s)
    ip, ix, d, g = problems.double_glazing(n, eps)
    S = IRKSolver(A, b, c, (ip, ix, d), h, (n, n), precision=precision, rtol=1e-12, device=dev)
    S.set_source(g)
    return S


def oracle_adjoint(n, eps, h, lam, s=5):
    Ao, bo, _ = oracle_tableau("radau_iia", s)
    Ko, go = double_glazing(n, eps)
    st = DirectStepper(Ao, bo, Ko, h, go)
    psi = st.adjoint_stages(h * np.outer(bo, lam))
    return psi, lam - Ko.T @ psi.sum(axis=0)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


@pytest.mark.parametrize("n,precision", [(64, "fp64"), (64, "mixed"), (128, "mixed")])
def test_transposed_adjoint_matches_oracle(dev, n, precision):
    say("case transposed adjoint", n, precision)
    eps, h = 0.005, 5e-3
    S = make(n, eps, h, dev, precision)
    rng = np.random.default_rng(41)
    u = torch.tensor(rng.random(n * n), dtype=torch.float64, device=dev)
    lam = rng.standard_normal(n * n)
    lam_n, psi, _ = S.adjoint_step(u, torch.tensor(lam, dtype=torch.float64, device=dev))
    psi_ref, lam_ref = oracle_adjoint(n, eps, h, lam)
    e_psi, e_lam = rel(psi.cpu().numpy(), psi_ref), rel(lam_n.cpu().numpy(), lam_ref)
    say("  psi rel err %.2e  lam rel err %.2e  iterations %d" % (e_psi, e_lam,
                                                                 S.last_stats.iters))
    assert e_psi <= 1e-9 and e_lam <= 1e-9
    S.close()


def test_transposed_adjoint_dot_product(dev):
    say("case transposed adjoint dot product")
    n, eps, h = 96, 0.005, 5e-3
    S = make(n, eps, h, dev)
    rng = np.random.default_rng(42)
    u = torch.tensor(rng.standard_normal(n * n), dtype=torch.float64, device=dev)
    lam = torch.tensor(rng.standard_normal(n * n), dtype=torch.float64, device=dev)
    zero = torch.zeros_like(u)
    Su = S.step(u) - S.step(zero)
    lam_n, _, _ = S.adjoint_step(u, lam)
    lhs, rhs = float(torch.dot(Su, lam)), float(torch.dot(u, lam_n))
    say("  <Su,lam> %.15e  <u,S^T lam> %.15e" % (lhs, rhs))
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)
    S.close()


def test_transposed_adjoint_after_operator_update(dev):
    say("case transposed adjoint after update_operator")
    n, h = 64, 5e-3
    S = make(n, 0.005, h, dev)
    rng = np.random.default_rng(43)
    u = torch.tensor(rng.random(n * n), dtype=torch.float64, device=dev)
    lam = rng.standard_normal(n * n)
    lt = torch.tensor(lam, dtype=torch.float64, device=dev)
    S.adjoint_step(u, lt)  # sets up the transposed solver for eps = 0.005
    ip, ix, d, g = problems.double_glazing(n, 0.02)
    S.update_operator((ip, ix, d))
    S.set_source(g)
    lam_n, psi, _ = S.adjoint_step(u, lt)
    psi_ref, lam_ref = oracle_adjoint(n, 0.02, h, lam)
    e_psi, e_lam = rel(psi.cpu().numpy(), psi_ref), rel(lam_n.cpu().numpy(), lam_ref)
    say("  psi rel err %.2e  lam rel err %.2e" % (e_psi, e_lam))
    assert e_psi <= 1e-9 and e_lam <= 1e-9
    S.close()
