"""GPU tests of the piecewise-constant multigrid interpolation (P = R^T),
the option for advection-dominated operators at large time steps (the
double-glazing problem of Sec. 3.2 with eps = 0.005, where the Galerkin
coarse operators under linear interpolation stop being M-matrices).

* one preconditioner application equals the oracle's V-cycle reading with
  the same interpolation (double glazing and heat, FP64 and mixed);
* steps of the eps = 0.005 double glazing at h_t = 1 converge and match the
  oracle's exact steps.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.amg import apply_vcycle_preconditioner
from oracle.ldu import coefficient_matrix
from oracle.operators import double_glazing, heat_K
from oracle.step import EigenStepper, run_steps
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


@pytest.mark.parametrize("which,n,h,precision", [("dg", 128, 1.0, "fp64"), ("dg", 128, 1.0, "mixed"),
                                                 ("heat", 256, 1e-2, "fp64"),
                                                 ("heat", 256, 1e-2, "mixed")])
def test_constant_interp_preconditioner_matches_oracle(dev, which, n, h, precision):
    from paper_2010_11377_amd.solver import IRKSolver
    say("case constant interpolation preconditioner %s n=%d h=%g %s" % (which, n, h, precision))
    A, b, c = tableaux.tableau("radau_iia", 3)
    K = problems.double_glazing(n, 0.005)[:3] if which == "dg" else problems.heat(n)
    S = IRKSolver(A, b, c, K, h, (n, n), precision=precision, interp="constant", device=dev)
    v = np.random.default_rng(12).standard_normal((3, n * n))
    z = S.apply_preconditioner(torch.tensor(v.ravel(), dtype=torch.float64, device=dev))
    z = z.cpu().numpy().reshape(3, n * n)
    cr = S.options.coarse_ratio
    S.close()
    Ko = double_glazing(n, 0.005)[0] if which == "dg" else heat_K(n)
    Ao, _, _ = oracle_tableau("radau_iia", 3)
    ref = apply_vcycle_preconditioner(coefficient_matrix(Ao, "LD"), Ko, h, v, n, n,
                                      interp="constant", coarse_ratio=cr)
    err = np.linalg.norm(z - ref) / np.linalg.norm(ref)
    say("  rel err %.2e" % err)
    assert err < (1e-11 if precision == "fp64" else 2e-5)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_double_glazing_large_step_converges(dev, precision):
    from paper_2010_11377_amd.solver import IRKSolver
    n, h, steps = 128, 1.0, 3
    say("case double glazing eps=0.005 h=1 constant interpolation %s" % precision)
    A, b, c = tableaux.tableau("radau_iia", 3)
    ip, ix, d, g = problems.double_glazing(n, 0.005)
    S = IRKSolver(A, b, c, (ip, ix, d), h, (n, n), precision=precision, interp="constant",
                  rtol=1e-10, max_iter=400, device=dev)
    S.set_source(torch.tensor(g, dtype=torch.float64, device=dev))
    u = torch.zeros(n * n, dtype=torch.float64, device=dev)
    its = []
    for _ in range(steps):
        u = S.step(u)
        its.append(S.last_stats.iters)
    S.close()
    Ko, go = double_glazing(n, 0.005)
    Ao, bo, _ = oracle_tableau("radau_iia", 3)
    ref = run_steps(EigenStepper(Ao, bo, Ko, h, g=go), np.zeros(n * n), steps)
    err = np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref)
    say("  iterations %s, rel err %.2e" % (its, err))
    assert err < 1e-8
