"""GPU tests of restarted FGMRES (short restart lengths) and of the iteration
cap: the step reaches the oracle's exact step through many restart cycles,
with the next column's preconditioner enqueued ahead of the convergence check
at every column but the last of a cycle; a capped solve reports that it did
not converge and still returns its best iterate; a step written over its own
input equals the out-of-place step.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.operators import heat_K
from oracle.step import DirectStepper, run_steps
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


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("restart", [2, 3, 5])
def test_restarted_fgmres_matches_oracle(dev, precision, restart):
    from paper_2010_11377_amd.solver import IRKSolver
    n, h, steps = 64, 2e-3, 3
    say("case restart %d %s" % (restart, precision))
    A, b, c = tableaux.tableau("radau_iia", 3)
    S = IRKSolver(A, b, c, problems.heat(n), h, (n, n), precision=precision, restart=restart,
                  max_iter=600, rtol=1e-10, device=dev)
    u0 = workloads.fourier_modes(n, seed=0)
    u = torch.tensor(u0, dtype=torch.float64, device=dev)
    its, rst = [], []
    for _ in range(steps):
        u = S.step(u)
        its.append(S.last_stats.iters)
        rst.append(S.last_stats.restarts)
    S.close()
    Ao, bo, _ = oracle_tableau("radau_iia", 3)
    ref = run_steps(DirectStepper(Ao, bo, heat_K(n), h), u0, steps)
    err = np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref)
    say("  iterations %s, restarts %s, rel err %.2e" % (its, rst, err))
    assert min(rst) > 0
    assert err < 1e-8


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_iteration_cap(dev, precision):
    from paper_2010_11377_amd.binding import IRK_E_NOT_CONVERGED
    from paper_2010_11377_amd.solver import IRKSolver
    n, h = 64, 2e-3
    A, b, c = tableaux.tableau("gauss", 2)
    S = IRKSolver(A, b, c, problems.heat(n), h, (n, n), precision=precision, max_iter=3,
                  rtol=1e-12, device=dev)
    u0 = torch.tensor(workloads.fourier_modes(n, seed=0), dtype=torch.float64, device=dev)
    u1 = S.step(u0, allow_not_converged=True)
    assert S.last_stats.iters == 3 and S.last_status == IRK_E_NOT_CONVERGED
    # the best iterate after three iterations is a step closer to the exact one
    # than no step at all
    Ao, bo, _ = oracle_tableau("gauss", 2)
    ref = run_steps(DirectStepper(Ao, bo, heat_K(n), h), u0.cpu().numpy(), 1)
    e1 = np.linalg.norm(u1.cpu().numpy() - ref)
    e0 = np.linalg.norm(u0.cpu().numpy() - ref)
    say("case iteration cap %s: error %.2e (no step %.2e)" % (precision, e1, e0))
    assert e1 < 0.1 * e0
    S.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("restart", [40, 3])
def test_in_place_step(dev, precision, restart):
    """irk_step with u_{n+1} in the buffer of u_n (allowed by the interface)
    returns exactly the out-of-place result, also through restart cycles."""
    from paper_2010_11377_amd.solver import IRKSolver
    n, h = 80, 2e-3
    say("case in-place step restart %d %s" % (restart, precision))
    A, b, c = tableaux.tableau("radau_iia", 3)
    S = IRKSolver(A, b, c, problems.heat(n), h, (n, n), precision=precision, restart=restart,
                  max_iter=600, rtol=1e-10, device=dev)
    u = torch.tensor(workloads.fourier_modes(n, seed=2), dtype=torch.float64, device=dev)
    v = u.clone()
    for _ in range(3):
        u = S.step(u)
        S.step(v, out=v)
        assert torch.equal(u, v)
    S.close()
