"""GPU tests of the second classical Gram-Schmidt pass (option reorth: 1 always,
2 when the first pass removed more than half of ||w||^2) against the oracle's
exact step, beside the default single pass (reorth 0).  The grid (100 x 100,
three stages) gives the vector kernels of the second pass a ragged last block;
short restarts run the pass across several restart cycles.
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


def run(dev, precision, reorth, restart, n, h, steps):
    from paper_2010_11377_amd.solver import IRKSolver
    A, b, c = tableaux.tableau("radau_iia", 3)
    S = IRKSolver(A, b, c, problems.heat(n), h, (n, n), precision=precision, reorth=reorth,
                  restart=restart, max_iter=600, rtol=1e-10, device=dev)
    u = torch.tensor(workloads.fourier_modes(n, seed=0), dtype=torch.float64, device=dev)
    its = []
    for _ in range(steps):
        u = S.step(u)
        its.append(S.last_stats.iters)
    S.close()
    return u.cpu().numpy(), its


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
@pytest.mark.parametrize("reorth,restart", [(1, 40), (2, 40), (1, 3), (2, 3)])
def test_second_pass_matches_oracle(dev, precision, reorth, restart):
    n, h, steps = 100, 2e-3, 3
    say("case reorth %d restart %d %s" % (reorth, restart, precision))
    u, its = run(dev, precision, reorth, restart, n, h, steps)
    u0, its0 = run(dev, precision, 0, restart, n, h, steps)
    Ao, bo, _ = oracle_tableau("radau_iia", 3)
    ref = run_steps(DirectStepper(Ao, bo, heat_K(n), h), workloads.fourier_modes(n, seed=0),
                    steps)
    err = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    err0 = np.linalg.norm(u0 - ref) / np.linalg.norm(ref)
    say("  iterations %s (single pass %s), rel err %.2e (single pass %.2e)"
        % (its, its0, err, err0))
    assert err < 1e-8
    # the basis is orthogonal to working precision either way: the second pass
    # may save an iteration on a restart boundary but never changes the count
    # by more than one
    assert all(abs(a - b) <= 1 for a, b in zip(its, its0))
