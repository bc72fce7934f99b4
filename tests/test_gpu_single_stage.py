"""GPU tests of the degenerate one-stage methods: implicit midpoint (Gauss 1)
and backward Euler (Radau IIA 1).  With s = 1 the stage system is the single
block M + h a_11 K, every preconditioner kind reduces to one V-cycle on it,
and the step must still reach the oracle's exact step (96 x 96 grid)."""
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
@pytest.mark.parametrize("family", ["gauss", "radau_iia"])
def test_one_stage_matches_oracle(dev, family, precision):
    from paper_2010_11377_amd.solver import IRKSolver
    n, h, steps = 96, 5e-3, 4
    say("case one stage %s %s" % (family, precision))
    A, b, c = tableaux.tableau(family, 1)
    u0 = workloads.fourier_modes(n, seed=1)
    Ao, bo, _ = oracle_tableau(family, 1)
    ref = run_steps(DirectStepper(Ao, bo, heat_K(n), h), u0, steps)
    outs = {}
    for kind in ("LD", "J"):
        S = IRKSolver(A, b, c, problems.heat(n), h, (n, n), precision=precision, precond=kind,
                      rtol=1e-11, device=dev)
        u = torch.tensor(u0, dtype=torch.float64, device=dev)
        its = []
        for _ in range(steps):
            u = S.step(u)
            its.append(S.last_stats.iters)
        S.close()
        outs[kind] = u
        err = np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref)
        say("  %s: iterations %s, rel err %.2e" % (kind, its, err))
        assert err < 1e-9
    # one block: P_LD and P_J are the same operator, so the runs are identical
    assert torch.equal(outs["LD"], outs["J"])
