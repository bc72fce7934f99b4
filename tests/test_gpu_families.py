"""GPU step parity for the method families of Sec. 2 (Table 1) that the
paper's experiments use beyond the configured workloads: Lobatto IIIC
s = 2..5 and Radau IIA s = 6, 7, with the paper's time-step rule of Sec. 5.1
h_t = h_x^((p+1)/q) (p = 2, q the temporal order: 2s - 1 for Radau IIA,
2s - 2 for Lobatto IIIC).

Heat on a 128^2 grid, the 8-mode initial value (seed 0), three steps, FGMRES
tolerance 1e-13, in both precisions.  The oracle is the exact sine-transform
stepper, applied to the same input as each GPU step: every step's result must
match the exact step to 1e-9 relative L2.  Per step, not accumulated: at these
time steps (0.026 to 0.33 beyond Lobatto IIIC 2) one step shrinks the 8-mode
field by a factor 60 to 400, so after three steps the solution is 1e-5 to
1e-8 of the initial one and an accumulated relative error would measure the
decay, not the solve.  For the same reason the tolerance is 1e-13 (at 1e-12
the first Lobatto IIIC 5 step, which keeps 1/400 of the field, is off by
1.4e-9 of its result, 3.5e-12 of its input).  The accumulated error relative
to the initial norm is checked beside it.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.step import HeatDSTStepper, run_steps
from oracle.tableau import tableau as oracle_tableau
from paper_2010_11377_amd import problems, tableaux, workloads

pytestmark = pytest.mark.gpu

CASES = [("lobatto_iiic", 2), ("lobatto_iiic", 3), ("lobatto_iiic", 4), ("lobatto_iiic", 5),
         ("radau_iia", 6), ("radau_iia", 7)]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("family,s", CASES)
def test_family_steps_match_oracle(dev, family, s, precision):
    from paper_2010_11377_amd.solver import IRKSolver
    n, steps = 128, 3
    hx = 1.0 / (n + 1)
    q = 2 * s - 1 if family == "radau_iia" else 2 * s - 2
    h = hx ** (3.0 / q)
    A, b, c = tableaux.tableau(family, s)
    S = IRKSolver(A, b, c, problems.heat(n), h, (n, n), precision=precision, rtol=1e-13,
                  restart=60, max_iter=600, device=dev)
    u0 = workloads.fourier_modes(n, seed=0)
    Ao, bo, _ = oracle_tableau(family, s)
    exact = HeatDSTStepper(Ao, bo, n, h)
    u = torch.tensor(u0, dtype=torch.float64, device=dev)
    its, errs = [], []
    for _ in range(steps):
        un = u.cpu().numpy()
        u = S.step(u)
        its.append(S.last_stats.iters)
        ref = exact.step(un)
        errs.append(np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref))
    ref = run_steps(exact, u0, steps)
    acc = np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(u0)
    say("case %s s=%d %s h_t=%.4g: iterations %s, per-step rel err %s, after %d steps "
        "%.2e of ||u0|| (||u_%d|| / ||u0|| = %.1e)" % (
            family, s, precision, h, its, ["%.1e" % e for e in errs], steps, acc, steps,
            np.linalg.norm(ref) / np.linalg.norm(u0)))
    assert max(errs) <= 1e-9
    assert acc <= 1e-12
    S.close()
