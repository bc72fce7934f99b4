"""GPU test of irk_step_noalloc (the step on the library's static scratch,
no device allocation in the call) against irk_step, through the C ABI.

Two solvers, used one after the other on the one static array: a 96 x 96
Radau IIA 3 heat solver, then a smaller 48 x 48 Gauss-Legendre 2 one, in
both precisions; two calls in a row each (the second solver's calls find the
first's data in the scratch).  Each result must equal irk_step's bit for bit
(the same kernels in the same order on other buffers) and the stage count
and iterations must agree.  A solver whose step does not fit the array is
refused with IRK_E_INVALID before any kernel runs.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.operators import heat_K
from oracle.step import DirectStepper
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


def _solver(dev, family, s, n, h, precision):
    from paper_2010_11377_amd.solver import IRKSolver
    A, b, c = tableaux.tableau(family, s)
    return IRKSolver(A, b, c, problems.heat(n), h, (n, n), precision=precision, rtol=1e-10,
                     device=dev)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_noalloc_step_equals_step(dev, precision):
    cases = [("radau_iia", 3, 96, 1e-3), ("gauss", 2, 48, 1e-2)]   # second one smaller
    for family, s, n, h in cases:
        say("case noalloc %s %s s=%d n=%d" % (precision, family, s, n))
        S = _solver(dev, family, s, n, h, precision)
        u = torch.tensor(workloads.fourier_modes(n, seed=0), dtype=torch.float64, device=dev)
        for call in range(2):
            ref = S.step(u)
            it_ref = S.last_stats.iters
            out = torch.empty_like(u)
            S.step_noalloc(u, out)
            it = S.last_stats.iters
            same = bool(torch.equal(out, ref))
            err = float(torch.linalg.norm(out - ref) / torch.linalg.norm(ref))
            say("  call %d: iterations %d / %d, bit-identical %s, rel diff %.1e" % (
                call, it, it_ref, same, err))
            assert it == it_ref
            assert same
            u = out
        # and against the oracle's exact step
        Ao, bo, _ = oracle_tableau(family, s)
        un = u.cpu().numpy()
        out = torch.empty_like(u)
        S.step_noalloc(u, out)
        ex = DirectStepper(Ao, bo, heat_K(n), h).step(un)
        e = np.linalg.norm(out.cpu().numpy() - ex) / np.linalg.norm(ex)
        say("  against the oracle: rel err %.2e" % e)
        assert e <= 1e-8
        S.close()


def test_noalloc_refuses_a_step_beyond_the_scratch(dev):
    from paper_2010_11377_amd.binding import IRK_E_INVALID, IRKError
    n = 256
    S = _solver(dev, "gauss", 7, n, 1e-3, "fp64")   # about 300 MB of step buffers
    u = torch.zeros(n * n, dtype=torch.float64, device=dev)
    with pytest.raises(IRKError) as ei:
        S.step_noalloc(u, torch.empty_like(u))
    assert ei.value.status == IRK_E_INVALID
    assert "scratch" in str(ei.value)
    say("  refused: %s" % ei.value)
    S.close()
