"""GPU tests of the preconditioner replayed from HIP graphs (option graphs = 1,
opt-in) against direct launches (graphs = 0, the default).

Both run the same kernels in the same order on the same data, so every
result must be bit-identical.  Each test replays the captured graphs many
times with the solver's own eager work (SpMM, Gram-Schmidt, Givens, host
synchronisation) between replays and compares every step:

* forward steps, FP32 V-cycles and FP64, several grids and tableaux;
* the preconditioner entry point called repeatedly on new inputs;
* left preconditioning (FP64);
* the adjoint step, and an operator update, which must drop the captured
  graphs (their kernel arguments point at the replaced operators);
* the graph cache: one graph per Krylov column, one replay per iteration (and
  at most one per step for a column enqueued ahead of the convergence check).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

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


def pair(dev, family, s, K, n, h, **kw):
    from paper_2010_11377_amd.solver import IRKSolver
    A, b, c = tableaux.tableau(family, s)
    g = IRKSolver(A, b, c, K, h, (n, n), graphs=True, device=dev, **kw)
    d = IRKSolver(A, b, c, K, h, (n, n), graphs=False, device=dev, **kw)
    return g, d


@pytest.mark.parametrize("family,s,n,h,steps,precision", [
    ("gauss", 2, 64, 1e-2, 4, "mixed"),
    ("radau_iia", 3, 256, 1e-3, 5, "mixed"),
    ("radau_iia", 3, 256, 1e-3, 3, "fp64"),
    ("gauss", 7, 512, 1e-3, 3, "mixed"),
    ("radau_iia", 5, 96, 5e-3, 3, "fp64"),
])
def test_steps_identical(dev, family, s, n, h, steps, precision):
    say("case graph steps %s s=%d n=%d h=%g %s" % (family, s, n, h, precision))
    G, D = pair(dev, family, s, problems.heat(n), n, h, precision=precision)
    ug = torch.tensor(workloads.fourier_modes(n, seed=0), dtype=torch.float64, device=dev)
    ud = ug.clone()
    iters, most = 0, 0
    for k in range(steps):
        ug = G.step(ug)
        ud = D.step(ud)
        assert G.last_stats.iters == D.last_stats.iters
        iters += G.last_stats.iters
        most = max(most, G.last_stats.iters)
        assert torch.equal(ug, ud), "step %d differs" % k
    ng, reps = G.graph_stats()
    say("  %d graphs, %d replays, %d iterations" % (ng, reps, iters))
    # one replay per Krylov iteration, plus at most one per step for a column
    # enqueued ahead of a convergence check that then stopped the iteration;
    # one graph per column used
    assert iters <= reps <= iters + steps and 1 <= ng <= most + 1
    assert D.graph_stats() == (0, 0)
    G.close()
    D.close()


def test_preconditioner_entry_point_identical(dev):
    n, h = 128, 1e-2
    say("case graph preconditioner n=%d" % n)
    G, D = pair(dev, "radau_iia", 3, problems.heat(n), n, h, precision="mixed")
    rng = np.random.default_rng(5)
    for r in range(4):
        v = torch.tensor(rng.standard_normal(3 * n * n), dtype=torch.float64, device=dev)
        assert torch.equal(G.apply_preconditioner(v), D.apply_preconditioner(v)), r
    assert G.graph_stats() == (1, 4)
    G.close()
    D.close()


def test_left_identical(dev):
    n, h = 128, 2e-3
    say("case graph left n=%d" % n)
    G, D = pair(dev, "radau_iia", 3, problems.heat(n), n, h, side="left")
    ug = torch.tensor(workloads.fourier_modes(n, seed=0), dtype=torch.float64, device=dev)
    ud = ug.clone()
    for k in range(3):
        ug = G.step(ug)
        ud = D.step(ud)
        assert torch.equal(ug, ud), k
    assert G.graph_stats()[1] > 0
    G.close()
    D.close()


def test_adjoint_and_operator_update_identical(dev):
    n, h = 64, 2e-3
    say("case graph adjoint + operator update n=%d" % n)
    kn = np.exp(workloads.gaussian_random_field(n + 2, seed=3))
    G, D = pair(dev, "radau_iia", 3, problems.kappa_diffusion(kn), n, h, rtol=1e-12)
    rng = np.random.default_rng(9)
    u = torch.tensor(rng.standard_normal(n * n), dtype=torch.float64, device=dev)
    lam = torch.tensor(rng.standard_normal(n * n), dtype=torch.float64, device=dev)
    assert torch.equal(G.step(u), D.step(u))
    ag, ad = G.adjoint_step(u, lam), D.adjoint_step(u, lam)
    for x, y in zip(ag, ad):
        assert torch.equal(x, y)
    assert G.graph_stats()[0] > 0
    K2 = problems.kappa_diffusion(kn * 1.5)
    G.update_operator(K2)
    D.update_operator(K2)
    assert G.graph_stats()[0] == 0
    for _ in range(2):
        assert torch.equal(G.step(u), D.step(u))
        ag, ad = G.adjoint_step(u, lam), D.adjoint_step(u, lam)
        for x, y in zip(ag, ad):
            assert torch.equal(x, y)
    G.close()
    D.close()
