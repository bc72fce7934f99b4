"""GPU tests of the per-class kernel timing (irk_profile_select / irk_profile_read),
which the benchmark's roofline figure comes from: the launch count and the
algorithmic bytes of the timed class follow from the iteration counts, the
timed steps return exactly the results of untimed ones (with and without the
preconditioner graphs), and an unknown class is refused.
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


def solver(dev, n, graphs):
    from paper_2010_11377_amd.solver import IRKSolver
    A, b, c = tableaux.tableau("radau_iia", 3)
    return IRKSolver(A, b, c, problems.heat(n), 1e-3, (n, n), precision="mixed",
                     graphs=graphs, device=dev)


def run(S, u0, steps):
    u, its = u0.clone(), []
    for _ in range(steps):
        u = S.step(u)
        its.append(S.last_stats.iters)
        assert S.last_stats.restarts == 0  # the byte counts below assume one cycle
    torch.cuda.synchronize()
    return u, its


@pytest.mark.parametrize("graphs", [False, True])
def test_profiled_classes(dev, graphs):
    n, steps, s = 256, 3, 3
    say("case profile classes graphs=%s" % graphs)
    S = solver(dev, n, graphs)
    u0 = torch.tensor(workloads.fourier_modes(n, seed=0), dtype=torch.float64, device=dev)
    ref, its = run(S, u0, steps)
    sN = s * n * n
    zb, vb = 4.0 * sN, 8.0 * sN  # FP32 preconditioned column, FP64 basis column
    # the first cycle's V_0 = 1 (x) f: the SpMM passes read one of its s blocks
    v0save = 8.0 * (sN - n * n)

    # Kronecker SpMM + first Gram-Schmidt update: once per iteration, reading z
    # and columns 0..j and writing column j+1 (constant coefficients: no matrix
    # bytes)
    S.profile_select("spmm_update")
    u, its2 = run(S, u0, steps)
    p = S.profile_read()
    assert torch.equal(u, ref) and its2 == its
    assert p["launches"] == sum(its)
    want = sum(zb + vb * (j + 2) - v0save for it in its for j in range(it))
    assert p["bytes"] == want
    assert p["ms"] > 0.0
    say("  spmm_update: %d launches, %.3f ms, %.0f bytes" % (p["launches"], p["ms"], p["bytes"]))

    S.profile_select("spmm_dots")
    u, _ = run(S, u0, steps)
    p = S.profile_read()
    assert torch.equal(u, ref)
    assert p["launches"] == sum(its)
    assert p["bytes"] == sum(zb + vb * (j + 1) - v0save for it in its for j in range(it))

    # the coupling pass runs once per coupled stage and preconditioner
    # application (the first block under P_LD has no coupling terms: its finest
    # passes form float(scale v_0) on load): once per iteration, plus at most
    # one column per step enqueued ahead of a convergence check that then
    # stopped the iteration
    S.profile_select("couple")
    u, _ = run(S, u0, steps)
    p = S.profile_read()
    assert torch.equal(u, ref)
    assert (s - 1) * sum(its) <= p["launches"] <= (s - 1) * (sum(its) + steps)

    # no second Gram-Schmidt pass by default: its classes never launch
    S.profile_select("vec_update")
    u, _ = run(S, u0, steps)
    assert torch.equal(u, ref) and S.profile_read()["launches"] == 0

    # selecting again resets the counters; stopping keeps them readable
    S.profile_select("vtail")
    assert S.profile_read() == {"launches": 0, "ms": 0.0, "bytes": 0.0}
    S.profile_select(None)
    u, _ = run(S, u0, steps)
    assert torch.equal(u, ref)
    S.close()


def test_unknown_class_refused(dev):
    from paper_2010_11377_amd import binding as B
    S = solver(dev, 64, False)
    for kc in (-2, len(B.KERNEL_CLASSES), 99):
        assert S.lib.irk_profile_select(S._h, kc) == B.IRK_E_INVALID
    S.close()
