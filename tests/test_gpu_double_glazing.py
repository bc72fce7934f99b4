"""GPU tests of the double-glazing configuration (Sec. 3.2, (3.3)): 1024^2
interior grid on [-1, 1]^2, eps = 1/200, first-order upwind advection, hot
east wall, Radau IIA 5, h_t = 5e-3, 20 steps, FP32 V-cycles inside FP64
FGMRES.

At the full size the whole 20-step run is compared with the oracle's
eigen-decoupled exact stepper (one real and two complex sparse LUs of the
1024^2 blocks, minimum-degree ordering, factored in threads: about a minute of
host time).  Every fifth step is also checked by properties that hold at any
size: the stage vectors the GPU returns satisfy the stage system
``(I + h A (x) K) k = 1 (x) (g - K u_n)`` to the solver tolerance (residual
evaluated on the CPU with the oracle's K), and
``u_{n+1} = u_n + h sum_i b_i k_i``.  The same comparison runs at 512^2.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.operators import double_glazing
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


def solver_for(n, dev, rtol=1e-9):
    from paper_2010_11377_amd.solver import IRKSolver
    A, b, c = tableaux.tableau("radau_iia", 5)
    ip, ix, d, g = problems.double_glazing(n, 0.005)
    S = IRKSolver(A, b, c, (ip, ix, d), 5e-3, (n, n), precision="mixed", rtol=rtol, device=dev)
    S.set_source(g)
    return S


@pytest.mark.timeout(900)
def test_double_glazing_1024_against_oracle(dev):
    say("case DG 1024 oracle and properties")
    n, h, steps = 1024, 5e-3, 20
    S = solver_for(n, dev)
    info = S.info()
    say("  hierarchy", info)
    assert not info["constant_coeff"]
    Ko, go = double_glazing(n, 0.005)
    Ao, bo, _ = oracle_tableau("radau_iia", 5)
    s = 5
    u = torch.zeros(n * n, dtype=torch.float64, device=dev)
    its, states = [], []
    for step in range(steps):
        un = u.cpu().numpy()
        u, k = S.step_stages(u)
        its.append(S.last_stats.iters)
        states.append(u.cpu().numpy())
        if step % 5 == 0 or step == steps - 1:
            kk = k.cpu().numpy()
            f = go - Ko @ un
            Kk = np.stack([Ko @ kk[i] for i in range(s)])
            res = np.tile(f, (s, 1)) - (kk + h * (Ao @ Kk))
            rel = np.linalg.norm(res) / (np.sqrt(s) * np.linalg.norm(f))
            u1 = states[-1]
            upd = np.linalg.norm(u1 - (un + h * (bo @ kk))) / np.linalg.norm(u1)
            say("  step %2d iters %d  stage residual %.2e  update %.2e" % (step, its[-1], rel, upd))
            assert rel <= 2e-9
            assert upd <= 1e-13
    ufin = states[-1]
    assert ufin.min() > -1e-8 and ufin.max() < 1.0 + 1e-8   # discrete maximum principle
    say("  iterations", its)
    S.close()
    say("  oracle: factoring the 1024^2 blocks")
    st = EigenStepper(Ao, bo, Ko, h, go, permc_spec="MMD_AT_PLUS_A", workers=3)
    ref = np.zeros(n * n)
    worst = 0.0
    for step in range(steps):
        ref = st.step(ref)
        err = np.linalg.norm(states[step] - ref) / np.linalg.norm(ref)
        worst = max(worst, err)
        if step % 5 == 0 or step == steps - 1:
            say("  step %2d rel err vs oracle %.2e" % (step, err))
    say("  worst rel err over the 20 steps %.2e" % worst)
    assert worst <= 1e-8


def test_double_glazing_512_against_oracle(dev):
    say("case DG 512 oracle")
    n, h, steps = 512, 5e-3, 20
    S = solver_for(n, dev)
    u = torch.zeros(n * n, dtype=torch.float64, device=dev)
    for _ in range(steps):
        u = S.step(u)
    Ko, go = double_glazing(n, 0.005)
    Ao, bo, _ = oracle_tableau("radau_iia", 5)
    ref = run_steps(EigenStepper(Ao, bo, Ko, h, go), np.zeros(n * n), steps)
    err = np.linalg.norm(u.cpu().numpy() - ref) / np.linalg.norm(ref)
    say("  rel err %.2e" % err)
    assert err <= 1e-8
    S.close()
