"""GPU parity of the HIP path against the CPU oracle, through the C ABI.

Element-by-element comparisons on seeded inputs at sizes the oracle solves in
seconds (several 256-thread tiles plus a ragged tail), the configured grids
where the oracle has an exact fast route (heat: sine transform), and
property checks (stage-system residual) at the largest double-glazing grid.

Tolerances:
* Kronecker SpMM (FP64): 1e-14 relative (a few roundings per entry);
* exact preconditioner (coarse level = whole grid) FP64: 1e-11; FP32: 1e-5;
* IRK steps: 1e-8 relative L2 after all steps, the accuracy target of the
  FGMRES outer iteration (residual tolerance rtol per step).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle.ldu import coefficient_matrix
from oracle.operators import double_glazing, heat_K, kappa_diffusion_K
from oracle.precond import apply_inverse, assemble
from oracle.step import DirectStepper, EigenStepper, HeatDSTStepper, run_steps, stage_matrix
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


def Solver(*args, **kw):
    from paper_2010_11377_amd.solver import IRKSolver
    return IRKSolver(*args, **kw)


def T(x, dev):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))


# ------------------------------------------------------------------ SpMM
@pytest.mark.parametrize("case", ["heat40_s1", "heat40_s2", "heat40_s3", "heat40_s7",
                                  "dg24_s5", "kappa20_s3"])
def test_kron_spmm(dev, case):
    say("case", case)
    rng = np.random.default_rng(11)
    if case.startswith("heat"):
        n = 40
        s = int(case.split("_s")[1])
        fam = "gauss" if s in (1, 2, 7) else "radau_iia"
        Kp, Ko = problems.heat(n), heat_K(n)
    elif case.startswith("dg"):
        n, s, fam = 24, 5, "radau_iia"
        Kp, Ko = problems.double_glazing(n, 0.005)[:3], double_glazing(n, 0.005)[0]
    else:
        n, s, fam = 20, 3, "radau_iia"
        kn = np.exp(workloads.gaussian_random_field(n + 2, seed=3))
        Kp, Ko = problems.kappa_diffusion(kn), kappa_diffusion_K(kn)
    h = 3e-3
    A, b, c = tableaux.tableau(fam, s)
    S = Solver(A, b, c, Kp, h, (n, n), device=dev)
    x = rng.standard_normal(s * n * n)
    y = S.apply_operator(T(x, dev)).cpu().numpy()
    Ao = oracle_tableau(fam, s)[0]
    ref = stage_matrix(Ao, Ko, h) @ x
    err = np.max(np.abs(y - ref)) / np.max(np.abs(ref))
    say("  spmm max rel err", err)
    assert err < 1e-14
    S.close()


# ------------------------------------------------------------------ preconditioner
@pytest.mark.parametrize("kind", ["LD", "DU", "GSL", "J"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_exact_preconditioner(dev, kind, precision):
    """coarse_max >= N: the V-cycle is a direct solve, so the GPU sweep must
    equal the oracle's exact block substitution (Sec. 4.2)."""
    say("case exact precond", kind, precision)
    n, s, h = 24, 3, 2e-3
    A, b, c = tableaux.tableau("radau_iia", s)
    Kp = problems.double_glazing(n, 0.005)[:3]
    S = Solver(A, b, c, Kp, h, (n, n), precond=kind, precision=precision, coarse_max=1024,
               device=dev)
    assert S.info()["levels"] == 1
    v = np.random.default_rng(5).standard_normal(s * n * n)
    z = S.apply_preconditioner(T(v, dev)).cpu().numpy()
    Ao = oracle_tableau("radau_iia", s)[0]
    ref = apply_inverse(coefficient_matrix(Ao, kind), double_glazing(n, 0.005)[0], h,
                        v.reshape(s, -1)).ravel()
    err = rel(z, ref)
    say("  rel err", err)
    assert err < (1e-11 if precision == "fp64" else 1e-5)
    S.close()


@pytest.mark.parametrize("problem", ["heat", "dg", "kappa"])
def test_vcycle_preconditioner_contracts(dev, problem):
    """With a real hierarchy, one V-cycle per block leaves a small relative
    residual || v - P z || / || v || (P assembled by the oracle)."""
    say("case vcycle contraction", problem)
    n, s, h = 64, 3, 1e-3
    A, b, c = tableaux.tableau("radau_iia", s)
    if problem == "heat":
        Kp, Ko = problems.heat(n), heat_K(n)
    elif problem == "dg":
        Kp, Ko = problems.double_glazing(n, 0.005)[:3], double_glazing(n, 0.005)[0]
    else:
        kn = np.exp(workloads.gaussian_random_field(n + 2, seed=3))
        Kp, Ko = problems.kappa_diffusion(kn), kappa_diffusion_K(kn)
    S = Solver(A, b, c, Kp, h, (n, n), device=dev)
    info = S.info()
    say("  levels", info)
    assert info["levels"] >= 3 and info["constant_coeff"] == (problem == "heat")
    v = np.random.default_rng(6).standard_normal(s * n * n)
    z = S.apply_preconditioner(T(v, dev)).cpu().numpy()
    Ao = oracle_tableau("radau_iia", s)[0]
    P = assemble(coefficient_matrix(Ao, "LD"), Ko, h)
    r = rel(P @ z, v)
    say("  relative preconditioner residual", r)
    assert r < 0.3
    S.close()


@pytest.mark.parametrize("problem,nx,ny,precision", [
    ("heat", 200, 136, "mixed"), ("heat", 200, 136, "fp64"), ("heat", 256, 256, "mixed"),
    ("heat", 512, 512, "mixed"), ("heat", 640, 416, "mixed"), ("heat", 1024, 1024, "mixed"),
    ("dg", 128, 128, "fp64"), ("dg", 128, 128, "mixed"),
    ("kappa", 128, 128, "fp64")])
def test_vcycle_preconditioner_matches_oracle(dev, problem, nx, ny, precision):
    """P_LD^-1 v with one V(2,2)-cycle per block against the oracle's plain
    sparse-matrix V-cycle (same hierarchy, smoother and transfers).  Grids
    span several register and LDS tiles with ragged edges, a mid level run by
    the multi-workgroup kernels and a one-workgroup tail."""
    from oracle.amg import apply_vcycle_preconditioner
    say("case vcycle vs oracle", problem, nx, ny, precision)
    s, h = 3, 1e-3
    A, b, c = tableaux.tableau("radau_iia", s)
    if problem == "heat":
        Kp, Ko = problems.heat(nx, ny=ny), heat_K(nx, ny=ny)
    elif problem == "dg":
        Kp, Ko = problems.double_glazing(nx, 0.005)[:3], double_glazing(nx, 0.005)[0]
    else:
        kn = np.exp(workloads.gaussian_random_field(nx + 2, seed=3))
        Kp, Ko = problems.kappa_diffusion(kn), kappa_diffusion_K(kn)
    S = Solver(A, b, c, Kp, h, (nx, ny), precision=precision, device=dev)
    say("  hierarchy", S.info())
    v = np.random.default_rng(12).standard_normal(s * nx * ny)
    z = S.apply_preconditioner(T(v, dev)).cpu().numpy()
    Ao = oracle_tableau("radau_iia", s)[0]
    ref = apply_vcycle_preconditioner(coefficient_matrix(Ao, "LD"), Ko, h, v.reshape(s, -1),
                                      nx, ny, nu=2, coarse_max=64,
                                      coarse_ratio=S.options.coarse_ratio).ravel()
    err = rel(z, ref)
    say("  rel err", err)
    assert err < (1e-11 if precision == "fp64" else 2e-5)
    S.close()


@pytest.mark.parametrize("problem,nx,ny,precision", [
    ("heat", 200, 136, "mixed"), ("heat", 200, 136, "fp64"), ("heat", 512, 512, "mixed"),
    ("heat", 512, 512, "fp64"), ("heat", 640, 416, "mixed"), ("heat", 1024, 1024, "mixed"),
    ("dg", 128, 128, "fp64"), ("dg", 256, 256, "mixed"), ("kappa", 128, 128, "fp64"),
    ("kappa", 192, 192, "mixed")])
def test_vcycle_jacobi_matches_oracle(dev, problem, nx, ny, precision):
    """The same with damped Jacobi smoothing (omega 0.8, two sweeps before and
    after the coarse correction) against the oracle's Jacobi V-cycle."""
    from oracle.amg import apply_vcycle_preconditioner
    say("case vcycle jacobi vs oracle", problem, nx, ny, precision)
    s, h = 3, 1e-3
    A, b, c = tableaux.tableau("radau_iia", s)
    if problem == "heat":
        Kp, Ko = problems.heat(nx, ny=ny), heat_K(nx, ny=ny)
    elif problem == "dg":
        Kp, Ko = problems.double_glazing(nx, 0.005)[:3], double_glazing(nx, 0.005)[0]
    else:
        kn = np.exp(workloads.gaussian_random_field(nx + 2, seed=3))
        Kp, Ko = problems.kappa_diffusion(kn), kappa_diffusion_K(kn)
    S = Solver(A, b, c, Kp, h, (nx, ny), precision=precision, smoother="jacobi",
               jacobi_omega=0.8, device=dev)
    say("  hierarchy", S.info())
    v = np.random.default_rng(12).standard_normal(s * nx * ny)
    z = S.apply_preconditioner(T(v, dev)).cpu().numpy()
    Ao = oracle_tableau("radau_iia", s)[0]
    ref = apply_vcycle_preconditioner(coefficient_matrix(Ao, "LD"), Ko, h, v.reshape(s, -1),
                                      nx, ny, nu=2, coarse_max=64,
                                      coarse_ratio=S.options.coarse_ratio, smoother="jacobi",
                                      omega=0.8).ravel()
    err = rel(z, ref)
    say("  rel err", err)
    assert err < (1e-11 if precision == "fp64" else 2e-5)
    S.close()


@pytest.mark.parametrize("problem,precision", [("heat", "mixed"), ("heat", "fp64"),
                                               ("dg", "mixed")])
def test_steps_with_jacobi_smoothing_match_oracle(dev, problem, precision):
    """Whole steps with damped Jacobi V-cycles reach the oracle's exact steps:
    heat 256^2 Gauss-Legendre 7 (h_t 1e-3, the 8-mode field) and double
    glazing 256^2 Radau IIA 5 (h_t 5e-3, from zero), five steps each."""
    say("case steps jacobi", problem, precision)
    n, steps = 256, 5
    if problem == "heat":
        fam, s, h = "gauss", 7, 1e-3
        A, b, c = tableaux.tableau(fam, s)
        S = Solver(A, b, c, problems.heat(n), h, (n, n), precision=precision, rtol=1e-10,
                   smoother="jacobi", device=dev)
        u0 = workloads.fourier_modes(n, seed=0)
        Ao, bo, _ = oracle_tableau(fam, s)
        ref = run_steps(HeatDSTStepper(Ao, bo, n, h), u0, steps)
    else:
        fam, s, h = "radau_iia", 5, 5e-3
        A, b, c = tableaux.tableau(fam, s)
        ip, ix, d, g = problems.double_glazing(n, 0.005)
        S = Solver(A, b, c, (ip, ix, d), h, (n, n), precision=precision, rtol=1e-10,
                   smoother="jacobi", device=dev)
        S.set_source(g)
        u0 = np.zeros(n * n)
        Ko, go = double_glazing(n, 0.005)
        Ao, bo, _ = oracle_tableau(fam, s)
        ref = run_steps(EigenStepper(Ao, bo, Ko, h, go), u0, steps)
    u = T(u0, dev)
    its = []
    for _ in range(steps):
        u = S.step(u)
        its.append(S.last_stats.iters)
    err = rel(u.cpu().numpy(), ref)
    say("  iterations %s, rel err %.2e" % (its, err))
    assert err <= 1e-8
    S.close()


# ------------------------------------------------------------------ steps
def test_step_c1_gl2_32(dev):
    """32x32 heat, sin(pi x) sin(pi y), GL2, h = 0.01, 10 steps, rtol 1e-10."""
    say("case C1")
    n, h, steps = 32, 0.01, 10
    A, b, c = tableaux.tableau("gauss", 2)
    S = Solver(A, b, c, problems.heat(n), h, (n, n), rtol=1e-10, device=dev)
    u0 = workloads.sine_mode(n)
    u = T(u0, dev)
    iters = []
    for _ in range(steps):
        u = S.step(u)
        iters.append(S.last_stats.iters)
    Ao, bo, _ = oracle_tableau("gauss", 2)
    ref = run_steps(DirectStepper(Ao, bo, heat_K(n), h), u0, steps)
    err = rel(u.cpu().numpy(), ref)
    say("  iters", iters, "rel err", err)
    assert err < 1e-9
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_step_c2_radau3_512(dev, precision):
    """512x512 heat, 8 random Fourier modes, Radau IIA3, h = 1e-3, 50 steps."""
    say("case C2", precision)
    n, h, steps = 512, 1e-3, 50
    A, b, c = tableaux.tableau("radau_iia", 3)
    # per-step residual 1e-9 keeps the error after 50 steps below 1e-8
    S = Solver(A, b, c, problems.heat(n), h, (n, n), precision=precision, rtol=1e-9, device=dev)
    u0 = workloads.fourier_modes(n, seed=0)
    u = T(u0, dev)
    its = []
    for _ in range(steps):
        u = S.step(u)
        its.append(S.last_stats.iters)
    Ao, bo, _ = oracle_tableau("radau_iia", 3)
    ref = run_steps(HeatDSTStepper(Ao, bo, n, h), u0, steps)
    err = rel(u.cpu().numpy(), ref)
    say("  iters", its[:5], "... mean %.1f" % np.mean(its), "rel err", err)
    assert err < 1e-8
    S.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_step_c4_gl7_2048(dev, precision):
    """2048x2048 heat, GL7, h = 1e-3, 10 steps (the benchmark workload)."""
    say("case C4", precision)
    n, h, steps = 2048, 1e-3, 10
    A, b, c = tableaux.tableau("gauss", 7)
    S = Solver(A, b, c, problems.heat(n), h, (n, n), precision=precision, rtol=1e-9, device=dev)
    u0 = workloads.fourier_modes(n, seed=0)
    u = T(u0, dev)
    its = []
    for _ in range(steps):
        u = S.step(u)
        its.append(S.last_stats.iters)
    S.close()
    Ao, bo, _ = oracle_tableau("gauss", 7)
    ref = run_steps(HeatDSTStepper(Ao, bo, n, h, workers=8), u0, steps)
    err = rel(u.cpu().numpy(), ref)
    say("  iters", its, "rel err", err)
    assert err < 1e-8


def test_step_c3_double_glazing_256(dev):
    """Double glazing at 256^2, Radau IIA5, h = 5e-3, 20 steps, FP32 V-cycles."""
    say("case C3-256")
    n, eps, h, steps = 256, 0.005, 5e-3, 20
    A, b, c = tableaux.tableau("radau_iia", 5)
    ip, ix, d, g = problems.double_glazing(n, eps)
    S = Solver(A, b, c, (ip, ix, d), h, (n, n), precision="mixed", device=dev)
    S.set_source(g)
    u = torch.zeros(n * n, dtype=torch.float64, device=dev)
    its = []
    for _ in range(steps):
        u = S.step(u)
        its.append(S.last_stats.iters)
    Ao, bo, _ = oracle_tableau("radau_iia", 5)
    Ko, go = double_glazing(n, eps)
    ref = run_steps(EigenStepper(Ao, bo, Ko, h, go), np.zeros(n * n), steps)
    err = rel(u.cpu().numpy(), ref)
    say("  iters", its, "rel err", err)
    assert err < 1e-8
    S.close()


def test_step_edge_cases(dev):
    say("case edge")
    # backward Euler (s = 1) on a grid that is not a multiple of the block size
    n, h = 30, 1e-2
    A, b, c = tableaux.tableau("radau_iia", 1)
    S = Solver(A, b, c, problems.heat(n), h, (n, n), rtol=1e-12, device=dev)
    u0 = workloads.white_noise(n, seed=4)
    u1 = S.step(T(u0, dev)).cpu().numpy()
    ref = DirectStepper(np.array([[1.0]]), np.array([1.0]), heat_K(n), h).step(u0)
    assert rel(u1, ref) < 1e-10
    # zero data: exact zero step, no iterations
    z = S.step(torch.zeros(n * n, dtype=torch.float64, device=dev))
    assert S.last_stats.iters == 0 and float(z.abs().max()) == 0.0
    S.close()
    # odd coarsest grid (50 -> 25, dense 625)
    n = 50
    A, b, c = tableaux.tableau("radau_iia", 2)
    S = Solver(A, b, c, problems.heat(n), h, (n, n), rtol=1e-10, device=dev)
    assert S.info()["levels"] == 2
    u0 = workloads.white_noise(n, seed=5)
    u1 = S.step(T(u0, dev)).cpu().numpy()
    Ao, bo, _ = oracle_tableau("radau_iia", 2)
    assert rel(u1, DirectStepper(Ao, bo, heat_K(n), h).step(u0)) < 1e-8
    # max_iter = 1 -> not converged, best iterate still written
    S2 = Solver(A, b, c, problems.heat(n), h, (n, n), rtol=1e-12, max_iter=1, device=dev)
    out = S2.step(T(u0, dev), allow_not_converged=True)
    from paper_2010_11377_amd import binding as B
    assert S2.last_stats.iters == 1
    with pytest.raises(B.IRKError):
        S2.step(T(u0, dev))
    assert np.isfinite(out.cpu().numpy()).all()
    # non-finite input
    bad = u0.copy()
    bad[7] = np.nan
    with pytest.raises(B.IRKError) as ei:
        S.step(T(bad, dev))
    assert ei.value.status == B.IRK_E_NONFINITE
    S.close()
    S2.close()
    # a grid that does not coarsen to <= 1024 unknowns is rejected
    n = 66
    with pytest.raises(B.IRKError):
        Solver(A, b, c, problems.heat(n), h, (n, n), device=dev)


def test_deterministic(dev):
    say("case determinism")
    n, h = 128, 1e-3
    A, b, c = tableaux.tableau("radau_iia", 3)
    S = Solver(A, b, c, problems.heat(n), h, (n, n), precision="mixed", device=dev)
    u0 = T(workloads.white_noise(n, seed=9), dev)
    a = S.step(u0).cpu().numpy()
    bb = S.step(u0).cpu().numpy()
    assert np.array_equal(a, bb)
    S.close()
