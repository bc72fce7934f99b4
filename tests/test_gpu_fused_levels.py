"""GPU tests of the paired intermediate levels (two nine-point levels per
launch in each direction of the FP32 V-cycle).

A node of a paired level goes through the same operations as in the
one-level passes; the compiler may contract a multiply and an add into one
FMA differently in the two kernels, so the FP32 results agree to rounding
(observed: 4e-7 of max |z|), not bit for bit.  A solver with the pairs (the
default) is compared with one without them (fuse_levels=False) on P_LD^-1 v
for heat grids whose hierarchies pair every intermediate level (512^2 ..
2048^2), ragged grids where only some levels pair (640 x 416, 512 x 256), a
grid with no pair (256^2), cycles that end inside a pair (small
coarse ratios), and whole steps; in FP64 the two agree to 1e-13.  Blocks
whose cycle ends on the tail's first level run that level's smoothing as one
multi-workgroup pass (k_s9smooth) with the option on and through the
one-workgroup tail with it off, so these comparisons cover that pass too
(every grid here has such blocks, the 256^2 one no pair).  A wrong class, halo or hand-over would
show as an O(1) error at the nodes it touches.  The oracle comparison of the
V-cycle itself runs in test_gpu_parity.py on the default (paired) path.
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


def pair_of_solvers(nx, ny, dev, fam="gauss", s=7, h=1e-3, precision="mixed", **kw):
    from paper_2010_11377_amd.solver import IRKSolver
    A, b, c = tableaux.tableau(fam, s)
    K = problems.heat(nx, ny=ny)
    on = IRKSolver(A, b, c, K, h, (nx, ny), precision=precision, device=dev, **kw)
    off = IRKSolver(A, b, c, K, h, (nx, ny), precision=precision, fuse_levels=False, device=dev,
                    **kw)
    return on, off


def compare(z_on, z_off, nx, ny, tol=1e-5):
    diff = int((z_on != z_off).sum())
    dmax = float((z_on - z_off).abs().max() / z_off.abs().max())
    say("  differing entries %d of %d, max diff / max |z| %.3e" % (diff, z_on.numel(), dmax))
    assert dmax <= tol
    return diff


@pytest.mark.parametrize("nx,ny,precision", [
    (256, 256, "mixed"), (512, 512, "mixed"), (1024, 1024, "mixed"), (2048, 2048, "mixed"),
    (640, 416, "mixed"), (512, 256, "mixed"), (512, 512, "fp64"), (1024, 1024, "fp64"),
    (640, 416, "fp64")])
def test_paired_vcycle(dev, nx, ny, precision):
    say("case paired V-cycle", nx, ny, precision)
    on, off = pair_of_solvers(nx, ny, dev, precision=precision)
    say("  hierarchy", on.info())
    v = torch.tensor(np.random.default_rng(12).standard_normal(7 * nx * ny), dtype=torch.float64,
                     device=dev)
    z_on = on.apply_preconditioner(v)
    z_off = off.apply_preconditioner(v)
    torch.cuda.synchronize()
    compare(z_on, z_off, nx, ny, tol=1e-5 if precision == "mixed" else 1e-13)
    on.close()
    off.close()


@pytest.mark.parametrize("ratio", [8.0, 64.0])
def test_paired_vcycle_cycle_end(dev, ratio):
    """Blocks whose cycle ends at an intermediate level: the pair that holds
    the end level takes a zero coarse correction."""
    say("case paired V-cycle, coarse ratio", ratio)
    n = 1024
    on, off = pair_of_solvers(n, n, dev, coarse_ratio=ratio)
    v = torch.tensor(np.random.default_rng(13).standard_normal(7 * n * n), dtype=torch.float64,
                     device=dev)
    z_on = on.apply_preconditioner(v)
    z_off = off.apply_preconditioner(v)
    torch.cuda.synchronize()
    compare(z_on, z_off, n, n)
    on.close()
    off.close()


def test_paired_steps(dev):
    say("case paired steps 1024^2 GL7")
    n = 1024
    on, off = pair_of_solvers(n, n, dev)
    u0 = torch.tensor(workloads.fourier_modes(n, seed=0), dtype=torch.float64, device=dev)
    u_on, u_off = u0, u0
    for _ in range(3):
        u_on = on.step(u_on)
        u_off = off.step(u_off)
        say("  iterations", on.last_stats.iters, off.last_stats.iters)
        assert abs(on.last_stats.iters - off.last_stats.iters) <= 1
    torch.cuda.synchronize()
    rel = float((u_on - u_off).norm() / u_off.norm())
    say("  rel diff of the states %.3e" % rel)
    assert rel <= 1e-8
    on.close()
    off.close()
