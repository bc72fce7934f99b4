"""Pins for the oracle's exact IRK steps (Sec. 2; block system (3.2)).

Independent facts used:
* three routes -- assembled sparse LU, per-mode sine transform, eigen-
  decoupling of A -- reach the same step;
* ``sin(pi x) sin(pi y)`` is a discrete eigenvector of the heat operator, so
  ``u_n = R(-h lam_11)^n u_0`` with R the Pade approximant of exp (textbook
  closed form, independent of the tableau);
* against the semi-discrete solution ``exp(-lam_11 t) u_0`` the error falls at
  the order of Table 1 (2s for GL, 2s-1 for Radau IIA) when h_t halves;
* the discrete steady state of the double-glazing problem is a fixed point of
  every step.
"""
import math

import numpy as np
import pytest
import scipy.sparse.linalg as spla

from oracle.operators import double_glazing, heat_K, kappa_diffusion_K
from oracle.step import DirectStepper, EigenStepper, HeatDSTStepper, run_steps
from oracle.tableau import tableau
from paper_2010_11377_amd.workloads import fourier_modes, sine_mode, white_noise


def pade_value(k, j, z):
    P = sum(math.factorial(k + j - i) * math.factorial(k)
            / (math.factorial(k + j) * math.factorial(i) * math.factorial(k - i)) * z ** i
            for i in range(k + 1))
    Q = sum(math.factorial(k + j - i) * math.factorial(j)
            / (math.factorial(k + j) * math.factorial(i) * math.factorial(j - i)) * (-z) ** i
            for i in range(j + 1))
    return P / Q


@pytest.mark.parametrize("family,s", [("gauss", 2), ("radau_iia", 3), ("gauss", 4), ("lobatto_iiic", 3)])
def test_dst_matches_direct(family, s):
    n, h = 12, 0.01
    A, b, c = tableau(family, s)
    u0 = white_noise(n, seed=5)
    a = run_steps(DirectStepper(A, b, heat_K(n), h), u0, 3)
    d = run_steps(HeatDSTStepper(A, b, n, h), u0, 3)
    assert np.linalg.norm(a - d) <= 1e-12 * np.linalg.norm(a)


def test_eigen_matches_direct_double_glazing():
    n, eps, h = 16, 0.005, 5e-3
    A, b, c = tableau("radau_iia", 5)
    K, g = double_glazing(n, eps)
    u0 = np.zeros(n * n)
    a = run_steps(DirectStepper(A, b, K, h, g), u0, 4)
    e = run_steps(EigenStepper(A, b, K, h, g), u0, 4)
    assert np.linalg.norm(a - e) <= 1e-12 * np.linalg.norm(a)
    # the other fill-reducing ordering and threaded factorisation: same solve
    m = run_steps(EigenStepper(A, b, K, h, g, permc_spec="MMD_AT_PLUS_A", workers=3), u0, 4)
    assert np.linalg.norm(a - m) <= 1e-12 * np.linalg.norm(a)


def test_eigen_matches_direct_kappa():
    n, h = 10, 2e-3
    A, b, c = tableau("radau_iia", 3)
    kn = np.exp(0.5 * np.random.default_rng(7).standard_normal((n + 2, n + 2)))
    K = kappa_diffusion_K(kn)
    u0 = fourier_modes(n, seed=2)
    a = run_steps(DirectStepper(A, b, K, h), u0, 3)
    e = run_steps(EigenStepper(A, b, K, h), u0, 3)
    assert np.linalg.norm(a - e) <= 1e-12 * np.linalg.norm(a)


@pytest.mark.parametrize("family,s,kj", [("gauss", 2, (2, 2)), ("radau_iia", 3, (2, 3)),
                                          ("gauss", 7, (7, 7)), ("radau_iia", 5, (4, 5))])
def test_manufactured_eigenmode(family, s, kj):
    n, h, steps = 32, 0.01, 10
    hx = 1.0 / (n + 1)
    lam11 = 8.0 / hx ** 2 * math.sin(math.pi * hx / 2) ** 2
    A, b, c = tableau(family, s)
    u0 = sine_mode(n)
    u = run_steps(DirectStepper(A, b, heat_K(n), h), u0, steps)
    ref = pade_value(kj[0], kj[1], -h * lam11) ** steps * u0
    assert np.linalg.norm(u - ref) <= 1e-13 * np.linalg.norm(ref)


@pytest.mark.parametrize("family,s,p", [("gauss", 2, 4), ("radau_iia", 2, 3), ("radau_iia", 3, 5)])
def test_temporal_order(family, s, p):
    n, T = 32, 0.16
    hx = 1.0 / (n + 1)
    lam11 = 8.0 / hx ** 2 * math.sin(math.pi * hx / 2) ** 2
    A, b, c = tableau(family, s)
    u0 = sine_mode(n)
    errs = []
    hs = [0.04, 0.02, 0.01] if p >= 5 else [0.04, 0.02, 0.01, 0.005]
    for h in hs:
        nsteps = int(round(T / h))
        u = run_steps(HeatDSTStepper(A, b, n, h), u0, nsteps)
        errs.append(np.linalg.norm(u - math.exp(-lam11 * T) * u0) / np.linalg.norm(u0))
    ratios = [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]
    assert abs(math.log2(ratios[-1]) - p) < 0.3, (errs, ratios)


def test_double_glazing_steady_state_is_fixed_point():
    n, eps, h = 20, 0.005, 5e-3
    A, b, c = tableau("radau_iia", 5)
    K, g = double_glazing(n, eps)
    ustar = spla.spsolve(K.tocsc(), g)
    u1 = DirectStepper(A, b, K, h, g).step(ustar)
    assert np.linalg.norm(u1 - ustar) <= 1e-12 * np.linalg.norm(ustar)


def test_l_stable_step_kills_stiff_modes():
    """Radau IIA with h lam >> 1 sends the top sine mode towards R(-inf) = 0
    (R_{2,3}(z) ~ -3/z), GL keeps |R(-inf)| = 1."""
    n = 16
    A, b, c = tableau("radau_iia", 3)
    u0 = sine_mode(n, n, n)
    u = HeatDSTStepper(A, b, n, 1.0).step(u0)
    hlam = 8.0 * (n + 1) ** 2 * math.sin(n * math.pi / (2 * (n + 1))) ** 2
    assert np.linalg.norm(u) < 3.2 / hlam * np.linalg.norm(u0)
    A, b, c = tableau("gauss", 3)
    u = HeatDSTStepper(A, b, n, 1.0).step(u0)
    assert np.linalg.norm(u) > 0.95 * np.linalg.norm(u0)
