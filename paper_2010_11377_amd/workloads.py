"""Seeded synthetic inputs shared by the GPU path's tests, the benchmark and
the oracle checks.  This module holds input data only: grids of initial
values, random coefficient fields and random directions.  It contains none of
the solver's arithmetic and imports neither the oracle nor the HIP library.

All randomness is drawn from ``numpy.random.default_rng(seed)``.

Grid convention: ``n x n`` interior nodes of the square ``[lo, hi]^2``,
spacing ``h = (hi - lo) / (n + 1)``, flat index ``j * n + i`` with ``x``
fastest.
"""
import numpy as np


def interior_axis(n, lo=0.0, hi=1.0):
    h = (hi - lo) / (n + 1)
    return lo + h * np.arange(1, n + 1)


def sine_mode(n, p=1, q=1):
    """``sin(p pi x) sin(q pi y)`` on the interior of the unit square."""
    t = interior_axis(n)
    return (np.sin(q * np.pi * t)[:, None] * np.sin(p * np.pi * t)[None, :]).ravel()


def fourier_modes(n, seed=0, modes=8, max_freq=16):
    """Sum of ``modes`` products ``a_m sin(p_m pi x) sin(q_m pi y)`` with
    ``a_m ~ N(0, 1)`` and distinct ``(p_m, q_m)`` drawn uniformly from
    ``{1..max_freq}^2``."""
    rng = np.random.default_rng(seed)
    flat = rng.choice(max_freq * max_freq, size=modes, replace=False)
    amps = rng.standard_normal(modes)
    t = interior_axis(n)
    u = np.zeros((n, n))
    for f, a in zip(flat, amps):
        p = int(f % max_freq) + 1
        q = int(f // max_freq) + 1
        u += a * np.sin(q * np.pi * t)[:, None] * np.sin(p * np.pi * t)[None, :]
    return u.ravel()


def white_noise(n, seed=1):
    return np.random.default_rng(seed).standard_normal(n * n)


def gaussian_random_field(m, seed=3, length=0.1, sigma=0.5, lo=0.0, hi=1.0):
    """Zero-mean Gaussian random field on the full ``m x m`` node grid of
    ``[lo, hi]^2`` (boundary nodes included, spacing ``(hi-lo)/(m-1)``) with
    covariance ``sigma^2 exp(-r^2 / (2 length^2))``.  The kernel separates,
    ``C = C_y (x) C_x``, so a sample is ``B_y Z B_x^T`` with ``B = V sqrt(max(w,
    0))`` from the eigendecomposition of each 1-D factor."""
    t = np.linspace(lo, hi, m)
    d = t[:, None] - t[None, :]
    C1 = np.exp(-d * d / (2.0 * length * length))
    w, V = np.linalg.eigh(C1)
    B = V * np.sqrt(np.clip(w, 0.0, None))[None, :]
    Z = np.random.default_rng(seed).standard_normal((m, m))
    return sigma * (B @ Z @ B.T)


def fd_directions(m, count=16, first_seed=100):
    """``count`` standard normal fields of shape (m, m), seeds first_seed.."""
    return [np.random.default_rng(first_seed + k).standard_normal((m, m)) for k in range(count)]
