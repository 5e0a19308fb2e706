"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module draws random numbers and evaluates the initial data on a grid.
It contains none of the solver's arithmetic: no flux, no time scheme, no
preconditioner, no primal-dual step.  Both the CPU oracle and the GPU path
receive the arrays produced here as plain inputs.

Workload recipe (the paper uses smooth random-free test data; the benchmark
family below extends its Burgers examples, Section 4.3, with seeded smooth
initial data):

    rng   = numpy.random.default_rng(seed)
    a_k   ~ U(0, 0.25),  k = 1..4
    th_k  ~ U(0, 2*pi),  k = 1..4
    u0(x) = 0.5 + sum_k a_k sin(2*pi*k*x + th_k)

evaluated at the finite-difference nodes x_j = j*h_x (Section 3.2), or at
arbitrary points (for Gauss-point projections).
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "fourier_coeffs",
    "fourier_u0",
    "fourier_u0_at",
    "fourier_u0_legendre",
    "sine_u0",
    "gaussian_bump_u0",
    "heat_gamma_at",
    "batch_shapes",
    "unit_directions",
]


def fourier_coeffs(seed: int):
    """Amplitudes a_k and phases th_k (k = 1..4) of the seeded Fourier sum."""
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.0, 0.25, 4)
    th = rng.uniform(0.0, 2.0 * np.pi, 4)
    return a, th


def fourier_u0_at(seed: int, x: np.ndarray, length: float = 1.0) -> np.ndarray:
    """u0(x) = 0.5 + sum_k a_k sin(2 pi k x / length + th_k) at points x (float64)."""
    a, th = fourier_coeffs(seed)
    x = np.asarray(x, dtype=np.float64)
    out = np.full(x.shape, 0.5)
    for k in range(4):
        out += a[k] * np.sin(2.0 * np.pi * (k + 1) * x / length + th[k])
    return out


def fourier_u0(seed: int, nx: int, length: float = 1.0) -> np.ndarray:
    """Seeded Fourier-sum initial data at the nodes x_j = j*length/nx."""
    x = np.arange(nx, dtype=np.float64) * (length / nx)
    return fourier_u0_at(seed, x, length)


def _sph_bessel_012(t: np.ndarray):
    """Spherical Bessel functions j_0, j_1, j_2 at t >= 0: the power series for t < 0.5
    (no cancellation), the trigonometric forms above."""
    t = np.asarray(t, dtype=np.float64)
    js = []
    for n in range(3):
        # series: sum_m (-1)^m t^(2m+n) / (2^m m! (2m+2n+1)!!)
        ser = np.zeros_like(t)
        df = 1.0
        for i in range(1, 2 * n + 2, 2):
            df *= i                      # (2n+1)!!
        term = t ** n / df
        for m in range(12):
            ser = ser + term
            term = -term * t * t / (2.0 * (m + 1) * (2 * m + 2 * n + 3))
        js.append(ser)
    big = t >= 0.5
    tb = np.where(big, t, 1.0)
    s, c = np.sin(tb), np.cos(tb)
    closed = [s / tb, s / tb ** 2 - c / tb, (3.0 / tb ** 2 - 1.0) * s / tb - 3.0 * c / tb ** 2]
    return [np.where(big, closed[n], js[n]) for n in range(3)]


def fourier_u0_legendre(seed: int, nx: int, length: float = 1.0) -> np.ndarray:
    """Cell-wise L2 projection of the seeded Fourier sum onto the Legendre basis P_0, P_1, P_2
    (cells [j h, (j+1) h], local coordinate xi in [-1, 1]), in closed form: for a mode
    sin(w x + th) on a cell with centre x_c and t = w h / 2, the coefficient of P_n is
    (2n+1) Im(i^n e^{i(w x_c + th)}) j_n(t).  Returns (3, nx): coefficient-planar."""
    a, th = fourier_coeffs(seed)
    h = length / nx
    xc = (np.arange(nx, dtype=np.float64) + 0.5) * h
    out = np.zeros((3, nx))
    out[0] += 0.5
    for k in range(4):
        w = 2.0 * np.pi * (k + 1) / length
        phi = w * xc + th[k]
        j0, j1, j2 = _sph_bessel_012(np.array(w * h / 2.0))
        out[0] += a[k] * np.sin(phi) * j0
        out[1] += a[k] * 3.0 * np.cos(phi) * j1
        out[2] += a[k] * -5.0 * np.sin(phi) * j2
    return out


def sine_u0(nx: int, length: float = 1.0) -> np.ndarray:
    """u0 = sin(2 pi x / length) at the nodes (linear-advection example)."""
    x = np.arange(nx, dtype=np.float64) * (length / nx)
    return np.sin(2.0 * np.pi * x / length)


def traffic_u0_at(x: np.ndarray) -> np.ndarray:
    """Piecewise-constant traffic density of Section 4.3 on [0, 2): 0.1 on [1, 2], 0.25 elsewhere."""
    x = np.asarray(x, dtype=np.float64)
    return np.where((x >= 1.0) & (x <= 2.0), 0.1, 0.25)


def traffic_u0(nx: int, length: float = 2.0) -> np.ndarray:
    """traffic_u0_at at the nodes x_j = j*length/nx."""
    return traffic_u0_at(np.arange(nx, dtype=np.float64) * (length / nx))


def gaussian_bump_u0(nx: int) -> np.ndarray:
    """u0 = exp(-64 (x - 1/2)^2) on [0,1) (heat example, Section 4.1)."""
    x = np.arange(nx, dtype=np.float64) / nx
    return np.exp(-64.0 * (x - 0.5) ** 2)


def heat_gamma_at(x: np.ndarray) -> np.ndarray:
    """Diffusion coefficient gamma(x) = 0.5 + 0.1 sin(2 pi x) (Section 4.1)."""
    return 0.5 + 0.1 * np.sin(2.0 * np.pi * np.asarray(x, dtype=np.float64))


def batch_shapes(seed: int, count: int = 256,
                 nx_choices=(256, 512, 1024, 2048, 4096),
                 nt_choices=(64, 128, 256, 512)):
    """Seeded (nx, nt, u0-seed) triples for a batch of independent problems.

    Sizes are drawn uniformly from the given sets; every problem gets its own
    initial-data seed derived from the batch seed.
    """
    rng = np.random.default_rng(seed)
    nx = rng.choice(np.asarray(nx_choices), size=count)
    nt = rng.choice(np.asarray(nt_choices), size=count)
    seeds = rng.integers(0, 2**31 - 1, size=count)
    return [(int(a), int(b), int(c)) for a, b, c in zip(nx, nt, seeds)]


def unit_directions(seed: int, n: int, count: int) -> np.ndarray:
    """`count` random unit vectors in R^n (Gaussian, normalised), float64."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((count, n))
    return v / np.linalg.norm(v, axis=1, keepdims=True)
