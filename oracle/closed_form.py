"""Closed forms for linear upwind backward Euler (oracle; test infrastructure only).

For u_t + a u_x = 0 (a > 0) with first-order upwinding and backward Euler
(Sections 2.1, 3.1), a Fourier mode e^{2 pi i k x} is multiplied per step by

    g_k = 1 / (1 + nu (1 - e^{-2 pi i k h_x}))      nu = a h_t / h_x,

so for u0 = sin(2 pi x) the scheme's solution is u^l_j = Im(g_1^l e^{2 pi i x_j}).
These are exact statements about the discrete scheme (not about the PDE).
"""
from __future__ import annotations

import numpy as np


def amplification(nx: int, nu: float, k) -> np.ndarray:
    """BE-upwind amplification factor g_k for wavenumber(s) k on [0, 1)."""
    k = np.asarray(k)
    return 1.0 / (1.0 + nu * (1.0 - np.exp(-2j * np.pi * k / nx)))


def advection_sine_solution(nx: int, nt: int, nu: float) -> np.ndarray:
    """u^l_j = Im(g^l e^{2 pi i j / nx}), l = 0..nt, for u0 = sin(2 pi x)."""
    g = amplification(nx, nu, 1)
    x = np.arange(nx) / nx
    lv = np.arange(nt + 1)[:, None]
    return np.imag(g ** lv * np.exp(2j * np.pi * x)[None, :])


def advection_solution(u0: np.ndarray, nt: int, nu: float) -> np.ndarray:
    """Scheme solution for arbitrary periodic data: each FFT mode times g_k^l."""
    nx = u0.shape[-1]
    g = amplification(nx, nu, np.fft.fftfreq(nx, 1.0 / nx))
    uh = np.fft.fft(u0)
    lv = np.arange(nt + 1)[:, None]
    return np.fft.ifft(g[None, :] ** lv * uh[None, :], axis=1).real


def advection_terminal_gradient(u0: np.ndarray, target: np.ndarray, nt: int, nu: float, hx: float):
    """d/du0 of h_x sum_j (u^{N_t}_j - target_j)^2 for the linear scheme.

    u^{N_t} = G^{N_t} u0 with G circulant (symbol g_k); the gradient is
    2 h_x (G^T)^{N_t} (u^{N_t} - target), and G^T has symbol conj(g_k).
    """
    nx = u0.shape[-1]
    k = np.fft.fftfreq(nx, 1.0 / nx)
    g = amplification(nx, nu, k)
    ut = np.fft.ifft(g ** nt * np.fft.fft(u0)).real
    res = 2.0 * hx * (ut - target)
    return np.fft.ifft(np.conj(g) ** nt * np.fft.fft(res)).real
