"""Step S0: the spatial operator (paper Sec. 3, eq. (3.2): periodic 2nd-order central
differences).  (L u)_i = c_minus[i] u_{i-1} + c_zero[i] u_i + c_plus[i] u_{i+1},
indices mod n.  Oracle code: plain, dense, float64."""
from __future__ import annotations

import numpy as np


def _rows(coeffs, n: int) -> np.ndarray:
    c = np.asarray(coeffs, dtype=np.float64)
    if c.ndim == 1:
        return np.repeat(c[:, None], n, axis=1)
    assert c.shape == (3, n)
    return c


def dense_operator(n: int, coeffs) -> np.ndarray:
    """O1: the n x n periodic tridiagonal matrix of the stencil."""
    c = _rows(coeffs, n)
    L = np.zeros((n, n))
    for i in range(n):
        L[i, (i - 1) % n] += c[0, i]
        L[i, i] += c[1, i]
        L[i, (i + 1) % n] += c[2, i]
    return L


def apply_stencil(coeffs, u: np.ndarray) -> np.ndarray:
    """L u for a vector (n,) or a block (n, k), straight from the stencil definition."""
    n = u.shape[0]
    c = _rows(coeffs, n)
    if u.ndim == 2:
        c = c[:, :, None]
    return c[0] * np.roll(u, 1, axis=0) + c[1] * u + c[2] * np.roll(u, -1, axis=0)


def stencil_symbol(n: int, coeffs) -> np.ndarray:
    """Eigenvalues of the circulant L on the Fourier modes e^{2 pi i k x}, in numpy FFT
    order: lambda_k = c0 + c_minus e^{-2 pi i k/n} + c_plus e^{2 pi i k/n}."""
    c = np.asarray(coeffs, dtype=np.float64)
    assert c.ndim == 1, "spectral route needs constant coefficients"
    k = np.arange(n)
    return c[1] + c[0] * np.exp(-2j * np.pi * k / n) + c[2] * np.exp(2j * np.pi * k / n)
