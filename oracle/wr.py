"""Step S10: waveform relaxation for viscous Burgers (paper Secs. 2.3-2.4, Fig. 2.4).

Semi-discrete Burgers (eq. (4.1), central differences, Sec. 4.1):
    u' = A u + N(u),   A = nu D2,   N(u)_i = -u_i (u_{i+1} - u_{i-1}) / (2h).
Iteration k -> k+1 treats the nonlinearity as a known source g_k(t) = N(u_k(t))
(eq. (2.10)), plus an external source f(x, t) when the problem carries one (the
manufactured source of Sec. 4.1).  With the Jacobian correction (eqs. (2.12)-(2.13), windowed as in
eq. (2.14)) the operator on window j is A + Jbar_j, where Jbar_j is the time average
of dN/du(u_k(t)) over the window (trapezoid rule over the window's samples), and the
source is g_k - Jbar_j u_k.  The shifted source of eq. (2.16) is read as
    g_hat = (A + Jbar_j) u0 + g_k(t) - Jbar_j u_k(t)
(the paper's printed hat on u_k would add a spurious Jbar_j u0; this reading keeps
the fixed point: at u_{k+1} = u_k the correction terms cancel).  Iterate 0 is the
constant extension u_0(t) = u(0).  Windows are solved independently (eq. (2.19)) and
superposed (eq. (2.20)); the subsolution of window j is continued homogeneously
through the later windows with their own operators A + Jbar_i.
"""
from __future__ import annotations

import math

import numpy as np

from .compress import compress, fit_cubic_spline, fit_time_polynomial, source_samples, spline_generator
from .march import march_segments, source_segments, time_generator
from .compress import chebyshev_vandermonde
from .operator import apply_stencil


def burgers_nonlinear(u: np.ndarray, h: float) -> np.ndarray:
    """N(u) = -u * D1 u (advective form), for (n,) or (n, k)."""
    return -u * (np.roll(u, -1, axis=0) - np.roll(u, 1, axis=0)) / (2 * h)


def burgers_jacobian(u: np.ndarray, h: float) -> np.ndarray:
    """Stencil rows (3, n) of dN/du at u: [u_i/(2h), -(u_{i+1}-u_{i-1})/(2h), -u_i/(2h)]."""
    return np.stack([u / (2 * h), -(np.roll(u, -1) - np.roll(u, 1)) / (2 * h), -u / (2 * h)])


def _trapezoid_weights(t: np.ndarray) -> np.ndarray:
    w = np.zeros_like(t)
    dt = np.diff(t)
    w[:-1] += dt / 2
    w[1:] += dt / 2
    return w / (t[-1] - t[0])


class _Win:
    def __init__(self, n, coeffs, u0, t0, t1, ts, G, **kw):
        self.n, self.coeffs, self.u0, self.t0, self.t1 = n, coeffs, u0, t0, t1
        self.t_samples, self.G, self.shift = ts, G, True
        self.__dict__.update(kw)


def wr_burgers(bp, route: str = "dense", return_history: bool = False):
    """K waveform-relaxation iterations; returns u_K at every window sample time,
    shape (n, P*s) in window-major order (window boundaries appear twice)."""
    n, P, s = bp.n, bp.P, bp.s
    h = 1.0 / n
    A = np.array([bp.nu / h**2, -2 * bp.nu / h**2, bp.nu / h**2])
    u0 = np.asarray(bp.u0, dtype=np.float64)
    times = [bp.window_times(j) for j in range(P)]
    all_t = np.concatenate(times)
    Uk = np.repeat(u0[:, None], P * s, axis=1)
    hist = []
    for _ in range(bp.K):
        models, opers = [], []
        for j in range(P):
            uk = Uk[:, j * s:(j + 1) * s]
            if bp.jacobian:
                wts = _trapezoid_weights(times[j])
                Jbar = sum(wts[i] * burgers_jacobian(uk[:, i], h) for i in range(s))
            else:
                Jbar = np.zeros((3, n))
            Lj = A[:, None] + Jbar
            if not bp.jacobian and route == "spectral":
                Lj = A.copy()
            Graw = burgers_nonlinear(uk, h) - apply_stencil(Jbar, uk)
            if getattr(bp, "forcing", None) is not None:  # external source f(x, t) (Sec. 4.1)
                Graw = Graw + np.asarray(bp.forcing)[:, j * s:(j + 1) * s]
            Ghat = source_samples(Lj, u0, Graw, True)
            m, U, C, sig, tail, _ = compress(Ghat, bp.svd_tol, bp.rank_max)
            if getattr(bp, "source_fit", 0) == 1:  # piecewise-cubic p(t)
                mdl = dict(m=m, q=4 * m, spline=True, Cp=fit_cubic_spline(C, times[j]) if m else None,
                           Bz=np.hstack([U, np.zeros((n, 3 * m))]) if m else None,
                           Kz=spline_generator(m) if m else None)
                models.append((mdl, None, None, m, 4 * m))
                opers.append(Lj)
                continue
            q, Pi, res, _ = fit_time_polynomial(C, times[j], times[j][0], times[j][-1],
                                                bp.fit_tol, bp.q_max)
            B = U @ Pi if m > 0 else None
            K = time_generator(q, times[j][0], times[j][-1]) if q else None
            w0 = chebyshev_vandermonde(np.array([-1.0]), q)[0] if q else None
            models.append((B, K, w0, m, q))
            opers.append(Lj)
        V = np.zeros((n, P * s))
        for j in range(P):
            B, K, w0, m, q = models[j]
            if isinstance(B, dict):  # spline pieces of window j
                specs = source_segments(B, opers[j], times[j][0], times[j][-1], times[j])
            else:
                specs = [(times[j][0], times[j][-1], opers[j], B, K, w0)]
            for i in range(j + 1, P):
                specs.append((times[i][0], times[i][-1], opers[i], None, None, None))
            specs.append((times[-1][-1], math.inf, opers[-1], None, None, None))
            V[:, j * s:] += march_segments(route, n, specs, np.zeros(n), times[j][0], all_t[j * s:])
        Unew = u0[:, None] + V
        inc = float(np.linalg.norm(Unew - Uk) / max(np.linalg.norm(Unew), 1e-300))
        hist.append(dict(increment=inc, ranks=[mm[3] for mm in models], qs=[mm[4] for mm in models]))
        Uk = Unew
    return (Uk, hist) if return_history else Uk
