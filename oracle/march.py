"""Ground truth for steps S5-S8: the exact solution of the semi-discrete problem with the
compressed source, per Paraexp window, and its superposition.

Paper Sec. 2.1: EBK approximates the exact solution of u' = A u + U p(t) (eq. (2.1)
with the source of eq. (2.3)) by projection onto a block Krylov space; the oracle
computes that exact solution directly.  Sec. 2.2: each window j carries the shifted
source only on [T_{j-1}, T_j) (eq. (2.7)), its subsolution v_j starts from zero
(eq. (2.8)), is continued homogeneously after T_j, and u = u0 + sum_j v_j (eq. (2.9)).

The polynomial source is made autonomous by augmentation: with
w(t) = [T_0(x(t)), ..., T_{q-1}(x(t))] (Chebyshev basis of the window, x = (2t - t0 -
t1)/(t1 - t0)) one has w' = K w with a constant nilpotent K, and

    d/dt [v; w] = [[L, U Pi], [0, K]] [v; w],

so the window solution at any time is one matrix exponential of this augmented
matrix applied to [v(t0); w(t0)].

With the piecewise-cubic source (the paper's choice, Sec. 3) each spline piece
[t_i, t_{i+1}] is a segment of its own: the state carries the piece's Taylor
coefficients z_j = p^(j)(t) / j! (blocks of m), z' = K z with K the shift
z_j' = (j + 1) z_{j+1}, the source is U z_0, and at t_i the polynomial part restarts
from the piece's coefficients.  The augmented matrix [[L, [U 0 0 0]], [0, K]] is the
same for every piece, so its exponentials are shared.
"""
from __future__ import annotations

import math
from typing import List, Optional

import numpy as np

from .compress import (chebyshev_vandermonde, compress, fit_cubic_spline, fit_time_polynomial, source_samples,
                       spline_generator)
from .expm import expm
from .operator import dense_operator, stencil_symbol


def time_generator(q: int, t0: float, t1: float) -> np.ndarray:
    """K with w' = K w for w_k(t) = T_k(x(t)).  From T_k' = 2k sum_{j<k, k-j odd} T_j
    (the j = 0 term counted once, i.e. with weight k), and dx/dt = 2/(t1 - t0)."""
    D = np.zeros((q, q))
    for k in range(1, q):
        for j in range(k - 1, -1, -2):
            D[k, j] = k if j == 0 else 2 * k
    return (2.0 / (t1 - t0)) * D


def window_model(p):
    """S1-S4 of one window: shifted samples, truncated SVD, Chebyshev fit (or, with
    p.source_fit == 1, the piecewise-cubic spline).

    Returns a dict with B = U Pi (n, q) (so that the fitted source is B w(t)), K, the
    window start vector w(t0) = [T_k(-1)], and diagnostics; for the spline also Cp
    (pieces, 4, m) and the shared piece matrices."""
    Ghat = source_samples(p.coeffs, p.u0, p.G, p.shift)
    m, U, C, sig, tail, f1 = compress(Ghat, p.svd_tol, p.rank_max)
    if getattr(p, "source_fit", 0) == 1:
        Cp = fit_cubic_spline(C, p.t_samples) if m > 0 else None
        Bz = np.hstack([U, np.zeros((p.n, 3 * m))]) if m > 0 else np.zeros((p.n, 0))
        return dict(m=m, q=4 * m, U=U, C=C, Cp=Cp, Bz=Bz, Kz=spline_generator(m) if m > 0 else None,
                    spline=True, sigma=sig, svd_tail=tail, fit_resid=0.0, flags=f1)
    q, Pi, res, f2 = fit_time_polynomial(C, p.t_samples, p.t0, p.t1, p.fit_tol, p.q_max)
    B = U @ Pi if m > 0 else np.zeros((p.n, 0))
    K = time_generator(q, p.t0, p.t1)
    w0 = chebyshev_vandermonde(np.array([-1.0]), q)[0] if q > 0 else np.zeros(0)
    return dict(m=m, q=q, U=U, C=C, Pi=Pi, B=B, K=K, w0=w0, sigma=sig, svd_tail=tail,
                fit_resid=res, flags=f1 | f2)


def _delta_key(d: float) -> float:
    return float(np.round(d, 14))


class _Segment:
    """Time interval [ta, tb) with operator coefficients and an optional fitted source.
    Segments with the same `key` share B, K and coefficients (their exponentials are
    cached once); `cheb` marks a Chebyshev-basis source (w(t) = [T_k(x(t))])."""

    def __init__(self, ta, tb, coeffs, B=None, K=None, w_a=None, key=None, cheb=True):
        self.ta, self.tb, self.coeffs = float(ta), float(tb), coeffs
        q = 0 if K is None else K.shape[0]
        self.q = q if (B is not None and q > 0) else 0
        self.B, self.K, self.w_a = B, K, w_a
        self.key = id(self) if key is None else key
        self.cheb = cheb


class _DenseStepper:
    def __init__(self, n):
        self.n = n
        self.cache = {}

    def _aug(self, seg):
        key = ("A", seg.key)
        if key not in self.cache:
            L = dense_operator(self.n, seg.coeffs)
            if seg.q:
                A = np.zeros((self.n + seg.q, self.n + seg.q))
                A[:self.n, :self.n] = L
                A[:self.n, self.n:] = seg.B
                A[self.n:, self.n:] = seg.K
            else:
                A = L
            self.cache[key] = A
        return self.cache[key]

    def to_state(self, x):
        return np.asarray(x, dtype=np.float64).copy()

    def to_vector(self, st):
        return st

    def advance(self, seg, st, w, delta):
        key = ("E", seg.key, _delta_key(delta))
        if key not in self.cache:
            self.cache[key] = expm(_delta_key(delta) * self._aug(seg))
        E = self.cache[key]
        if seg.q:
            z = E @ np.concatenate([st, w])
            return z[:self.n], z[self.n:]
        return E @ st, w


class _SpectralStepper:
    """Same exponential, block-diagonalised by the DFT (constant coefficients only):
    mode k carries the (1+q) x (1+q) matrix [[lambda_k, (F B)_k], [0, K]]."""

    def __init__(self, n):
        self.n = n
        self.cache = {}

    def to_state(self, x):
        return np.fft.fft(np.asarray(x, dtype=np.float64))

    def to_vector(self, st):
        return np.fft.ifft(st).real

    def _aug(self, seg):
        key = ("A", seg.key)
        if key not in self.cache:
            lam = stencil_symbol(self.n, seg.coeffs)
            if seg.q:
                A = np.zeros((self.n, 1 + seg.q, 1 + seg.q), dtype=np.complex128)
                A[:, 0, 0] = lam
                A[:, 0, 1:] = np.fft.fft(seg.B, axis=0)
                A[:, 1:, 1:] = seg.K
            else:
                A = lam
            self.cache[key] = A
        return self.cache[key]

    def advance(self, seg, st, w, delta):
        d = _delta_key(delta)
        key = ("E", seg.key, d)
        A = self._aug(seg)
        if not seg.q:
            return np.exp(d * A) * st, w
        if key not in self.cache:
            self.cache[key] = expm(d * A)
        E = self.cache[key]
        z = np.concatenate([st[:, None], np.broadcast_to(w, (self.n, seg.q))], axis=1)
        z = np.einsum("kij,kj->ki", E, z)
        # w evolves identically in every mode (real polynomial part); take mode 0's copy
        return z[:, 0], z[0, 1:].real.copy()


_GROWTH = 100.0


def _chebyshev_w(seg, t):
    """w(t) = [T_k(x(t))], x = (2t - ta - tb) / (tb - ta), of a source segment."""
    x = (2.0 * t - seg.ta - seg.tb) / (seg.tb - seg.ta)
    return chebyshev_vandermonde(np.array([x]), seg.q)[0]


def _march(route, n, segments: List[_Segment], x0, t_start, t_out):
    """Advance the state through consecutive segments, recording it at t_out."""
    stepper = _SpectralStepper(n) if route == "spectral" else _DenseStepper(n)
    st = stepper.to_state(x0)
    t = float(t_start)
    si = 0
    w = segments[0].w_a.copy() if segments[0].q else None
    out = np.zeros((n, len(t_out)))
    for k, tk in enumerate(t_out):
        tk = float(tk)
        if tk < t_start:
            raise ValueError("output time before the start of the march")
        while t < tk:
            seg = segments[si]
            te = min(tk, seg.tb)
            if te > t:
                if seg.q and seg.cheb:
                    # The polynomial block's exponential over a long step multiplies
                    # rounding by the Chebyshev re-expansion coefficients of the shift
                    # (about (1 + sqrt(2c))^q for a shift of c = 2 step / window in x),
                    # which reaches 1e12 for q = 32 over a whole window.  Since
                    # exp(d A) = exp(d A / m)^m, a long step is taken as m equal pieces
                    # whose growth factor stays below _GROWTH, each starting from the
                    # exact w(t) = [T_k(x(t))] that the augmented system carries.
                    c_max = 0.5 * (_GROWTH ** (1.0 / seg.q) - 1.0) ** 2
                    m = max(1, int(math.ceil(2.0 * (te - t) / (seg.tb - seg.ta) / c_max)))
                    d = (te - t) / m
                    for i in range(m):
                        w = _chebyshev_w(seg, t + i * d)
                        st, w = stepper.advance(seg, st, w, d)
                else:
                    st, w = stepper.advance(seg, st, w, te - t)
                t = te
            if t >= seg.tb and si + 1 < len(segments):
                si += 1
                w = segments[si].w_a.copy() if segments[si].q else None
        out[:, k] = stepper.to_vector(st)
    return out


def source_segments(mdl, coeffs, t0, t1, t_samples, key=None):
    """The source-carrying segments of a window: one Chebyshev segment [t0, t1], or one
    segment per spline piece [t_i, t_{i+1}] sharing one augmented matrix."""
    if not mdl.get("spline"):
        return [_Segment(t0, t1, coeffs, mdl["B"] if mdl["q"] else None, mdl["K"], mdl["w0"])]
    if mdl["m"] == 0:
        return [_Segment(t0, t1, coeffs)]
    key = ("spline", id(mdl)) if key is None else key
    ts = np.asarray(t_samples, dtype=np.float64)
    return [_Segment(ts[i], ts[i + 1], coeffs, mdl["Bz"], mdl["Kz"], mdl["Cp"][i].reshape(-1), key=key, cheb=False)
            for i in range(len(ts) - 1)]


def _auto_route(p, route):
    if route != "auto":
        return route
    return "spectral" if (np.asarray(p.coeffs).ndim == 1 and p.n > 768) else "dense"


def solve_window(p, route: str = "auto", model: Optional[dict] = None):
    """One window: v(t_k) (shift) or u(t_k) (no shift) at p.t_out.  Outputs before the
    window start are zero for the shifted problem (the subsolution vanishes there)."""
    route = _auto_route(p, route)
    mdl = model or window_model(p)
    n = p.n
    segs = source_segments(mdl, p.coeffs, p.t0, p.t1, p.t_samples) + [_Segment(p.t1, math.inf, p.coeffs)]
    t_out = np.asarray(p.t_out, dtype=np.float64)
    out = np.zeros((n, len(t_out)))
    later = t_out >= p.t0
    if not p.shift and not np.all(later):
        raise ValueError("unshifted problem needs t_out >= t0")
    x0 = np.zeros(n) if p.shift else np.asarray(p.u0, dtype=np.float64)
    if np.any(later):
        out[:, later] = _march(route, n, segs, x0, p.t0, t_out[later])
    return out, mdl


def solve_windows_superposed(probs, route: str = "auto"):
    """Paraexp: u(t_k) = u0 + sum_j v_j(t_k) over independent windows (eq. (2.9))."""
    u0 = np.asarray(probs[0].u0, dtype=np.float64)
    total = None
    for p in probs:
        assert p.shift
        v, _ = solve_window(p, route)
        total = v if total is None else total + v
    return u0[:, None] + total


def solve_sequential(probs, route: str = "auto"):
    """The serial counterpart: one march of the shifted state through the windows in
    order, the source switching at each T_j, then u0 + state (used to pin eq. (2.9))."""
    route = _auto_route(probs[0], route)
    n = probs[0].n
    segs = []
    for p in probs:
        mdl = window_model(p)
        segs += source_segments(mdl, p.coeffs, p.t0, p.t1, p.t_samples)
    segs.append(_Segment(probs[-1].t1, math.inf, probs[-1].coeffs))
    u0 = np.asarray(probs[0].u0, dtype=np.float64)
    out = _march(route, n, segs, np.zeros(n), probs[0].t0, probs[0].t_out)
    return u0[:, None] + out


def march_segments(route, n, seg_specs, x0, t_start, t_out):
    """Public form of the segment march for the waveform-relaxation oracle: seg_specs is a
    list of (ta, tb, coeffs, B or None, K or None, w_a or None) tuples or of segments made
    by source_segments."""
    segs = [s if isinstance(s, _Segment) else _Segment(*s) for s in seg_specs]
    return _march(route, n, segs, x0, t_start, t_out)
