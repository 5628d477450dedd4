"""Steps S1-S4: source samples, truncated SVD, polynomial fit in time.

Paper Sec. 2.1: the source is sampled at s times, G = [g(t_1) ... g(t_s)]
(eq. (2.2)); the thin SVD G = U~ S~ V~^T is truncated to the m largest singular
values so that g(t) ~= U p(t) (eq. (2.3)); p(t) interpolates the coefficients of
the retained columns.  Sec. 2.2 shifts the source by A u0 (eq. (2.6)).

Readings of points the paper leaves open (listed in the design doc):
  * truncation: m is the smallest r with sqrt(sum_{i>r} sigma_i^2) <= svd_tol*||G||_F,
    singular values <= 1e-14 sigma_1 are never kept, a cut inside a cluster
    (|sigma_m - sigma_{m+1}| <= 1e-12 sigma_1) keeps the whole cluster, and m is
    capped at rank_max;
  * p(t), default: one least-squares polynomial per window, of the smallest degree
    q-1 whose relative Frobenius fit residual over the samples is <= fit_tol, capped
    at q_max; it is represented in the Chebyshev basis T_k(x), x = (2t - t0 - t1)/(t1 - t0);
  * p(t), piecewise (the paper's own choice of Sec. 3, "piecewise cubic polynomials"):
    the cubic spline interpolating each coefficient row at the samples, with
    not-a-knot end conditions (the third derivative continuous at the second and the
    second-to-last sample).
"""
from __future__ import annotations

import numpy as np

from .operator import apply_stencil

FLAG_RANK_CAPPED = 4
FLAG_FIT_CAPPED = 8


def source_samples(coeffs, u0: np.ndarray, G: np.ndarray, shift: bool) -> np.ndarray:
    """S1: G_hat = G + (L u0) 1^T when the Paraexp shift is on (eq. (2.6))."""
    G = np.asarray(G, dtype=np.float64)
    if not shift:
        return G.copy()
    return G + apply_stencil(coeffs, u0)[:, None]


def compress(Ghat: np.ndarray, svd_tol: float, rank_max: int):
    """S2-S3: thin SVD (LAPACK) and the truncation rule.

    Returns (m, U, C, sigma, tail, flags) with U (n, m) orthonormal, C = U^T G_hat
    (m, s) the coefficients at the sample times, and tail the dropped energy
    sqrt(sum_{i>=m} sigma_i^2) relative to ||G_hat||_F."""
    n, s = Ghat.shape
    Ut, sig, _ = np.linalg.svd(Ghat, full_matrices=False)
    fro = float(np.sqrt(np.sum(sig**2)))
    flags = 0
    if fro == 0.0 or sig[0] == 0.0:
        return 0, np.zeros((n, 0)), np.zeros((0, s)), sig, 0.0, 0
    # tails[r] = sqrt(sum_{i >= r} sigma_i^2), r = 0..len(sig)
    sq = sig**2
    tails = np.sqrt(np.concatenate([np.cumsum(sq[::-1])[::-1], [0.0]]))
    m = int(np.argmax(tails <= svd_tol * fro))
    while m > 0 and sig[m - 1] <= 1e-14 * sig[0]:
        m -= 1
    while 0 < m < len(sig) and abs(sig[m - 1] - sig[m]) <= 1e-12 * sig[0] and sig[m] > 1e-14 * sig[0]:
        m += 1
    if m > rank_max:
        m = rank_max
        flags |= FLAG_RANK_CAPPED
    U = Ut[:, :m].copy()
    C = U.T @ Ghat
    return m, U, C, sig, float(tails[m] / fro), flags


def chebyshev_vandermonde(x: np.ndarray, q: int) -> np.ndarray:
    """(len(x), q) matrix of T_k(x_i), k < q, by the three-term recurrence."""
    V = np.zeros((len(x), q))
    if q > 0:
        V[:, 0] = 1.0
    if q > 1:
        V[:, 1] = x
    for k in range(2, q):
        V[:, k] = 2 * x * V[:, k - 1] - V[:, k - 2]
    return V


def fit_time_polynomial(C: np.ndarray, t_samples: np.ndarray, t0: float, t1: float,
                        fit_tol: float, q_max: int):
    """S4: least-squares fit of each row of C by sum_{k<q} Pi[:, k] T_k(x(t)).

    Returns (q, Pi (m, q), relative residual, flags)."""
    m, s = C.shape
    if m == 0:
        return 0, np.zeros((0, 0)), 0.0, 0
    x = (2 * np.asarray(t_samples) - t0 - t1) / (t1 - t0)
    qcap = min(q_max, s)
    Vfull = chebyshev_vandermonde(x, qcap)
    cn = float(np.linalg.norm(C))
    last = None
    for q in range(1, qcap + 1):
        Vq = Vfull[:, :q]
        coef, *_ = np.linalg.lstsq(Vq, C.T, rcond=None)   # (q, m)
        Pi = coef.T
        res = float(np.linalg.norm(C - Pi @ Vq.T)) / cn if cn > 0 else 0.0
        last = (q, Pi, res)
        if res <= fit_tol:
            return q, Pi, res, 0
    q, Pi, res = last
    return q, Pi, res, FLAG_FIT_CAPPED


def fit_cubic_spline(C: np.ndarray, t_samples: np.ndarray) -> np.ndarray:
    """S4, piecewise: the not-a-knot cubic spline through each row of C (m, s) at the
    sample times.  Returns Cp (s-1, 4, m): on piece i, p(t) = sum_k Cp[i, k] (t - t_i)^k.

    Written from the definition: unknown second derivatives M_0..M_{s-1}; at interior
    samples the first derivative is continuous,
        h_{i-1} M_{i-1} + 2 (h_{i-1} + h_i) M_i + h_i M_{i+1}
            = 6 ((y_{i+1} - y_i) / h_i - (y_i - y_{i-1}) / h_{i-1}),
    and at the second and second-to-last sample the third derivative is continuous
    (M_1 - M_0) / h_0 = (M_2 - M_1) / h_1 (not-a-knot); the dense system is solved as
    it stands.  Three samples give the parabola through them, two the straight line."""
    C = np.asarray(C, dtype=np.float64)
    t = np.asarray(t_samples, dtype=np.float64)
    m, s = C.shape
    h = np.diff(t)
    M = np.zeros((s, m))
    if s >= 4:
        A = np.zeros((s, s))
        rhs = np.zeros((s, m))
        for i in range(1, s - 1):
            A[i, i - 1] = h[i - 1]
            A[i, i] = 2 * (h[i - 1] + h[i])
            A[i, i + 1] = h[i]
            rhs[i] = 6 * ((C[:, i + 1] - C[:, i]) / h[i] - (C[:, i] - C[:, i - 1]) / h[i - 1])
        A[0, 0], A[0, 1], A[0, 2] = h[1], -(h[0] + h[1]), h[0]
        A[s - 1, s - 3], A[s - 1, s - 2], A[s - 1, s - 1] = h[s - 2], -(h[s - 3] + h[s - 2]), h[s - 3]
        M = np.linalg.solve(A, rhs)
    elif s == 3:
        # one parabola: M constant, from the second divided difference
        dd = ((C[:, 2] - C[:, 1]) / h[1] - (C[:, 1] - C[:, 0]) / h[0]) / (t[2] - t[0])
        M = np.tile(2 * dd, (3, 1))
    Cp = np.zeros((s - 1, 4, m))
    for i in range(s - 1):
        Cp[i, 0] = C[:, i]
        Cp[i, 1] = (C[:, i + 1] - C[:, i]) / h[i] - h[i] * (2 * M[i] + M[i + 1]) / 6
        Cp[i, 2] = M[i] / 2
        Cp[i, 3] = (M[i + 1] - M[i]) / (6 * h[i])
    return Cp


def spline_generator(m: int) -> np.ndarray:
    """K (4m, 4m) with z' = K z for the Taylor coefficients z_j(t) = p^(j)(t) / j! of a
    cubic (blocks of m): z_j' = (j + 1) z_{j+1}, z_3' = 0."""
    K = np.zeros((4 * m, 4 * m))
    for j in range(3):
        K[j * m:(j + 1) * m, (j + 1) * m:(j + 2) * m] = (j + 1) * np.eye(m)
    return K
