"""Dense matrix exponential by scaling and squaring with the diagonal Pade [13/13]
approximant (Higham, SIAM J. Matrix Anal. Appl. 26 (2005), Algorithm 2.3), used by the
oracle for the exact exponential of the augmented matrix.  Batched over leading axes,
real or complex.  Test pins compare it with scipy.linalg.expm and with closed forms."""
from __future__ import annotations

import math

import numpy as np

# Higham 2005, Table 2.3: the largest ||A||_1 for which the [13/13] approximant has
# backward error below the double-precision unit roundoff.
THETA_13 = 5.371920351148152


def pade_coefficients(p: int = 13) -> np.ndarray:
    """Numerator coefficients of the diagonal [p/p] Pade approximant of e^x:
    c_k = (2p-k)! p! / ((2p)! k! (p-k)!),  N(x) = sum_k c_k x^k, D(x) = N(-x)."""
    f = math.factorial
    return np.array([f(2 * p - k) * f(p) / (f(2 * p) * f(k) * f(p - k)) for k in range(p + 1)],
                    dtype=np.float64)


def _pade13(A: np.ndarray) -> np.ndarray:
    c = pade_coefficients(13)
    n = A.shape[-1]
    I = np.broadcast_to(np.eye(n, dtype=A.dtype), A.shape)
    A2 = A @ A
    A4 = A2 @ A2
    A6 = A4 @ A2
    # even part V(A) and odd part U(A) of N(A) = V + U, D(A) = V - U
    U = A @ (A6 @ (c[13] * A6 + c[11] * A4 + c[9] * A2) + c[7] * A6 + c[5] * A4 + c[3] * A2 + c[1] * I)
    V = A6 @ (c[12] * A6 + c[10] * A4 + c[8] * A2) + c[6] * A6 + c[4] * A4 + c[2] * A2 + c[0] * I
    return np.linalg.solve(V - U, V + U)


def expm(A: np.ndarray) -> np.ndarray:
    """exp(A) for A of shape (..., N, N)."""
    A = np.asarray(A)
    if A.ndim == 2:
        return expm(A[None])[0]
    batch = A.shape[:-2]
    Af = A.reshape((-1,) + A.shape[-2:])
    out = np.empty_like(Af, dtype=np.result_type(Af.dtype, np.float64))
    norms = np.abs(Af).sum(axis=-2).max(axis=-1)          # ||A||_1 per matrix
    sq = np.zeros(len(Af), dtype=int)
    big = norms > THETA_13
    sq[big] = np.ceil(np.log2(norms[big] / THETA_13)).astype(int)
    for s in np.unique(sq):
        idx = np.nonzero(sq == s)[0]
        R = _pade13(Af[idx] / (2.0 ** s))
        for _ in range(int(s)):
            R = R @ R
        out[idx] = R
    return out.reshape(batch + A.shape[-2:])
