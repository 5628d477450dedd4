"""Problem generators for the Paraexp exp-action workloads (all float64, all seeded).

Grid convention (periodic, 2nd-order central differences, Sec. 3 of the paper):
x_i = i/n, i = 0..n-1, h = 1/n.  The right-hand-side operator L (the paper's A in
eq. (2.1), u' = A u + g) is a periodic 3-point stencil

    (L u)_i = c_minus[i] u_{i-1} + c_zero[i] u_i + c_plus[i] u_{i+1}

given either as 3 constants or as 3 length-n rows (per-point coefficients).

Sample times follow the paper's choices: Chebyshev(-Lobatto) nodes on each window
for the advection-diffusion runs (Sec. 3), uniform nodes for the Burgers waveform
relaxation runs (Sec. 4.2).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, List, Optional, Sequence

import numpy as np


@dataclasses.dataclass
class Problem:
    """One window subproblem u' = L u + g(t) on [t0, t1] (source zero after t1).

    shift=True solves the Paraexp-shifted problem of Sec. 2.2: v(t0) = 0 with
    source L u0 + g, and the outputs are v(t_k); shift=False solves for u
    itself from u(t0) = u0.
    """

    n: int
    coeffs: np.ndarray          # (3,) or (3, n): rows c_minus, c_zero, c_plus
    u0: np.ndarray              # (n,)
    t0: float
    t1: float
    t_samples: np.ndarray       # (s,) ascending, t_samples[0] = t0, t_samples[-1] = t1
    G: np.ndarray               # (n, s) raw source samples g(t_i), column-major use
    t_out: np.ndarray           # (n_out,) ascending absolute output times
    shift: bool = True
    krylov_steps: int = 30
    rank_max: int = 32
    q_max: int = 32
    tol: float = 1e-12
    svd_tol: float = 1e-13
    fit_tol: float = 1e-13
    name: str = ""
    krylov: int = 0             # 0: polynomial Krylov space, 1: shift-and-invert
    sai_shift: float = 0.0      # shift-and-invert: gamma / cycle step (0: default)
    source_fit: int = 0         # p(t): 0 one Chebyshev least-squares polynomial, 1 cubic spline

    @property
    def s(self) -> int:
        return int(self.t_samples.shape[0])

    @property
    def per_point(self) -> bool:
        return np.asarray(self.coeffs).ndim == 2


@dataclasses.dataclass
class BurgersProblem:
    """Viscous Burgers u_t + u u_x = nu u_xx + f on the periodic unit interval,
    solved by Paraexp waveform relaxation (Sec. 2.3-2.4) over P windows of [0, T]
    with s uniform samples per window (endpoints included)."""

    n: int
    nu: float
    T: float
    P: int
    s: int
    K: int
    u0: np.ndarray
    jacobian: bool = True
    krylov_steps: int = 80
    rank_max: int = 24
    q_max: int = 32
    tol: float = 1e-10
    svd_tol: float = 1e-10
    fit_tol: float = 1e-11
    name: str = ""
    krylov: int = 0
    sai_shift: float = 0.0
    forcing: Optional[np.ndarray] = None   # (n, P*s) external source samples, window-major
    source_fit: int = 0                    # p(t): 0 Chebyshev least squares, 1 cubic spline

    def window_times(self, j: int) -> np.ndarray:
        t0 = self.T * j / self.P
        t1 = self.T * (j + 1) / self.P
        return uniform_samples(t0, t1, self.s)


def grid(n: int) -> np.ndarray:
    return np.arange(n, dtype=np.float64) / n


def ade_coeffs(n: int, a: float, nu: float) -> np.ndarray:
    """Stencil of u_t + a u_x = nu u_xx (eq. (3.1)), central differences, h = 1/n."""
    h = 1.0 / n
    return np.array([nu / h**2 + a / (2 * h), -2 * nu / h**2, nu / h**2 - a / (2 * h)],
                    dtype=np.float64)


def burgers_diffusion_coeffs(n: int, nu: float) -> np.ndarray:
    """Linear part nu u_xx of the Burgers equation (eq. (4.1)), central differences."""
    return ade_coeffs(n, 0.0, nu)


def chebyshev_lobatto(t0: float, t1: float, s: int) -> np.ndarray:
    """s Chebyshev extrema on [t0, t1], ascending, endpoints included."""
    if s == 1:
        return np.array([t0], dtype=np.float64)
    i = np.arange(s, dtype=np.float64)
    t = 0.5 * (t0 + t1) - 0.5 * (t1 - t0) * np.cos(np.pi * i / (s - 1))
    t[0], t[-1] = t0, t1
    return t


def uniform_samples(t0: float, t1: float, s: int) -> np.ndarray:
    t = np.linspace(t0, t1, s, dtype=np.float64)
    t[0], t[-1] = t0, t1
    return t


def _periodic_distance(x: np.ndarray, c: float) -> np.ndarray:
    d = np.abs(x - c)
    return np.minimum(d, 1.0 - d)


def _cheb_T(d: int, y: np.ndarray) -> np.ndarray:
    """Chebyshev polynomial T_d(y) by the three-term recurrence (input generator only)."""
    t0, t1 = np.ones_like(y), y
    if d == 0:
        return t0
    for _ in range(d - 1):
        t0, t1 = t1, 2 * y * t1 - t0
    return t1


def smooth_field(rng: np.random.Generator, n: int, modes: int, deg: int):
    """u0 = sum of `modes` periodic Gaussians; g = sum_r sin(2 pi k_r x + th_r) * poly_r(t),
    poly_r = sum_{d<=deg} alpha_{rd} T_d(2t/T - 1)."""
    x = grid(n)
    c = rng.uniform(0.0, 1.0, modes)
    w = rng.uniform(0.01, 0.05, modes)
    k = rng.integers(1, 33, modes)
    th = rng.uniform(0.0, 2 * np.pi, modes)
    alpha = rng.standard_normal((modes, deg + 1))
    u0 = np.zeros(n)
    for r in range(modes):
        u0 += np.exp(-(_periodic_distance(x, c[r]) / w[r]) ** 2)
    spatial = np.stack([np.sin(2 * np.pi * k[r] * x + th[r]) for r in range(modes)], axis=1)

    def g_at(t: np.ndarray, T: float = 1.0) -> np.ndarray:
        y = 2.0 * np.asarray(t, dtype=np.float64) / T - 1.0
        temporal = np.stack([sum(alpha[r, d] * _cheb_T(d, y) for d in range(deg + 1))
                             for r in range(modes)], axis=0)   # (modes, s)
        return spatial @ temporal

    return u0, g_at


def config_c1(n: int = 256) -> Problem:
    """1-D advection-diffusion, n=256, a=1, nu=1e-2, T=1, Gaussian pulse, source
    sin(2 pi x) cos(4 pi t) at 64 Chebyshev-Lobatto times, 32 output times, l=30."""
    x = grid(n)
    u0 = np.exp(-((x - 0.3) / 0.05) ** 2)
    ts = chebyshev_lobatto(0.0, 1.0, 64)
    G = np.outer(np.sin(2 * np.pi * x), np.cos(4 * np.pi * ts))
    return Problem(n=n, coeffs=ade_coeffs(n, 1.0, 1e-2), u0=u0, t0=0.0, t1=1.0,
                   t_samples=ts, G=G, t_out=np.arange(1, 33) / 32.0, shift=True,
                   krylov_steps=30, rank_max=8, q_max=32, tol=1e-12, svd_tol=1e-13,
                   fit_tol=1e-13, name="c1_ade_n256")


def config_c2(n: int = 8192, seed: int = 2, krylov_steps: int = 60, s: int = 256,
              n_out: int = 32, tol: float = 1e-12) -> Problem:
    """1-D advection-diffusion, n=8192, a=1, nu=1e-3, T=1, u0 = 8 seeded Gaussians,
    source = 8 seeded Fourier modes x Chebyshev time polynomials of degree <= 6,
    256 Chebyshev-Lobatto samples, Krylov dimension 60, 32 output times."""
    rng = np.random.default_rng(seed)
    u0, g_at = smooth_field(rng, n, 8, 6)
    ts = chebyshev_lobatto(0.0, 1.0, s)
    return Problem(n=n, coeffs=ade_coeffs(n, 1.0, 1e-3), u0=u0, t0=0.0, t1=1.0,
                   t_samples=ts, G=g_at(ts), t_out=np.arange(1, n_out + 1) / n_out,
                   shift=True, krylov_steps=krylov_steps, rank_max=16, q_max=32, tol=tol,
                   svd_tol=1e-13, fit_tol=1e-13, name=f"c2_ade_n{n}")


def c2_source(n: int = 8192, seed: int = 2):
    """(u0, g_at) of config_c2 with the same seed: the source as a function of time, for
    sampling it on Paraexp windows."""
    rng = np.random.default_rng(seed)
    return smooth_field(rng, n, 8, 6)


def config_c3(n: int = 4096, K: int = 12, s: int = 512, jacobian: bool = True,
              krylov_steps: int = 80) -> BurgersProblem:
    """Viscous Burgers, n=4096, nu=5e-3, T=0.5, u0 = sin(2 pi x) + 0.5 sin(6 pi x),
    12 waveform-relaxation iterations, 512 uniform samples, rank <= 24, l = 80."""
    x = grid(n)
    u0 = np.sin(2 * np.pi * x) + 0.5 * np.sin(6 * np.pi * x)
    return BurgersProblem(n=n, nu=5e-3, T=0.5, P=1, s=s, K=K, u0=u0, jacobian=jacobian,
                          krylov_steps=krylov_steps, rank_max=24, name=f"c3_burgers_n{n}")


def config_c4(count: int = 512, seed: int = 4, n_lo: int = 512, n_hi: int = 16384,
              l_lo: int = 40, l_hi: int = 100, tol: float = 1e-9,
              indices: Optional[Sequence[int]] = None) -> List[Problem]:
    """512 independent advection-diffusion instances with seeded n, nu, a, rank and
    Krylov dimension; T=1, 64 Chebyshev-Lobatto samples, 32 output times.  `indices`
    builds only those instances (the same ones the full list holds)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_lo, n_hi + 1, count)
    nus = np.exp(rng.uniform(np.log(1e-4), np.log(1e-1), count))
    avs = rng.uniform(0.0, 2.0, count)
    rs = rng.integers(1, 9, count)
    ls = rng.integers(l_lo, l_hi + 1, count)
    seeds = rng.integers(0, 2**31 - 1, count)
    ts = chebyshev_lobatto(0.0, 1.0, 64)
    out = []
    for i in (range(count) if indices is None else indices):
        sub = np.random.default_rng(int(seeds[i]))
        u0, g_at = smooth_field(sub, int(ns[i]), int(rs[i]), 7)
        out.append(Problem(n=int(ns[i]), coeffs=ade_coeffs(int(ns[i]), float(avs[i]), float(nus[i])),
                           u0=u0, t0=0.0, t1=1.0, t_samples=ts, G=g_at(ts),
                           t_out=np.arange(1, 33) / 32.0, shift=True,
                           krylov_steps=int(ls[i]), rank_max=16, q_max=32, tol=tol,
                           svd_tol=1e-13, fit_tol=1e-13, name=f"c4_{i}"))
    return out


def config_c4_subset(count: int = 8, seed: int = 4, n_lo: int = 64, n_hi: int = 384) -> List[Problem]:
    """Same recipe as the 512-instance batch but with small grids (parity-test size)."""
    return config_c4(count=count, seed=seed, n_lo=n_lo, n_hi=n_hi, l_lo=12, l_hi=30, tol=1e-12)


def ade_windows(n: int, coeffs: np.ndarray, u0: np.ndarray, g_at: Callable, T: float, P: int,
                s: int, t_out: np.ndarray, sampler=chebyshev_lobatto, **kw) -> List[Problem]:
    """Split [0, T] into P equal windows (Sec. 2.2); window j carries the source on
    [T_{j-1}, T_j) only, samples it at s nodes, and reports outputs for all t_out."""
    probs = []
    for j in range(P):
        t0, t1 = T * j / P, T * (j + 1) / P
        ts = sampler(t0, t1, s)
        probs.append(Problem(n=n, coeffs=coeffs, u0=u0, t0=t0, t1=t1, t_samples=ts,
                             G=g_at(ts), t_out=np.asarray(t_out, dtype=np.float64),
                             shift=True, name=f"window{j}", **kw))
    return probs


def split_windows(p: Problem, P: int, g_at: Callable, s: Optional[int] = None) -> List[Problem]:
    """Paraexp windows of an existing single-window problem (same operator, u0, outputs)."""
    kw = dict(krylov_steps=p.krylov_steps, rank_max=p.rank_max, q_max=p.q_max, tol=p.tol,
              svd_tol=p.svd_tol, fit_tol=p.fit_tol)
    return ade_windows(p.n, p.coeffs, p.u0, g_at, p.t1 - p.t0, P, s or p.s, p.t_out, **kw)


def manufactured_ade(n: int = 1000, P: int = 8, s: int = 100, nu: float = 1e-2, a: float = 1.0,
                     T: float = 1.0, **kw):
    """Five travelling pulses u = 1/2 - 1/2 cos(10 pi (x - t)) (eq. (3.6)) with the source
    f = u_t + a u_x - nu u_xx evaluated at the grid points; returns (windows, exact(x, t))."""
    x = grid(n)
    u0 = 0.5 - 0.5 * np.cos(10 * np.pi * x)

    def f_at(t):
        t = np.asarray(t, dtype=np.float64)
        ph = 10 * np.pi * (x[:, None] - t[None, :])
        # u_t = -5 pi sin(ph), a u_x = 5 a pi sin(ph), -nu u_xx = -50 nu pi^2 cos(ph)
        return (a - 1.0) * 5 * np.pi * np.sin(ph) - 50 * nu * np.pi**2 * np.cos(ph)

    def exact(t):
        return 0.5 - 0.5 * np.cos(10 * np.pi * (x - t))

    wins = ade_windows(n, ade_coeffs(n, a, nu), u0, f_at, T, P, s, np.array([T]), **kw)
    return wins, exact


def sawtooth_wave(xi: np.ndarray, eps: float = 0.1, kmax: int = 100):
    """Smoothed sawtooth of Sec. 4.1 (eq. 4.2): u(xi) = 1/2 - sum_{k<=kmax} sin(2 pi k xi)
    Phi(k, eps) / (pi k), Phi = (pi k eps / 2) / sinh(pi k eps / 2); returns u, u', u''."""
    xi = np.asarray(xi, dtype=np.float64)
    u = np.full(xi.shape, 0.5)
    du = np.zeros(xi.shape)
    d2u = np.zeros(xi.shape)
    for k in range(1, kmax + 1):
        z = np.pi * k * eps / 2
        c = (z / np.sinh(z)) / (np.pi * k)
        arg = 2 * np.pi * k * xi
        u -= c * np.sin(arg)
        du -= c * 2 * np.pi * k * np.cos(arg)
        d2u += c * (2 * np.pi * k) ** 2 * np.sin(arg)
    return u, du, d2u


def manufactured_burgers(n: int = 100, nu: float = 1e-2, T: float = 0.1, P: int = 1, s: int = 50, K: int = 8,
                         speed: float = 0.5, **kw):
    """Travelling smoothed sawtooth of Sec. 4.1: u(x, t) = sawtooth(xi), xi = x - speed t +
    1/2, an exact solution of u_t + u u_x = nu u_xx + f with f = (u - speed) u_xi - nu u_xixi
    (eq. 4.1 with the manufactured source), sampled at the WR samples of every window.
    Returns (BurgersProblem, exact(t) -> u(x, t) on the grid)."""
    x = grid(n)

    def exact(t):
        return sawtooth_wave(x - speed * t + 0.5)[0]

    bp = BurgersProblem(n=n, nu=nu, T=T, P=P, s=s, K=K, u0=exact(0.0), name=f"sawtooth_n{n}_P{P}", **kw)
    cols = []
    for j in range(P):
        for t in bp.window_times(j):
            u, du, d2u = sawtooth_wave(x - speed * t + 0.5)
            cols.append((u - speed) * du - nu * d2u)
    bp.forcing = np.stack(cols, axis=1)
    return bp, exact


def random_ade_problem(seed: int, n: int, modes: int = 3, deg: int = 4, s: int = 24,
                       krylov_steps: int = 12, n_out: int = 5, a: float = 1.0, nu: float = 1e-2,
                       T: float = 0.25, shift: bool = True, per_point: bool = False,
                       tol: float = 1e-12) -> Problem:
    """Small seeded instance for parity tests (ragged n, few modes, short horizon)."""
    rng = np.random.default_rng(seed)
    u0, g_at = smooth_field(rng, n, modes, deg)
    ts = chebyshev_lobatto(0.0, T, s)
    G = g_at(ts, T)
    coeffs = ade_coeffs(n, a, nu)
    if per_point:
        x = grid(n)
        bump = 1.0 + 0.3 * np.sin(2 * np.pi * x + rng.uniform(0, 2 * np.pi))
        c = np.stack([coeffs[0] * bump, coeffs[1] * bump, coeffs[2] * bump])
        coeffs = c
    t_out = np.sort(rng.uniform(0.0, T, n_out - 1))
    t_out = np.concatenate([t_out, [T]])
    return Problem(n=n, coeffs=coeffs, u0=u0, t0=0.0, t1=T, t_samples=ts, G=G, t_out=t_out,
                   shift=shift, krylov_steps=krylov_steps, rank_max=16, q_max=24, tol=tol,
                   svd_tol=1e-13, fit_tol=1e-13, name=f"rand{seed}_n{n}")
