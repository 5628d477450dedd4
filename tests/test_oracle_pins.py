"""Pins of the CPU oracle against facts that do not come from the oracle itself:
closed forms, an independent integrator, a library routine, invariants, and the
number the paper prints (Table 1).  CPU only."""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle
import synth
from oracle.march import march_segments

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def _problem(n, coeffs, u0, G, ts, t_out, shift, **kw):
    return synth.Problem(n=n, coeffs=np.asarray(coeffs, dtype=np.float64), u0=u0, t0=float(ts[0]),
                         t1=float(ts[-1]), t_samples=ts, G=G, t_out=np.asarray(t_out, dtype=np.float64),
                         shift=shift, **kw)


# ---------------------------------------------------------------- expm (library pin)
@pytest.mark.parametrize("scale", [0.01, 0.5, 3.0, 40.0, 300.0])
def test_expm_matches_scipy(scale):
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 30))
    A = scale * (A - 3.0 * np.eye(30)) / np.linalg.norm(A, 1)
    assert rel(oracle.expm(A), scipy.linalg.expm(A)) < 1e-12


def test_expm_closed_forms():
    th = 2.7
    R = oracle.expm(np.array([[0.0, -th], [th, 0.0]]))
    assert np.allclose(R, [[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]], atol=1e-14)
    N = np.diag(np.ones(4), 1) * 1.5                    # nilpotent: exp is a finite sum
    E = oracle.expm(N)
    ref = sum(np.linalg.matrix_power(N, k) / math.factorial(k) for k in range(5))
    assert np.max(np.abs(E - ref)) < 1e-13
    d = np.array([-50.0, -1.0, 0.0, 2.0])
    assert np.allclose(oracle.expm(np.diag(d)), np.diag(np.exp(d)), rtol=1e-13, atol=0)


def test_pade_coefficients_reproduce_exp():
    # the [13/13] approximant must match e^x to roundoff for |x| <= 1
    c = oracle.pade_coefficients(13)
    for x in [-1.0, -0.3, 0.2, 1.0]:
        num = sum(c[k] * x**k for k in range(14))
        den = sum(c[k] * (-x) ** k for k in range(14))
        assert abs(num / den - math.exp(x)) < 1e-15 * math.exp(abs(x))


# ---------------------------------------------------------------- time generator
def test_time_generator_translates_chebyshev_vector():
    q, t0, t1 = 12, 0.3, 0.8
    K = oracle.time_generator(q, t0, t1)
    for ta, tb in [(0.3, 0.45), (0.3, 0.8), (0.5, 0.61)]:
        xa, xb = [(2 * t - t0 - t1) / (t1 - t0) for t in (ta, tb)]
        wa = np.polynomial.chebyshev.chebvander(np.array([xa]), q - 1)[0]
        wb = np.polynomial.chebyshev.chebvander(np.array([xb]), q - 1)[0]
        # K is nilpotent, so its exponential is the finite Taylor sum
        E = sum(np.linalg.matrix_power((tb - ta) * K, j) / math.factorial(j) for j in range(q))
        assert np.max(np.abs(E @ wa - wb)) < 1e-14 * np.abs(E).sum(axis=1).max()


# ---------------------------------------------------------------- P1 Fourier-mode decay
@pytest.mark.parametrize("route", ["dense", "spectral"])
@pytest.mark.parametrize("a,nu", [(1.0, 1e-2), (0.0, 1e-2), (1.0, 0.0)])
def test_p1_fourier_mode_decay(route, a, nu):
    n, k = 64, 3
    h = 1.0 / n
    x = synth.grid(n)
    ts = synth.chebyshev_lobatto(0.0, 1.0, 8)
    t_out = np.array([0.1, 0.5, 1.0, 1.7])
    p = _problem(n, synth.ade_coeffs(n, a, nu), np.cos(2 * np.pi * k * x), np.zeros((n, 8)), ts,
                 t_out, shift=False)
    out, _ = oracle.solve_window(p, route)
    # semi-discrete symbol of the central-difference stencil
    lam = -(4 * nu / h**2) * math.sin(math.pi * k / n) ** 2 - 1j * (a / h) * math.sin(2 * math.pi * k / n)
    ref = np.stack([np.real(np.exp(lam * t) * np.exp(2j * np.pi * k * x)) for t in t_out], axis=1)
    assert rel(out, ref) < 1e-12


# ---------------------------------------------------------------- P2 phi-response
@pytest.mark.parametrize("route", ["dense", "spectral"])
def test_p2_phi_response_constant_and_linear_source(route):
    n, k, a, nu = 48, 2, 0.7, 3e-2
    h = 1.0 / n
    x = synth.grid(n)
    al, be, a0 = 1.3, -2.1, 0.4
    T = 0.6
    ts = synth.chebyshev_lobatto(0.0, T, 10)
    G = np.outer(np.cos(2 * np.pi * k * x), al + be * ts)
    t_out = np.array([0.05, 0.3, 0.6, 0.9])          # the last one is after the window
    p = _problem(n, synth.ade_coeffs(n, a, nu), a0 * np.cos(2 * np.pi * k * x), G, ts, t_out,
                 shift=False)
    out, mdl = oracle.solve_window(p, route)
    assert mdl["m"] == 1 and mdl["q"] == 2
    lam = -(4 * nu / h**2) * math.sin(math.pi * k / n) ** 2 - 1j * (a / h) * math.sin(2 * math.pi * k / n)

    def phi1(z):
        return (np.exp(z) - 1) / z

    def phi2(z):
        return (np.exp(z) - 1 - z) / z**2

    def y(t):
        return np.exp(lam * t) * a0 + al * t * phi1(lam * t) + be * t**2 * phi2(lam * t)

    cols = []
    for t in t_out:
        yt = y(t) if t <= T else np.exp(lam * (t - T)) * y(T)
        cols.append(np.real(yt * np.exp(2j * np.pi * k * x)))
    assert rel(out, np.stack(cols, axis=1)) < 1e-12


# ---------------------------------------------------------------- P3 RK4 brute force
def _rk4(coeffs, u0, g_at, t_end, dt):
    u = u0.copy()
    t = 0.0
    nsteps = int(round(t_end / dt))
    for _ in range(nsteps):
        f = lambda tt, uu: oracle.apply_stencil(coeffs, uu) + g_at(np.array([tt]))[:, 0]
        k1 = f(t, u)
        k2 = f(t + dt / 2, u + dt / 2 * k1)
        k3 = f(t + dt / 2, u + dt / 2 * k2)
        k4 = f(t + dt, u + dt * k3)
        u = u + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        t += dt
    return u


@pytest.mark.parametrize("per_point", [False, True])
@pytest.mark.parametrize("shift", [True, False])
def test_p3_rk4_brute_force(per_point, shift):
    n, T = 24, 0.2
    rng = np.random.default_rng(7)
    u0, g_at = synth.smooth_field(rng, n, 2, 3)
    ts = synth.chebyshev_lobatto(0.0, T, 12)
    coeffs = synth.ade_coeffs(n, 1.0, 1e-2)
    if per_point:
        bump = 1.0 + 0.3 * np.sin(2 * np.pi * synth.grid(n))
        coeffs = np.stack([coeffs[0] * bump, coeffs[1] * bump, coeffs[2] * bump])
    gT = lambda t: g_at(t, T)
    p = _problem(n, coeffs, u0, gT(ts), ts, [T], shift=shift)
    out, mdl = oracle.solve_window(p, "dense")
    u_or = (u0 + out[:, 0]) if shift else out[:, 0]
    u_rk = _rk4(coeffs, u0, gT, T, 2e-5)
    assert mdl["q"] == 4          # cubic time dependence is fitted exactly
    assert rel(u_or, u_rk) < 1e-11


# ---------------------------------------------------------------- P4 two routes agree
def test_p4_dense_and_spectral_agree_c1():
    p = synth.config_c1()
    od, md = oracle.solve_window(p, "dense")
    osp, ms = oracle.solve_window(p, "spectral")
    assert md["m"] == ms["m"] == 2
    assert rel(osp, od) < 1e-12


# ---------------------------------------------------------------- P5 superposition
@pytest.mark.parametrize("route", ["dense", "spectral"])
def test_p5_superposition_equals_sequential_march(route):
    rng = np.random.default_rng(11)
    n = 80
    u0, g_at = synth.smooth_field(rng, n, 3, 5)
    t_out = np.array([0.1, 0.25, 0.5, 0.8, 1.0])
    wins = synth.ade_windows(n, synth.ade_coeffs(n, 1.0, 5e-3), u0, g_at, 1.0, 4, 16, t_out,
                             krylov_steps=10, rank_max=8, q_max=16, tol=1e-12, svd_tol=1e-13,
                             fit_tol=1e-13)
    sup = oracle.solve_windows_superposed(wins, route)
    seq = oracle.solve_sequential(wins, route)
    assert rel(sup, seq) < 1e-13


# ---------------------------------------------------------------- P6 paper's Table 1
def _golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    vals = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    return vals


def test_p6_manufactured_ade_reproduces_table1_serial_error():
    n, nu, a = 1000, 1e-2, 1.0
    wins, exact = synth.manufactured_ade(n=n, P=8, s=100, krylov_steps=20, rank_max=8, q_max=32,
                                         tol=1e-12, svd_tol=1e-12, fit_tol=1e-13)
    u = oracle.solve_windows_superposed(wins, "spectral")[:, 0]
    # semi-discrete closed form: only Fourier mode 5 (10 pi x) is excited
    h = 1.0 / n
    x = synth.grid(n)
    kk = 5
    lam = -(4 * nu / h**2) * math.sin(math.pi * kk / n) ** 2 - 1j * (a / h) * math.sin(2 * math.pi * kk / n)
    om = 10 * np.pi
    # u = 1/2 - 1/2 Re(e^{i om x} y(t)), y(0) = 1, forcing of y: 100 nu pi^2 e^{-i om t}
    c = 100 * nu * np.pi**2 * (1.0 / 1.0)
    y = np.exp(lam) * 1.0 + c * (np.exp(lam) - np.exp(-1j * om)) / (lam + 1j * om)
    u_semi = 0.5 - 0.5 * np.real(np.exp(1j * om * x) * y)
    assert rel(u, u_semi) < 1e-10
    err = rel(u, exact(1.0))
    paper = _golden("table1_serial_error.txt")["serial_error"]
    assert abs(err - paper) / paper < 0.01
    assert wins[0].n == 1000 and oracle.window_model(wins[0])["m"] == 2


# ---------------------------------------------------------------- P8 Theorem 1
def test_p8_singular_value_decay_with_window_length():
    n = 200
    x = synth.grid(n)
    prof = np.stack([np.sin(2 * np.pi * k * x + 0.3 * k) for k in (1, 3, 4, 7)], axis=1)
    rates = np.array([0.7, -1.3, 2.1, -0.4])

    def ratios(dT):
        ts = synth.chebyshev_lobatto(0.0, dT, 16)
        G = prof @ np.exp(np.outer(rates, ts))
        sig = np.linalg.svd(G, compute_uv=False)
        return sig / sig[0]

    r1, r2 = ratios(0.2), ratios(0.1)
    assert 0.35 < r2[1] / r1[1] < 0.65          # sigma_2 / sigma_1 ~ dT
    assert 0.15 < r2[2] / r1[2] < 0.35          # sigma_3 / sigma_1 ~ dT^2
    # the oracle's compression sees the same singular values (independent eigen route)
    m, U, C, sig, tail, _ = oracle.compress(prof @ np.exp(np.outer(rates, synth.chebyshev_lobatto(0, 0.2, 16))), 1e-3, 8)
    G = prof @ np.exp(np.outer(rates, synth.chebyshev_lobatto(0, 0.2, 16)))
    ev = np.sqrt(np.clip(np.sort(np.linalg.eigvalsh(G.T @ G))[::-1], 0, None))
    assert np.allclose(sig[:3], ev[:3], rtol=1e-10)
    assert np.allclose(U.T @ U, np.eye(m), atol=1e-13)
    assert abs(np.linalg.norm(G - U @ C) / np.linalg.norm(G) - tail) < 1e-12


# ---------------------------------------------------------------- P9 exact ranks
def test_p9_exact_ranks():
    p1 = synth.config_c1()
    assert oracle.window_model(p1)["m"] == 2
    p2 = synth.config_c2(n=1024, s=64)
    mdl = oracle.window_model(p2)
    assert mdl["m"] == 7 and mdl["q"] == 7
    # constant source: exact with m = 1 and a constant p (Sec. 3.1)
    n = 64
    x = synth.grid(n)
    ts = synth.chebyshev_lobatto(0.0, 1.0, 9)
    p3 = _problem(n, synth.ade_coeffs(n, 1.0, 1e-2), np.exp(-((x - 0.5) / 0.1) ** 2),
                  np.zeros((n, 9)), ts, [1.0], shift=True)
    m3 = oracle.window_model(p3)
    assert m3["m"] == 1 and m3["q"] == 1


# ---------------------------------------------------------------- P10 mass
def test_p10_mass_balance():
    p = synth.random_ade_problem(3, 96, T=0.4)
    out, mdl = oracle.solve_window(p, "dense")
    # d/dt sum(v) = sum(fitted source) because the stencil columns sum to zero
    assert abs(np.sum(p.coeffs)) < 1e-9 * np.max(np.abs(p.coeffs))
    gx, gw = np.polynomial.legendre.leggauss(40)
    colsum = mdl["B"].sum(axis=0)
    for k, t in enumerate(p.t_out):
        tt = p.t0 + (t - p.t0) * (gx + 1) / 2
        xx = (2 * tt - p.t0 - p.t1) / (p.t1 - p.t0)
        W = np.polynomial.chebyshev.chebvander(xx, mdl["q"] - 1)
        integral = (t - p.t0) / 2 * gw @ (W @ colsum)
        assert abs(out[:, k].sum() - integral) < 1e-9 * max(1.0, abs(integral))


# ---------------------------------------------------------------- P11 dissipativity
def test_p11_homogeneous_norm_nonincreasing():
    n = 128
    x = synth.grid(n)
    ts = synth.chebyshev_lobatto(0.0, 1.0, 4)
    t_out = np.linspace(0.05, 1.0, 20)
    p = _problem(n, synth.ade_coeffs(n, 1.0, 1e-3), np.exp(-((x - 0.4) / 0.03) ** 2),
                 np.zeros((n, 4)), ts, t_out, shift=False)
    out, _ = oracle.solve_window(p, "spectral")
    norms = np.linalg.norm(out, axis=0)
    assert np.all(np.diff(norms) <= 1e-14 * norms[0])


# ---------------------------------------------------------------- WR vs RK4 of the nonlinear ODE
@pytest.mark.parametrize("jacobian", [True, False])
@pytest.mark.parametrize("P", [1, 2])
def test_wr_burgers_converges_to_rk4_solution(jacobian, P):
    n = 32
    x = synth.grid(n)
    bp = synth.workloads.BurgersProblem(n=n, nu=0.05, T=0.1, P=P, s=16, K=10 if jacobian else 16,
                                        u0=np.sin(2 * np.pi * x) + 0.5 * np.sin(6 * np.pi * x),
                                        jacobian=jacobian, rank_max=16, q_max=16, svd_tol=1e-13,
                                        fit_tol=1e-12)
    U, hist = oracle.wr_burgers(bp, "dense", return_history=True)
    h = 1.0 / n

    def f(uu):
        # right-hand side of the semi-discrete Burgers system written out here, not taken
        # from the oracle: nu (u_{i+1} - 2 u_i + u_{i-1}) / h^2 - u_i (u_{i+1} - u_{i-1}) / (2h)
        up, um = np.concatenate([uu[1:], uu[:1]]), np.concatenate([uu[-1:], uu[:-1]])
        return bp.nu * (up - 2.0 * uu + um) / h**2 - uu * (up - um) / (2.0 * h)

    u = bp.u0.copy()
    dt = 1e-5
    for _ in range(int(round(bp.T / dt))):
        k1 = f(u); k2 = f(u + dt / 2 * k1); k3 = f(u + dt / 2 * k2); k4 = f(u + dt * k3)
        u = u + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    assert rel(U[:, -1], u) < 1e-8
    assert hist[-1]["increment"] < 1e-9


def test_wr_spectral_picard_matches_dense():
    n = 64
    x = synth.grid(n)
    bp = synth.workloads.BurgersProblem(n=n, nu=0.02, T=0.1, P=1, s=10, K=3, u0=np.sin(2 * np.pi * x),
                                        jacobian=False, rank_max=10, q_max=10)
    a = oracle.wr_burgers(bp, "dense")
    b = oracle.wr_burgers(bp, "spectral")
    assert rel(a, b) < 1e-11


# ---------------------------------------------------------------- Burgers nonlinearity and Jacobian
@pytest.mark.parametrize("n", [16, 64, 256, 1000])
def test_burgers_nonlinear_closed_form_on_a_sine(n):
    """N(u)_i = -u_i (u_{i+1} - u_{i-1}) / (2h) on u = sin(2 pi x): the central difference of
    a sine is exact up to the factor sin(2 pi h) / (2 pi h), so
    N_i = -sin(2 pi x_i) cos(2 pi x_i) sin(2 pi h) / h (Sec. 4.1, eq. burgersEq discretised)."""
    h = 1.0 / n
    x = np.arange(n) / n
    got = oracle.burgers_nonlinear(np.sin(2 * np.pi * x), h)
    want = -np.sin(2 * np.pi * x) * np.cos(2 * np.pi * x) * np.sin(2 * np.pi * h) / h
    assert np.max(np.abs(got - want)) <= 1e-12 * np.max(np.abs(want))
    # block input: column by column, a phase-shifted sine in the second column
    U = np.stack([np.sin(2 * np.pi * x), np.sin(2 * np.pi * x + 0.7)], axis=1)
    G = oracle.burgers_nonlinear(U, h)
    want2 = -np.sin(2 * np.pi * x + 0.7) * np.cos(2 * np.pi * x + 0.7) * np.sin(2 * np.pi * h) / h
    assert np.max(np.abs(G[:, 0] - want)) <= 1e-12 * np.max(np.abs(want))
    assert np.max(np.abs(G[:, 1] - want2)) <= 1e-12 * np.max(np.abs(want2))


def _sawtooth(xi, eps=0.1, kmax=100):
    """Smoothed sawtooth of Sec. 4.1 (eq. modifiedSawtooth) and its exact derivative:
    u = 1/2 - sum_k sin(2 pi k xi) Phi_k / (pi k), Phi_k = (pi k eps/2) / sinh(pi k eps/2)."""
    k = np.arange(1, kmax + 1)[:, None]
    a = np.pi * k * eps / 2
    phi = a / np.sinh(a)
    u = 0.5 - np.sum(np.sin(2 * np.pi * k * xi) * phi / (np.pi * k), axis=0)
    ux = -np.sum(2 * np.cos(2 * np.pi * k * xi) * phi, axis=0)
    return u, ux


def test_burgers_nonlinear_second_order_on_the_smoothed_sawtooth():
    """The advective discretisation is consistent with -u u_x to second order: on the
    paper's manufactured solution (Sec. 4.1, at t = 0.3) halving h cuts the error by 4."""
    errs = []
    for n in (256, 512, 1024, 2048):
        x = np.arange(n) / n
        u, ux = _sawtooth(x - 0.5 * 0.3 + 0.5)
        errs.append(np.max(np.abs(oracle.burgers_nonlinear(u, 1.0 / n) - (-u * ux))))
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(np.abs(ratios - 4.0) < 0.1), ratios


@pytest.mark.parametrize("seed", [0, 1])
def test_burgers_jacobian_is_the_derivative_of_the_nonlinearity(seed):
    """J(u) v = (N(u + e v) - N(u - e v)) / (2e) for every direction v.  N is quadratic, so
    the central difference is exact apart from rounding (Sec. 2.3, eq. jacobian).  The
    product J v is formed here from the three stencil rows by explicit indexing."""
    rng = np.random.default_rng(seed)
    n = 96
    h = 1.0 / n
    u = rng.standard_normal(n)
    J = oracle.burgers_jacobian(u, h)
    assert J.shape == (3, n)
    for _ in range(3):
        v = rng.standard_normal(n)
        Jv = np.array([J[0, i] * v[i - 1] + J[1, i] * v[i] + J[2, i] * v[(i + 1) % n] for i in range(n)])
        e = 1e-3
        fd = (oracle.burgers_nonlinear(u + e * v, h) - oracle.burgers_nonlinear(u - e * v, h)) / (2 * e)
        assert rel(Jv, fd) < 1e-10
    # the dense Jacobian built entry by entry from partial derivatives of N_i
    D = np.zeros((n, n))
    for i in range(n):
        for j in range(n):
            ej = np.zeros(n)
            ej[j] = 1.0
            D[i, j] = (oracle.burgers_nonlinear(u + ej, h)[i] - oracle.burgers_nonlinear(u - ej, h)[i]) / 2.0
    assert rel(oracle.dense_operator(n, J), D) < 1e-12


# ---------------------------------------------------------------- truncation rule (reading #8)
def _matrix_with_spectrum(sig, n=200, s=40, seed=3):
    rng = np.random.default_rng(seed)
    Uq, _ = np.linalg.qr(rng.standard_normal((n, len(sig))))
    Vq, _ = np.linalg.qr(rng.standard_normal((s, len(sig))))
    return (Uq * np.asarray(sig)) @ Vq.T


def _rank_by_eckart_young(sig, svd_tol):
    """Brute force: the smallest r whose best rank-r approximation (Eckart-Young) leaves
    a Frobenius error <= svd_tol ||G||_F, from the singular values by direct summation."""
    fro = math.sqrt(sum(v * v for v in sig))
    for r in range(len(sig) + 1):
        if math.sqrt(sum(v * v for v in sig[r:])) <= svd_tol * fro:
            return r
    return len(sig)


@pytest.mark.parametrize("svd_tol", [0.3, 3e-2, 1e-3, 1e-6, 1e-9])
def test_truncation_energy_rule_is_eckart_young(svd_tol):
    sig = [3.0, 1.0, 0.4, 1e-2, 3e-4, 1e-5, 2e-7, 5e-9, 1e-10]
    G = _matrix_with_spectrum(sig)
    m, U, C, got_sig, tail, flags = oracle.compress(G, svd_tol, 30)
    assert m == _rank_by_eckart_young(sig, svd_tol)
    # the reported tail is the relative Frobenius error of the kept factorisation
    assert abs(np.linalg.norm(G - U @ C) / np.linalg.norm(G) - tail) < 1e-13


def test_truncation_keeps_a_cluster_whole():
    """sigma_3 and sigma_4 differ by 4e-13 sigma_1: a cut between them by the energy rule
    alone (m = 3) is widened to keep both (reading #8)."""
    sig = [1.0, 0.5, 0.1, 0.1 - 4e-13, 1e-6, 1e-7]
    G = _matrix_with_spectrum(sig)
    fro = math.sqrt(sum(v * v for v in sig))
    svd_tol = 0.09                                  # tail after 3 is 0.0887 ||G||_F
    assert _rank_by_eckart_young(sig, svd_tol) == 3
    m, *_ = oracle.compress(G, svd_tol, 30)
    assert m == 4
    # a gap of 1e-9 sigma_1 is not a cluster
    sig2 = [1.0, 0.5, 0.1, 0.1 - 1e-9, 1e-6, 1e-7]
    m2, *_ = oracle.compress(_matrix_with_spectrum(sig2), svd_tol, 30)
    assert m2 == 3
    assert fro > 0


def test_truncation_floor_and_cap():
    """Singular values at or below 1e-14 sigma_1 are never kept, whatever svd_tol asks;
    values just above it are; rank_max caps m and sets the flag."""
    sig = [1.0, 0.3, 5e-13, 2e-13, 5e-15]
    G = _matrix_with_spectrum(sig)
    m, *_ = oracle.compress(G, 0.0, 30)
    assert m == 4
    m, *_rest, flags = oracle.compress(G, 0.0, 2)
    assert m == 2 and flags & 4
    # svd_tol = 1e-13 of ||G||_F (~1.04): both 5e-13 and 2e-13 are needed
    assert _rank_by_eckart_young(sig, 1e-13) == 4
    m, *_ = oracle.compress(G, 1e-13, 30)
    assert m == 4


def test_wr_with_the_manufactured_sawtooth_source_reaches_a_second_order_floor():
    # Sec. 4.1: with the manufactured source the waveform-relaxation iterate converges to
    # the semi-discrete solution, whose distance to the exact travelling sawtooth is the
    # O(dx^2) error of the central differences (the floor of the paper's error histories)
    floors = []
    for n in (100, 200):
        bp, exact = synth.manufactured_burgers(n=n, P=1, s=50, K=8)
        U = oracle.wr_burgers(bp, "dense")
        ex = np.stack([exact(t) for t in bp.window_times(0)], axis=1)
        floors.append(np.linalg.norm(U - ex) / np.linalg.norm(ex))
    assert 3.6 < floors[0] / floors[1] < 4.5, floors


def test_cubic_spline_fit_matches_scipy():
    # the piecewise-cubic p(t) of Sec. 3 ("piecewise cubic polynomials"), read as the
    # not-a-knot interpolating spline: same coefficients as scipy's CubicSpline
    from scipy.interpolate import CubicSpline
    from oracle.compress import fit_cubic_spline
    rng = np.random.default_rng(11)
    for s in (3, 4, 5, 9, 64):
        t = np.sort(rng.uniform(0.0, 1.0, s))
        t[0], t[-1] = 0.0, 1.0
        C = rng.standard_normal((4, s))
        Cp = fit_cubic_spline(C, t)
        ref = CubicSpline(t, C.T, bc_type="not-a-knot").c   # (4, s-1, m), highest power first
        for k in range(4):  # relative to the largest coefficient of that power, or to 1
            scale = max(np.abs(ref[3 - k]).max(), 1.0)
            assert np.abs(Cp[:, k, :] - ref[3 - k]).max() <= 1e-12 * scale, (s, k)
    # two samples: the straight line
    Cp = fit_cubic_spline(np.array([[1.0, 3.0]]), np.array([0.0, 0.5]))
    assert np.allclose(Cp[0, :, 0], [1.0, 4.0, 0.0, 0.0])


def test_spline_source_of_a_cubic_in_time_equals_the_polynomial_route():
    # a source that is cubic in time is reproduced exactly by the spline, so the piecewise
    # march (one segment per piece, Taylor-coefficient state) equals the single
    # Chebyshev-polynomial march; dense and spectral routes agree on the pieces
    p = synth.random_ade_problem(5, 64, modes=3, deg=3, s=12, krylov_steps=12, n_out=5)
    r_cheb, _ = oracle.solve_window(p, "dense")
    p.source_fit = 1
    r_dense, _ = oracle.solve_window(p, "dense")
    r_spec, _ = oracle.solve_window(p, "spectral")
    assert np.linalg.norm(r_dense - r_cheb) <= 1e-12 * np.linalg.norm(r_cheb)
    assert np.linalg.norm(r_spec - r_dense) <= 1e-12 * np.linalg.norm(r_dense)
