"""The piecewise-cubic source p(t) (Sec. 3: the paper's implementation takes p as piecewise
cubic polynomials; here the not-a-knot spline through the coefficient samples) on the GPU
path, through the C ABI, against the oracle (which marches one segment per spline piece
with the piece's Taylor coefficients as the polynomial state).

Both Krylov spaces; the FP64 bar 1e-10 on grids the dense oracle route finishes in
seconds, on the n = 8192 workload with the spectral route, and in the Burgers waveform
relaxation."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def gpu_out(t):
    return t.detach().cpu().numpy().T


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_04567_amd as pe
    c = pe.Context(0)
    yield c
    c.close()


def test_spline_compression_matches_oracle(ctx):
    p = synth.random_ade_problem(7, 300, modes=4, deg=9, s=33, krylov_steps=16, n_out=4)
    p.source_fit = 1
    got = ctx.compress(p)
    mdl = oracle.window_model(p)
    assert got["m"] == mdl["m"] and got["q"] == 4
    U = got["U"].detach().cpu().numpy().T          # (n, m)
    Pw = got["Pw"].detach().cpu().numpy()          # (pieces, 4, m)
    for i in (0, 7, len(Pw) - 1):
        assert rel(U @ Pw[i].T, mdl["U"] @ mdl["Cp"][i].T) < 1e-11, i


@pytest.mark.parametrize("krylov", [0, 1])
@pytest.mark.parametrize("case", ["rand", "rand_perpoint", "rand_noshift"])
def test_spline_solve_matches_dense_oracle(ctx, case, krylov):
    p = synth.random_ade_problem(8, 150, modes=3, deg=7, s=25, krylov_steps=14, n_out=6,
                                 per_point=case == "rand_perpoint", shift=case != "rand_noshift")
    p.source_fit = 1
    p.krylov = krylov
    ref, _ = oracle.solve_window(p, "dense")
    outs, reps = ctx.solve_batch([p])
    assert not reps[0]["flags"] & 1, reps[0]
    assert rel(gpu_out(outs[0]), ref) < FP64_TOL, reps[0]


def test_spline_c2_full_size(ctx):
    # the n = 8192 workload with the spline source on 257 uniform samples (256 pieces of
    # equal length, so the oracle's piece exponential is shared and every output is a
    # sample time): every sample is a restart point of the march
    p = synth.config_c2()
    _, g_at = synth.c2_source(p.n, 2)
    p.t_samples = synth.uniform_samples(0.0, 1.0, 257)
    p.G = g_at(p.t_samples)
    p.source_fit = 1
    p.krylov = 1
    ref, _ = oracle.solve_window(p, "spectral")
    outs, reps = ctx.solve_batch([p])
    assert not reps[0]["flags"] & 1, reps[0]
    got = gpu_out(outs[0])
    assert rel(got, ref) < FP64_TOL, reps[0]
    # each of the 257 outputs (every one a spline knot and a restart point), on the scale
    # of the largest
    per_out = np.linalg.norm(got - ref, axis=0) / np.linalg.norm(ref, axis=0).max()
    assert per_out.max() < FP64_TOL, per_out.max()


def test_spline_wr_matches_dense_oracle(ctx):
    bp, _ = synth.manufactured_burgers(n=96, P=2, s=21, K=3, tol=1e-12, svd_tol=1e-13, fit_tol=1e-12)
    bp.source_fit = 1
    bp.krylov = 1
    ref = oracle.wr_burgers(bp, "dense")
    U, reps, inc = ctx.wr_burgers(bp)
    assert rel(U.detach().cpu().numpy().T, ref) < FP64_TOL, (reps, inc)
