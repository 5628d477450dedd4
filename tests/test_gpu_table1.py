"""The paper's parallel-efficiency workload (Sec. 3.2, Table 1) on the GPU path.

Manufactured advection-diffusion problem with five travelling pulses, a = 1,
nu = 1e-2, dx = 1e-3 (n = 1000), 100 samples per window, rank-2 source; the interval
[0, 1] is split into P windows that are solved as one batch and superposed on the GPU.
Pins: (1) the superposed GPU solution equals the oracle's (spectral route) to the FP64
bar; (2) its error against the exact PDE solution at T = 1 reproduces the serial
error of Table 1 (tests/golden/table1_serial_error.txt) within 1% for every P -- the
Paraexp split does not change the result, which is the paper's claim for PEBK.  Every P of
the table (1 to 32) with both Krylov spaces."""
import os

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def golden(name):
    vals = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", name)):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            vals[k] = float(v)
    return vals


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_04567_amd as pe
    c = pe.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("krylov", [0, 1])
@pytest.mark.parametrize("P", [1, 2, 4, 8, 16, 32])
def test_table1_manufactured_ade_on_gpu(ctx, P, krylov):
    # krylov 0: the polynomial block Krylov space; 1: shift-and-invert
    wins, exact = synth.manufactured_ade(n=1000, P=P, s=100, krylov_steps=20, rank_max=8, q_max=32,
                                         tol=1e-12, svd_tol=1e-12, fit_tol=1e-13)
    for w in wins:
        w.krylov = krylov
    outs, reps = ctx.solve_batch(wins)
    assert all(r["rank"] == 2 for r in reps)
    u = ctx.superpose(wins[0].u0, outs).detach().cpu().numpy()[0]
    ref = oracle.solve_windows_superposed(wins, "spectral")[:, 0]
    assert rel(u, ref) < 1e-10
    err = rel(u, exact(1.0))
    paper = golden("table1_serial_error.txt")["serial_error"]
    assert abs(err - paper) / paper < 0.01, err
