"""The batched workload: 512 independent advection-diffusion instances (seeded n in
512..16384, nu log-uniform in [1e-4, 1e-1], a in [0, 2], source rank 1-8, Krylov dimension
40-100, 64 Chebyshev-Lobatto samples, 32 outputs), every instance solved on the GPU in
batches of 128 through pe_solve_batch with the shift-and-invert Krylov space.

Pins: every instance converges (no flags), and 25 instances spread over the batch match
the CPU oracle's spectral route (exact exponential of the augmented system per Fourier
mode, Sec. 2.1 eq. 2.4 with the fitted source of eq. 2.3).  The workload's own step
tolerance (1e-9 per unit time, relative to max(|u0|, |y|)) is used, so the bar is ten
times that tolerance over the unit horizon rather than the 1e-10 of the tighter-tolerance
parity tests: several instances (nu ~ 1e-4 at n ~ 1.3e4, |L| ~ 1e5-1e6) cannot resolve a
residual below about eps |L| |u| per unit time, so a 1e-11 tolerance is out of their
reach with either Krylov space.  Each chunk prints its time and largest cycle count."""
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-9
BAR = 10 * TOL
CHUNK = 128


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_04567_amd as pe
    c = pe.Context(0)
    yield c
    c.close()


def test_c4_all_512_instances(ctx):
    import paper_1509_04567_amd as pe
    probs = synth.config_c4(tol=TOL)
    for p in probs:
        p.krylov = pe.PE_KRYLOV_SAI
    check = set(range(0, 512, 512 // 24))
    errs, cycles = {}, []
    for c0 in range(0, len(probs), CHUNK):
        chunk = probs[c0:c0 + CHUNK]
        t0 = time.perf_counter()
        outs, reps = ctx.solve_batch(chunk)
        dt = time.perf_counter() - t0
        cycles += [r["cycles"] for r in reps]
        print(f"C4 instances {c0}..{c0 + len(chunk) - 1}: {dt:.2f} s, cycles max {max(r['cycles'] for r in reps)}",
              flush=True)
        for i, (p, o, r) in enumerate(zip(chunk, outs, reps)):
            assert r["flags"] & 1 == 0, (c0 + i, r)
            if c0 + i in check:
                ref, _ = oracle.solve_window(p, "spectral")
                errs[c0 + i] = rel(o.detach().cpu().numpy().T, ref)
                print(f"  instance {c0 + i}: n={p.n} l={p.krylov_steps} rel L2 {errs[c0 + i]:.2e}", flush=True)
        del outs
    worst = max(errs.values())
    print(f"C4: {len(probs)} instances, cycles mean {np.mean(cycles):.1f} max {max(cycles)}, "
          f"worst sampled rel L2 {worst:.2e}", flush=True)
    assert worst < BAR, errs
