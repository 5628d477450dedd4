"""pe_compress_noalloc (the compression entry point for callers that cannot allocate)
against pe_compress, through the C ABI, on two calls in a row -- the second on a smaller
problem, so the fixed scratch still holds the first call's data -- and its size limit.

Both entry points run the same kernels on the same inputs with fixed-order reductions,
so their results must agree bit for bit (integer results exactly, and U, Pi and the
singular values too)."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_04567_amd as pe
    c = pe.Context(0)
    yield c
    c.close()


def test_noalloc_compress_matches_compress_on_two_calls(ctx):
    import torch
    big = synth.config_c2(n=8192)          # 8192 x 256 samples: 48 MiB of scratch
    small = synth.config_c1()              # 256 x 64, after the big one
    for p in (big, small):
        print(f"noalloc compress: {p.name} n={p.n} s={p.s}", flush=True)
        ref = ctx.compress(p)
        got = ctx.compress(p, noalloc=True)
        assert got["m"] == ref["m"] and got["q"] == ref["q"]
        assert got["report"] == ref["report"]
        assert np.array_equal(got["sigma"], ref["sigma"])
        assert torch.equal(got["U"], ref["U"])
        assert torch.equal(got["Pi"], ref["Pi"])
        assert ref["m"] > 0


def test_noalloc_compress_rejects_problems_beyond_the_scratch(ctx):
    import paper_1509_04567_amd as pe
    x = synth.grid(1 << 16)
    ts = synth.chebyshev_lobatto(0.0, 1.0, 128)   # 65536 x 128 samples: over 128 MiB of scratch
    G = np.outer(np.sin(2 * np.pi * x), np.cos(ts))
    p = synth.Problem(n=x.size, coeffs=synth.ade_coeffs(x.size, 1.0, 1e-3), u0=np.zeros(x.size), t0=0.0, t1=1.0,
                      t_samples=ts, G=G, t_out=np.array([1.0]), shift=False, krylov_steps=10, rank_max=4,
                      q_max=16, tol=1e-10, svd_tol=1e-13, fit_tol=1e-12)
    with pytest.raises(pe.PeError) as ei:
        ctx.compress(p, noalloc=True)
    assert ei.value.status == pe.PE_ERR_UNSUPPORTED
    assert ctx.compress(p)["m"] == 1        # the allocating entry point still takes it
