"""Tile autotuning of the block orthogonalisation kernels (pe_autotune), through the C ABI.

The tuned tiling only partitions the rows of each block step differently (the batched
pipeline of Sec. 2.2 over the block Arnoldi of eq. 2.4), so a solve on a tuned context
must still match the oracle to the same bars as the default tiling: FP64 1e-10 against the
dense route on small grids, and on the n = 8192 advection-diffusion workload against the
spectral route.  The cache file round-trips the choices."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
MIXED_TOL = 1e-7


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(b), 1e-300))


def gpu_out(t):
    return t.detach().cpu().numpy().T


@pytest.fixture()
def pe():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1509_04567_amd as pe
    return pe


def test_autotune_choices_are_admissible_and_cached(pe, tmp_path):
    cache = str(tmp_path / "tiles.txt")
    ctx = pe.Context(0)
    try:
        shapes = [(8192, 16, pe.PE_FP64), (8192, 16, pe.PE_MIXED), (600, 3, pe.PE_FP64)]
        assert ctx.autotune(shapes, cache) == 17 + 17 + 4
        table = ctx.autotune_table()
        print("tuned tiles", table, flush=True)
        assert set(table) == ({(13, bw, mx) for bw in range(1, 18) for mx in (0, 1)}
                              | {(10, bw, 0) for bw in range(1, 5)})
        for (nlog2, bw, _), (ru, rp) in table.items():
            assert ru in (64, 128, 256, 512) and ru <= 1 << nlog2
            assert rp in (16, 32, 64, 128, 256) and rp * bw <= 1024
        # keys already known are not timed again
        assert ctx.autotune(shapes[:1], None) == 0
    finally:
        ctx.close()
    ctx2 = pe.Context(0)
    try:
        assert ctx2.autotune(shapes, cache) == 0
        assert ctx2.autotune_table() == table
    finally:
        ctx2.close()


@pytest.mark.parametrize("krylov", [0, 1])
def test_solve_with_non_default_tiles_matches_oracle(pe, tmp_path, krylov):
    # every block width of the 513..1024 bucket forced onto tiles the default never picks
    # (update chunks of 256 rows, projection chunks of 16): the march must be unchanged
    cache = tmp_path / "tiles.txt"
    cache.write_text("".join(f"10 {bw} {mx} 256 16\n" for bw in range(1, 9) for mx in (0, 1)))
    p = synth.random_ade_problem(31, 600, modes=3, deg=7, s=25, krylov_steps=14, n_out=5)
    p.krylov = krylov
    ref, _ = oracle.solve_window(p, "dense")
    ctx = pe.Context(0)
    try:
        assert ctx.autotune([], str(cache)) == 0
        assert ctx.autotune_table()[(10, 4, 0)] == (256, 16)
        outs, reps = ctx.solve_batch([p])
    finally:
        ctx.close()
    assert not reps[0]["flags"] & 1, reps[0]
    assert rel(gpu_out(outs[0]), ref) < FP64_TOL, reps[0]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_c2_full_size_on_tuned_tiles(pe, prec):
    precision = pe.PE_FP64 if prec == "fp64" else pe.PE_MIXED
    p = synth.config_c2() if prec == "fp64" else synth.config_c2(tol=1e-8)
    p.krylov = 1
    ref, _ = oracle.solve_window(p, "spectral")
    ctx = pe.Context(0)
    try:
        ctx.autotune([(p.n, p.rank_max, precision)])
        print("tuned tiles", ctx.autotune_table(), flush=True)
        outs, reps = ctx.solve_batch([p], precision=precision)
    finally:
        ctx.close()
    assert not reps[0]["flags"] & 1, reps[0]
    assert rel(gpu_out(outs[0]), ref) < (FP64_TOL if prec == "fp64" else MIXED_TOL), reps[0]


def test_cache_lines_with_invalid_chunk_heights_are_skipped(pe, tmp_path):
    cache = tmp_path / "tiles.txt"
    cache.write_text("10 4 0 100 16\n10 3 0 256 20\n10 2 0 128 32\n10 5 0 8192 32\n")
    ctx = pe.Context(0)
    try:
        assert ctx.autotune([], str(cache)) == 0
        assert ctx.autotune_table() == {(10, 2, 0): (128, 32)}
    finally:
        ctx.close()
