"""pe_workspace_query: host-only sizing of the device workspace (no GPU needed)."""
import pytest

import synth


@pytest.fixture(scope="module")
def pe():
    import paper_1509_04567_amd as pe
    try:
        pe.load_library()
    except ImportError:
        pytest.skip("library not built")
    return pe


def _lower_bound(p, beta=8):
    # the Krylov basis, (l + 1) blocks of n x b_w, and the seven N x N matrices of the
    # projected exponential, N = l b_w + q, at the largest rank and order allowed
    bw = min(p.rank_max, len(p.t_samples)) + 1
    q = min(p.q_max, len(p.t_samples))
    N = p.krylov_steps * bw + q
    return beta * (p.krylov_steps + 1) * p.n * bw + 8 * 7 * N * N


def test_query_covers_basis_and_projected_matrices(pe):
    for p in (synth.config_c1(), synth.config_c2(), synth.random_ade_problem(3, 333)):
        b = pe.workspace_query([p])
        assert b >= _lower_bound(p)
        assert b <= 3 * _lower_bound(p) + (64 << 20)


def test_query_monotone_in_sizes_and_batch(pe):
    p = synth.config_c2(n=4096)
    q = synth.config_c2(n=4096)
    q.krylov_steps = p.krylov_steps + 20
    bp, bq = pe.workspace_query([p]), pe.workspace_query([q])
    assert bq > bp
    assert pe.workspace_query([p, q]) >= bp + bq - (8 << 20)  # both marches live together
    assert pe.workspace_query([p], pe.PE_MIXED) < bp           # fp32 basis
    assert pe.workspace_query([]) == 0


def test_query_rejects_unsupported_sizes(pe):
    p = synth.random_ade_problem(4, 64)
    p.rank_max = 32
    with pytest.raises(pe.PeError) as ei:
        pe.workspace_query([p])
    assert ei.value.status == -5
    p = synth.random_ade_problem(4, 8)
    p.rank_max = 8
    with pytest.raises(pe.PeError) as ei:
        pe.workspace_query([p])
    assert ei.value.status == -1


def test_every_block_width_has_a_geometry_at_every_size(pe):
    # block widths 1..32 on grids from 4 to 2^20 points: every cycle geometry fits
    # (wide blocks on long grids fall back to the global-memory TSQR combine)
    for n in (4, 33, 160, 1024, 8192, 65536, 1 << 20):
        for rank_max in sorted({0, 1, 7, 8, 9, 15, 16, 17, 24, 31}):
            if n < rank_max + 1:
                continue
            p = synth.random_ade_problem(1, 64, s=40)
            p.n, p.rank_max, p.krylov_steps = n, rank_max, 60
            assert pe.workspace_query([p]) > 0
    # the largest workload shape: 2^20 points, rank 32 samples, 120 block steps
    p = synth.random_ade_problem(1, 64, s=64)
    p.n, p.rank_max, p.krylov_steps = 1 << 20, 31, 120
    assert pe.workspace_query([p]) > 121 * (1 << 20) * 32 * 8
