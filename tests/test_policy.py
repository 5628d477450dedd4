"""CPU tests of the march's decision rules through the library's host-only entry points
(include/paraexp_policy.h): the step-size decision of a restart trial on synthetic error
ladders, and the second-Gram-Schmidt-pass rule of block Arnoldi on a numpy model of one
classical Gram-Schmidt pass.  No GPU: these functions touch no device."""
import math

import numpy as np
import pytest

pe = pytest.importorskip("paper_1509_04567_amd")


def ladder(errs, ys=None):
    ys = ys if ys is not None else [1.0] * len(errs)
    return np.array([v for pair in zip(errs, ys) for v in pair], dtype=np.float64)


BASE = dict(alpha=1e-3, tol=1e-10, ref=1.0, tspan=1.0, dmin=1e-13, krylov_steps=30)


def decide(errs, ys=None, **kw):
    args = dict(BASE)
    args.update(kw)
    return pe.policy_step(ladder(errs, ys), **args)


def test_accepts_the_largest_passing_level():
    # limit = 1e-10; levels 0..3 pass, 4..5 fail
    d = decide([1e-16, 1e-14, 1e-13, 5e-11, 2e-10, 1e-8])
    assert d["action"] == pe.PE_STEP_ACCEPT and d["level"] == 3
    assert d["step"] == pytest.approx(1e-3 * 8)
    assert d["rho"] == pytest.approx(0.5)
    assert d["flags"] == 0


def test_every_level_passes():
    d = decide([1e-20, 1e-19, 1e-18])
    assert d["action"] == pe.PE_STEP_ACCEPT and d["level"] == 2


def test_limit_scales_with_the_state_norm():
    # |y| = 100 raises the limit to 1e-8: level 2 (5e-9) passes
    d = decide([1e-12, 1e-10, 5e-9, 1e-7], ys=[100.0] * 4)
    assert d["level"] == 2


@pytest.mark.parametrize("bad", [math.nan, math.inf])
def test_nonfinite_estimate_at_level_zero_stops_the_march(bad):
    d = decide([bad, 1e-20, 1e-20])
    assert d["action"] == pe.PE_STEP_STOP
    assert d["flags"] & pe.FLAG_NOT_CONVERGED


def test_nonfinite_state_norm_at_level_zero_stops_the_march():
    d = decide([1e-20, 1e-20], ys=[math.nan, 1.0])
    assert d["action"] == pe.PE_STEP_STOP


def test_nonfinite_upper_levels_are_rejected_not_fatal():
    d = decide([1e-16, 1e-14, math.nan, math.inf])
    assert d["action"] == pe.PE_STEP_ACCEPT and d["level"] == 1


def test_all_rejected_reduces_the_step():
    d = decide([1e-6, 1e-4, 1e-2])
    assert d["action"] == pe.PE_STEP_REJECT
    # between 0.05 and 0.5 of the level-0 step
    assert 0.05 * 1e-3 <= d["step"] <= 0.5 * 1e-3
    # a small excess shrinks by half, a huge one by 20
    assert decide([2e-10])["step"] == pytest.approx(0.5e-3)
    assert decide([1e10])["step"] == pytest.approx(0.05e-3)


def test_all_rejected_at_the_minimum_step_stops():
    d = decide([1e-6, 1e-4], alpha=1e-13, dmin=1e-13)
    assert d["action"] == pe.PE_STEP_STOP and d["flags"] & pe.FLAG_NOT_CONVERGED


def test_rejections_reach_the_minimum_step_and_stop():
    """A ladder that never passes, fed back step after step, ends in STOP after a bounded
    number of trials (each cuts the step by at least 2) -- never an endless crawl."""
    alpha, trials = 1e-2, 0
    while True:
        d = decide([1.0, 1.0], alpha=alpha, dmin=1e-13)
        trials += 1
        if d["action"] == pe.PE_STEP_STOP:
            break
        assert d["action"] == pe.PE_STEP_REJECT and d["step"] < alpha
        alpha = d["step"]
        assert trials < 60
    assert trials <= math.ceil(math.log2(1e-2 / 1e-13)) + 1


def test_happy_breakdown_flag():
    d = decide([0.0, 0.0, 0.0], ys=[1.0, 1.0, 1.0])
    assert d["action"] == pe.PE_STEP_ACCEPT and d["level"] == 2
    assert d["flags"] & pe.FLAG_BREAKDOWN


@pytest.mark.parametrize("p", [6.0, 14.0])
def test_local_order_is_measured_from_two_levels(p):
    # err ~ step^p: level k+1 is 2^p times level k
    errs = [1e-14 * 2 ** (p * k) for k in range(6)]
    d = decide(errs, tol=1e-14 * 2 ** (p * 3) * 1.01)
    assert d["level"] == 3
    assert d["pexp"] == pytest.approx(p)


def test_step_growth():
    assert pe.policy_step_growth(1.0, 10.0, 30) == pytest.approx(0.95)
    assert pe.policy_step_growth(1e-30, 10.0, 30) == 4.0
    assert pe.policy_step_growth(1e30, 10.0, 30) == 0.5
    # err ~ step^p: a ratio 2^-p allows twice the step (times the 0.95 margin)
    assert pe.policy_step_growth(2.0 ** -8, 8.0, 30) == pytest.approx(1.9)


# ---------------------------------------------------------------- second Gram-Schmidt pass
def _one_cgs_pass(V, W):
    """One classical Gram-Schmidt pass of the block W against the orthonormal V, then the
    in-block QR (numpy), as the first pass of a block Arnoldi step computes them."""
    S = V.T @ W
    Wp = W - V @ S
    Q1, R1 = np.linalg.qr(Wp)
    sgn = np.sign(np.diag(R1))
    sgn[sgn == 0] = 1.0
    return Q1 * sgn, (R1.T * sgn).T


def _old_rule(R, Rn, kappa=0.3):
    # the rule this replaces: every column of R keeps kappa of its pre-projection norm
    return all(np.linalg.norm(R[:, b]) >= kappa * Rn[b] for b in range(R.shape[0]))


def test_reorth_rule_catches_nearly_parallel_columns():
    """Two columns that keep most of their norm through the projection but are nearly
    parallel to each other: the column-norm rule would skip the second pass, and the new
    block is then far from orthogonal to the basis; the R^{-1} rule asks for it."""
    rng = np.random.default_rng(0)
    n, k = 2000, 40
    V, _ = np.linalg.qr(rng.standard_normal((n, k)))
    a = 0.8 * V @ rng.standard_normal(k) / math.sqrt(k) + 0.6 * rng.standard_normal(n) / math.sqrt(n)
    b = rng.standard_normal(n) / math.sqrt(n)
    W = np.stack([a, a + 1e-9 * b, rng.standard_normal(n) / math.sqrt(n)], axis=1)
    Rn = np.linalg.norm(W, axis=0)
    Q1, R1 = _one_cgs_pass(V, W)
    loss = np.max(np.abs(V.T @ Q1))
    assert loss > 1e-10                      # a second pass is needed
    assert _old_rule(R1, Rn)                 # ... which the column-norm rule would skip
    assert not pe.policy_reorth_skip(R1, Rn, 0.3)


def test_reorth_rule_skips_a_well_conditioned_block():
    rng = np.random.default_rng(1)
    n, k = 2000, 40
    V, _ = np.linalg.qr(rng.standard_normal((n, k)))
    W = 0.5 * V @ rng.standard_normal((k, 4)) / math.sqrt(k) + rng.standard_normal((n, 4)) / math.sqrt(n)
    Rn = np.linalg.norm(W, axis=0)
    Q1, R1 = _one_cgs_pass(V, W)
    assert np.max(np.abs(V.T @ Q1)) < 1e-14
    assert pe.policy_reorth_skip(R1, Rn, 0.3)


def test_reorth_rule_deflated_and_degenerate_inputs():
    R = np.array([[2.0, 0.3], [0.0, 0.0]])   # column 1 deflated: zero diagonal and row
    assert pe.policy_reorth_skip(R, np.array([2.0, 1.0]), 0.3)
    # a column that lost 99% of its norm to the projection
    assert not pe.policy_reorth_skip(np.array([[0.01]]), np.array([1.0]), 0.3)
    assert pe.policy_reorth_skip(np.array([[0.5]]), np.array([1.0]), 0.3)
    assert not pe.policy_reorth_skip(np.array([[math.nan]]), np.array([1.0]), 0.3)
