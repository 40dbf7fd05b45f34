"""Pins for the variation oracle (Supplementary Sec. S.I: SBX, Eq. (S.6)-(S.7);
polynomial mutation, Eq. (S.8)-(S.11)) and the row gather (Eq. (13)):
closed forms at special draws, the SBX spread distribution, invariants.
CPU only."""
from __future__ import annotations

import numpy as np
import pytest


def _pop(rng, n, d, lo=-2.0, hi=3.0):
    return rng.uniform(lo, hi, (n, d)).astype(np.float32)


def test_sbx_half_draw_copies_parents_and_pm_half_draw_is_identity(oracle_mod):
    rng = np.random.default_rng(1)
    X = _pop(rng, 40, 7)
    lo, hi = np.full(7, -2.0, np.float32), np.full(7, 3.0, np.float32)
    out = oracle_mod.sbx_pm(X, lo, hi, 15.0, 20.0, np.full((20, 7), 0.5, np.float32),
                            np.full((40, 7), 0.5, np.float32))
    np.testing.assert_array_equal(out, X.astype(np.float64))


@pytest.mark.parametrize("eta_c", [0.0, 2.0, 15.0, 30.0])
def test_sbx_spread_follows_its_distribution(oracle_mod, eta_c):
    """Children keep the parents' mean, and their spread |c1 - c2| / |x1 - x2|
    is the SBX spread factor b whose distribution is P(b <= t) = t^(eta+1)/2
    for t <= 1 and 1 - 1/(2 t^(eta+1)) above: the draw m is recovered from it."""
    rng = np.random.default_rng(2)
    n, d = 400, 5
    X = _pop(rng, n, d, 0.4, 0.6)
    m = rng.uniform(0.01, 0.99, (n // 2, d)).astype(np.float32)
    lo, hi = np.full(d, -1e6, np.float32), np.full(d, 1e6, np.float32)
    out = oracle_mod.sbx_pm(X, lo, hi, eta_c, 20.0, m, np.full((n, d), 0.5, np.float32))
    x1, x2 = X[: n // 2].astype(np.float64), X[n // 2:].astype(np.float64)
    c1, c2 = out[: n // 2], out[n // 2:]
    np.testing.assert_allclose(c1 + c2, x1 + x2, rtol=0, atol=1e-12)
    ok = np.abs(x1 - x2) > 1e-3
    b = np.abs(c1 - c2)[ok] / np.abs(x1 - x2)[ok]
    e = eta_c + 1.0
    cdf = np.where(b <= 1.0, b ** e / 2.0, 1.0 - 1.0 / (2.0 * b ** e))
    np.testing.assert_allclose(cdf, m.astype(np.float64)[ok], rtol=0, atol=1e-8)


def test_pm_extreme_draws_reach_the_bounds(oracle_mod):
    """Draw 0 moves a variable to its lower bound and draw 1 to its upper
    bound, for any position inside the bounds."""
    rng = np.random.default_rng(3)
    d = 6
    lo = rng.uniform(-3, 0, d).astype(np.float32)
    hi = (lo + rng.uniform(0.5, 4, d)).astype(np.float32)
    X = (lo + rng.uniform(0, 1, (30, d)) * (hi - lo)).astype(np.float32)
    keep = np.full((15, d), 0.5, np.float32)
    for draw, want in ((0.0, lo), (1.0, hi)):
        out = oracle_mod.sbx_pm(X, lo, hi, 10.0, 20.0, keep, np.full((30, d), draw, np.float32))
        np.testing.assert_allclose(out, np.broadcast_to(want.astype(np.float64), out.shape), rtol=0,
                                   atol=1e-12)


@pytest.mark.parametrize("eta_m", [0.0, 5.0, 20.0])
def test_pm_stays_in_bounds_and_is_monotone_in_the_draw(oracle_mod, eta_m):
    rng = np.random.default_rng(4)
    d = 4
    lo, hi = np.zeros(d, np.float32), np.ones(d, np.float32)
    X = np.repeat(rng.uniform(0, 1, (1, d)), 64, axis=0).astype(np.float32)
    draws = np.repeat(np.linspace(0, 1, 64, dtype=np.float32)[:, None], d, axis=1)
    out = oracle_mod.sbx_pm(X, lo, hi, 10.0, eta_m, np.full((32, d), 0.5, np.float32), draws)
    assert np.all(out >= -1e-12) and np.all(out <= 1 + 1e-12)
    assert np.all(np.diff(out, axis=0) >= -1e-12)
    np.testing.assert_allclose(out[draws == np.float32(0.5)], X[draws == np.float32(0.5)], atol=1e-15)


def test_children_outside_the_bounds_are_clipped(oracle_mod):
    X = np.array([[0.9, 0.1], [0.1, 0.9]], np.float32)
    lo, hi = np.zeros(2, np.float32), np.ones(2, np.float32)
    m = np.array([[0.999, 0.999]], np.float32)            # spread factor about 1.3
    out = oracle_mod.sbx_pm(X, lo, hi, 0.0, 20.0, m, np.full((2, 2), 0.5, np.float32))
    B = 1.0 / (2.0 - 2.0 * np.float64(np.float32(0.999)))
    c1 = ((1 + B) * 0.9 + (1 - B) * 0.1) / 2.0            # above 1 -> clipped
    assert c1 > 1.0 and out[0, 0] == 1.0 and out[1, 0] == 0.0


def test_rejects_bad_inputs(oracle_mod):
    X = np.zeros((4, 2), np.float32)
    ok = np.full((2, 2), 0.3, np.float32), np.full((4, 2), 0.3, np.float32)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.sbx_pm(X, np.ones(2), np.ones(2), 1.0, 1.0, *ok)          # l == u
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.sbx_pm(X, np.zeros(2), np.ones(2), -1.0, 1.0, *ok)
    bad = ok[1].copy()
    bad[1, 0] = np.nan
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.sbx_pm(X, np.zeros(2), np.ones(2), 1.0, 1.0, ok[0], bad)


def test_gather_rows(oracle_mod):
    rng = np.random.default_rng(5)
    X = rng.random((50, 9)).astype(np.float32)
    idx = rng.choice(50, 20, replace=False).astype(np.int32)
    np.testing.assert_array_equal(oracle_mod.gather_rows(X, idx), X[idx])
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.gather_rows(X, np.array([0, 50], np.int32))
