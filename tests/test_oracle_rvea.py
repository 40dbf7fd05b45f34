"""Pins for the TensorRVEA selection oracle (Supplementary Sec. S.V,
Alg. S.12): a hand-worked case, closed forms, special cases and invariants.
CPU only."""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rvea_apd.json")


def _golden():
    with open(GOLDEN) as fh:
        return json.load(fh)


def test_hand_worked(oracle_mod):
    g = _golden()
    F = np.asarray(g["objs"], np.float32)
    V = np.asarray(g["refs"], np.float32)
    np.testing.assert_allclose(oracle_mod.rvea_gamma(V), g["gamma"], rtol=0, atol=1e-12)
    for c in g["cases"]:
        r = oracle_mod.rvea_select(F, V, c["t"], c["t_max"], c["alpha"])
        assert r.elite.tolist() == c["elite"], c
        assert r.assign.tolist() == g["assign"]
        np.testing.assert_allclose(r.theta, g["theta"], rtol=0, atol=1e-6)
    r = oracle_mod.rvea_select(F, V, 10, 10, 2.0)
    np.testing.assert_allclose(r.apd, g["apd_at_t_max"], rtol=1e-6)


def test_gamma_closed_forms(oracle_mod):
    # directions at multiples of pi/8: neighbours pi/8 apart
    a = np.arange(5) * math.pi / 8
    V = np.stack([np.cos(a), np.sin(a)], 1).astype(np.float32)
    np.testing.assert_allclose(oracle_mod.rvea_gamma(V), math.pi / 8, rtol=0, atol=1e-6)
    # simplex lattice p = 2 in three objectives: every vertex has a mid-edge
    # point at 45 degrees and every mid-edge point a vertex at 45 degrees
    D = workloads.das_dennis(3, 2).astype(np.float32)
    np.testing.assert_allclose(oracle_mod.rvea_gamma(D), math.pi / 4, rtol=0, atol=1e-12)


def test_rejects_duplicate_and_bad_references(oracle_mod):
    F = np.random.default_rng(0).uniform(0, 1, (20, 3)).astype(np.float32)
    V = workloads.das_dennis(3, 2).astype(np.float32)
    dup = np.concatenate([V, V[:1] * 2.0])            # same direction twice
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.rvea_select(F, dup, 1, 10)
    neg = V.copy()
    neg[2, 0] = -0.1
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.rvea_select(F, neg, 1, 10)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.rvea_select(F, V[:1], 1, 10)        # gamma needs two references
    bad = F.copy()
    bad[3, 1] = np.nan
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.rvea_select(bad, V, 1, 10)


def _brute_angles(F, V):
    """Angles by the textbook formula with numpy's arccos (float64)."""
    Fp = F.astype(np.float64) - F.astype(np.float64).min(0)
    Vn = V.astype(np.float64) / np.linalg.norm(V.astype(np.float64), axis=1, keepdims=True)
    nrm = np.linalg.norm(Fp, axis=1)
    cos = (Fp @ Vn.T) / np.where(nrm > 0, nrm, 1.0)[:, None]
    return np.arccos(np.clip(cos, -1.0, 1.0)), nrm


@pytest.mark.parametrize("name,N", [("small", 200), ("ties", 1500), ("large", 1500), ("many", 800)])
def test_penalty_zero_keeps_smallest_norm(oracle_mod, name, N):
    """t = 0: APD = ||F'|| exactly, so each elite is its partition's point
    closest to the ideal point; partitions are the smallest angles."""
    w = workloads.make(name, N=N)
    r = oracle_mod.rvea_select(w.objs, w.refs, 0, 10, 2.0)
    ang, nrm = _brute_angles(w.objs, w.refs)
    np.testing.assert_allclose(r.apd, nrm, rtol=1e-14, atol=0)
    srt = np.sort(ang, axis=1)
    clear = (srt[:, 1] - srt[:, 0]) > 1e-9            # no near-equal smallest angles
    assert np.array_equal(r.assign[clear], np.argmin(ang, axis=1)[clear])
    np.testing.assert_allclose(r.theta, ang[np.arange(w.N), r.assign], rtol=0, atol=1e-7)
    for j in range(w.H):
        members = np.nonzero(r.assign == j)[0]
        if members.size == 0:
            assert r.elite[j] == -1
        else:
            assert r.elite[j] == members[np.argmin(r.apd[members])]


def test_points_on_reference_directions(oracle_mod):
    """Points placed on the reference directions (with the ideal point at the
    origin) have angle 0, so APD = norm at any penalty, and each partition's
    elite is its shortest point."""
    V = workloads.das_dennis(3, 4).astype(np.float64)
    rng = np.random.default_rng(3)
    scale = rng.choice([0.5, 1.0, 2.0, 4.0], size=(V.shape[0], 3))
    F = np.concatenate([V * scale[:, q:q + 1] for q in range(3)] + [np.eye(3) * 8.0, np.zeros((1, 3))])
    F = F.astype(np.float32)                            # dyadic multiples: exact
    r = oracle_mod.rvea_select(F, V.astype(np.float32), 7, 10, 2.0)
    nH = V.shape[0]
    for q in range(3):
        on = np.arange(q * nH, (q + 1) * nH)
        assert np.array_equal(r.assign[on], np.arange(nH))
        np.testing.assert_allclose(r.theta[on], 0.0, atol=1e-7)
    # the origin point (the ideal point itself): partition 0, APD 0, the elite of 0
    assert r.assign[-1] == 0 and r.apd[-1] == 0.0 and r.elite[0] == F.shape[0] - 1
    for j in range(1, nH):
        members = np.nonzero(r.assign == j)[0]
        assert r.elite[j] == members[np.argmin(np.linalg.norm(F[members].astype(np.float64), axis=1))]


@pytest.mark.parametrize("shift", [-3, 2])
def test_power_of_two_scaling(oracle_mod, shift):
    w = workloads.make("ties", N=2000)
    a = oracle_mod.rvea_select(w.objs, w.refs, 3, 10, 2.0)
    b = oracle_mod.rvea_select(np.ldexp(w.objs, shift).astype(np.float32), w.refs, 3, 10, 2.0)
    assert np.array_equal(a.elite, b.elite) and np.array_equal(a.assign, b.assign)
    assert np.array_equal(a.theta, b.theta)
    assert np.array_equal(np.ldexp(a.apd, shift), b.apd)


def test_translation_invariance(oracle_mod):
    w = workloads.make("ties", N=2000)          # multiples of 1/256: the shift is exact
    c = np.array([0.5, -1.25, 3.0], np.float32)
    a = oracle_mod.rvea_select(w.objs, w.refs, 4, 10, 2.0)
    b = oracle_mod.rvea_select(w.objs + c, w.refs, 4, 10, 2.0)
    for k in ("elite", "assign", "apd", "theta"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k


@pytest.mark.parametrize("name,N", [("small", 200), ("large", 2000), ("many", 1000)])
def test_invariants_and_penalty_monotone(oracle_mod, name, N):
    w = workloads.make(name, N=N)
    prev = None
    for t in (0, 2, 5, 10):
        r = oracle_mod.rvea_select(w.objs, w.refs, t, 10, 2.0)
        for j in range(w.H):
            members = np.nonzero(r.assign == j)[0]
            if members.size == 0:
                assert r.elite[j] == -1 and r.gap[j] == -1.0
                continue
            e = r.elite[j]
            assert r.assign[e] == j and r.apd[e] == r.apd[members].min()
            assert e == members[r.apd[members] == r.apd[e]].min()       # lowest index on ties
            if members.size > 1:
                s = np.sort(r.apd[members])
                assert r.gap[j] == pytest.approx((s[1] - s[0]) / s[1], abs=1e-15)
        if prev is not None:
            assert np.all(r.apd >= prev.apd) and np.array_equal(r.assign, prev.assign)
        prev = r
