"""Pins for the TensorHypE selection oracle (Sec. IV-C; Supplementary
Alg. S.10, S.11): a hand-worked lattice case, the alpha weights in closed
form, exact areas when the sample draws form a lattice, a Monte Carlo check,
and selection invariants.  CPU only."""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

import workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hype_lattice.json")


def _lattice(G, M=2):
    g = (np.arange(G) + 0.5) / G
    return np.stack(np.meshgrid(*([g] * M), indexing="ij"), -1).reshape(-1, M).astype(np.float32)


def test_hand_worked(oracle_mod):
    with open(GOLDEN) as fh:
        c0 = json.load(fh)
    F = np.asarray(c0["objs"], np.float32)
    U = _lattice(c0["grid"])
    _, cnt = oracle_mod.hype_hv(F, c0["vref"], U, 1)
    assert cnt.reshape(4, 4).tolist() == c0["counts_by_column"]
    for c in c0["cases"]:
        s = oracle_mod.hype_select(F, c0["vref"], U, c["n"])
        assert s.k == c["k"] and s.selected.tolist() == c["selected"] and s.rank.tolist() == c0["rank"]
        want = [-math.inf if v is None else v for v in c["d"]]
        np.testing.assert_allclose(s.d, want, rtol=1e-15, atol=0)


@pytest.mark.parametrize("k,N", [(1, 7), (4, 10), (9, 10), (10, 10), (57, 400), (300, 400)])
def test_alpha_closed_form(oracle_mod, k, N):
    """alpha_c = C(k-1, c-1) / (c C(N-1, c-1)); with k = N every alpha_c is 1/c."""
    a = oracle_mod.hype_alpha(k, N)
    want = [math.comb(k - 1, c - 1) / (c * math.comb(N - 1, c - 1)) for c in range(1, k + 1)]
    np.testing.assert_allclose(a, want, rtol=1e-12, atol=1e-300)
    if k == N:
        np.testing.assert_allclose(a, 1.0 / np.arange(1, k + 1), rtol=1e-15)


def _union_area(pts):
    """Area of the union of the boxes [x, 1] x [y, 1] (a staircase sweep)."""
    pts = sorted((float(x), float(y)) for x, y in pts)
    area, ymin = 0.0, 1.0
    for q, (x, y) in enumerate(pts):
        xnext = pts[q + 1][0] if q + 1 < len(pts) else 1.0
        ymin = min(ymin, y)
        area += (xnext - x) * (1.0 - ymin)
    return area


def _dyadic_points(rng, n, G):
    """Points on the 1/G grid in [0, 1)^2, with f_l = (0, 0) held by two of them."""
    P = rng.integers(0, G, size=(n, 2)) / G
    P[0, 0] = 0.0
    P[1, 1] = 0.0
    return P.astype(np.float32)


@pytest.mark.parametrize("seed", range(4))
def test_lattice_draws_give_exact_areas(oracle_mod, seed):
    """Draws at the centres of a G x G lattice integrate boxes with corners on
    the 1/G grid exactly: with k = N the estimates add up to the dominated
    area (each sample split evenly among its dominators), and with k = 1 each
    estimate is the area the point alone dominates."""
    G = 64
    rng = np.random.default_rng(seed)
    F = _dyadic_points(rng, 40, G)
    U = _lattice(G)
    N = F.shape[0]
    hv, _ = oracle_mod.hype_hv(F, [1.0, 1.0], U, N)
    assert hv.sum() == pytest.approx(_union_area(F), rel=1e-12)
    hv1, _ = oracle_mod.hype_hv(F, [1.0, 1.0], U, 1)
    total = _union_area(F)
    for p in range(N):
        excl = total - _union_area(np.delete(F, p, axis=0))
        assert hv1[p] == pytest.approx(excl, abs=1e-12), p


def test_random_draws_converge(oracle_mod):
    """Uniform random draws: the k = 1 estimates approach the exclusive areas
    (within five standard errors of a binomial proportion)."""
    rng = np.random.default_rng(11)
    F = _dyadic_points(rng, 12, 16)
    s = 400_000
    U = rng.random((s, 2), dtype=np.float64).astype(np.float32)
    hv1, _ = oracle_mod.hype_hv(F, [1.0, 1.0], U, 1)
    total = _union_area(F)
    for p in range(F.shape[0]):
        excl = total - _union_area(np.delete(F, p, axis=0))
        se = math.sqrt(max(excl * (1 - excl), 1e-12) / s)
        assert abs(hv1[p] - excl) <= 5 * se + 1e-12, (p, hv1[p], excl)


@pytest.mark.parametrize("shift", [-2, 3])
def test_power_of_two_scaling(oracle_mod, shift):
    w = workloads.make("ties", N=1500)
    vref = (w.objs.max(0) * 1.125).astype(np.float32)
    U = np.random.default_rng(3).random((2000, 3)).astype(np.float32)
    a = oracle_mod.hype_select(w.objs, vref, U, 700)
    b = oracle_mod.hype_select(np.ldexp(w.objs, shift).astype(np.float32),
                               np.ldexp(vref, shift).astype(np.float32), U, 700)
    assert np.array_equal(a.selected, b.selected)
    S = a.rank <= a.last_front
    assert np.array_equal(np.ldexp(a.d[S], 3 * shift), b.d[S])


@pytest.mark.parametrize("name,N,n", [("small", 200, 100), ("ties", 2000, 1000), ("large", 1500, 700),
                                      ("many", 800, 400)])
def test_selection_invariants(oracle_mod, name, N, n):
    w = workloads.make(name, N=N)
    M = w.objs.shape[1]
    vref = (w.objs.max(0) * 1.1).astype(np.float32)
    U = np.random.default_rng(N).random((3000, M)).astype(np.float32)
    s = oracle_mod.hype_select(w.objs, vref, U, n)
    r, L = oracle_mod.ranks(w.objs)
    l, nb, nl = oracle_mod.last_front(r, n)
    assert np.array_equal(s.rank, r) and s.last_front == l and s.k == nb + nl - n
    sel = np.zeros(w.N, bool)
    sel[s.selected] = True
    assert s.selected.size == n and np.all(np.diff(s.selected) > 0)
    assert np.all(sel[r < l]) and not np.any(sel[r > l])
    Fl = np.nonzero(r == l)[0]
    chosen, rest = Fl[sel[Fl]], Fl[~sel[Fl]]
    if rest.size and chosen.size:
        assert s.d[chosen].min() >= s.d[rest].max()
    assert np.all(s.d[r > l] == -np.inf) and np.all(s.d[r <= l] >= 0)
