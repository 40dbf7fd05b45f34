"""Pins for the CPU oracle: hand-worked cases, brute force, closed forms,
special cases and invariants.  CPU only."""
from __future__ import annotations

import itertools
import json
import math
import os

import numpy as np
import pytest

import workloads
from tests import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_worked.json")


def _cases():
    with open(GOLDEN) as fh:
        return json.load(fh)["cases"]


# ---------------------------------------------------------------------------
# Hand-worked examples (every stage)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("case", _cases(), ids=lambda c: c["name"])
def test_hand_worked(oracle_mod, case):
    o = oracle_mod
    F = np.asarray(case["objs"], np.float32)
    refs = np.asarray(case["refs"], np.float32)
    K = case["K"]
    din, dout = o.dominance(F)
    assert din.tolist() == case["dom_in"]
    assert dout.tolist() == case["dom_out"]
    r, L = o.ranks(F)
    assert r.tolist() == case["rank"]
    l, nb, nl = o.last_front(r, K)
    assert (l, nb, nl) == (case["last_front"], case["n_before"], case["last_front_size"])
    nz = o.normalize(F, r, l)
    assert nz.z.tolist() == case["z"]
    assert nz.extreme.tolist() == case["extreme"]
    np.testing.assert_allclose(nz.a, case["a"], rtol=1e-15)
    assert nz.fallback == case["fallback"]
    niche, dist, gap = o.associate(F, r, l, nz.z, nz.a, refs)
    assert niche.tolist() == case["niche"]
    for i, (num, den) in enumerate(zip(case["dist_num"], case["dist_den"])):
        if num is None:
            assert dist[i] == -1.0
        else:
            assert abs(dist[i] - num / den) <= 1e-12
    rho = o.niche_count(r, niche, l, refs.shape[0])
    assert rho.tolist() == case["rho"]
    sel = o.select(F, refs, K)
    assert sel.selected.tolist() == case["selected"]
    assert sel.rank.tolist() == case["rank"]
    assert sel.dom_in.tolist() == case["dom_in"]


# ---------------------------------------------------------------------------
# Dominance counts and ranks against brute force
# ---------------------------------------------------------------------------
def _grid_inputs():
    rng = np.random.default_rng(11)
    out = []
    for M in (2, 3, 5, 10):
        for n in (1, 2, 7, 64, 300):
            out.append(rng.integers(0, 4, size=(n, M)).astype(np.float32))
    # exhaustive lattices: every point of {0,1,2}^3 and {0,1}^5, plus duplicates
    g3 = np.asarray(list(itertools.product(range(3), repeat=3)), np.float32)
    out.append(g3)
    out.append(np.concatenate([g3, g3[::3]]))
    out.append(np.asarray(list(itertools.product(range(2), repeat=5)), np.float32))
    # real-valued shells with negative values and -0.0 / +0.0 mixed
    f = workloads.make("small", N=150).objs.copy()
    f[::7, 0] = -0.0
    f[1::7, 0] = 0.0
    f[2::11] -= 0.75
    out.append(f)
    return out


@pytest.mark.parametrize("F", _grid_inputs(), ids=lambda F: f"{F.shape[0]}x{F.shape[1]}")
def test_dominance_and_ranks_bruteforce(oracle_mod, F):
    D = bf.dominance_matrix(F)
    din, dout = oracle_mod.dominance(F)
    assert din.tolist() == D.sum(axis=0).tolist()
    assert dout.tolist() == D.sum(axis=1).tolist()
    assert din.sum() == dout.sum()
    r, L = oracle_mod.ranks(F)
    assert r.tolist() == bf.deb_fronts(F).tolist()
    assert r.tolist() == bf.longest_chain_ranks(F).tolist()
    assert L == int(r.max()) + 1
    for j in range(0, F.shape[0], max(1, F.shape[0] // 17)):
        assert oracle_mod.dominance_one(F, j) == (din[j], dout[j])


def test_dominance_single_pair(oracle_mod):
    F = np.asarray([[1, 2], [1, 3], [1, 2], [0, 5]], np.float32)
    assert oracle_mod.dominates(F, 0, 1)
    assert not oracle_mod.dominates(F, 1, 0)
    assert not oracle_mod.dominates(F, 0, 2)  # identical rows
    assert not oracle_mod.dominates(F, 0, 3) and not oracle_mod.dominates(F, 3, 0)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ranks_two_objective_sweep(oracle_mod, seed):
    rng = np.random.default_rng(seed)
    F = rng.integers(0, 40, size=(2000, 2)).astype(np.float32)  # many ties and duplicates
    r, _ = oracle_mod.ranks(F)
    assert r.tolist() == bf.ranks_2d_sweep(F).tolist()


def test_ranks_two_objective_sweep_real(oracle_mod):
    F = workloads.sphere_shell(np.random.default_rng(5), 3000, 2, lambda g, n: g.uniform(0, 0.5, n), 0.2)
    F = F.astype(np.float32)
    r, _ = oracle_mod.ranks(F)
    assert r.tolist() == bf.ranks_2d_sweep(F).tolist()


# ---------------------------------------------------------------------------
# Analytic fronts
# ---------------------------------------------------------------------------
def _dyadic_simplex(p=256, step=9):
    pts = []
    for i in range(0, p + 1, step):
        for j in range(0, p + 1 - i, step):
            pts.append((i / p, j / p, (p - i - j) / p))
    return np.asarray(pts, np.float32)


def test_dyadic_simplex_all_front0(oracle_mod):
    F = _dyadic_simplex()
    assert np.all(F.astype(np.float64).sum(axis=1) == 1.0)
    r, L = oracle_mod.ranks(F)
    assert L == 1 and np.all(r == 0)
    din, dout = oracle_mod.dominance(F)
    assert din.sum() == 0 and dout.sum() == 0


def test_nested_dyadic_shells(oracle_mod):
    S = _dyadic_simplex(step=13)
    F = np.concatenate([S, 2 * S, 4 * S])
    perm = np.random.default_rng(3).permutation(F.shape[0])
    F = F[perm]
    shell = np.repeat([0, 1, 2], S.shape[0])[perm]
    r, L = oracle_mod.ranks(F)
    assert L == 3
    assert r.tolist() == shell.tolist()


def test_positive_unit_sphere_front0(oracle_mod):
    rng = np.random.default_rng(7)
    g = np.abs(rng.standard_normal((1500, 3)))
    F = (g / np.linalg.norm(g, axis=1, keepdims=True)).astype(np.float32)
    # float32 rounding could in principle create a dominating pair: confirm first
    assert not bf.dominance_matrix(F).any()
    r, L = oracle_mod.ranks(F)
    assert L == 1 and np.all(r == 0)


# ---------------------------------------------------------------------------
# Invariants on the synthetic workloads
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,N", [("small", 200), ("ties", 2500), ("large", 2000), ("many", 1500)])
def test_front_invariants(oracle_mod, name, N):
    w = workloads.make(name, N=N)
    F = w.objs
    r, L = oracle_mod.ranks(F)
    D = bf.dominance_matrix(F)
    din, dout = oracle_mod.dominance(F)
    assert din.sum() == dout.sum() == D.sum()
    assert set(np.unique(r).tolist()) == set(range(L))           # fronts partition [N]
    dom_rank = np.where(D, r[:, None], -1)                        # rank of each dominator
    assert np.all(dom_rank.max(axis=0) < r) or np.all((dom_rank.max(axis=0) < r) | (din == 0))
    for j in range(F.shape[0]):                                   # no own/later-front dominator
        doms = np.nonzero(D[:, j])[0]
        assert np.all(r[doms] < r[j])
        if r[j] > 0:                                              # a dominator one front earlier
            assert np.any(r[doms] == r[j] - 1)
        else:
            assert doms.size == 0


# ---------------------------------------------------------------------------
# Last front
# ---------------------------------------------------------------------------
def test_last_front_closed_form(oracle_mod):
    w = workloads.make("ties", N=3000)
    r, L = oracle_mod.ranks(w.objs)
    sizes = np.bincount(r)
    cum = np.cumsum(sizes)
    for K in (1, int(sizes[0]), int(sizes[0]) + 1, 1500, int(cum[2]), 2999, 3000):
        l, nb, nl = oracle_mod.last_front(r, K)
        assert l == int(np.searchsorted(cum, K))
        assert nb == (int(cum[l - 1]) if l > 0 else 0)
        assert nl == int(sizes[l])
        assert 1 <= K - nb <= nl
        assert l == int(np.sort(r)[K - 1])
    l, nb, nl = oracle_mod.last_front(r, 3000)                   # K = N
    assert l == L - 1 and K - 0 >= 0 and 3000 - nb == sizes[L - 1]
    l, nb, nl = oracle_mod.last_front(r, int(sizes[0]))           # K = |F_0|
    assert l == 0 and nb == 0 and nl == sizes[0]


# ---------------------------------------------------------------------------
# Normalisation closed forms
# ---------------------------------------------------------------------------
def test_normalize_axis_extremes(oracle_mod):
    s = np.asarray([2.0, 0.5, 8.0, 1.0], np.float32)
    M = s.size
    axis = np.diag(s)
    rng = np.random.default_rng(1)
    interior = rng.uniform(0.25, 1.0, size=(40, M)).astype(np.float32)
    F = np.concatenate([interior[:20], axis, interior[20:]])
    r = np.zeros(F.shape[0], np.int32)
    nz = oracle_mod.normalize(F, r, 0)
    assert nz.z.tolist() == [0.0] * M
    assert nz.extreme.tolist() == [20 + k for k in range(M)]
    assert nz.a.tolist() == s.astype(np.float64).tolist()      # powers of two: exact
    assert nz.fallback == 0


def test_normalize_linear_front_with_vertices(oracle_mod):
    F = np.concatenate([np.eye(3, dtype=np.float32), _dyadic_simplex(step=17)])
    r = np.zeros(F.shape[0], np.int32)
    nz = oracle_mod.normalize(F, r, 0)
    assert nz.z.tolist() == [0.0, 0.0, 0.0]
    assert nz.a.tolist() == [1.0, 1.0, 1.0]
    assert nz.fallback == 0


def test_normalize_singular_takes_nadir(oracle_mod):
    # the same point is extreme for both axes -> E has two equal rows
    F = np.asarray([[1, 1], [3, 4], [4, 2], [2, 5]], np.float32)
    r = np.zeros(4, np.int32)
    nz = oracle_mod.normalize(F, r, 0)
    assert nz.z.tolist() == [1.0, 1.0]
    assert nz.extreme.tolist() == [0, 0]
    assert nz.fallback == 1
    assert nz.a.tolist() == [3.0, 4.0]                            # max_S (f - z)


def test_normalize_zero_nadir_guard(oracle_mod):
    F = np.asarray([[1, 2], [1, 3], [1, 5]], np.float32)          # objective 0 constant
    r = np.zeros(3, np.int32)
    nz = oracle_mod.normalize(F, r, 0)
    assert nz.fallback == 2
    assert nz.a.tolist() == [1.0, 3.0]


def test_normalize_negative_intercept_takes_nadir(oracle_mod):
    # Worked by hand: z = 0; ASF_0 is least for point 0 (5); ASF_1 for point 4
    # (1e6); ASF_2 ties at 4e6 between points 1 and 4 -> lowest index 1.
    # E = [[5,0,0],[1,4,0],[4,2,3]]: b = (1/5, 1/5, -1/15) -> a negative
    # intercept, so the nadir max_S f = (5, 5, 4) is used.
    F = np.asarray([[5, 0, 0], [4, 2, 3], [0, 5, 2], [5, 4, 4], [1, 4, 0]], np.float32)
    nz = oracle_mod.normalize(F, np.zeros(5, np.int32), 0)
    assert nz.extreme.tolist() == [0, 4, 1]
    b = np.linalg.solve(F.astype(np.float64)[nz.extreme], np.ones(3))
    assert b[2] < 0
    assert nz.fallback == 1
    assert nz.a.tolist() == [5.0, 5.0, 4.0]
    # a zero intercept component (b_k = 0) is rejected the same way
    F2 = np.asarray([[4, 3, 3], [3, 5, 1], [4, 4, 0], [2, 5, 3], [0, 4, 4]], np.float32)
    nz2 = oracle_mod.normalize(F2, np.zeros(5, np.int32), 0)
    b2 = np.linalg.solve(F2.astype(np.float64)[nz2.extreme] - nz2.z, np.ones(3))
    assert abs(b2[1]) < 1e-15 and nz2.fallback == 1


def test_ideal_over_S_equals_global_min(oracle_mod):
    for name, N in (("small", 200), ("ties", 3000), ("large", 3000)):
        w = workloads.make(name, N=N)
        r, _ = oracle_mod.ranks(w.objs)
        l, _, _ = oracle_mod.last_front(r, w.K)
        nz = oracle_mod.normalize(w.objs, r, l)
        assert nz.z.tolist() == w.objs.astype(np.float64).min(axis=0).tolist()


@pytest.mark.parametrize("shift", [-3, 5])
def test_power_of_two_scaling_metamorphic(oracle_mod, shift):
    w = workloads.make("ties", N=2500)
    a = oracle_mod.select(w.objs, w.refs, w.K)
    b = oracle_mod.select(np.ldexp(w.objs, shift).astype(np.float32), w.refs, w.K)
    assert a.selected.tolist() == b.selected.tolist()
    assert a.rank.tolist() == b.rank.tolist()
    assert a.niche.tolist() == b.niche.tolist()
    assert a.dist.tolist() == b.dist.tolist()


# ---------------------------------------------------------------------------
# Association
# ---------------------------------------------------------------------------
def test_point_on_reference_line(oracle_mod):
    refs = workloads.das_dennis(3, 4).astype(np.float32)
    F = np.concatenate([np.eye(3, dtype=np.float32), refs * np.float32(0.75)])
    r = np.zeros(F.shape[0], np.int32)
    nz = oracle_mod.normalize(F, r, 0)
    # the scaled axis directions are the extreme points: a = 0.75 on every axis,
    # so f' = f / 0.75 keeps every scaled reference point on its own line
    assert nz.a.tolist() == [0.75, 0.75, 0.75] and nz.z.tolist() == [0.0, 0.0, 0.0]
    niche, dist, gap = oracle_mod.associate(F, r, 0, nz.z, nz.a, refs)
    for t in range(refs.shape[0]):
        i = 3 + t
        if np.count_nonzero(refs[t]) == 0:
            continue
        assert niche[i] == t
        assert dist[i] < 1e-12


def test_association_matches_paper_formula(oracle_mod):
    w = workloads.make("large", N=3000)
    r, _ = oracle_mod.ranks(w.objs)
    l, _, _ = oracle_mod.last_front(r, w.K)
    nz = oracle_mod.normalize(w.objs, r, l)
    niche, dist, gap = oracle_mod.associate(w.objs, r, l, nz.z, nz.a, w.refs)
    S = r <= l
    fp = (w.objs.astype(np.float64) - nz.z) / nz.a
    Dp = bf.paper_distance(fp[S], w.refs)
    # argmin agrees wherever the top two are not within the printed formula's
    # own cancellation error; values agree to that error
    sel = gap[S] > 1e-6
    assert np.all(np.argmin(Dp, axis=1)[sel] == niche[S][sel])
    assert np.max(np.abs(Dp.min(axis=1) - dist[S])) < 1e-7
    assert np.all(niche[~S] == -1) and np.all(dist[~S] == -1.0)
    # brute force in the residual form with numpy, over every reference
    rh = w.refs.astype(np.float64) / np.linalg.norm(w.refs.astype(np.float64), axis=1, keepdims=True)
    s = fp[S] @ rh.T
    res = np.linalg.norm(fp[S][:, None, :] - s[:, :, None] * rh[None, :, :], axis=2)
    assert np.all(np.argmin(res, axis=1)[sel] == niche[S][sel])
    np.testing.assert_allclose(res.min(axis=1), dist[S], rtol=0, atol=1e-14)


# ---------------------------------------------------------------------------
# Niching: sequential loop vs key-sort; special cases
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", range(8))
def test_niching_loop_equals_keysort(oracle_mod, seed):
    rng = np.random.default_rng(100 + seed)
    N = int(rng.integers(5, 400))
    H = int(rng.integers(1, 12))
    rank = rng.integers(0, 3, size=N).astype(np.int32)
    l = 1
    if not np.any(rank == l):
        rank[0] = l
    niche = rng.integers(0, H, size=N).astype(np.int32)
    niche[rank > l] = -1
    dist = np.round(rng.uniform(0, 1, size=N), 2)                 # many equal distances
    rho = oracle_mod.niche_count(rank, niche, l, H)
    nl = int(np.sum(rank == l))
    for R in sorted({1, nl, max(1, nl // 2), max(1, nl // 3)}):
        got = oracle_mod.niching(rank, niche, dist, l, H, R, rho)
        want = bf.keysort_niching(rank, niche, dist, l, rho, R)
        assert got.tolist() == want.tolist()
        assert got.sum() == R and np.all(rank[got] == l)


def test_niching_special_cases(oracle_mod):
    rng = np.random.default_rng(9)
    N, H = 60, 5
    rank = np.ones(N, np.int32)
    rank[:10] = 0
    niche = rng.integers(0, H, N).astype(np.int32)
    dist = rng.uniform(0, 1, N)
    rho = oracle_mod.niche_count(rank, niche, 1, H)
    # R = |F_l| selects all of F_l
    assert oracle_mod.niching(rank, niche, dist, 1, H, 50, rho).tolist() == (rank == 1).tolist()
    # all of F_l in one reference: its R closest
    n1 = niche.copy()
    n1[rank == 1] = 3
    got = oracle_mod.niching(rank, n1, dist, 1, H, 7, rho)
    idx = np.nonzero(rank == 1)[0]
    want = idx[np.argsort(dist[idx], kind="stable")[:7]]
    assert sorted(np.nonzero(got)[0].tolist()) == sorted(want.tolist())
    # all rho = 0 and every reference populated: first H picks = each ref's closest
    zero = np.zeros(H, np.int32)
    got = oracle_mod.niching(np.ones(N, np.int32), niche, dist, 1, H, H, zero)
    want = [min(np.nonzero(niche == j)[0], key=lambda i: (dist[i], i)) for j in range(H)]
    assert sorted(np.nonzero(got)[0].tolist()) == sorted(want)


# ---------------------------------------------------------------------------
# Whole selection
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,N", [("small", 200), ("ties", 3000), ("large", 3000), ("many", 2000)])
def test_select_invariants(oracle_mod, name, N):
    w = workloads.make(name, N=N)
    s = oracle_mod.select(w.objs, w.refs, w.K)
    sel = s.selected
    assert sel.size == w.K and np.all(np.diff(sel) > 0)
    r = s.rank
    l = s.last_front
    assert np.all(np.isin(np.nonzero(r < l)[0], sel))
    assert np.all(r[sel] <= l)
    assert s.num_from_last == w.K - int(np.sum(r < l))
    assert 1 <= s.num_from_last <= s.last_front_size == int(np.sum(r == l))
    assert s.num_fronts == int(r.max()) + 1
    assert np.all((s.niche >= 0) == (r <= l)) and np.all(s.niche < w.H)


def test_select_rejects_bad_arguments(oracle_mod):
    w = workloads.make("small")
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.select(w.objs, w.refs, 0)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.select(w.objs, w.refs, w.N + 1)
    bad = w.objs.copy()
    bad[3, 1] = np.nan
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.select(bad, w.refs, w.K)
    bad = w.objs.copy()
    bad[5, 0] = np.inf
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.select(bad, w.refs, w.K)
    with pytest.raises(oracle_mod.OracleError):
        oracle_mod.select(w.objs[:, :1], w.refs[:, :1], 10)         # M = 1


# ---------------------------------------------------------------------------
# Near-tie gap of the association (the quantity that exempts a point from the
# exact niche comparison): top two distances over every reference
# ---------------------------------------------------------------------------
def _numpy_top_two(fp, refs):
    """Residual distances of every row to every reference line (NumPy), and
    the relative gap (d2 - d1) / d2 of the two smallest."""
    rh = refs.astype(np.float64) / np.linalg.norm(refs.astype(np.float64), axis=1, keepdims=True)
    s = fp @ rh.T
    res = np.linalg.norm(fp[:, None, :] - s[:, :, None] * rh[None, :, :], axis=2)
    if res.shape[1] == 1:
        return res, np.full(res.shape[0], np.inf)
    two = np.partition(res, 1, axis=1)[:, :2]
    return res, (two[:, 1] - two[:, 0]) / np.maximum(two[:, 1], 1e-300)


@pytest.mark.parametrize("name,N", [("small", 200), ("ties", 2000), ("large", 1500), ("many", 1200)])
def test_gap_matches_top_two_over_all_references(oracle_mod, name, N):
    w = workloads.make(name, N=N)
    r, _ = oracle_mod.ranks(w.objs)
    l, _, _ = oracle_mod.last_front(r, w.K)
    nz = oracle_mod.normalize(w.objs, r, l)
    niche, dist, gap = oracle_mod.associate(w.objs, r, l, nz.z, nz.a, w.refs)
    S = r <= l
    fp = (w.objs.astype(np.float64)[S] - nz.z) / nz.a
    res, g = _numpy_top_two(fp, w.refs)
    np.testing.assert_allclose(gap[S], g, rtol=0, atol=1e-9)
    assert np.all(gap[~S] == -1.0)
    clear = g > 1e-9
    assert np.all(np.argmin(res, axis=1)[clear] == niche[S][clear])
    # the oracle's near-tie count is the number of admitted points under 1e-6
    s = oracle_mod.select(w.objs, w.refs, w.K)
    assert s.near_ties == int(np.sum(gap[S] < 1e-6))


def test_gap_single_reference_and_exact_ties(oracle_mod):
    # M = 2, references along the axes: every point on the diagonal is exactly
    # as far from both lines (d = its coordinate), so the gap is exactly 0 and
    # the lower reference index wins; the ideal point itself (f' = 0) ties too.
    # The vertices (0,1) and (1,0) make z = 0 and a = 1, so f' = f.
    F = np.asarray([[0, 1], [1, 0], [0.25, 0.25], [0.5, 0.5], [0.375, 0.125], [0.125, 0.375],
                    [0.75, 0.75]], np.float32)
    refs = np.asarray([[1, 0], [0, 1]], np.float32)
    r, _ = oracle_mod.ranks(F)
    assert r.tolist() == [0, 0, 0, 1, 0, 0, 2]
    nz = oracle_mod.normalize(F, r, 2)
    assert nz.z.tolist() == [0.0, 0.0] and nz.a.tolist() == [1.0, 1.0]
    niche, dist, gap = oracle_mod.associate(F, r, 2, nz.z, nz.a, refs)
    for i in (2, 3, 6):
        assert gap[i] == 0.0 and niche[i] == 0 and dist[i] == float(F[i, 0])
    assert niche[4] == 0 and dist[4] == 0.125 and gap[4] == pytest.approx(2.0 / 3.0, abs=1e-15)
    assert niche[5] == 1 and dist[5] == 0.125
    assert niche[0] == 1 and niche[1] == 0 and gap[0] == 1.0 and gap[1] == 1.0
    one = refs[:1]
    _, _, g1 = oracle_mod.associate(F, r, 2, nz.z, nz.a, one)
    assert np.all(np.isinf(g1))
    s = oracle_mod.select(F, refs, 6)                # l = 1: S = {r <= 1} holds points 2 and 3
    assert s.last_front == 1 and s.near_ties == 2


# ---------------------------------------------------------------------------
# One-shot niche selection (Sec. IV-A.5, Alg. S.4, Alg. S.6)
# ---------------------------------------------------------------------------
def _oneshot_golden():
    with open(os.path.join(os.path.dirname(__file__), "golden", "oneshot_niching.json")) as fh:
        return json.load(fh)


def test_oneshot_hand_worked(oracle_mod):
    c = _oneshot_golden()
    rank = np.asarray(c["rank"], np.int32)
    niche = np.asarray(c["niche"], np.int32)
    dist = np.asarray(c["dist"], np.float64)
    rho = oracle_mod.niche_count(rank, niche, c["l"], c["H"])
    assert rho.tolist() == c["rho"]
    for R, want in c["oneshot"].items():
        got, ne = oracle_mod.niching_oneshot(rank, niche, dist, c["l"], c["H"], int(R), rho)
        assert np.nonzero(got)[0].tolist() == want and ne == c["n_empty"]
    for R, want in c["exact"].items():
        got = oracle_mod.niching(rank, niche, dist, c["l"], c["H"], int(R), rho)
        assert np.nonzero(got)[0].tolist() == want


def _random_niching_case(rng):
    N = int(rng.integers(5, 300))
    H = int(rng.integers(1, 16))
    rank = rng.integers(0, 3, size=N).astype(np.int32)
    l = 1
    if not np.any(rank == l):
        rank[0] = l
    niche = rng.integers(0, H, size=N).astype(np.int32)
    niche[rank > l] = -1
    dist = np.round(rng.uniform(0, 1, size=N), 2)
    return rank, niche, dist, l, H


@pytest.mark.parametrize("seed", range(12))
def test_oneshot_against_loop_and_rules(oracle_mod, seed):
    rng = np.random.default_rng(500 + seed)
    rank, niche, dist, l, H = _random_niching_case(rng)
    rho = oracle_mod.niche_count(rank, niche, l, H)
    Fl = np.nonzero(rank == l)[0]
    # closest member (distance, index) of every reference with rho = 0 and members
    closest = []
    for j in range(H):
        m = [i for i in Fl if niche[i] == j]
        if rho[j] == 0 and m:
            closest.append(min(m, key=lambda i: (dist[i], i)))
    closest = sorted(closest)
    for R in sorted({1, len(Fl), max(1, len(closest)), max(1, len(Fl) // 2)}):
        got, ne = oracle_mod.niching_oneshot(rank, niche, dist, l, H, R, rho)
        assert ne == len(closest)
        assert got.sum() == R and np.all(rank[got] == l)
        sel = np.nonzero(got)[0].tolist()
        if R == len(closest):
            # every empty niche admits its closest member first in the loop too
            assert got.tolist() == oracle_mod.niching(rank, niche, dist, l, H, R, rho).tolist()
            assert got.tolist() == bf.keysort_niching(rank, niche, dist, l, rho, R).tolist()
        if R <= len(closest):
            assert sel == closest[:R]
        else:
            rest = [i for i in Fl if i not in closest]
            assert sel == sorted(closest + rest[:R - len(closest)])


def test_oneshot_whole_selection(oracle_mod):
    w = workloads.make("ties", N=3000)
    a = oracle_mod.select(w.objs, w.refs, w.K)
    b = oracle_mod.select(w.objs, w.refs, w.K, niching="oneshot")
    assert b.rank.tolist() == a.rank.tolist() and b.niche.tolist() == a.niche.tolist()
    l = a.last_front
    assert np.all(np.isin(np.nonzero(a.rank < l)[0], b.selected))
    assert b.selected.size == w.K and np.all(np.diff(b.selected) > 0)
    assert np.all(b.rank[b.selected] <= l)
