"""GPU parity: TensorHypE selection (Sec. IV-C; Supplementary Alg. S.10,
S.11) through the C ABI against the CPU oracle, on the same seeded draws.

Ranks are bit-exact.  Hypervolume estimates agree to 1e-10 relative (the
library forms the alpha products in chunks).  The kept set is exact unless the
oracle's estimates at the last front's cut differ by less than 1e-9 relative;
there every kept member must have an estimate at least the cut's."""
from __future__ import annotations

import json
import math
import os

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hype_lattice.json")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2503_20286_amd as nsga3
    nsga3.load()
    oracle.lib()


def _gpu_hype(F, vref, U, n, ctx=None):
    import torch
    import paper_2503_20286_amd as nsga3
    o = torch.from_numpy(np.ascontiguousarray(F, np.float32)).cuda()
    v = torch.from_numpy(np.ascontiguousarray(vref, np.float32)).cuda()
    u = torch.from_numpy(np.ascontiguousarray(U, np.float32)).cuda()
    r = nsga3.hype_select(o, v, u, n, ctx=ctx)
    torch.cuda.synchronize()
    return r.selected.cpu().numpy(), r.d.cpu().numpy(), r.rank.cpu().numpy(), r.info()


def _draws(seed, s, M):
    return np.random.default_rng(seed).random((s, M)).astype(np.float32)


def _vref(F):
    return (F.max(0).astype(np.float64) * 1.1 + 0.01).astype(np.float32)


def _compare(F, vref, U, n):
    sel, d, rank, info = _gpu_hype(F, vref, U, n)
    o = oracle.hype_select(F, vref, U, n)
    assert info.status == 0
    assert np.array_equal(rank, o.rank)
    assert (info.last_front, info.num_fronts, info.last_front_size) == \
        (o.last_front, o.num_fronts, o.last_front_size)
    S = o.rank <= o.last_front
    assert np.all(d[~S] == -np.inf)
    np.testing.assert_allclose(d[S], o.d[S], rtol=1e-10, atol=1e-300)
    if np.array_equal(sel, o.selected):
        return
    # a near-tie at the cut: the kept set must still be a valid cut
    Fl = np.nonzero(o.rank == o.last_front)[0]
    R = n - int(np.sum(o.rank < o.last_front))
    cut = np.sort(o.d[Fl])[::-1][R - 1]
    kept = np.zeros(F.shape[0], bool)
    kept[sel] = True
    assert sel.size == n and np.all(kept[o.rank < o.last_front])
    assert np.all(o.d[Fl[kept[Fl]]] >= cut * (1 - 1e-9))
    assert np.all(o.d[Fl[~kept[Fl]]] <= cut * (1 + 1e-9))


def test_hand_worked_lattice():
    with open(GOLDEN) as fh:
        g = json.load(fh)
    F = np.asarray(g["objs"], np.float32)
    G = g["grid"]
    c = (np.arange(G) + 0.5) / G
    U = np.stack(np.meshgrid(c, c, indexing="ij"), -1).reshape(-1, 2).astype(np.float32)
    for case in g["cases"]:
        sel, d, rank, info = _gpu_hype(F, g["vref"], U, case["n"])
        assert sel.tolist() == case["selected"] and rank.tolist() == g["rank"]
        want = [-math.inf if v is None else v for v in case["d"]]
        np.testing.assert_allclose(d, want, rtol=1e-12, atol=0)


@pytest.mark.parametrize("name,N,s", [("small", None, 4000), ("ties", 3000, 5000),
                                      ("large", 5000, 3000), ("many", 3000, 2000)])
def test_workload_parity(name, N, s):
    w = workloads.make(name, N=N)
    U = _draws(7 + w.N, s, w.M)
    print(f"hype {name} N={w.N} M={w.M} s={s}", flush=True)
    for n in sorted({1, w.N // 3, w.N // 2, w.N}):
        _compare(w.objs, _vref(w.objs), U, n)


def test_last_front_fits_exactly_and_ragged_sizes():
    w = workloads.make("ties", N=2000, seed=13)
    r, _ = oracle.ranks(w.objs)
    sizes = np.bincount(r)
    U = _draws(5, 1500, 3)
    for n in (int(sizes[0]), int(sizes[:2].sum()), int(sizes[0]) + 1):   # k = 0, k = 0, k > 0
        _compare(w.objs, _vref(w.objs), U, n)
    for N in (1, 2, 63, 64, 65, 513):
        v = workloads.make("large", N=N, seed=90)
        _compare(v.objs, _vref(v.objs), _draws(N, 700, 5), max(1, N // 2))


@pytest.mark.parametrize("M", [2, 4, 8, 16])
def test_objective_counts(M):
    rng = np.random.default_rng(400 + M)
    F = workloads.sphere_shell(rng, 1500, M, lambda g, n: g.uniform(0, 0.4, n), 0.2).astype(np.float32)
    _compare(F, _vref(F), _draws(M, 2500, M), 700)


def test_duplicates_and_reference_point_inside():
    """Integer data with many identical points (equal estimates: the lower
    index is kept), and a reference point below some points (they dominate no
    sample)."""
    rng = np.random.default_rng(17)
    F = rng.integers(0, 6, size=(1200, 3)).astype(np.float32)
    F = np.concatenate([F, F[:300]])
    _compare(F, np.array([4.5, 4.5, 4.5], np.float32), _draws(3, 3000, 3), 700)


def test_full_size_ties_workload():
    """N = 20,000 merged points (a population of 10,000), M = 3, 10,000 draws."""
    w = workloads.make("ties")
    print(f"hype full N={w.N}", flush=True)
    _compare(w.objs, _vref(w.objs), _draws(2024, 10_000, 3), w.N // 2)


def test_bad_inputs():
    import torch
    import paper_2503_20286_amd as nsga3
    w = workloads.make("small")
    U = _draws(1, 500, 3)
    bad = U.copy()
    bad[3, 1] = np.nan
    assert _gpu_hype(w.objs, _vref(w.objs), bad, 100)[3].status == -2
    o = torch.from_numpy(w.objs).cuda()
    v = torch.from_numpy(_vref(w.objs)).cuda()
    u = torch.from_numpy(U).cuda()
    for n in (0, w.N + 1):
        with pytest.raises(nsga3.NativeError):
            nsga3.hype_select(o, v, u, n)
    _compare(w.objs, _vref(w.objs), U, 100)     # the context still works
