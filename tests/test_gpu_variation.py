"""GPU parity: simulated binary crossover and polynomial mutation
(Supplementary Sec. S.I) and the row gather (Eq. (13)) through the C ABI,
against the float64 oracle; and one whole generation (variation, merge,
selection, gather).

The library computes the operators in float32 with hardware base-2
logarithms and exponentials; the tolerance 1e-5 (u - l) + 1e-6 max(|l|, |u|)
per variable covers the float32 error of the spread factor (a few ulps of B,
times |x1 - x2| <= u - l) and of the mutation step (an absolute error of about
1e-7 of the normalised step near draw 1/2, times u - l)."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2503_20286_amd as nsga3
    nsga3.load()
    oracle.lib()


def _t(a, dtype=np.float32):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype)).cuda()


def _gpu_var(X, lo, hi, ec, em, rs, rp):
    import torch
    import paper_2503_20286_amd as nsga3
    out, st = nsga3.sbx_pm(_t(X), _t(lo), _t(hi), ec, em, _t(rs), _t(rp))
    torch.cuda.synchronize()
    return out.cpu().numpy(), int(st.item())


def _case(seed, n, d):
    rng = np.random.default_rng(seed)
    lo = rng.uniform(-4, 1, d).astype(np.float32)
    hi = (lo + rng.uniform(0.5, 6, d)).astype(np.float32)
    X = (lo + rng.random((n, d)) * (hi - lo)).astype(np.float32)
    h = n // 2
    return X, lo, hi, rng.random((h, d)).astype(np.float32), rng.random((2 * h, d)).astype(np.float32)


@pytest.mark.parametrize("n,d", [(2, 1), (3, 5), (1000, 37), (2001, 64), (512, 4096)])
@pytest.mark.parametrize("ec,em", [(15.0, 20.0), (2.0, 5.0), (30.0, 0.0)])
def test_sbx_pm_parity(n, d, ec, em):
    X, lo, hi, rs, rp = _case(n * 31 + d, n, d)
    got, st = _gpu_var(X, lo, hi, ec, em, rs, rp)
    want = oracle.sbx_pm(X, lo, hi, ec, em, rs, rp)
    assert st == 0
    tol = 1e-5 * (hi - lo).astype(np.float64) + 1e-6 * np.maximum(np.abs(lo), np.abs(hi))
    err = np.abs(got.astype(np.float64) - want)
    assert np.all(err <= tol), float((err / tol).max())
    assert np.all(got >= lo) and np.all(got <= hi)


def test_identity_draws_copy_the_parents_exactly():
    X, lo, hi, rs, rp = _case(5, 400, 12)
    got, st = _gpu_var(X, lo, hi, 10.0, 20.0, np.full_like(rs, 0.5), np.full_like(rp, 0.5))
    assert st == 0 and np.array_equal(got, X)


def test_extreme_mutation_draws_reach_the_bounds():
    X, lo, hi, rs, rp = _case(6, 300, 8)
    keep = np.full_like(rs, 0.5)
    for draw, want in ((0.0, lo), (1.0, hi)):
        got, st = _gpu_var(X, lo, hi, 10.0, 20.0, keep, np.full_like(rp, draw))
        assert st == 0
        np.testing.assert_allclose(got, np.broadcast_to(want, got.shape), rtol=0,
                                   atol=float(1e-5 * (hi - lo).max()))


def test_bad_bounds_report_status():
    import torch
    import paper_2503_20286_amd as nsga3
    X, lo, hi, rs, rp = _case(7, 100, 8)
    hi2 = hi.copy()
    hi2[3] = lo[3]
    assert _gpu_var(X, lo, hi2, 10.0, 20.0, rs, rp)[1] == -2
    with pytest.raises(nsga3.NativeError):
        nsga3.sbx_pm(_t(X), _t(lo), _t(hi), -1.0, 20.0, _t(rs), _t(rp))
    with pytest.raises(ValueError):
        nsga3.sbx_pm(_t(X), _t(lo), _t(hi), 1.0, 20.0, _t(rs[:10]), _t(rp))


@pytest.mark.parametrize("d", [1, 7, 64, 4096])
def test_gather_rows(d):
    import torch
    import paper_2503_20286_amd as nsga3
    rng = np.random.default_rng(d)
    X = rng.random((3000, d)).astype(np.float32)
    idx = rng.choice(3000, 1200, replace=False).astype(np.int32)
    out, st = nsga3.gather_rows(_t(X), _t(idx, np.int32))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert np.array_equal(out.cpu().numpy(), oracle.gather_rows(X, idx))
    bad = idx.copy()
    bad[5] = 3000
    out, st = nsga3.gather_rows(_t(X), _t(bad, np.int32))
    torch.cuda.synchronize()
    assert int(st.item()) == -1
    o = out.cpu().numpy()
    ok = np.arange(bad.size) != 5
    assert np.array_equal(o[ok], X[bad[ok]])


def _objectives(P):
    """A synthetic three-objective test function of this suite (not from the
    paper): the first two variables place a point on a curved front, the rest
    push it outward."""
    x0, x1, rest = P[:, 0].astype(np.float64), P[:, 1].astype(np.float64), P[:, 2:].astype(np.float64)
    g = 1.0 + np.sum((rest - 0.5) ** 2, axis=1)
    f = np.stack([g * x0 * x1, g * x0 * (1 - x1), g * (1 - x0 ** 2)], axis=1)
    return f.astype(np.float32)


def test_one_generation():
    """Variation of a population, evaluation, merge, selection of n from the
    2n merged points, and the gather of the next population: each step
    checked against the oracle on the GPU's own inputs."""
    import torch
    import paper_2503_20286_amd as nsga3
    n, d = 1000, 30
    rng = np.random.default_rng(42)
    lo, hi = np.zeros(d, np.float32), np.ones(d, np.float32)
    P = rng.random((n, d)).astype(np.float32)
    rs, rp = rng.random((n // 2, d)).astype(np.float32), rng.random((n, d)).astype(np.float32)
    Q, st = _gpu_var(P, lo, hi, 20.0, 20.0, rs, rp)
    assert st == 0
    ref_Q = oracle.sbx_pm(P, lo, hi, 20.0, 20.0, rs, rp)
    assert np.all(np.abs(Q - ref_Q) <= 1e-5)
    merged = np.concatenate([P, Q])
    F = _objectives(merged)
    refs = workloads.das_dennis(3, 12).astype(np.float32)
    res = nsga3.select(_t(F), _t(refs), n)
    torch.cuda.synchronize()
    sel = res.selected.cpu().numpy()
    want = oracle.select(F, refs, n, with_counts=False)
    assert np.array_equal(sel, want.selected)
    nxt, st = nsga3.gather_rows(_t(merged), res.selected)
    torch.cuda.synchronize()
    assert int(st.item()) == 0 and np.array_equal(nxt.cpu().numpy(), merged[sel])
