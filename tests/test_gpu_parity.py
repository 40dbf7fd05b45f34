"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Ranks, fronts, dominance counts, l, |F_l|, R and the selected indices must be
bit-exact.  Reference-line indices must match except where the oracle's two
closest lines are within 1e-6 relative distance; distances must agree within
1e-5 * max(1, ||f'||) of the float64 oracle."""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_helpers import compare_full, dist_close, gpu_select

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "hand_worked.json")


def _zero(rep):
    bad = {k: v for k, v in rep.items() if k != "near_ties" and v}
    assert not bad, f"mismatches: {rep}"


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2503_20286_amd as nsga3
    nsga3.load()
    oracle.lib()


def test_hand_worked_cases():
    with open(GOLDEN) as fh:
        cases = json.load(fh)["cases"]
    for c in cases:
        F = np.asarray(c["objs"], np.float32)
        R = np.asarray(c["refs"], np.float32)
        g = gpu_select(F, R, c["K"])
        assert g["selected"].tolist() == c["selected"], c["name"]
        assert g["rank"].tolist() == c["rank"]
        assert g["dom_in"].tolist() == c["dom_in"]
        assert g["dom_out"].tolist() == c["dom_out"]
        assert g["niche"].tolist() == c["niche"]
        info = g["info"]
        assert (info.status, info.last_front, info.last_front_size) == (0, c["last_front"], c["last_front_size"])
        for i, (num, den) in enumerate(zip(c["dist_num"], c["dist_den"])):
            if num is None:
                assert g["dist"][i] == -1.0
            else:
                assert abs(g["dist"][i] - num / den) <= 1e-6


@pytest.mark.parametrize("name,N", [("small", None), ("ties", 3000), ("large", 5000), ("many", 4000),
                                    ("ties", None)])
def test_workload_full_parity(name, N):
    w = workloads.make(name, N=N)
    print(f"case {name} N={w.N} M={w.M} H={w.H} K={w.K}", flush=True)
    g = gpu_select(w.objs, w.refs, w.K)
    _zero(compare_full(w.objs, w.refs, w.K, g))


@pytest.mark.parametrize("N", [1, 2, 3, 63, 64, 65, 1023, 1024, 1025, 4097])
def test_sizes_and_ragged_tails(N):
    w = workloads.make("large", N=N, seed=77)
    for K in sorted({1, max(1, N // 2), N}):
        print(f"ragged N={N} K={K}", flush=True)
        g = gpu_select(w.objs, w.refs, K)
        _zero(compare_full(w.objs, w.refs, K, g))


def test_duplicates_and_equal_sums():
    rng = np.random.default_rng(5)
    base = rng.integers(0, 6, size=(700, 3)).astype(np.float32)
    F = np.concatenate([base, base[:300], base[::-1][:200]])       # many identical rows
    R = workloads.das_dennis(3, 5).astype(np.float32)
    for K in (1, 37, 600, F.shape[0]):
        g = gpu_select(F, R, K)
        _zero(compare_full(F, R, K, g))


def test_long_chain_many_fronts():
    # points on a line: each dominates every later one -> N fronts
    t = np.arange(600, dtype=np.float32)
    F = np.stack([t, 2 * t + 1, t + 3], axis=1)[np.random.default_rng(1).permutation(600)]
    R = workloads.das_dennis(3, 4).astype(np.float32)
    g = gpu_select(F, R, 300)
    assert g["info"].num_fronts == 600
    _zero(compare_full(F, R, 300, g))


@pytest.mark.parametrize("M", [2, 4, 7, 8, 12, 16])
def test_objective_counts(M):
    rng = np.random.default_rng(M)
    F = workloads.sphere_shell(rng, 1500, M, lambda g, n: g.uniform(0, 0.4, n), 0.2).astype(np.float32)
    p = {2: 20, 4: 5, 7: 2, 8: 2, 12: 1, 16: 1}[M]
    R = workloads.das_dennis(M, p).astype(np.float32)
    g = gpu_select(F, R, 700)
    _zero(compare_full(F, R, 700, g))


def _fallback_inputs(kind, N=900, seed=7):
    """Inputs whose intercepts take each fallback of the a5 solve: two equal
    objectives give two equal extreme rows (singular hyperplane, nadir used);
    a constant objective also gives a zero nadir entry (replaced by 1)."""
    rng = np.random.default_rng(seed)
    F = rng.uniform(0, 1, (N, 3)).astype(np.float32)
    if kind == "equal_objectives":
        F[:, 2] = F[:, 1]
    else:
        F[:, 0] = 0.25
    return F, workloads.das_dennis(3, 6).astype(np.float32)


@pytest.mark.parametrize("kind,code", [("equal_objectives", 1), ("constant_objective", 2)])
def test_intercept_fallbacks(kind, code):
    F, R = _fallback_inputs(kind)
    g = gpu_select(F, R, F.shape[0] // 2)
    assert g["info"].intercept_fallback == code
    _zero(compare_full(F, R, F.shape[0] // 2, g))


def test_negative_and_signed_zero_objectives():
    w = workloads.make("ties", N=2000, seed=9)
    F = w.objs.copy() - np.float32(0.75)
    F[::5, 1] = -0.0
    F[1::5, 1] = 0.0
    g = gpu_select(F, w.refs, 1000)
    _zero(compare_full(F, w.refs, 1000, g))


def test_exact_equidistant_points_take_stagewise_check():
    """Points (a, a, b) with a > b on the unit sphere are exactly as far from
    the first axis line as from the second (both residuals sum a*a + b*b), so
    the oracle's top-two gap is 0: the comparison must take its stage-wise
    branch (oracle niching on the GPU's own association) and still agree."""
    rng = np.random.default_rng(21)
    a = np.linspace(0.6, 0.7, 40)
    tie = np.stack([a, a, np.sqrt(1.0 - 2.0 * a * a)], axis=1)
    rest = workloads.sphere_shell(rng, 500, 3, lambda g, n: g.uniform(0, 0.5, n), 0.2)
    F = np.concatenate([np.eye(3), tie, rest]).astype(np.float32)
    R = np.eye(3, dtype=np.float32)
    K = F.shape[0] // 2
    g = gpu_select(F, R, K)
    rep = compare_full(F, R, K, g)
    assert rep["near_ties"] >= 40, rep
    _zero(rep)


def test_nonfinite_and_bad_reference_report_status():
    w = workloads.make("small")
    bad = w.objs.copy()
    bad[17, 2] = np.nan
    assert gpu_select(bad, w.refs, w.K)["info"].status == -2
    bad = w.objs.copy()
    bad[3, 0] = np.inf
    assert gpu_select(bad, w.refs, w.K)["info"].status == -2
    R = w.refs.copy()
    R[4, 1] = -0.5
    assert gpu_select(w.objs, R, w.K)["info"].status == -2
    R = w.refs.copy()
    R[0] = 0.0
    assert gpu_select(w.objs, R, w.K)["info"].status == -2
    # the context keeps working after a device-side error
    g = gpu_select(w.objs, w.refs, w.K)
    _zero(compare_full(w.objs, w.refs, w.K, g))


def test_host_checked_errors():
    import torch
    import paper_2503_20286_amd as nsga3
    w = workloads.make("small")
    o = torch.from_numpy(w.objs).cuda()
    r = torch.from_numpy(w.refs).cuda()
    for K in (0, w.N + 1):
        with pytest.raises(nsga3.NativeError) as e:
            nsga3.select(o, r, K)
        assert e.value.code == -1
    with pytest.raises(nsga3.NativeError):
        nsga3.select(o[:, :1].contiguous(), r[:, :1].contiguous(), 10)   # M = 1
    big = torch.zeros((4, 17), dtype=torch.float32, device="cuda")
    with pytest.raises(nsga3.NativeError):
        nsga3.select(big, torch.ones((3, 17), dtype=torch.float32, device="cuda"), 2)


def test_repeat_calls_bit_identical_and_smaller_after_larger():
    w = workloads.make("ties", N=6000)
    a = gpu_select(w.objs, w.refs, w.K)
    b = gpu_select(w.objs, w.refs, w.K)
    for k in ("selected", "rank", "niche", "dist", "dom_in", "dom_out"):
        assert np.array_equal(a[k], b[k]), k
    s = workloads.make("small")
    g = gpu_select(s.objs, s.refs, s.K)
    _zero(compare_full(s.objs, s.refs, s.K, g))


def test_power_of_two_scaling_gives_identical_outputs():
    w = workloads.make("large", N=4000)
    a = gpu_select(w.objs, w.refs, w.K)
    b = gpu_select(np.ldexp(w.objs, 3).astype(np.float32), w.refs, w.K)
    for k in ("selected", "rank", "niche", "dist", "dom_in", "dom_out"):
        assert np.array_equal(a[k], b[k]), k


# ---------------------------------------------------------------------------
# Full-size workloads (the shapes the benchmark times): every point compared
# with the oracle's whole selection (ranks, both dominance counts, niches,
# distances, selected indices, front statistics).
# ---------------------------------------------------------------------------
_ORACLE_FULL = {}


def _oracle_full(name):
    """(workload, oracle selection) at the workload's full size, computed once
    per test session (tens of seconds of CPU at N = 200,000)."""
    if name not in _ORACLE_FULL:
        w = workloads.make(name)
        print(f"oracle {name} N={w.N} M={w.M} H={w.H} K={w.K}", flush=True)
        _ORACLE_FULL[name] = (w, oracle.select(w.objs, w.refs, w.K, with_counts=True))
    return _ORACLE_FULL[name]


@pytest.mark.parametrize("name,assoc", [("large", "fp32"), ("many", "fp32"), ("many", "bf16")])
def test_full_size_every_point(name, assoc):
    import paper_2503_20286_amd as nsga3
    w, s = _oracle_full(name)
    mode = nsga3.ASSOC_BF16 if assoc == "bf16" else nsga3.ASSOC_FP32
    ctx = nsga3.Context(0, assoc=mode)
    ctx.reserve(w.N, w.M, w.H)           # the benchmark's launch configuration
    print(f"full-size {name} {assoc} N={w.N}", flush=True)
    g = gpu_select(w.objs, w.refs, w.K, ctx=ctx)
    rep = compare_full(w.objs, w.refs, w.K, g, s=s)
    print(f"full-size {name} {assoc}: {rep}", flush=True)
    _zero(rep)
    assert int(g["dom_in"].sum()) == int(g["dom_out"].sum())
    ctx.close()


# ---------------------------------------------------------------------------
# Matrix-core (bfloat16) screening of the association: same contract.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,N", [("small", None), ("ties", 3000), ("large", 5000), ("many", 4000)])
def test_bf16_association_parity(name, N):
    import paper_2503_20286_amd as nsga3
    w = workloads.make(name, N=N)
    print(f"bf16 case {name} N={w.N} M={w.M} H={w.H}", flush=True)
    g = gpu_select(w.objs, w.refs, w.K, assoc=nsga3.ASSOC_BF16)
    _zero(compare_full(w.objs, w.refs, w.K, g))


@pytest.mark.parametrize("M", [2, 7, 8, 9, 16])
def test_bf16_objective_counts(M):
    import paper_2503_20286_amd as nsga3
    rng = np.random.default_rng(100 + M)
    F = workloads.sphere_shell(rng, 1200, M, lambda g, n: g.uniform(0, 0.4, n), 0.2).astype(np.float32)
    p = {2: 40, 7: 2, 8: 2, 9: 2, 16: 1}[M]
    R = workloads.das_dennis(M, p).astype(np.float32)
    g = gpu_select(F, R, 600, assoc=nsga3.ASSOC_BF16)
    _zero(compare_full(F, R, 600, g))


# ---------------------------------------------------------------------------
# One-shot niche selection (Sec. IV-A.5, Alg. S.4, Alg. S.6) against the
# oracle's one-shot form.
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("name,N,assoc", [("small", None, "fp32"), ("ties", 3000, "fp32"),
                                          ("large", 5000, "fp32"), ("many", 4000, "bf16"),
                                          ("ties", None, "fp32")])
def test_oneshot_niching_parity(name, N, assoc):
    import paper_2503_20286_amd as nsga3
    w = workloads.make(name, N=N)
    mode = nsga3.ASSOC_BF16 if assoc == "bf16" else nsga3.ASSOC_FP32
    print(f"oneshot {name} N={w.N} {assoc}", flush=True)
    for K in sorted({1, w.K, w.N}):
        g = gpu_select(w.objs, w.refs, K, assoc=mode, niching=nsga3.NICHING_ONESHOT)
        _zero(compare_full(w.objs, w.refs, K, g, niching="oneshot"))


def test_oneshot_surplus_shortfall_and_exact_fill():
    """K chosen so that the last front's shortfall R is below, equal to and
    above the number of empty-niche picks |E| (last front 0 and 1; 496
    references, so that many niches are empty)."""
    import paper_2503_20286_amd as nsga3
    w = workloads.make("ties", N=4000, seed=12)
    refs = workloads.das_dennis(3, 30).astype(np.float32)
    r, _ = oracle.ranks(w.objs)
    sizes = np.bincount(r)
    for l in (0, 1):
        nb = int(sizes[:l].sum())
        s = oracle.select(w.objs, refs, nb + 1, with_counts=False)
        assert s.last_front == l
        rho = oracle.niche_count(s.rank, s.niche, l, refs.shape[0])
        _, ne = oracle.niching_oneshot(s.rank, s.niche, s.dist, l, refs.shape[0], 1, rho)
        assert ne >= 3
        for R in (1, ne - 1, ne, ne + 1, int(sizes[l])):
            K = nb + R
            print(f"oneshot l={l} |E|={ne} R={R}", flush=True)
            g = gpu_select(w.objs, refs, K, niching=nsga3.NICHING_ONESHOT)
            assert g["info"].last_front == l and g["info"].num_from_last == R
            _zero(compare_full(w.objs, refs, K, g, niching="oneshot"))


def test_oneshot_full_size_every_point():
    import paper_2503_20286_amd as nsga3
    w, s = _oracle_full("large")
    l = s.last_front
    rho = oracle.niche_count(s.rank, s.niche, l, w.H)
    chosen, _ = oracle.niching_oneshot(s.rank, s.niche, s.dist, l, w.H, s.num_from_last, rho)
    want = np.nonzero((s.rank < l) | chosen)[0]
    g = gpu_select(w.objs, w.refs, w.K, niching=nsga3.NICHING_ONESHOT)
    assert np.array_equal(g["rank"], s.rank)
    assert np.array_equal(g["niche"], s.niche)
    assert np.array_equal(g["selected"], want)


def test_oneshot_plan_matches_single_calls():
    """Batched plans of a one-shot context run as graphs of single calls."""
    import torch
    import paper_2503_20286_amd as nsga3
    ws = workloads.make_batch(10, n_lo=50, n_hi=4000, base_seed=8800)
    probs = [(torch.from_numpy(w.objs).cuda(), torch.from_numpy(w.refs).cuda(), w.K) for w in ws]
    ctx = nsga3.Context(0, niching=nsga3.NICHING_ONESHOT)
    plan = nsga3.Plan(probs, ctx=ctx)
    for _ in range(2):
        plan.launch()
        torch.cuda.synchronize()
        for b, (o, r, K) in enumerate(probs):
            single = nsga3.select(o, r, K, ctx=ctx)
            torch.cuda.synchronize()
            assert torch.equal(plan.results[b].selected, single.selected), b
    for b in (0, 4, 9):
        w = ws[b]
        res = plan.results[b]
        g = {k: getattr(res, k).cpu().numpy() for k in ("selected", "rank", "niche", "dist",
                                                        "dom_in", "dom_out")}
        g["info"] = res.info()
        _zero(compare_full(w.objs, w.refs, w.K, g, niching="oneshot"))
    plan.close()
    ctx.close()


@pytest.mark.parametrize("name,N", [("ties", 3000), ("large", 5000), ("many", 3000)])
def test_pairwise_compare_path_parity(name, N, monkeypatch):
    """The pairwise-compare dominance kernels (kept beside the block-bitset
    ones) must give the same results."""
    import paper_2503_20286_amd as nsga3
    monkeypatch.setenv("NSGA3_PAIRWISE", "1")
    ctx = nsga3.Context(0)
    monkeypatch.delenv("NSGA3_PAIRWISE")
    w = workloads.make(name, N=N)
    g = gpu_select(w.objs, w.refs, w.K, ctx=ctx)
    _zero(compare_full(w.objs, w.refs, w.K, g))
    ctx.close()


@pytest.mark.parametrize("separate", ["0", "1"])
def test_out_degree_forms_parity(separate, monkeypatch):
    """Out-degrees counted inside the in-degree probes (NSGA3_SEPARATE_OUT=0)
    and by their own backward pass (=1) give the oracle's counts for every
    objective count (the default picks one form by M)."""
    import paper_2503_20286_amd as nsga3
    monkeypatch.setenv("NSGA3_SEPARATE_OUT", separate)
    ctx = nsga3.Context(0)
    monkeypatch.delenv("NSGA3_SEPARATE_OUT")
    rng = np.random.default_rng(40)
    cases = [workloads.make("ties", N=3000), workloads.make("large", N=5000),
             workloads.make("many", N=3000)]
    for w in cases:
        g = gpu_select(w.objs, w.refs, w.K, ctx=ctx)
        _zero(compare_full(w.objs, w.refs, w.K, g))
    F = rng.integers(0, 50, size=(2500, 2)).astype(np.float32)   # dense two-objective dominance
    R = workloads.das_dennis(2, 30).astype(np.float32)
    g = gpu_select(F, R, 1200, ctx=ctx)
    _zero(compare_full(F, R, 1200, g))
    ctx.close()


@pytest.mark.parametrize("wide", ["0", "1"])
def test_wide_table_counts_parity(wide, monkeypatch):
    """All-pairs counts with 128-member tables (NSGA3_WIDE_TABLES=1, the
    default for 4 <= M <= 10) and with 64-member tables (=0), and peeling
    levels with 128-member front tables (NSGA3_WIDE_LEVELS=1, opt-in) or
    64-member ones, give the oracle's counts and ranks: every M of the wide
    range, ragged sizes around the 128-member blocks (1, 127, 128, 129, 2,049),
    ties and duplicates, with and without the count outputs."""
    import paper_2503_20286_amd as nsga3
    monkeypatch.setenv("NSGA3_WIDE_TABLES", wide)
    monkeypatch.setenv("NSGA3_WIDE_LEVELS", wide)
    ctx = nsga3.Context(0)
    monkeypatch.delenv("NSGA3_WIDE_TABLES")
    monkeypatch.delenv("NSGA3_WIDE_LEVELS")
    rng = np.random.default_rng(41)
    for M in (4, 5, 6, 7, 8, 9, 10, 11):
        for N in (1, 127, 128, 129, 2049):
            F = rng.integers(0, 6, size=(N, M)).astype(np.float32)  # ties and duplicates
            R = np.abs(rng.standard_normal((20, M))).astype(np.float32) + 0.05
            K = max(1, N // 2)
            print(f"wide={wide} M={M} N={N}", flush=True)
            g = gpu_select(F, R, K, ctx=ctx)
            _zero(compare_full(F, R, K, g))
    w = workloads.make("large", N=6000, seed=44)
    g = gpu_select(w.objs, w.refs, w.K, ctx=ctx, want_counts=False)
    s = oracle.select(w.objs, w.refs, w.K, with_counts=False)
    assert np.array_equal(g["rank"], s.rank)
    ctx.close()


@pytest.mark.parametrize("tail_block,levels", [(True, 2), (False, 1), (True, 5)])
def test_peeling_tails(tail_block, levels, monkeypatch):
    """Levels beyond the enqueued ones are finished by the cooperative tail or
    by the single-workgroup tail; both must give the oracle's ranks."""
    import paper_2503_20286_amd as nsga3
    monkeypatch.setenv("NSGA3_TAIL_BLOCK", "1" if tail_block else "0")
    monkeypatch.setenv("NSGA3_HOST_LEVELS", str(levels))
    ctx = nsga3.Context(0)
    monkeypatch.delenv("NSGA3_TAIL_BLOCK")
    monkeypatch.delenv("NSGA3_HOST_LEVELS")
    for name, N in (("ties", 4000), ("large", 3000)):
        w = workloads.make(name, N=N)
        g = gpu_select(w.objs, w.refs, w.K, ctx=ctx)
        _zero(compare_full(w.objs, w.refs, w.K, g))
    t = np.arange(300, dtype=np.float32)
    F = np.stack([t, 2 * t + 1, t + 3], axis=1)[np.random.default_rng(2).permutation(300)]
    R = workloads.das_dennis(3, 4).astype(np.float32)
    g = gpu_select(F, R, 150, ctx=ctx)
    assert g["info"].num_fronts == 300
    _zero(compare_full(F, R, 150, g))
    ctx.close()
