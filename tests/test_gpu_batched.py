"""GPU: batched plans (many selections in one graph launch).  Every output of
every instance must equal a single nsga3_select call on the same instance, on
every replay, with new data in the same buffers; sampled instances are also
checked against the oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_helpers import compare_full

pytestmark = pytest.mark.gpu

FIELDS = ("selected", "rank", "niche", "dist", "dom_in", "dom_out")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2503_20286_amd as nsga3
    nsga3.load()
    oracle.lib()


@pytest.fixture(params=["engine", "engine_phased", "graph"])
def plan_mode(request, monkeypatch):
    """engine: per-class branches that overlap; engine_phased: every class's
    counts between the two engine phases; graph: a graph of single calls."""
    monkeypatch.delenv("NSGA3_PLAN_MODE", raising=False)
    monkeypatch.delenv("NSGA3_PLAN_OVERLAP", raising=False)
    if request.param == "graph":
        monkeypatch.setenv("NSGA3_PLAN_MODE", "graph")
    elif request.param == "engine_phased":
        monkeypatch.setenv("NSGA3_PLAN_OVERLAP", "0")
    return request.param


def _host(sel):
    return {k: None if getattr(sel, k) is None else getattr(sel, k).cpu().numpy() for k in FIELDS}


def _dev(ws):
    import torch
    return [(torch.from_numpy(w.objs).cuda(), torch.from_numpy(w.refs).cuda(), w.K) for w in ws]


def _check_against_single(plan, probs, tag):
    import torch
    import paper_2503_20286_amd as nsga3
    for b, (o, r, K) in enumerate(probs):
        single = nsga3.select(o, r, K)
        torch.cuda.synchronize()
        a, s = _host(plan.results[b]), _host(single)
        for k in FIELDS:
            assert np.array_equal(a[k], s[k]), (tag, b, k)
        ia, is_ = plan.results[b].info(), single.info()
        assert (ia.status, ia.last_front, ia.num_fronts, ia.last_front_size, ia.num_from_last,
                ia.intercept_fallback, ia.near_ties) == \
               (is_.status, is_.last_front, is_.num_fronts, is_.last_front_size,
                is_.num_from_last, is_.intercept_fallback, is_.near_ties), (tag, b)


def test_plan_matches_single_calls_and_oracle(plan_mode):
    import torch
    import paper_2503_20286_amd as nsga3
    ws = workloads.make_batch(24, n_lo=1, n_hi=3000, base_seed=7000)
    probs = _dev(ws)
    print("plan", plan_mode, flush=True)
    plan = nsga3.Plan(probs)
    print("plan info", plan.info(), flush=True)
    for rep in range(3):  # several replays, each checked
        plan.launch()
        torch.cuda.synchronize()
        _check_against_single(plan, probs, (plan_mode, rep))
        for b in range(len(probs)):
            assert plan.results[b].info().status == 0
    for b in (0, 5, 23):
        w = ws[b]
        g = _host(plan.results[b])
        g["info"] = plan.results[b].info()
        rep = compare_full(w.objs, w.refs, w.K, g)
        assert not {k: v for k, v in rep.items() if k != "near_ties" and v}, rep
    plan.close()


def test_benchmark_batch_against_oracle():
    """The 512-instance batch the benchmark times (N_b in [200, 20000], M_b in
    {2, 3, 5}), captured with autotuning as the benchmark does; the largest
    instance of each objective count and 16 seeded random ones are compared
    with the oracle element by element."""
    import torch
    import paper_2503_20286_amd as nsga3
    ws = workloads.make_batch(512)
    probs = _dev(ws)
    ctx = nsga3.Context(0, autotune=True)
    ctx.reserve(max(w.N for w in ws), 5, 210)
    plan = nsga3.Plan(probs, ctx=ctx)
    for _ in range(2):
        plan.launch()
    torch.cuda.synchronize()
    pick = set()
    for M in sorted({w.M for w in ws}):
        pick.add(max((b for b, w in enumerate(ws) if w.M == M), key=lambda b: ws[b].N))
    pick |= set(np.random.default_rng(512).choice(len(ws), size=16, replace=False).tolist())
    for b in sorted(pick):
        w = ws[b]
        print(f"batch instance {b}: N={w.N} M={w.M} H={w.H} K={w.K}", flush=True)
        g = _host(plan.results[b])
        g["info"] = plan.results[b].info()
        rep = compare_full(w.objs, w.refs, w.K, g)
        assert not {k: v for k, v in rep.items() if k != "near_ties" and v}, (b, rep)
    plan.close()
    ctx.close()


def test_plan_replay_with_new_data_in_same_buffers(plan_mode):
    import torch
    import paper_2503_20286_amd as nsga3
    ws = workloads.make_batch(12, n_lo=1, n_hi=3000, base_seed=8000)
    probs = _dev(ws)
    plan = nsga3.Plan(probs)
    plan.launch()
    torch.cuda.synchronize()
    for b, (o, r, K) in enumerate(probs):  # new data, same shapes
        w = workloads.make_instance(9000 + b, o.shape[0], o.shape[1])
        o.copy_(torch.from_numpy(w.objs).cuda())
    torch.cuda.synchronize()
    for rep in range(2):
        x = torch.ones(1 << 20, device="cuda")  # eager work between replays
        (x * 2).sum().item()
        plan.launch()
        torch.cuda.synchronize()
        _check_against_single(plan, probs, (plan_mode, "new", rep))
    plan.close()


def test_engine_edge_instances():
    """Mixed objective counts in one plan (one engine launch per M), sizes 1,
    2, ragged tile boundaries, duplicates, K = 1 and K = N, and a long chain."""
    import torch
    import paper_2503_20286_amd as nsga3
    rng = np.random.default_rng(11)
    cases = []
    for (N, M) in [(1, 2), (2, 3), (3, 5), (64, 4), (1023, 2), (1024, 3), (1025, 5), (2049, 7),
                   (4097, 2), (700, 16), (300, 9)]:
        f = rng.integers(0, 6, size=(N, M)).astype(np.float32)  # ties and duplicates
        refs = workloads.das_dennis(M, 3 if M <= 5 else 1).astype(np.float32)
        for K in sorted({1, max(1, N // 3), N}):
            cases.append((f, refs, K))
    a = np.arange(600, dtype=np.float32)
    chain = np.stack([a, a], axis=1)  # a total order: 600 fronts
    cases.append((chain, workloads.das_dennis(2, 5).astype(np.float32), 300))
    # M = 2 ranking pass: runs of identical points across 64-point batches, and
    # more fronts than its table holds (7000 > 6144: the level peel takes over)
    a3 = np.repeat(np.arange(700, dtype=np.float32), 3)
    cases.append((np.stack([a3, a3], axis=1), workloads.das_dennis(2, 5).astype(np.float32), 1000))
    g2 = rng.integers(0, 40, size=(3000, 2)).astype(np.float32)
    cases.append((g2, workloads.das_dennis(2, 5).astype(np.float32), 1500))
    a7 = np.arange(7000, dtype=np.float32)
    cases.append((np.stack([a7, a7], axis=1), workloads.das_dennis(2, 5).astype(np.float32), 3500))
    # lists longer than one split item takes (32768 entries): the two-stage
    # level split (per-item counts, then ordered writes)
    big = workloads.make_instance(9500, 40000, 3)
    cases.append((big.objs, big.refs, big.K))
    # intercept fallbacks: equal objectives (singular), a constant objective (zero nadir)
    for col in (2, 0):
        f = rng.uniform(0, 1, (900, 3)).astype(np.float32)
        if col == 2:
            f[:, 2] = f[:, 1]
        else:
            f[:, 0] = 0.25
        cases.append((f, workloads.das_dennis(3, 6).astype(np.float32), 450))
    probs = [(torch.from_numpy(np.ascontiguousarray(f)).cuda(),
              torch.from_numpy(np.ascontiguousarray(r)).cuda(), K) for (f, r, K) in cases]
    plan = nsga3.Plan(probs)
    plan.launch()
    torch.cuda.synchronize()
    _check_against_single(plan, probs, "edge")
    for b, (f, r, K) in enumerate(cases):
        g = _host(plan.results[b])
        g["info"] = plan.results[b].info()
        rep = compare_full(f, r, K, g)
        assert not {k: v for k, v in rep.items() if k != "near_ties" and v}, (b, rep)
    plan.close()


def test_engine_bad_instance_is_isolated():
    """A non-finite objective or a bad reference row in one instance sets that
    instance's status and leaves every other instance exact."""
    import torch
    import paper_2503_20286_amd as nsga3
    ws = workloads.make_batch(6, n_lo=100, n_hi=900, base_seed=8100)
    probs = _dev(ws)
    probs[1][0][3, 0] = float("nan")
    probs[4][1][2, 0] = -1.0
    plan = nsga3.Plan(probs)
    plan.launch()
    torch.cuda.synchronize()
    for b in range(len(probs)):
        st = plan.results[b].info().status
        if b in (1, 4):
            assert st == -2, (b, st)  # NSGA3_E_NONFINITE
        else:
            assert st == 0
            o, r, K = probs[b]
            single = nsga3.select(o, r, K)
            torch.cuda.synchronize()
            a, s = _host(plan.results[b]), _host(single)
            for k in FIELDS:
                assert np.array_equal(a[k], s[k]), (b, k)
    plan.close()


def test_autotuned_plan_matches_single_calls():
    """Autotuning picks work-item shapes by timing; results must not change."""
    import torch
    import paper_2503_20286_amd as nsga3
    ws = workloads.make_batch(18, n_lo=100, n_hi=12000, base_seed=8200)
    probs = _dev(ws)
    ctx = nsga3.Context(0, autotune=True)
    plan = nsga3.Plan(probs, ctx=ctx)
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        _check_against_single(plan, probs, ("autotuned", rep))
    plan2 = nsga3.Plan(probs, ctx=ctx)  # tuned shapes come from the context's cache
    plan2.launch()
    torch.cuda.synchronize()
    _check_against_single(plan2, probs, "cached")
    plan.close()
    plan2.close()
    ctx.close()


def test_tuned_shapes_persist_across_contexts(tmp_path):
    """nsga3_tuned_save / nsga3_tuned_load: a second context that loads the
    first one's file holds the same shapes, and its autotuned plan (which then
    times nothing) gives the single calls' results; malformed files and files
    from another device are rejected without changing the context."""
    import torch
    import paper_2503_20286_amd as nsga3
    ws = workloads.make_batch(10, n_lo=100, n_hi=9000, base_seed=8250)
    probs = _dev(ws)
    ctx = nsga3.Context(0, autotune=True)
    plan = nsga3.Plan(probs, ctx=ctx)
    plan.close()
    shapes = ctx.tuned_shapes()
    assert shapes
    path = tmp_path / "tuned.txt"
    ctx.save_tuned(path)
    ctx.close()
    ctx2 = nsga3.Context(0, autotune=True)
    assert ctx2.tuned_shapes() == []
    ctx2.load_tuned(path)
    assert ctx2.tuned_shapes() == shapes
    plan2 = nsga3.Plan(probs, ctx=ctx2)
    assert ctx2.tuned_shapes() == shapes  # every group came from the file
    plan2.launch()
    torch.cuda.synchronize()
    _check_against_single(plan2, probs, "loaded")
    plan2.close()
    lines = path.read_text().splitlines()
    bad = tmp_path / "bad.txt"
    bad.write_text("\n".join(lines + ["5 1 8 -3 0"]) + "\n")  # negative tail length
    other = tmp_path / "other.txt"
    head = lines[0].split()
    other.write_text("\n".join([" ".join(head[:3] + [str(int(head[3]) + 1)])] + lines[1:]) + "\n")
    ctx3 = nsga3.Context(0)
    with pytest.raises(nsga3.NativeError) as e1:
        ctx3.load_tuned(bad)
    assert e1.value.code == nsga3.E_INVALID
    with pytest.raises(nsga3.NativeError) as e2:
        ctx3.load_tuned(other)
    assert e2.value.code == nsga3.E_UNSUPPORTED
    with pytest.raises(nsga3.NativeError):
        ctx3.load_tuned(tmp_path / "missing.txt")
    assert ctx3.tuned_shapes() == []
    ctx3.close()
    ctx2.close()


def test_plan_rejects_bad_descriptor():
    import torch
    import paper_2503_20286_amd as nsga3
    w = workloads.make("small")
    o = torch.from_numpy(w.objs).cuda()
    r = torch.from_numpy(w.refs).cuda()
    with pytest.raises(nsga3.NativeError):
        nsga3.Plan([(o, r, w.K), (o, r, w.N + 1)])


def test_engine_pairwise_counts_match(monkeypatch):
    """The batched plan's pairwise count launch (NSGA3_PAIRWISE=1) gives the
    same outputs as its block-bitset launch."""
    import torch
    import paper_2503_20286_amd as nsga3
    ws = workloads.make_batch(9, n_lo=50, n_hi=6000, base_seed=8300)
    probs = _dev(ws)
    plan = nsga3.Plan(probs)
    plan.launch()
    torch.cuda.synchronize()
    a = [_host(r) for r in plan.results]
    monkeypatch.setenv("NSGA3_PAIRWISE", "1")
    plan2 = nsga3.Plan(probs)
    plan2.launch()
    torch.cuda.synchronize()
    for b, r in enumerate(plan2.results):
        h = _host(r)
        for k in FIELDS:
            assert np.array_equal(a[b][k], h[k]), (b, k)
    plan.close()
    plan2.close()


@pytest.mark.parametrize("separate", ["0", "1"])
def test_engine_out_degree_forms_match(separate, monkeypatch):
    """Batched counts with out-degrees from the in-degree probes or from the
    backward pass, for every objective count, equal single calls."""
    import torch
    import paper_2503_20286_amd as nsga3
    ws = workloads.make_batch(9, n_lo=50, n_hi=6000, base_seed=8400)
    probs = _dev(ws)
    monkeypatch.setenv("NSGA3_SEPARATE_OUT", separate)
    ctx = nsga3.Context(0)
    plan = nsga3.Plan(probs, ctx=ctx)
    plan.launch()
    torch.cuda.synchronize()
    monkeypatch.delenv("NSGA3_SEPARATE_OUT")
    _check_against_single(plan, probs, ("out", separate))
    plan.close()
    ctx.close()


@pytest.mark.parametrize("wide", ["0", "1"])
def test_engine_wide_table_counts_match_oracle(wide, monkeypatch):
    """Batched counts over 128-member tables (NSGA3_ENGINE_WIDE=1, opt-in, for
    4 <= M <= 10) and over 64-member tables (the default) give the oracle's
    outputs: every M of the wide range and one beyond it, sizes around the
    128-member blocks (1, 127, 128, 129, 2,049), ties and duplicates."""
    import torch
    import paper_2503_20286_amd as nsga3
    monkeypatch.setenv("NSGA3_ENGINE_WIDE", wide)
    ctx = nsga3.Context(0)
    monkeypatch.delenv("NSGA3_ENGINE_WIDE")
    rng = np.random.default_rng(43)
    cases = []
    for M in (4, 5, 6, 7, 8, 9, 10, 11):
        for N in (1, 127, 128, 129, 2049):
            F = rng.integers(0, 6, size=(N, M)).astype(np.float32)  # ties and duplicates
            R = np.abs(rng.standard_normal((20, M))).astype(np.float32) + 0.05
            cases.append((F, R, max(1, N // 2)))
    probs = [(torch.from_numpy(F).cuda(), torch.from_numpy(R).cuda(), K) for F, R, K in cases]
    print(f"wide={wide}: {len(cases)} instances", flush=True)
    plan = nsga3.Plan(probs, ctx=ctx)
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        for b, (F, R, K) in enumerate(cases):
            g = _host(plan.results[b])
            g["info"] = plan.results[b].info()
            bad = {k: v for k, v in compare_full(F, R, K, g).items() if k != "near_ties" and v}
            assert not bad, (wide, rep, b, F.shape, bad)
    plan.close()
    ctx.close()


def test_engine_split_chunk_boundaries():
    """Level lists whose lengths sit on and around the engine split's
    512-entry chunks (one-item splits), and one list just over the one-item
    limit of 32,768 entries (two-stage splits in 512-entry items): every
    output equals single calls, and the small instances equal the oracle."""
    import torch
    import paper_2503_20286_amd as nsga3
    sizes = [(511, 3), (512, 3), (513, 5), (1023, 5), (1025, 3), (2049, 5), (32769, 3)]
    ws = [workloads.make_instance(9100 + i, N, M) for i, (N, M) in enumerate(sizes)]
    probs = _dev(ws)
    print("sizes", sizes, flush=True)
    plan = nsga3.Plan(probs)
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        _check_against_single(plan, probs, ("split", rep))
    for b, w in enumerate(ws):
        if w.N > 4096:
            continue
        g = _host(plan.results[b])
        g["info"] = plan.results[b].info()
        bad = {k: v for k, v in compare_full(w.objs, w.refs, w.K, g).items()
               if k != "near_ties" and v}
        assert not bad, (b, w.N, w.M, bad)
    plan.close()
