"""GPU: code paths that the workload-shaped tests do not reach.

* Many reference directions: H > 2048 takes the niche-count and bucket-cursor
  paths with global atomics (the per-work-group tallies hold 2048 references)
  and H > 4096 the niche threshold search over global memory (its LDS copy
  holds 4096), in both association modes.
* Workspace allocation failures (the configured cap and an injected failure):
  the call reports NSGA3_E_NOMEM, enqueues nothing, and the context (or a new
  plan) works afterwards.
"""
from __future__ import annotations

import numpy as np
import pytest

import oracle
import workloads
from tests.gpu_helpers import compare_full, gpu_select

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2503_20286_amd as nsga3
    nsga3.load()
    oracle.lib()


def _zero(rep):
    bad = {k: v for k, v in rep.items() if k != "near_ties" and v}
    assert not bad, f"mismatches: {rep}"


# Das-Dennis sets with M = 3: p = 63 gives 2080 directions, p = 99 gives 5050.
@pytest.mark.parametrize("p,assoc", [(63, "fp32"), (63, "bf16"), (99, "fp32"), (99, "bf16")])
def test_many_reference_directions(p, assoc):
    import paper_2503_20286_amd as nsga3
    w = workloads.make("small", N=6000, seed=31)
    R = workloads.das_dennis(3, p).astype(np.float32)
    mode = nsga3.ASSOC_BF16 if assoc == "bf16" else nsga3.ASSOC_FP32
    print(f"H={R.shape[0]} {assoc}", flush=True)
    for K in (w.N // 2, w.N // 5):
        g = gpu_select(w.objs, R, K, assoc=mode)
        _zero(compare_full(w.objs, R, K, g))


def test_workspace_cap_reports_nomem_and_context_recovers():
    import torch
    import paper_2503_20286_amd as nsga3
    small = workloads.make("small")
    big = workloads.make("ties", N=8000)
    need_small = nsga3.workspace_size(small.N, small.M, small.H)
    need_big = nsga3.workspace_size(big.N, big.M, big.H)
    assert need_big > need_small
    ctx = nsga3.Context(0, max_workspace_bytes=need_small)
    g = gpu_select(small.objs, small.refs, small.K, ctx=ctx)
    _zero(compare_full(small.objs, small.refs, small.K, g))
    o = torch.from_numpy(big.objs).cuda()
    r = torch.from_numpy(big.refs).cuda()
    with pytest.raises(nsga3.NativeError) as e:
        nsga3.select(o, r, big.K, ctx=ctx)
    assert e.value.code == -3
    with pytest.raises(nsga3.NativeError) as e:
        ctx.reserve(big.N, big.M, big.H)
    assert e.value.code == -3
    with pytest.raises(nsga3.NativeError) as e:          # plans honour the cap too
        nsga3.Plan([(o, r, big.K)], ctx=ctx)
    assert e.value.code == -3
    g = gpu_select(small.objs, small.refs, small.K, ctx=ctx)   # still usable
    _zero(compare_full(small.objs, small.refs, small.K, g))
    ctx.close()


def test_injected_allocation_failure_then_success(monkeypatch):
    import torch
    import paper_2503_20286_amd as nsga3
    w = workloads.make("ties", N=5000)
    o = torch.from_numpy(w.objs).cuda()
    r = torch.from_numpy(w.refs).cuda()
    ctx = nsga3.Context(0)
    monkeypatch.setenv("NSGA3_TEST_FAIL_ALLOC", "1")
    with pytest.raises(nsga3.NativeError) as e:
        nsga3.select(o, r, w.K, ctx=ctx)
    assert e.value.code == -3
    with pytest.raises(nsga3.NativeError) as e:
        nsga3.Plan([(o, r, w.K)], ctx=ctx)
    assert e.value.code == -3
    monkeypatch.delenv("NSGA3_TEST_FAIL_ALLOC")
    g = gpu_select(w.objs, w.refs, w.K, ctx=ctx)
    _zero(compare_full(w.objs, w.refs, w.K, g))
    plan = nsga3.Plan([(o, r, w.K)], ctx=ctx)
    plan.launch()
    torch.cuda.synchronize()
    assert torch.equal(plan.results[0].selected, torch.from_numpy(g["selected"]).cuda())
    plan.close()
    ctx.close()


def test_repeated_calls_follow_the_previous_level_profile():
    """A context sizes each call's peeling launches from the previous call's
    level sizes: the levels it enqueues, the table-build grids, and the last
    levels finished by one work-group.  Repeating a workload takes the
    one-work-group tail; switching workloads makes the expectation stale in
    both directions (too many enqueued levels, or a tail too large for one
    work-group, which the grid then peels).  Every call must match the
    oracle exactly."""
    import paper_2503_20286_amd as nsga3
    cases = {
        "ties": workloads.make("ties", N=8000, seed=41),
        "large": workloads.make("large", N=6000, seed=42),
        "small": workloads.make("small", N=200, seed=43),
    }
    refsel = {k: oracle.select(w.objs, w.refs, w.K, with_counts=True) for k, w in cases.items()}
    ctx = nsga3.Context(0)
    for name in ("ties", "ties", "ties", "large", "ties", "large", "large", "small", "ties"):
        w = cases[name]
        print(name, w.N, w.M, refsel[name].num_fronts, flush=True)
        g = gpu_select(w.objs, w.refs, w.K, ctx=ctx)
        _zero(compare_full(w.objs, w.refs, w.K, g, s=refsel[name]))
    ctx.close()
