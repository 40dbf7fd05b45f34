"""GPU: batched plans (many selections in one graph launch) must reproduce the
single-call results bit for bit, on every replay, with new data in the same
buffers, and match the oracle."""
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


def _host(sel):
    return {k: None if getattr(sel, k) is None else getattr(sel, k).cpu().numpy() for k in FIELDS}


def _make(B, seed, n_hi=3000):
    return workloads.make_batch(B, n_lo=1, n_hi=n_hi, base_seed=seed)


def test_plan_matches_single_calls_and_oracle():
    import torch
    import paper_2503_20286_amd as nsga3
    ws = _make(24, 7000)
    probs = [(torch.from_numpy(w.objs).cuda(), torch.from_numpy(w.refs).cuda(), w.K) for w in ws]
    plan = nsga3.Plan(probs)
    print("plan", plan.info(), flush=True)
    for rep in range(3):  # several replays, each checked
        plan.launch()
        torch.cuda.synchronize()
        for b, (o, r, K) in enumerate(probs):
            single = nsga3.select(o, r, K)
            torch.cuda.synchronize()
            a, s = _host(plan.results[b]), _host(single)
            for k in FIELDS:
                assert np.array_equal(a[k], s[k]), (rep, b, k)
            assert plan.results[b].info().status == 0
    for b in (0, 5, 23):
        w = ws[b]
        g = _host(plan.results[b])
        g["info"] = plan.results[b].info()
        rep = compare_full(w.objs, w.refs, w.K, g)
        assert not {k: v for k, v in rep.items() if k != "near_ties" and v}, rep
    plan.close()


def test_plan_replay_with_new_data_in_same_buffers():
    import torch
    import paper_2503_20286_amd as nsga3
    ws = _make(12, 8000)
    probs = [(torch.from_numpy(w.objs).cuda(), torch.from_numpy(w.refs).cuda(), w.K) for w in ws]
    plan = nsga3.Plan(probs)
    plan.launch()
    torch.cuda.synchronize()
    for b, (o, r, K) in enumerate(probs):  # new data, same shapes
        w = workloads.make_instance(9000 + b, o.shape[0], o.shape[1])
        o.copy_(torch.from_numpy(w.objs).cuda())
    torch.cuda.synchronize()
    for rep in range(2):
        plan.launch()
        torch.cuda.synchronize()
        for b, (o, r, K) in enumerate(probs):
            single = nsga3.select(o, r, K)
            torch.cuda.synchronize()
            a, s = _host(plan.results[b]), _host(single)
            for k in FIELDS:
                assert np.array_equal(a[k], s[k]), (rep, b, k)
    plan.close()


def test_plan_rejects_bad_descriptor():
    import torch
    import paper_2503_20286_amd as nsga3
    w = workloads.make("small")
    o = torch.from_numpy(w.objs).cuda()
    r = torch.from_numpy(w.refs).cuda()
    with pytest.raises(nsga3.NativeError):
        nsga3.Plan([(o, r, w.K), (o, r, w.N + 1)])
