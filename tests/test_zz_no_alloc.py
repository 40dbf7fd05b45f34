"""GPU: the allocation-free entry point (nsga3_select_noalloc) against
nsga3_select on the same inputs, two calls in a row (the second smaller, so
the shared scratch array holds the first call's data when it starts), and
the size limit."""
from __future__ import annotations

import numpy as np
import pytest

import workloads

pytestmark = pytest.mark.gpu

FIELDS = ("selected", "rank", "niche", "dist", "dom_in", "dom_out")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    import paper_2503_20286_amd as nsga3
    nsga3.load()


def _host(sel):
    out = {k: getattr(sel, k).cpu().numpy() for k in FIELDS}
    out["info"] = sel.info()
    return out


def _both(w, K):
    import torch
    import paper_2503_20286_amd as nsga3
    o = torch.from_numpy(w.objs).cuda()
    r = torch.from_numpy(w.refs).cuda()
    out = nsga3.alloc_outputs(w.N, K, o.device)
    nsga3.select_noalloc(o, r, K, out=out)
    torch.cuda.synchronize()
    a = _host(out)
    b = _host(nsga3.select(o, r, K))
    return a, b


def _same(a, b, tag):
    for k in FIELDS:
        assert np.array_equal(a[k], b[k]), (tag, k)
    assert a["info"] == b["info"], tag
    assert a["info"].status == 0, tag


def test_noalloc_matches_select_twice_second_smaller():
    big = workloads.make("ties", N=20000)
    small = workloads.make("large", N=3000, seed=5)
    for tag, w, K in (("first", big, big.K), ("second", small, small.K // 3)):
        print(f"noalloc {tag}: N={w.N} M={w.M} H={w.H} K={K}", flush=True)
        a, b = _both(w, K)
        _same(a, b, tag)


def test_noalloc_size_limit_and_recovery():
    import torch
    import paper_2503_20286_amd as nsga3
    w = workloads.make("large", N=120000)          # workspace about 44 MiB > 32 MiB
    assert nsga3.workspace_size(w.N, w.M, w.H) > 32 << 20
    o = torch.from_numpy(w.objs).cuda()
    r = torch.from_numpy(w.refs).cuda()
    out = nsga3.alloc_outputs(w.N, w.K, o.device)
    with pytest.raises(nsga3.NativeError) as e:
        nsga3.select_noalloc(o, r, w.K, out=out)
    assert e.value.code == -3
    s = workloads.make("small")
    a, b = _both(s, s.K)
    _same(a, b, "after rejection")
