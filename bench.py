"""Benchmark: merged-population points/s through the whole NSGA-III
environmental selection on one MI355X.

One step = one nsga3_select call (every stage: keys and presort, dominance
counts, front peeling, normalisation, association, niche selection) over the
large workload (N=200,000 merged points, M=5 objectives, H=210 Das-Dennis
directions (p=6), K=100,000; sphere shell f = r*u, r = 1 + Exp(rate 4), 20% of
points with r = 1), inputs resident in device memory.

Prints one JSON line (rank 0, N=1).  The roofline object covers the dominant
phase (the dominance counts: block-table build, in-degree and out-degree
kernels): algorithmic work M*N*(N-1)/2 pair-objective compares per launch
(every unordered pair decided once) divided by the phase's duration from HIP
events the library records on its stream, against the vector-ALU compare
peak 256 CUs x 64 lanes x 2.4 GHz; traffic is the phase's HBM bytes from
FETCH_SIZE / WRITE_SIZE counters (profiles/dominance_count_large_traffic.json).
The "batched" object times 512 selections of mixed N and M in one graph
launch.  The CPU baseline is the float64 oracle on a bounded sample of the
same recipe, scaled to N=200,000 by the O(N^2) cost of its dominance stages.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "merged-pop points/sec through NSGA-III selection (N=200k,M=5); batched sel/s"
PEAK_CMP_PER_S = 256 * 64 * 2.4e9          # vector-ALU lane operations per second
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "dominance_count_large_traffic.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=["large", "many", "ties", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-n", type=int, default=140000)
    ap.add_argument("--check", action="store_true", help="verify one timed result (sampled)")
    ap.add_argument("--assoc", default="fp32", choices=["fp32", "bf16"],
                    help="association screening precision (re-scoring is float64 in both)")
    ap.add_argument("--precision-report", action="store_true",
                    help="instead of the throughput line: float32 vs bfloat16 association on the "
                         "workload, errors against the float64 oracle and the phase times")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched measurement (512 selections in one graph launch)")
    ap.add_argument("--batch", type=int, default=512, help="instances in the batched plan")
    ap.add_argument("--batch-only-m", type=int, default=0,
                    help="diagnostics: keep only the batch's instances with this M")
    ap.add_argument("--engine-stats", action="store_true",
                    help="add the batched engine's per-stage block times (separate plan)")
    ap.add_argument("--plan-compare", action="store_true",
                    help="also time the batch as a graph of single selections")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="first run a plain device copy of this many MiB (three times), whose "
                         "FETCH_SIZE / WRITE_SIZE counters scale those of the library's kernels")
    return ap.parse_args()


def cpu_baseline(name: str, N_full: int, n_sample: int):
    """Times the oracle on N=n_sample points of the same recipe and scales the
    time by (N_full / n_sample)^2 (its dominance count and peeling are O(N^2))."""
    import oracle
    import workloads
    w = workloads.make(name, N=n_sample)
    oracle.lib()
    t0 = time.perf_counter()
    oracle.select(w.objs, w.refs, w.K, with_counts=True)
    dt = time.perf_counter() - t0
    t_full = dt * (N_full / n_sample) ** 2
    return {
        "value": N_full / t_full,
        "unit": "points/s",
        "cores": oracle.num_threads(),
        "kind": "oracle",
        "sample": (f"float64 C oracle (OpenMP) on the first-recipe sample N={n_sample} of workload "
                   f"'{name}' (same seed and shape recipe): {dt:.2f} s; scaled by (N/n)^2 to "
                   f"N={N_full}: {t_full:.1f} s per selection"),
    }


def precision_report(args, w, objs, refs):
    """One JSON line: association error of each screening precision against the
    float64 oracle (on the GPU's own ranks, which both modes share), selection
    agreement between the modes, and the association phase time of each."""
    import numpy as np
    import torch

    import oracle
    import paper_2503_20286_amd as nsga3
    modes = {"fp32": nsga3.ASSOC_FP32, "bf16": nsga3.ASSOC_BF16}
    out = {}
    res = {}
    for name, mode in modes.items():
        ctx = nsga3.Context(0, assoc=mode)
        ctx.reserve(w.N, w.M, w.H)
        r = nsga3.select(objs, refs, w.K, ctx=ctx)
        for _ in range(args.warmup):
            nsga3.select(objs, refs, w.K, ctx=ctx, out=r)
        torch.cuda.synchronize()
        ctx.profile(True)
        for _ in range(args.steps):
            nsga3.select(objs, refs, w.K, ctx=ctx, out=r)
        torch.cuda.synchronize()
        ms, calls = ctx.phase_times()
        ctx.profile(False)
        res[name] = {k: getattr(r, k).cpu().numpy() for k in ("selected", "rank", "niche", "dist")}
        res[name]["info"] = r.info()
        out[name] = {"associate_ms": ms[4] / calls, "total_ms": sum(ms) / calls}
        ctx.close()
    rank = res["fp32"]["rank"]
    assert np.array_equal(rank, res["bf16"]["rank"])
    l = res["fp32"]["info"].last_front
    nz = oracle.normalize(w.objs, rank, l)
    niche, dist, gap = oracle.associate(w.objs, rank, l, nz.z, nz.a, w.refs)
    S = rank <= l
    tie = S & (gap < 1e-6)
    fpn = np.linalg.norm((w.objs.astype(np.float64) - nz.z) / nz.a, axis=1)
    for name in modes:
        g = res[name]
        mism = (g["niche"] != niche) & S
        dd = np.abs(g["dist"].astype(np.float64) - dist)[S]
        out[name].update({
            "niche_mismatch_outside_ties": int(np.sum(mism & ~tie)),
            "niche_mismatch_at_ties": int(np.sum(mism & tie)),
            "max_abs_dist_err": float(dd.max()),
            "max_rel_dist_err": float((dd / np.maximum(1.0, fpn[S])).max()),
            "near_ties_reported": g["info"].near_ties,
        })
    line = {
        "metric": "association error vs float64 oracle, float32 and bfloat16 screening",
        "workload": f"{args.workload}: N={w.N} M={w.M} H={w.H} K={w.K}",
        "admitted_points": int(S.sum()),
        "oracle_near_ties": int(tie.sum()),
        "selection_identical_across_modes": bool(np.array_equal(res["fp32"]["selected"],
                                                                res["bf16"]["selected"])),
        "modes": out,
    }
    print(json.dumps(line), flush=True)


def batched(args):
    """Batched form: ``args.batch`` independent selections (N_b uniform in
    [200, 20000], M_b from {2, 3, 5}, K_b = N_b/2) captured once into a plan
    and replayed; compared with the same instances as back-to-back single
    calls on one stream."""
    import torch

    import paper_2503_20286_amd as nsga3
    import workloads
    ws = workloads.make_batch(args.batch)
    if args.batch_only_m:
        ws = [w for w in ws if w.M == args.batch_only_m]
    probs = [(torch.from_numpy(w.objs).cuda(), torch.from_numpy(w.refs).cuda(), w.K) for w in ws]
    ctx = nsga3.Context(0, autotune=True)
    ctx.reserve(max(w.N for w in ws), 5, 210)
    t0 = time.perf_counter()
    plan = nsga3.Plan(probs, ctx=ctx)  # times candidate work-item shapes per (M, N range)
    t_create = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    for _ in range(max(args.warmup, 1)):
        plan.launch(stream)
    torch.cuda.synchronize()
    bad = [b for b, r in enumerate(plan.results) if r.info().status != 0]
    if bad:
        raise SystemExit(f"batched selection reported a status on instances {bad[:8]}")
    steps = max(1, args.steps // 2)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(stream)
    for _ in range(steps):
        plan.launch(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    ms_graph = start.elapsed_time(stop) / steps
    # the same instances as single calls, one after another
    outs = [nsga3.select(o, r, K, ctx=ctx) for (o, r, K) in probs]
    torch.cuda.synchronize()
    start.record(stream)
    for (o, r, K), out in zip(probs, outs):
        nsga3.select(o, r, K, ctx=ctx, out=out)
    stop.record(stream)
    torch.cuda.synchronize()
    ms_single = start.elapsed_time(stop)
    same = all(torch.equal(a.selected, b.selected) and torch.equal(a.rank, b.rank)
               for a, b in zip(plan.results, outs))
    info = plan.info()
    plan.close()
    tuned = ctx.tuned_shapes()
    n_pts = sum(w.N for w in ws)
    extra = {}
    # the same batch with the fixed default shapes, for comparison
    dctx = nsga3.Context(0)
    pd = nsga3.Plan(probs, ctx=dctx)
    pd.launch(stream)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        pd.launch(stream)
    stop.record(stream)
    torch.cuda.synchronize()
    extra["default_shapes_ms_per_launch"] = start.elapsed_time(stop) / steps
    pd.close()
    dctx.close()
    if args.engine_stats:
        pctx = nsga3.Context(0)
        pctx.profile(True)
        p2 = nsga3.Plan(probs, ctx=pctx)
        for _ in range(2):
            p2.launch(stream)
        torch.cuda.synchronize()
        st = p2.stage_times()
        extra["engine_block_ms_per_launch"] = {
            "stages": {k: {"item": v["item_ms"] / 2, "epilogue": v["epilogue_ms"] / 2,
                           "items": v["items"] // 2} for k, v in st["stages"].items()},
            "probe": st["probe_ms"] / 2, "idle": st["idle_ms"] / 2}
        p2.close()
        pctx.close()
    if args.plan_compare:
        os.environ["NSGA3_PLAN_MODE"] = "graph"
        try:
            p3 = nsga3.Plan(probs, ctx=ctx)
        finally:
            del os.environ["NSGA3_PLAN_MODE"]
        p3.launch(stream)
        torch.cuda.synchronize()
        start.record(stream)
        for _ in range(steps):
            p3.launch(stream)
        stop.record(stream)
        torch.cuda.synchronize()
        extra["graph_of_single_calls_ms"] = start.elapsed_time(stop) / steps
        p3.close()
    return {
        "value": len(ws) / (ms_graph / 1e3),
        "unit": "selections/s",
        "ms_per_launch": ms_graph,
        "points_per_s": n_pts / (ms_graph / 1e3),
        "instances": len(ws),
        "total_points": n_pts,
        "graph_branches": info["branches"],
        "graph_nodes": info["nodes"],
        "plan_create_s_with_autotune": t_create,
        "tuned_shapes": tuned,
        "single_calls_ms": ms_single,
        "single_calls_sel_per_s": len(ws) / (ms_single / 1e3),
        "speedup_vs_single_calls": ms_single / ms_graph,
        "identical_to_single_calls": bool(same),
        "steps": steps,
        **extra,
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the selection runs on a single MI355X)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2503_20286_amd as nsga3
    import workloads

    if not torch.cuda.is_available():
        print("no HIP device visible", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    nsga3.load()
    w = workloads.make(args.workload)
    dev = torch.device("cuda:0")
    objs = torch.from_numpy(w.objs).to(dev)
    refs = torch.from_numpy(w.refs).to(dev)
    if args.precision_report:
        precision_report(args, w, objs, refs)
        return
    ctx = nsga3.Context(0, assoc=nsga3.ASSOC_BF16 if args.assoc == "bf16" else nsga3.ASSOC_FP32)
    ctx.reserve(w.N, w.M, w.H)
    stream = torch.cuda.current_stream(dev)
    out = nsga3.select(objs, refs, w.K, ctx=ctx)
    for _ in range(args.warmup):
        nsga3.select(objs, refs, w.K, ctx=ctx, out=out)
    torch.cuda.synchronize()
    info = out.info()
    if info.status != 0:
        raise SystemExit(f"selection reported status {info.status}")

    ctx.profile(True)
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_host = time.perf_counter()
    start.record(stream)
    for _ in range(args.steps):
        nsga3.select(objs, refs, w.K, ctx=ctx, out=out)
    stop.record(stream)
    torch.cuda.synchronize()
    t_host = time.perf_counter() - t_host
    ms_total = start.elapsed_time(stop)
    phase_ms, calls = ctx.phase_times()
    ctx.profile(False)
    ms_per_step = ms_total / args.steps
    phases = {name: phase_ms[q] / max(calls, 1) for q, name in enumerate(nsga3.PHASES)}

    if args.check:
        import oracle
        sel = out.selected.cpu().numpy()
        rank = out.rank.cpu().numpy()
        l, nb, nl = oracle.last_front(rank, w.K)
        assert sel.size == w.K and np.all(np.diff(sel) > 0)
        assert np.all(rank[sel] <= l)

    N, M = w.N, w.M
    cmp_per_launch = M * N * (N - 1) / 2.0
    t_dom = phases["dominance_count"] / 1e3
    achieved = cmp_per_launch / t_dom / 1e12
    peak = PEAK_CMP_PER_S / 1e12
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as fh:
            tr = json.load(fh)
        if tr.get("workload") == args.workload:
            traffic = tr.get("bytes_per_launch")
    res = {
        "metric": METRIC,
        "value": N / (ms_per_step / 1e3),
        "unit": "points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: N={N} M={M} H={w.H} K={w.K}",
            "N": N, "M": M, "H": w.H, "K": w.K,
            "compute": "u32 order keys (exact f32 dominance, block bitsets); f64 normalisation "
                       f"and re-scoring; {args.assoc} association screening",
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "alu",
            "kernel": "dominance counts (k_build_blocks + k_fwd_all + k_bwd_all, block bitsets)",
            "achieved": achieved,
            "peak": peak,
            "unit": "Tcmp/s",
            "frac": achieved / peak,
            "traffic": traffic,
            "work_per_launch": f"{cmp_per_launch:.4e} pair-objective compares (M*N*(N-1)/2: every "
                               "unordered pair decided once)",
            "frac_counts_and_peeling": cmp_per_launch / ((phases["dominance_count"] + phases["peel"])
                                                          / 1e3) / PEAK_CMP_PER_S,
        },
        "phases_ms": phases,
        "fronts": {"num_fronts": info.num_fronts, "last_front": info.last_front,
                   "last_front_size": info.last_front_size, "num_from_last": info.num_from_last,
                   "near_ties": info.near_ties, "intercept_fallback": info.intercept_fallback},
        "host_wall_s": t_host,
    }
    if not args.no_batch:
        res["batched"] = batched(args)
    if not args.no_cpu_baseline:
        res["cpu_baseline"] = cpu_baseline(args.workload, N, min(args.cpu_sample_n, N))
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
