"""Benchmark: merged-population points/s through the whole NSGA-III
environmental selection on one MI355X.

One step = one nsga3_select call (every stage: keys and presort, dominance
counts, front peeling, normalisation, association, niche selection) over the
large workload (N=200,000 merged points, M=5 objectives, H=210 Das-Dennis
directions (p=6), K=100,000; sphere shell f = r*u, r = 1 + Exp(rate 4), 20% of
points with r = 1), inputs resident in device memory.  The timed loop records
no per-phase events; phase times come from a separate loop with the library's
phase events on.

Prints one JSON line (rank 0, N=1).  The roofline object covers the dominant
phase (the dominance counts): algorithmic work M*N*(N-1)/2 pair-objective
compares per launch (every unordered pair decided once) divided by the phase's
event-timed duration, against the vector-ALU rate 256 CUs x 64 lanes x 2.4 GHz.
The block-bitset kernels decide 64 pairs per probe, so this is an effective
pair-decision rate, not a VALU utilisation, and it can exceed 1; the issue
utilisation is roofline.valu_issue: the phase's counted VALU instructions
(SQ_INSTS_VALU, profiles/dominance_count_large_counters.json) over its event
time against 1024 SIMDs x 2.4 GHz / 4.  traffic is the phase's HBM bytes from
FETCH_SIZE / WRITE_SIZE counters (profiles/dominance_count_large_traffic.json).

The float64 oracle runs once on the whole workload: its wall time is the
cpu_baseline, and its outputs are compared element by element with the timed
selection ("parity": mismatch counts, all must be 0).  "c5" runs the
many-objective workload (N=100,000, M=10, H=275) with float32 and bfloat16
association screening against the oracle; "batched" times 512 selections of
mixed N and M in one graph launch.
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
COUNTERS_FILE = os.path.join(ROOT, "profiles", "dominance_count_large_counters.json")
VALU_ISSUE_PER_S = 256 * 4 * 2.4e9 / 4       # wave64 VALU instructions per second


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="large", choices=["large", "many", "ties", "small"])
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle (cpu_baseline and parity objects)")
    ap.add_argument("--no-c5", action="store_true",
                    help="skip the many-objective float32 / bfloat16 comparison")
    ap.add_argument("--no-oneshot", action="store_true",
                    help="skip the one-shot niching report")
    ap.add_argument("--no-rvea", action="store_true",
                    help="skip the TensorRVEA selection report")
    ap.add_argument("--no-hype", action="store_true",
                    help="skip the TensorHypE selection report")
    ap.add_argument("--no-variation", action="store_true",
                    help="skip the SBX / polynomial mutation and gather report")
    ap.add_argument("--assoc", default="fp32", choices=["fp32", "bf16"],
                    help="association screening precision (re-scoring is float64 in both)")
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


def cpu_baseline(w):
    """The float64 oracle on the whole workload, once, with every host core;
    plus one-thread timings of the small (N=200) and ties (N=20,000) workloads.
    Returns (baseline object, oracle selection)."""
    import oracle
    import workloads
    oracle.lib()
    t0 = time.perf_counter()
    ref = oracle.select(w.objs, w.refs, w.K, with_counts=True)
    dt = time.perf_counter() - t0
    cores = oracle.num_threads()
    single = {}
    oracle.set_num_threads(1)
    try:
        for name, reps in (("small", 3), ("ties", 1)):
            s = workloads.make(name)
            ts = []
            for _ in range(reps):
                t1 = time.perf_counter()
                oracle.select(s.objs, s.refs, s.K, with_counts=True)
                ts.append(time.perf_counter() - t1)
            t = sorted(ts)[len(ts) // 2]
            single[name] = {"N": s.N, "M": s.M, "s_per_selection": t, "points_per_s": s.N / t}
    finally:
        oracle.set_num_threads(0)
    return {
        "value": w.N / dt,
        "unit": "points/s",
        "cores": cores,
        "kind": "oracle",
        "sample": (f"float64 C oracle (OpenMP, {cores} threads) once on the whole workload "
                   f"(N={w.N}, M={w.M}, H={w.H}, K={w.K}; ranks, both dominance counts, "
                   f"selection): {dt:.2f} s"),
        "single_thread": single,
    }, ref


def parity(w, g, ref):
    """Mismatch counts of a GPU selection against the oracle's (ranks, counts,
    selection and front statistics exact; reference lines exact outside the
    oracle's near-ties; distances within 1e-5 * max(1, ||f'||))."""
    import numpy as np

    import oracle
    l = ref.last_front
    nz = oracle.normalize(w.objs, ref.rank, l)
    niche, dist, gap = oracle.associate(w.objs, ref.rank, l, nz.z, nz.a, w.refs)
    S = ref.rank <= l
    tie = S & (gap < 1e-6)
    fpn = np.linalg.norm((w.objs.astype(np.float64) - nz.z) / nz.a, axis=1)
    gd = g["dist"].astype(np.float64)
    derr = np.abs(gd - dist)
    info = g["info"]
    out = {
        "rank": int(np.sum(g["rank"] != ref.rank)),
        "selected": int(np.setxor1d(g["selected"], ref.selected).size),
        "niche_outside_ties": int(np.sum((g["niche"] != niche) & S & ~tie)),
        "dist_outside_tol": int(np.sum(S & ~tie & (derr > 1e-5 * np.maximum(1.0, fpn)))
                                + np.sum(~S & (gd != -1.0))),
        "max_abs_dist_err": float(derr[S & ~tie].max()) if np.any(S & ~tie) else 0.0,
        "front_stats": int((info.last_front, info.num_fronts, info.last_front_size,
                            info.num_from_last, info.intercept_fallback) !=
                           (ref.last_front, ref.num_fronts, ref.last_front_size,
                            ref.num_from_last, ref.intercept_fallback)),
        "near_ties": int(tie.sum()),
    }
    if g.get("dom_in") is not None:
        out["dom_in"] = int(np.sum(g["dom_in"] != ref.dom_in))
        out["dom_out"] = int(np.sum(g["dom_out"] != ref.dom_out))
    return out


def _host(res):
    return {"selected": res.selected.cpu().numpy(), "rank": res.rank.cpu().numpy(),
            "niche": res.niche.cpu().numpy(), "dist": res.dist.cpu().numpy(),
            "dom_in": None if res.dom_in is None else res.dom_in.cpu().numpy(),
            "dom_out": None if res.dom_out is None else res.dom_out.cpu().numpy(),
            "info": res.info()}


def _time_calls(fn, steps, stream):
    import torch
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    for _ in range(steps):
        fn()
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps


def _phase_pass(ctx, fn, steps):
    """Phase times (ms per call) from the library's HIP events, in a loop of
    its own so that the headline loop records none."""
    import torch

    import paper_2503_20286_amd as nsga3
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(steps):
        fn()
    torch.cuda.synchronize()
    ms, calls = ctx.phase_times()
    ctx.profile(False)
    return {name: ms[q] / max(calls, 1) for q, name in enumerate(nsga3.PHASES)}


def oneshot_report(args, w, objs, refs, g_exact, ref):
    """The one-shot niche selection on the same workload: time per selection
    and of the niching phase, its agreement with the oracle's one-shot form,
    and the quality delta against the exact loop (selection difference and
    how many references the selected set covers)."""
    import numpy as np
    import torch

    import oracle
    import paper_2503_20286_amd as nsga3
    ctx = nsga3.Context(0, niching=nsga3.NICHING_ONESHOT)
    ctx.reserve(w.N, w.M, w.H)
    r = nsga3.select(objs, refs, w.K, ctx=ctx)

    def call():
        nsga3.select(objs, refs, w.K, ctx=ctx, out=r)
    for _ in range(args.warmup):
        call()
    ms = _time_calls(call, args.steps, torch.cuda.current_stream())
    ph = _phase_pass(ctx, call, args.steps)
    g = _host(r)
    ctx.close()
    out = {"ms_per_selection": ms, "niching_ms": ph["niching"]}
    if ref is not None:
        l = ref.last_front
        rho = oracle.niche_count(ref.rank, ref.niche, l, w.H)
        chosen, ne = oracle.niching_oneshot(ref.rank, ref.niche, ref.dist, l, w.H,
                                            ref.num_from_last, rho)
        want = np.nonzero((ref.rank < l) | chosen)[0]
        out["selected_mismatch_vs_oracle_oneshot"] = int(np.setxor1d(g["selected"], want).size)
        out["empty_niche_picks"] = int(ne)
    cov = {}
    for name, x in (("exact", g_exact), ("oneshot", g)):
        nic = x["niche"][x["selected"]]
        cnt = np.bincount(nic, minlength=w.H)
        cov[name] = {"refs_covered": int(np.sum(cnt > 0)), "max_niche_count": int(cnt.max())}
    out["quality_vs_exact"] = {
        "selected_differ": int(np.setdiff1d(g["selected"], g_exact["selected"]).size),
        **{f"{k}_{m}": v for k, d in cov.items() for m, v in d.items()},
    }
    return out


def rvea_report(args, w, objs, refs):
    """TensorRVEA selection (Supplementary Alg. S.12) on the same workload:
    time per call, its screening rate against the float32 vector peak, and
    parity with the float64 oracle (partitions exact; elites exact outside
    APD near-ties)."""
    import numpy as np
    import torch

    import oracle
    import paper_2503_20286_amd as nsga3
    t, t_max, alpha = 5, 10, 2.0
    ctx = nsga3.Context(0)
    r = nsga3.rvea_select(objs, refs, t, t_max, alpha, ctx=ctx)
    for _ in range(args.warmup):
        nsga3.rvea_select(objs, refs, t, t_max, alpha, ctx=ctx)
    ms = _time_calls(lambda: nsga3.rvea_select(objs, refs, t, t_max, alpha, ctx=ctx), args.steps,
                     torch.cuda.current_stream())
    r = nsga3.rvea_select(objs, refs, t, t_max, alpha, ctx=ctx)
    torch.cuda.synchronize()
    e, a, apd = r.elite.cpu().numpy(), r.assign.cpu().numpy(), r.apd.cpu().numpy()
    ctx.close()
    s = oracle.rvea_select(w.objs, w.refs, t, t_max, alpha)
    tie = s.gap < 1e-12
    # screening: two float32 passes of H dot products of length M per point
    flops = 2.0 * 2.0 * w.N * w.H * w.M
    return {
        "t": t, "t_max": t_max, "alpha": alpha,
        "ms_per_selection": ms,
        "points_per_s": w.N / (ms / 1e3),
        "screen_tflop_s": flops / (ms / 1e3) / 1e12,
        "screen_frac_of_fp32_peak": flops / (ms / 1e3) / 157.3e12,
        "parity": {
            "assign_mismatch": int(np.sum(a != s.assign)),
            "elite_mismatch_outside_ties": int(np.sum((e != s.elite) & ~tie)),
            "max_rel_apd_err": float(np.max(np.abs(apd - s.apd) / np.maximum(s.apd, 1e-300))),
            "apd_near_tie_partitions": int(np.sum(tie)),
        },
        "nonempty_partitions": int(np.sum(e >= 0)),
    }


def hype_report(args):
    """TensorHypE selection (Sec. IV-C; Supplementary Alg. S.10, S.11): the
    ties workload (N = 20,000 merged points of a population of 10,000, M = 3)
    with 10,000 Monte Carlo draws, timed and compared with the oracle; and
    the large workload (N = 200,000, M = 5) timed."""
    import numpy as np
    import torch

    import oracle
    import paper_2503_20286_amd as nsga3
    import workloads
    out = {}
    for name, check in (("ties", True), ("large", False)):
        w = workloads.make(name)
        s = 10_000
        U = np.random.default_rng(2024).random((s, w.M)).astype(np.float32)
        vref = (w.objs.max(0).astype(np.float64) * 1.1 + 0.01).astype(np.float32)
        o = torch.from_numpy(w.objs).cuda()
        v = torch.from_numpy(vref).cuda()
        u = torch.from_numpy(U).cuda()
        n = w.N // 2
        ctx = nsga3.Context(0)
        r = nsga3.hype_select(o, v, u, n, ctx=ctx)
        for _ in range(args.warmup):
            nsga3.hype_select(o, v, u, n, ctx=ctx)
        ms = _time_calls(lambda: nsga3.hype_select(o, v, u, n, ctx=ctx), args.steps,
                         torch.cuda.current_stream())
        r = nsga3.hype_select(o, v, u, n, ctx=ctx)
        torch.cuda.synchronize()
        info = r.info()
        rec = {"workload": f"{name}: N={w.N} M={w.M} n={n} s={s}", "ms_per_selection": ms,
               "points_per_s": w.N / (ms / 1e3), "last_front": info.last_front,
               "last_front_size": info.last_front_size,
               "sample_point_tests_per_s": float(s) * w.N / (ms / 1e3)}
        if check:
            sel = r.selected.cpu().numpy()
            d = r.d.cpu().numpy()
            ref = oracle.hype_select(w.objs, vref, U, n)
            S = ref.rank <= ref.last_front
            rec["parity"] = {
                "rank_mismatch": int(np.sum(r.rank.cpu().numpy() != ref.rank)),
                "selected_mismatch": int(np.setxor1d(sel, ref.selected).size),
                "max_rel_hv_err": float(np.max(np.abs(d[S] - ref.d[S]) /
                                               np.maximum(np.abs(ref.d[S]), 1e-300))),
            }
        ctx.close()
        out[name] = rec
    return out


def variation_report(args):
    """SBX and polynomial mutation (Supplementary Sec. S.I) of a population of
    n = 10,000 with d = 4,096 variables (the decision-space size of the
    paper's largest robot-control problems), and the gather of 10,000 rows:
    HBM rooflines (algorithmic bytes: every input read once, every output
    written once)."""
    import torch

    import paper_2503_20286_amd as nsga3
    n, d = 10_000, 4096
    h = n // 2
    g = torch.Generator(device="cuda").manual_seed(7)
    X = torch.rand((n, d), device="cuda", generator=g)
    lo = torch.zeros(d, device="cuda")
    hi = torch.ones(d, device="cuda")
    rs = torch.rand((h, d), device="cuda", generator=g)
    rp = torch.rand((2 * h, d), device="cuda", generator=g)
    out = torch.empty((2 * h, d), device="cuda")
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    for _ in range(args.warmup):
        nsga3.sbx_pm(X, lo, hi, 20.0, 20.0, rs, rp, out=out, status=st)
    ms = _time_calls(lambda: nsga3.sbx_pm(X, lo, hi, 20.0, 20.0, rs, rp, out=out, status=st),
                     args.steps, torch.cuda.current_stream())
    var_bytes = 4.0 * (2 * h * d + h * d + 2 * h * d + 2 * h * d + 2 * d)
    idx = torch.randperm(2 * h, device="cuda", generator=g)[:h].to(torch.int32).contiguous()
    rows = torch.empty((h, d), device="cuda")
    for _ in range(args.warmup):
        nsga3.gather_rows(out, idx, out=rows, status=st)
    ms_g = _time_calls(lambda: nsga3.gather_rows(out, idx, out=rows, status=st), args.steps,
                       torch.cuda.current_stream())
    g_bytes = 4.0 * (2 * h * d + h)     # h rows read and written, indices read
    torch.cuda.synchronize()
    return {
        "workload": f"n={n} d={d}",
        "sbx_pm": {"ms": ms, "bytes": var_bytes, "achieved_GB_s": var_bytes / (ms / 1e3) / 1e9,
                   "frac_of_hbm_peak": var_bytes / (ms / 1e3) / 8e12, "status": int(st.item())},
        "gather": {"rows": h, "ms": ms_g, "bytes": g_bytes,
                   "achieved_GB_s": g_bytes / (ms_g / 1e3) / 1e9,
                   "frac_of_hbm_peak": g_bytes / (ms_g / 1e3) / 8e12},
    }


def c5_report(args):
    """Many-objective workload with float32 and bfloat16 association
    screening: whole-selection and association times, and each mode's
    association and selection against the float64 oracle."""
    import numpy as np
    import torch

    import oracle
    import paper_2503_20286_amd as nsga3
    import workloads
    w = workloads.make("many")
    objs = torch.from_numpy(w.objs).cuda()
    refs = torch.from_numpy(w.refs).cuda()
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    ref = oracle.select(w.objs, w.refs, w.K, with_counts=False)
    t_oracle = time.perf_counter() - t0
    out = {"workload": f"many: N={w.N} M={w.M} H={w.H} K={w.K}",
           "oracle_s_without_counts": t_oracle}
    sel = {}
    for name, mode in (("fp32", nsga3.ASSOC_FP32), ("bf16", nsga3.ASSOC_BF16)):
        ctx = nsga3.Context(0, assoc=mode)
        ctx.reserve(w.N, w.M, w.H)
        r = nsga3.select(objs, refs, w.K, ctx=ctx, want_counts=False)

        def call():
            nsga3.select(objs, refs, w.K, ctx=ctx, out=r, want_counts=False)
        for _ in range(args.warmup):
            call()
        ms = _time_calls(call, args.steps, stream)
        ph = _phase_pass(ctx, call, args.steps)
        g = _host(r)
        sel[name] = g["selected"]
        p = parity(w, g, ref)
        out[name] = {"ms_per_selection": ms, "associate_ms": ph["associate"],
                     "niche_mismatch_outside_ties": p["niche_outside_ties"],
                     "max_abs_dist_err": p["max_abs_dist_err"],
                     "rank_mismatch": p["rank"], "selected_mismatch": p["selected"],
                     "oracle_near_ties": p["near_ties"]}
        ctx.close()
    out["selection_identical_across_modes"] = bool(np.array_equal(sel["fp32"], sel["bf16"]))
    return out


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
    fields = ("selected", "rank", "niche", "dist", "dom_in", "dom_out")
    same = all(torch.equal(getattr(a, k), getattr(b, k)) for a, b in zip(plan.results, outs)
               for k in fields) and all(a.info() == b.info() for a, b in zip(plan.results, outs))
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

    def call():
        nsga3.select(objs, refs, w.K, ctx=ctx, out=out)

    t_host = time.perf_counter()
    ms_per_step = _time_calls(call, args.steps, stream)
    t_host = time.perf_counter() - t_host
    phases = _phase_pass(ctx, call, args.steps)
    g = _host(out)
    # the same selection without the optional dom_in / dom_out outputs: the
    # in-degrees are still computed (the peel needs them), the out-degrees,
    # which the selection never uses, are not
    lean = nsga3.select(objs, refs, w.K, ctx=ctx, want_counts=False)

    def call_lean():
        nsga3.select(objs, refs, w.K, ctx=ctx, out=lean)
    for _ in range(args.warmup):
        call_lean()
    lean_ms = _time_calls(call_lean, args.steps, stream)
    lean_same = bool(torch.equal(lean.selected, out.selected) and torch.equal(lean.rank, out.rank))

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
    valu = None
    if os.path.exists(COUNTERS_FILE):
        with open(COUNTERS_FILE) as fh:
            cn = json.load(fh)
        if cn.get("workload") == args.workload and cn.get("count_phase_valu_per_launch"):
            v = cn["count_phase_valu_per_launch"]
            valu = {"instructions_per_launch": v,
                    "frac_of_issue_peak": v / (t_dom * VALU_ISSUE_PER_S),
                    "source": os.path.relpath(COUNTERS_FILE, ROOT)}
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
            "kernel": "dominance counts (block bitsets: k_build_wide + k_fwd_all_wide, 128-member "
                      "tables, for 4 <= M <= 10; k_build_blocks + k_fwd_all, 64-member tables, "
                      "otherwise; out-degrees from the in-degree probes for M >= 4, a backward pass "
                      "k_bwd_all below)",
            "achieved": achieved,
            "peak": peak,
            "unit": "Tcmp/s",
            "frac": achieved / peak,
            "traffic": traffic,
            "work_per_launch": f"{cmp_per_launch:.4e} pair-objective compares (M*N*(N-1)/2: every "
                               "unordered pair decided once)",
            "note": "effective pair-decision rate: one block-bitset probe decides 64 or 128 pairs "
                    "with M key searches and M mask ANDs, so frac is not a VALU utilisation and can "
                    "exceed 1",
            "frac_counts_and_peeling": cmp_per_launch / ((phases["dominance_count"] + phases["peel"])
                                                          / 1e3) / PEAK_CMP_PER_S,
            # counted VALU instructions of the phase (rocprofv3 SQ_INSTS_VALU)
            # over this run's phase time against 1024 SIMDs x 2.4 GHz / 4
            "valu_issue": valu,
        },
        "phases_ms": phases,
        "without_count_outputs": {
            "ms_per_selection": lean_ms, "points_per_s": N / (lean_ms / 1e3),
            "same_selection_and_ranks": lean_same,
            "note": "dom_in and dom_out not requested (optional outputs): no out-degrees; the "
                    "headline value keeps every output"},
        "streaming_phases_gb_s": {
            # algorithmic HBM bytes of the streaming phases over their event time
            "prep_sort": N * M * 4 / (phases["prep_sort"] * 1e6),
            "associate": (N * M * 4 + w.H * M * 4 + 8 * N) / (phases["associate"] * 1e6),
            "niching_and_output": (w.K + 3 * N) * 4 / (phases["niching"] * 1e6),
        },
        "fronts": {"num_fronts": info.num_fronts, "last_front": info.last_front,
                   "last_front_size": info.last_front_size, "num_from_last": info.num_from_last,
                   "near_ties": info.near_ties, "intercept_fallback": info.intercept_fallback},
        "host_wall_s": t_host,
    }
    if not args.no_batch:
        res["batched"] = batched(args)
    ref = None
    if not args.no_cpu_baseline:
        res["cpu_baseline"], ref = cpu_baseline(w)
        res["parity"] = parity(w, g, ref)
    if not args.no_oneshot:
        res["oneshot_niching"] = oneshot_report(args, w, objs, refs, g, ref)
    if not args.no_rvea:
        res["rvea"] = rvea_report(args, w, objs, refs)
    if not args.no_hype and args.workload == "large":
        res["hype"] = hype_report(args)
    if not args.no_variation and args.workload == "large":
        res["variation"] = variation_report(args)
    if not args.no_c5 and args.workload == "large":
        res["c5"] = c5_report(args)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
