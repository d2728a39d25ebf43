#!/usr/bin/env python3
"""Benchmark of the UST estimator of diag(L^+) on one MI355X.

One step = one full ApproxDiagLpinv run (BFS tree and sample size, all tau trees sampled
with Wilson's algorithm, Algorithm 2 aggregation, the pivot-column solve and the
combination) on a graph already resident in HBM.  Default workload: R-MAT scale 22 (edge
factor 16, Graph500 a/b/c/d), largest component, unit weights, max-degree pivot, eps = 0.3
(tau = 9475), Philox seed 1.

Prints one JSON line: trees/s end to end (`value`), walk steps/s of the sampler, the
end-to-end time, a roofline entry for the dominant kernel and the CPU oracle's rate on a
bounded sample of the same workload (one host thread, and all host threads over disjoint
tree ranges).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
# VALU issue peak: one wave64 instruction per SIMD every 4 cycles (16-lane SIMDs for 32-bit
# integer work), 256 CUs x 4 SIMDs at 2.4 GHz
VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4
WORKLOADS = {
    "rmat16": dict(kind="rmat", scale=16, ef=16, seed=1),
    # weighted graphs (Section "Generalizations"): R-MAT 16 with conductances uniform in [1, 4)
    "rmat16w": dict(kind="rmat", scale=16, ef=16, seed=1, weights=("uniform", 1, 1.0, 4.0)),
    "grid32": dict(kind="grid", side=32, tau=1000),
    "rmat18": dict(kind="rmat", scale=18, ef=16, seed=1),
    "rmat20": dict(kind="rmat", scale=20, ef=16, seed=1),
    "rmat22": dict(kind="rmat", scale=22, ef=16, seed=1),
    "rhg1m": dict(kind="rhg", n=1_000_000, deg=20.0, gamma=3.0, seed=1),
    "batch64": dict(kind="batch", count=64, tau_cap=4096),
}
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2006_13679_amd", "csrc", f)
                  for f in ("ustd_kernels.hip", "ustd_solve.hip", "ustd_blocks.hip", "ustd_kernels.hpp", "ustd_device.hpp")]


def kernel_source_digest() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def make_workload(name: str):
    from paper_2006_13679_amd import graphgen as gg

    w = WORKLOADS[name]
    if w["kind"] == "rmat":
        g = gg.rmat(w["scale"], w["ef"], w["seed"])
        return g, gg.max_degree_pivot(g), 0, dict(workload="rmat-scale%d-ef%d" % (w["scale"], w["ef"]),
                                                  generator_seed=w["seed"])
    if w["kind"] == "rhg":
        g = gg.hyperbolic(w["n"], w["deg"], w["gamma"], seed=w["seed"])
        return g, gg.max_degree_pivot(g), 0, dict(workload="rhg-n%d-deg%g-gamma%g" % (w["n"], w["deg"], w["gamma"]),
                                                  generator_seed=w["seed"])
    g = gg.grid2d(w["side"])
    return g, gg.grid_center_pivot(w["side"]), w["tau"], dict(workload="grid%dx%d" % (w["side"], w["side"]))


def algorithmic_bytes(n: int, tau: int, steps: int, farness: int) -> dict:
    """Bytes the method must move: 20 B per walk step (the landing vertex's column entry, row
    bounds, flag word and tree test) plus 12 B per vertex and tree for the commit (sampler);
    18 B per (vertex, B-path edge) pair plus 12 B per vertex and tree for Algorithm 2
    (aggregation)."""
    return dict(sample=20 * steps + 12 * n * tau, aggregate=(18 * farness + 12 * n) * tau)


def load_traffic(kernel: str, workload: str):
    path = os.path.join(ROOT, "profiles", "%s_%s_traffic.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    if t.get("kernel_src_digest") != kernel_source_digest():
        return None  # counters were taken on an older kernel
    return t


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """Host threads for the parallel oracle leg: the CPUs this process may run on, at most
    OMP_NUM_THREADS when the environment sets it (the GPU machine's CPU share)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, n)


def cpu_baseline(g, u, tau, seed, budget_s: float, w=None):
    """The oracle as it stands on a bounded sample of the workload, scaled to the full tau,
    plus one full FP64 solve: first single-threaded (as many trees as fit in `budget_s`), then
    with every host thread taking a contiguous range of further trees (about `budget_s` of work
    per thread; trees are independent and counts integers, so this is the same computation).
    With conductances w, the oracle's weighted walk, aggregation and solve (single-threaded)."""
    import oracle

    oracle.build()
    t0 = time.perf_counter()
    if w is None:
        x, it, rr = oracle.solve(g.row_ptr, g.col, u, tol=1e-12)
        _, parB, _ = oracle.bfs(g.row_ptr, g.col, u)
    else:
        x, it, rr = oracle.solve_weighted(g.row_ptr, g.col, w, u, tol=1e-12)
        _, _, rmax = oracle.bpath_resistance(g.row_ptr, g.col, w, u)
        k = oracle.fixed_shift(tau, rmax)
    t_solve = time.perf_counter() - t0
    done, t_trees, chunk = 0, 0.0, 1
    while t_trees < budget_s and done < tau:
        c = min(chunk, tau - done)
        t0 = time.perf_counter()
        if w is None:
            oracle.trees(g.row_ptr, g.col, u, seed, done, c, want_parents=False, parB=parB)
        else:
            oracle.trees_weighted(g.row_ptr, g.col, w, u, seed, done, c, k, want_parents=False)
        t_trees += time.perf_counter() - t0
        done += c
        chunk = min(chunk * 2, 512)
    per_tree = t_trees / done
    one = tau / (per_tree * tau + t_solve)
    out = {"value": one, "unit": "trees/s", "cores": 1, "kind": "oracle", "cpu_model": cpu_model(),
           "sample": "%d of %d trees (%.1f s) + one FP64 Jacobi-PCG solve (%.2f s), single-threaded C; "
                     "value = tau / (per-tree time * tau + solve time)" % (done, tau, t_trees, t_solve),
           "ms_per_tree": per_tree * 1e3}
    th = host_threads()
    if w is not None or th < 2:
        return out
    per_thread = max(1, min(int(budget_s / per_tree), (tau - 1) // th + 1))
    cnt = min(per_thread * th, tau)
    t0 = time.perf_counter()
    oracle.trees_threads(g.row_ptr, g.col, u, seed, 0, cnt, th, parB=parB)
    t_par = time.perf_counter() - t0
    allc = tau / (t_par / cnt * tau + t_solve)
    return {"value": allc, "unit": "trees/s", "cores": th, "kind": "oracle", "cpu_model": cpu_model(),
            "sample": "%d of %d trees over %d host threads, contiguous tree ranges (%.1f s wall) + one FP64 "
                      "Jacobi-PCG solve (%.2f s, one thread); value = tau / (wall per tree * tau + solve time)"
                      % (cnt, tau, th, t_par, t_solve),
            "ms_per_tree": t_par / cnt * 1e3, "single_thread": out}


def run_batch(args):
    """Config of 64 mixed graphs (32 R-MAT, 32 grids) with tau capped at 4096.  The schedule is
    tuned (ustd_batch_autotune; cached in the JSON file USTD_TUNE_CACHE names, when set), one
    execution of the planned batch is captured in a HIP graph, and one step = one replay of that
    graph: the whole estimator for all members (set-up, sampling, Algorithm 2, solves,
    combination).  The one-shot batch call and per-graph FP64 calls are timed beside it."""
    import numpy as np
    import torch

    from paper_2006_13679_amd import api
    from paper_2006_13679_amd import graphgen as gg

    w = WORKLOADS[args.workload]
    members = gg.batch_members(w["count"], w["tau_cap"])
    dev = torch.device("cuda:0")
    mode = api.SOLVE_MIXED if args.solve == "mixed" else api.SOLVE_FP64
    graphs = [api.Graph.from_host(m["graph"].row_ptr, m["graph"].col, device=dev) for m in members]
    probs = [api.problem(G, pivot=m["pivot"], eps=0.3, seed=m["seed"], tau_cap=m["tau_cap"], solve_mode=mode,
                         solve_tol=1e-12) for G, m in zip(graphs, members)]
    ws = api.Workspace(dev)
    print("bench: batch of %d graphs, n total %d" % (len(members), sum(m["graph"].n for m in members)),
          file=sys.stderr, flush=True)
    # the one-shot call (plan, one eager execution, reports), for reference
    api.batch_diag_lpinv(graphs, probs, ws=ws, want_counts=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d_ref, _, reps_ref = api.batch_diag_lpinv(graphs, probs, ws=ws, want_counts=False)
    torch.cuda.synchronize()
    ms_one_shot = (time.perf_counter() - t0) * 1e3
    print("bench: one-shot batch %.1f ms" % ms_one_shot, file=sys.stderr, flush=True)

    tt = time.perf_counter()
    if args.no_tune:
        sched, tuned_ms, hit = api.Schedule(), 0.0, False
    else:
        sched, tuned_ms, hit = api.batch_autotune(graphs, probs, ws=ws, cache_path=os.environ.get("USTD_TUNE_CACHE"),
                                                  graph=True)
    tune_s = time.perf_counter() - tt
    print("bench: tuned schedule %s (%.1f ms, %s) in %.1f s" % (sched.as_dict(), tuned_ms,
                                                               "cached" if hit else "timed", tune_s),
          file=sys.stderr, flush=True)
    tp = time.perf_counter()
    plan = api.BatchPlan(graphs, probs, ws=ws, schedule=sched, want_counts=False)
    ms_plan = (time.perf_counter() - tp) * 1e3
    plan.execute()  # eager execution: phase times
    reps_eager = plan.reports()
    plan.capture()
    for i in range(args.warmup):
        plan.replay()
        torch.cuda.synchronize()
        print("bench: warmup replay %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        plan.replay()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1e3 / args.steps
    print("bench: %d timed graph replays in %.3f s" % (args.steps, wall), file=sys.stderr, flush=True)
    reps = plan.reports()
    for i in range(len(members)):  # the replayed graph gives the one-shot call's results
        assert torch.equal(plan.diags[i], d_ref[i]) and reps[i]["walk_steps"] == reps_ref[i]["walk_steps"], i
    tau = sum(r["tau"] for r in reps)
    steps = sum(r["walk_steps"] for r in reps)
    ms_sample, ms_ag = reps_eager[0]["ms_sample"], reps_eager[0]["ms_aggregate"]
    ms_solve = sum(r["ms_solve"] for r in reps_eager)
    ms_bfs = sum(r["ms_bfs"] for r in reps_eager)
    # the same members one call each, FP64 solve (the plain per-graph form), one pass
    pws = api.Workspace(dev)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for G, p in zip(graphs, probs):
        q = api.Problem.from_buffer_copy(p)
        q.solve_mode = api.SOLVE_FP64
        api.diag_lpinv_p(G, q, ws=pws, want_counts=False)
    torch.cuda.synchronize()
    ms_single = (time.perf_counter() - t1) * 1e3
    ab = 0
    for i, (m, r) in enumerate(zip(members, reps)):
        dist, _, _, _ = api.bfs(graphs[i], probs[i], ws=pws)
        ab += algorithmic_bytes(m["graph"].n, r["tau"], r["walk_steps"], int(dist.sum().item()))["sample"]
    achieved = ab / (ms_sample * 1e-3) / 1e9
    out = {
        "metric": "spanning trees/sec + walk steps/sec; end-to-end diag(L\u2020) time at \u03b5=0.3",
        "value": round(tau / (ms_step * 1e-3), 2), "unit": "trees/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32+fp64" if mode == api.SOLVE_FP64 else "int32+fp32/fp64", "data": "synthetic",
        "config": {"workload": "batch-%d-mixed-rmat10to16-grid16to256-taucap%d" % (w["count"], w["tau_cap"]),
                   "members": w["count"], "tau_total": tau, "n_total": sum(m["graph"].n for m in members),
                   "eps": 0.3, "solve": args.solve, "step": "one replay of the captured HIP graph"},
        "tuned_schedule": sched.as_dict(),
        "tuner": ({"from_cache": hit, "ms_per_graph_replay": round(tuned_ms, 3), "tuning_s": round(tune_s, 2)}
                  if not args.no_tune else "off: default schedule"),
        "plan_ms": round(ms_plan, 2),
        "one_shot_ms": round(ms_one_shot, 3),
        "walk_steps_per_s": round(steps / (ms_sample * 1e-3), 1),
        "sampling_trees_per_s": round(tau / (ms_sample * 1e-3), 1),
        "e2e_ms_eager": round(reps_eager[0]["ms_total"], 4),
        "phase_ms_eager": {"setup_bfs_at_plan": ms_bfs, "sample": ms_sample, "aggregate": ms_ag,
                           "solve": ms_solve},
        "pool_fills": reps[0]["n_batches"], "walk_steps": steps,
        "per_graph_fp64_ms": round(ms_single, 3), "batched_speedup_vs_per_graph_fp64": round(ms_single / ms_step, 3),
        "roofline": {"bound": "hbm", "kernel": "wilson_kernel", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                     "algorithmic_bytes_per_launch": ab, "launch_ms": round(ms_sample, 4)},
    }
    plan.close()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_batch(members, reps, args.cpu_budget)
    print(json.dumps(out), flush=True)


def run_edges(args):
    """Spanning-edge counts of q trees on the workload (effective resistance of every edge to
    +-eps w.h.p.); one step = sampling the q trees and counting their edges."""
    import numpy as np
    import torch

    from paper_2006_13679_amd import api

    g, u, _, cfg = make_workload(args.workload)
    dev = torch.device("cuda:0")
    G = api.Graph.from_host(g.row_ptr, g.col, device=dev)
    q = api.edge_sample_size(g.n, g.m, 0.3, 0.0)
    p = api.problem(G, pivot=u, eps=0.3, seed=1, trees_per_batch=args.trees_per_batch)
    ws = api.Workspace(dev)
    counts = torch.zeros(G.nnz, dtype=torch.int64, device=dev)
    for _ in range(args.warmup):
        counts.zero_()
        api.edge_counts(G, p, 0, q, counts=counts, ws=ws)
    torch.cuda.synchronize()
    reps = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        counts.zero_()
        _, r = api.edge_counts(G, p, 0, q, counts=counts, ws=ws)
        reps.append(r)
    torch.cuda.synchronize()
    ms_step = (time.perf_counter() - t0) * 1e3 / args.steps
    med = lambda k: float(np.median([r[k] for r in reps]))  # noqa: E731
    steps = reps[0]["walk_steps"]
    ms_sample, ms_count = med("ms_sample"), med("ms_aggregate")
    ab = 20 * steps + 12 * g.n * q
    achieved = ab / (ms_sample * 1e-3) / 1e9
    out = {
        "metric": "spanning trees/sec for all-edge effective resistances (spanning-edge counts) at eps=0.3",
        "value": round(q / (ms_step * 1e-3), 2), "unit": "trees/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": dict(cfg, n=g.n, m=g.m, pivot=u, eps=0.3, q=q, seed=1, task="edges"),
        "walk_steps_per_s": round(steps / (ms_sample * 1e-3), 1),
        "phase_ms": {"setup_bfs": med("ms_bfs"), "sample": ms_sample, "edge_count": ms_count},
        "roofline": {"bound": "hbm", "kernel": "wilson_kernel", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": None,
                     "algorithmic_bytes_per_launch": ab, "launch_ms": round(ms_sample, 4)},
    }
    if not args.no_cpu_baseline:
        import oracle

        oracle.build()
        done, t_used, chunk = 0, 0.0, 8
        while t_used < args.cpu_budget and done < q:
            c = min(chunk, q - done)
            t1 = time.perf_counter()
            par, _, _ = oracle.trees(g.row_ptr, g.col, u, 1, done, c, want_counts=False)
            oracle.edge_counts(g.row_ptr, g.col, par, u)
            t_used += time.perf_counter() - t1
            done += c
            chunk = min(chunk * 2, 256)
        out["cpu_baseline"] = {"value": done / t_used, "unit": "trees/s", "cores": 1, "kind": "oracle",
                               "sample": "%d of %d trees with their edge counts (%.1f s), single-threaded" %
                                         (done, q, t_used)}
    print(json.dumps(out), flush=True)


def cpu_baseline_batch(members, reps, budget_s: float):
    """The oracle on a bounded sample of the batch: two trees of every member (scaled to its
    tau) and the solve of every eighth member (scaled by eight)."""
    import oracle

    oracle.build()
    est, t_used, trees_done = 0.0, 0.0, 0
    for i, (m, r) in enumerate(zip(members, reps)):
        g = m["graph"]
        c = 2 if t_used < budget_s else 1
        t0 = time.perf_counter()
        oracle.trees(g.row_ptr, g.col, r["pivot"], m["seed"], 0, c, want_parents=False)
        dt = time.perf_counter() - t0
        t_used += dt
        trees_done += c
        est += dt / c * r["tau"]
        if i % 8 == 0:
            t0 = time.perf_counter()
            oracle.solve(g.row_ptr, g.col, r["pivot"], tol=1e-12)
            dt = time.perf_counter() - t0
            t_used += dt
            est += 8 * dt
    tau = sum(r["tau"] for r in reps)
    return {"value": tau / est, "unit": "trees/s", "cores": 1, "kind": "oracle",
            "sample": "%d trees over the 64 members (each scaled to its tau) + the FP64 solves of 8 members "
                      "(each scaled by 8), %.1f s of single-threaded C; value = total tau / estimated time"
                      % (trees_done, t_used)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat22", choices=sorted(WORKLOADS))
    ap.add_argument("--solve", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--trees-per-batch", type=int, default=0)
    ap.add_argument("--pivot", default="workload", choices=["workload", "sweep"],
                    help="the workload's pivot (max degree, or the grid centre), or the double-sweep pivot "
                         "(pivot = -2: the smallest eccentricity bound after ten BFS sweeps, found on the device)")
    ap.add_argument("--cpu-budget", type=float, default=12.0, help="seconds of oracle work for cpu_baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--variant", default="plain", choices=["plain", "blocks"],
                    help="Wilson variant of the timed leg: plain (rooted at the pivot), or blocks (one walk "
                         "per biconnected component of the graph, joined at the cut vertices)")
    ap.add_argument("--no-tune", action="store_true",
                    help="batch workload: replay the default schedule (no autotuning)")
    ap.add_argument("--no-variant-compare", action="store_true",
                    help="skip the one-run comparison of the two Wilson variants")
    ap.add_argument("--task", default="diag", choices=["diag", "edges"],
                    help="diag: diag(L+) (default); edges: spanning-edge counts of q = ceil(2 eps^-2 ln(2m/delta)) "
                         "trees, the effective resistance of every edge")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only copy MIB mebibytes device to device (calibrates HBM byte counters) and exit")
    ap.add_argument("--gather-probe", type=int, default=0, metavar="MIB",
                    help="only gather 2^24 random 4-byte words from a MIB-mebibyte array and exit (HBM bytes the "
                         "counters report per random access)")
    args = ap.parse_args()

    if args.copy_probe:
        import torch

        nbytes = args.copy_probe << 20
        src = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes}), flush=True)
        return

    if args.gather_probe:
        import torch

        words = (args.gather_probe << 20) // 4
        src = torch.arange(words, dtype=torch.int32, device="cuda:0")
        g = torch.Generator(device="cuda:0").manual_seed(7)
        idx = torch.randint(0, words, (1 << 24,), device="cuda:0", generator=g)
        torch.cuda.synchronize()
        out = src[idx]
        torch.cuda.synchronize()
        print(json.dumps({"gather_probe_words": 1 << 24, "array_bytes": words * 4, "check": int(out[:4].sum())}),
              flush=True)
        return

    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (trees would shard by range "
              "across GPUs with one all-reduce of the integer counts)", file=sys.stderr)
        sys.exit(2)
    if WORKLOADS[args.workload]["kind"] == "batch":
        run_batch(args)
        return
    if args.task == "edges":
        run_edges(args)
        return

    import numpy as np
    import torch

    from paper_2006_13679_amd import api

    g, u, tau_override, cfg = make_workload(args.workload)
    dev = torch.device("cuda:0")
    wspec = WORKLOADS[args.workload].get("weights")
    w = None
    if wspec:
        from paper_2006_13679_amd import graphgen as gg

        kind, wseed, lo, hi = wspec
        w = gg.edge_weights(g, wseed, kind, lo, hi)
        cfg = dict(cfg, workload="%s-weighted-%s%gto%g" % (cfg["workload"], kind, lo, hi),
                   weights="%s[%g,%g) seed %d" % (kind, lo, hi, wseed))
    G = api.Graph.from_host(g.row_ptr, g.col, device=dev, weight=w)
    mode = api.SOLVE_MIXED if args.solve == "mixed" else api.SOLVE_FP64
    if args.pivot == "sweep":
        u = -2  # chosen on the device in every call (its BFS sweeps are part of the timed set-up)
        cfg = dict(cfg, workload=cfg["workload"] + "-sweep-pivot")
    variant = api.WILSON_BLOCKS if args.variant == "blocks" else api.WILSON_PLAIN
    if variant == api.WILSON_BLOCKS:
        cfg = dict(cfg, workload=cfg["workload"] + "-blocks")
    p = api.problem(G, pivot=u, eps=0.3, seed=1, tau_override=tau_override, solve_mode=mode, solve_tol=1e-12,
                    trees_per_batch=args.trees_per_batch, wilson_variant=variant)
    ws = api.Workspace(dev)
    print("bench: %s n=%d m=%d pivot=%d" % (cfg["workload"], g.n, g.m, u), file=sys.stderr, flush=True)

    reps = []
    for i in range(args.warmup):
        api.diag_lpinv_p(G, p, ws=ws, want_counts=False)
        print("bench: warmup %d done" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        _, _, rep = api.diag_lpinv_p(G, p, ws=ws, want_counts=False)
        reps.append(rep)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    print("bench: %d timed steps in %.3f s" % (args.steps, wall), file=sys.stderr, flush=True)

    ms_step = wall * 1e3 / args.steps
    tau = reps[0]["tau"]
    u = reps[0]["pivot"]
    steps = reps[0]["walk_steps"]
    med = lambda k: float(np.median([r[k] for r in reps]))  # noqa: E731
    ms_sample, ms_iv, ms_ag = med("ms_sample"), med("ms_intervals"), med("ms_aggregate")

    diag_t, _, _ = api.diag_lpinv_p(G, p, ws=ws, want_counts=False)
    torch.cuda.synchronize()
    tc = time.perf_counter()
    for _ in range(10):
        api.centralities(diag_t)
    torch.cuda.synchronize()
    ms_central = (time.perf_counter() - tc) * 1e3 / 10
    pu = api.problem(G, pivot=u, eps=0.3, seed=1)
    dist, _, _, _ = api.bfs(G, pu, ws=ws)  # farness of the pivot, for the algorithmic-byte count
    farness = int(dist.sum().item())
    ab = algorithmic_bytes(g.n, tau, steps, farness)
    phases = {"sample": ms_sample, "aggregate": ms_ag}
    dom = max(phases, key=phases.get)
    kname = {"sample": "wilson", "aggregate": "aggregate"}[dom]
    # one launch of either kernel per batch of trees: per-launch bytes over the mean launch time
    launches = max(1, reps[0]["n_batches"])
    achieved = ab[dom] / (phases[dom] * 1e-3) / 1e9
    traffic = load_traffic(kname, cfg["workload"])
    roof = {"bound": "hbm", "kernel": kname + "_kernel", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": (traffic["bytes_per_launch"] if traffic else None),
            "algorithmic_bytes_per_launch": ab[dom] // launches, "launch_ms": round(phases[dom] / launches, 4),
            "launches": launches}
    if traffic and traffic.get("measured_ms_per_launch"):
        roof["traffic_gbs"] = round(traffic["bytes_per_launch"] / (roof["launch_ms"] * 1e-3) / 1e9, 1)
    # instruction-issue roofline of the same kernel: VALU wave instructions per launch (rocprofv3
    # SQ_INSTS_VALU of the current kernels) over this run's mean launch time
    issue = None
    if traffic and traffic.get("valu_wave_insts_per_launch"):
        v = traffic["valu_wave_insts_per_launch"]
        rate = v / (roof["launch_ms"] * 1e-3)
        issue = {"bound": "valu_issue", "kernel": kname + "_kernel", "achieved": round(rate, 1), "peak": VALU_ISSUE_PEAK,
                 "unit": "wave64 VALU instructions/s", "frac": round(rate / VALU_ISSUE_PEAK, 4),
                 "valu_per_walk_step": round(v / max(steps / launches, 1), 3)}

    # the pivot column in both precisions (the same problem otherwise): iterations, time, the
    # true residual and how far the mixed-precision column and diagonal are from the FP64 ones
    # at identical counts (Eq. diag-comp: diag[v] - diag'[v] = 2 (x[v] - x'[v]) - (x[u] - x'[u]))
    cmp = {}
    xs = {}
    for name, md in (("fp64", api.SOLVE_FP64), ("mixed", api.SOLVE_MIXED)):
        q = api.Problem.from_buffer_copy(p)
        q.solve_mode = md
        x, r = api.solve_pivot_column(G, q, ws=ws)
        xs[name] = x.double()
        cmp[name] = {"ms": round(r["ms_solve"], 3), "iters": r["solve_iters"], "reliable_updates": r["solve_outer"],
                     "relres": r["solve_relres"], "target": r["solve_tol"]}
    dx = (xs["mixed"] - xs["fp64"])
    cmp["mixed_vs_fp64_x_rel_inf"] = float(dx.abs().max() / xs["fp64"].abs().max())
    dd = 2.0 * dx - dx[u]
    dd[u] = dx[u]
    cmp["mixed_vs_fp64_diag_rel_inf"] = float(dd.abs().max() / diag_t.abs().max())
    cmp["mixed_speedup"] = round(cmp["fp64"]["ms"] / max(cmp["mixed"]["ms"], 1e-9), 3)

    # the other Wilson variant, one warm and one timed run of the same problem: sampling time and
    # walk steps beside the timed leg's (the per-component walks take fewer steps; the estimate
    # they give differs from the timed leg's by the sampling error only)
    vcmp = None
    if not args.no_variant_compare and w is None:
        other = api.WILSON_PLAIN if variant == api.WILSON_BLOCKS else api.WILSON_BLOCKS
        q = api.Problem.from_buffer_copy(p)
        q.wilson_variant = other
        api.diag_lpinv_p(G, q, ws=ws, want_counts=False)
        torch.cuda.synchronize()
        tv = time.perf_counter()
        _, _, ro = api.diag_lpinv_p(G, q, ws=ws, want_counts=False)
        torch.cuda.synchronize()
        wall_o = (time.perf_counter() - tv) * 1e3
        names = {api.WILSON_PLAIN: "plain", api.WILSON_BLOCKS: "blocks"}
        vcmp = {names[variant]: {"ms_sample": round(ms_sample, 3), "walk_steps": steps, "ms_step": round(ms_step, 3),
                                 "sampling_trees_per_s": round(tau / (ms_sample * 1e-3), 1)},
                names[other]: {"ms_sample": round(ro["ms_sample"], 3), "walk_steps": ro["walk_steps"],
                               "ms_step": round(wall_o, 3),
                               "sampling_trees_per_s": round(tau / (ro["ms_sample"] * 1e-3), 1)}}
        vcmp["blocks_sample_speedup"] = round(vcmp["plain"]["ms_sample"] / max(vcmp["blocks"]["ms_sample"], 1e-9), 3)
        vcmp["blocks_step_ratio"] = round(vcmp["blocks"]["walk_steps"] / max(vcmp["plain"]["walk_steps"], 1), 4)

    out = {
        "metric": "spanning trees/sec + walk steps/sec; end-to-end diag(L†) time at ε=0.3",
        "value": round(tau / (ms_step * 1e-3), 2),
        "unit": "trees/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32+fp64" if mode == api.SOLVE_FP64 else "int32+fp32/fp64",
        "data": "synthetic",
        "config": dict(cfg, n=g.n, m=g.m, pivot=u, ecc=reps[0]["ecc"], eps=0.3, tau=tau, seed=1,
                       solve=args.solve, trees_per_batch=reps[0]["trees_per_batch"], wilson_variant=args.variant),
        "walk_steps_per_s": round(steps / (ms_sample * 1e-3), 1),
        "sampling_trees_per_s": round(tau / (ms_sample * 1e-3), 1),
        "e2e_ms": round(med("ms_total"), 4),
        # sample and aggregate sum each batch's launch spans (two pools overlap); the solve runs on a
        # side stream beside the sampling, so its span is wall time, not kernel time (solve_compare
        # has the solve alone)
        "phase_ms": {"setup_bfs": med("ms_bfs"), "sample": ms_sample, "aggregate": ms_ag,
                     "solve_span_overlapped": med("ms_solve"), "combine": med("ms_combine")},
        "walk_steps": steps, "walk_draws": reps[0]["walk_draws"],
        "solve_iters": reps[0]["solve_iters"], "solve_relres": reps[0]["solve_relres"],
        "roofline": roof,
        "issue_roofline": issue,
        "centralities_ms": round(ms_central, 4),
        "solve_compare": cmp,
    }
    if vcmp:
        out["wilson_variant_compare"] = vcmp
    if not args.no_cpu_baseline:
        print("bench: timing the CPU oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(g, u, tau, 1, args.cpu_budget, w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
