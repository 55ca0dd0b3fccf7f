"""Benchmark: k-source shortest-path traversal + hybrid closeness estimate on one MI355X.

One step = one full estimate (sample draw, all k traversals, every estimator
of Sec. 2 for every node, outputs left in device memory) on a resident graph.
Headline workload: directed R-MAT scale 22 (a,b,c,d = .57,.19,.19,.05, 16 arcs
per node, duplicates and self-loops removed, largest strongly connected
component), k = 128 samples, round-trip distances (a forward and a reverse
batched 64-samples-per-word BFS per sample group).

Prints ONE JSON line.  `value` = GTEPS of the batched path = 2 k arcs / t for
the round trip (k m / t for undirected graphs, m the edges counted once) with
t the wall time of one step.  Also reported: the plain one-sample-at-a-time
GPU path, per-step latency percentiles, the roofline of the dominant kernel
(algorithmic bytes / its HIP-event-timed duration), and the CPU oracle timed
on a bounded sample of the same workload.  Under "configs" the same figures
for the other workloads (Barabasi-Albert 10k with k = 64, with the oracle's
exact all-pairs time and the estimators' error; R-MAT scale 20 with k = 256;
the weighted 2048 x 2048 grid with k = 64) and the 512-job serving mix at
0.5, 0.8 and 1.0 of its burst capacity.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
ATOMIC_PEAK_GPS = 27.0  # random 64-bit atomic minima completed per second, device-wide (measured, see profiles/)
METRIC = "GTEPS of k-source SSSP + hybrid estimate, batched vs plain; p99 job latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


SCATTER_KERNEL = "k_scatter_level"
MERGE_KERNEL = "k_group_level"


def bytes_per_arc(W: int) -> int:
    """Algorithmic bytes per arc of the scatter kernel: 4 B for the arc's end
    id + 8W B for the far end's words (a pull gathers the neighbour's seen
    mask; a push reads the target's pending words, the bits already pushed to
    it).  The one atomic OR per hub chunk, and the pushes' atomics, are left
    out."""
    return 4 + 8 * W


def merge_bytes_per_node(W: int) -> int:
    """Algorithmic bytes per node slot of a live group in the merge kernel:
    the row bound (4 B), the node's seen mask in, its pending words and its
    next seen mask (the level's snapshot) out, 8W B each."""
    return 4 + 24 * W


def merge_roofline(timings, W: int) -> dict:
    """The merge kernel (one launch per level after the scatter launch): its
    own pulls (arcs scanned minus the scatter's) at 4 + 8W B per arc, plus
    4 + 24W B per node slot of the live groups, over the level batches' time
    minus the scatter launches' (so the launch gaps count against it)."""
    launches = sum(t["scatter_launches"] for t in timings)
    ms = sum(t["kernel_ms"] - t["scatter_ms"] for t in timings)
    if launches == 0 or ms <= 0:
        return {"kernel": MERGE_KERNEL, "achieved": None, "frac": None}
    arcs = sum(t["arcs_scanned"] - t["scatter_arcs"] for t in timings)
    nodes = sum(t["nodes_visited"] for t in timings)
    per_launch = (arcs * bytes_per_arc(W) + nodes * merge_bytes_per_node(W)) / launches
    avg_ms = ms / launches
    achieved = per_launch / (avg_ms / 1e3) / 1e9
    return {"kernel": MERGE_KERNEL, "algorithmic_bytes_per_launch": int(per_launch),
            "avg_launch_us": round(avg_ms * 1e3, 2), "achieved": round(achieved, 1), "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "arcs_per_launch": int(arcs / launches)}


def source_digest(name: str = "bfs_batched.hip") -> str:
    import hashlib
    with open(os.path.join(ROOT, "paper_1409_0035_amd", "csrc", name), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(workload: str, tuning: dict, path: str | None = None):
    """HBM bytes per launch of the scatter kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes, each scaled by the same counter on a copy
    of known size; None once the kernel source or the graph builder has
    changed since, or when the run's launch knobs differ from the profiled
    ones."""
    if path is None:
        path = os.path.join(ROOT, "profiles", f"{SCATTER_KERNEL}_{workload}_pmc.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:  # keys may hold a colon ("sha256[:16]")
                key, _, val = line[2:].partition(": ")
                vals[key.strip()] = val.strip().strip("`")
    if vals.get("bfs_batched.hip sha256[:16]") != source_digest():
        return None
    # the graph builder decides the hub prefix and the node order the kernel gathers in
    if vals.get("ccgpu.hip sha256[:16]") != source_digest("ccgpu.hip"):
        return None
    prof_tuning = vals.get("tuning", "")
    bfs_knobs = ("alpha", "level_blocks", "scatter_blocks")
    if prof_tuning != ",".join(f"{kn}={tuning[kn]}" for kn in bfs_knobs):
        return None
    try:
        return float(vals["scaled HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def scatter_roofline(timings, W: int, workload: str, tuning: dict) -> dict:
    """Per-launch algorithmic bytes / average launch duration of the scatter
    kernel (one launch per level), both from the library's own counters and
    HIP events on the launch stream."""
    launches = sum(t["scatter_launches"] for t in timings)
    ms = sum(t["scatter_ms"] for t in timings)
    if launches == 0 or ms <= 0:
        return {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
                "traffic": None, "kernel": SCATTER_KERNEL}
    arcs = sum(t["scatter_arcs"] for t in timings)
    per_launch = arcs * bytes_per_arc(W) / launches
    avg_ms = ms / launches
    achieved = per_launch / (avg_ms / 1e3) / 1e9
    pull_ms = sum(t["pull_scatter_ms"] for t in timings)
    pull_arcs = sum(t["hub_arcs"] for t in timings)
    traffic = measured_traffic(workload, tuning)
    level_ms = sum(t["kernel_ms"] for t in timings)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
            "kernel": SCATTER_KERNEL, "algorithmic_bytes_per_launch": int(per_launch),
            "avg_launch_us": round(avg_ms * 1e3, 2), "launches_per_step": launches / len(timings),
            "bytes_per_arc": bytes_per_arc(W),
            # the counters' bytes over the same launch time, beside the algorithmic figure
            "traffic_gbs": None if traffic is None else round(traffic / (avg_ms / 1e3) / 1e9, 1),
            "traffic_frac": None if traffic is None else round(traffic / (avg_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4),
            # the scatter launches' share of the level batches (the rest: the merge launches and gaps)
            "share_of_level_kernels": round(ms / level_ms, 3) if level_ms > 0 else None,
            # masks gathered (or pushed along) per second: a random-access rate, between the device's
            # measured 66 G/s for random loads that miss L2 and 261 G/s for ones that hit it
            "gathers_g_per_s": round(arcs / (ms / 1e3) / 1e9, 2),
            "pull_levels_gbs": round(pull_arcs * bytes_per_arc(W) / (pull_ms / 1e3) / 1e9, 1) if pull_ms > 0 else None,
            # the level's other kernel, beside the dominant one
            "merge": merge_roofline(timings, W)}


def cpu_baseline(g, k, seed, rg=None, budget_s=24.0, exact_all_pairs=False):
    """The CPU oracle, as it stands, on a bounded sample of the same workload,
    on the host's cores.  Its two stages are timed apart and extrapolated to
    the whole estimate: the k searches (BFS / Dijkstra, both directions for a
    digraph) on all host threads and on one, for a prefix of the sources; and
    the estimator for every node by the oracle's Algorithm 1 accounting
    (estimate_tails, O(nk + kn log n)) over that prefix's distance columns,
    scaled to k columns.  With exact_all_pairs, also one search from every
    node (the exact S of Eq. (1)), on all threads and on one; the exact sums
    are returned for the estimator-error report."""
    import oracle

    threads = os.cpu_count() or 1
    samples = np.asarray(oracle.draw_samples(g.n, k, seed), dtype=np.int32)
    m = g.m if not g.directed else 2 * g.arcs
    # all threads: a prefix of the sources grown to about a third of the budget
    ks = min(k, threads)
    t0 = time.perf_counter()
    oracle.sample_distances(g, samples[:ks], threads=threads, reverse_graph=rg)
    t_batch = time.perf_counter() - t0
    ks = min(k, max(ks, int(ks * (budget_s / 3) / max(t_batch, 1e-3)) // threads * threads))
    t0 = time.perf_counter()
    D = oracle.sample_distances(g, samples[:ks], threads=threads, reverse_graph=rg)
    t_search_T = (time.perf_counter() - t0) / ks
    # one thread: one or two sources
    k1 = 1 if t_search_T * threads > 2.0 else 2
    t0 = time.perf_counter()
    oracle.sample_distances(g, samples[:k1], threads=1, reverse_graph=rg)
    t_search_1 = (time.perf_counter() - t0) / k1
    # the estimator over the prefix's columns, on all threads and on one
    t0 = time.perf_counter()
    oracle.estimate_tails(g, samples[:ks], D=D, threads=threads, adaptive_eps=())
    t_est_T = (time.perf_counter() - t0) * k / ks
    t0 = time.perf_counter()
    oracle.estimate_tails(g, samples[:ks], D=D, threads=1, adaptive_eps=())
    t_est_1 = (time.perf_counter() - t0) * k / ks
    del D
    total_T = k * t_search_T + t_est_T
    total_1 = k * t_search_1 + t_est_1
    out = {
        "value": round(k * m / total_T / 1e9, 5), "unit": "GTEPS", "cores": threads, "kind": "oracle",
        "sample": (f"searches from {ks} of the {k} sources on {threads} threads and {k1} on one thread, and the "
                   f"oracle's Algorithm 1 estimator for all {g.n} nodes over those {ks} columns; extrapolated to "
                   f"{k} sources: {total_T:.2f} s per estimate on {threads} threads, {total_1:.1f} s on one"),
        "per_estimate_s": {"threads": threads, "searches": round(k * t_search_T, 3), "estimator": round(t_est_T, 3),
                           "total": round(total_T, 3)},
        "single_thread": {"value": round(k * m / total_1 / 1e9, 5), "searches_s": round(k * t_search_1, 3),
                          "estimator_s": round(t_est_1, 3), "total_s": round(total_1, 3)},
    }
    exact = None
    if exact_all_pairs:
        t0 = time.perf_counter()
        exact = oracle.exact_sums(g, threads=threads, reverse_graph=rg)
        tT = time.perf_counter() - t0
        t1 = None
        if tT * threads < 30.0:
            t0 = time.perf_counter()
            oracle.exact_sums(g, threads=1, reverse_graph=rg)
            t1 = time.perf_counter() - t0
        out["exact_all_pairs_s"] = {"threads": round(tT, 3), "single_thread": None if t1 is None else round(t1, 3)}
    return out, exact


def estimator_error(ctx, gh, g, k, seed, exact, cc):
    """Average relative error |S^ - S| / S of each estimator against the exact
    S (Eq. (1)), over every node and over 1000 random query nodes (as the
    paper's experiments report it), from the library's outputs."""
    res = cc.cc_estimate(ctx.handle, gh, k, seed=seed,
                         outputs=("S_hyb", "S_samp", "S_piv", "S_pub", "S_ad", "S_sweep"))
    res["S_hyb_eps_1/10"] = cc.cc_estimate(ctx.handle, gh, k, seed=seed, eps=(1, 10), outputs=("S_hyb",))["S_hyb"]
    S = exact.astype(np.float64)
    q = np.random.default_rng(1000 + seed).choice(g.n, size=min(1000, g.n), replace=False)
    names = {"S_samp": "sampling", "S_piv": "pivoting", "S_pub": "pivoting upper bound",
             "S_hyb": f"hybrid eps=1/{int(round(math.sqrt(k)))}", "S_hyb_eps_1/10": "hybrid eps=1/10",
             "S_ad": "adaptive eps (Sec. 4)", "S_sweep": "threshold sweep (Algorithm 2)"}
    out = {}
    for f, label in names.items():
        e = np.abs(res[f].astype(np.float64) - S) / S
        out[label] = {"all_nodes": round(float(e.mean()), 5), "1000_queries": round(float(e[q].mean()), 5)}
    return out


def beta_bench(args, graphgen, cc, torch):
    """Sec. 5 for every node: K timed node-weighted estimates (weighted sample
    drawn on the host, k traversals, distance rows, beta-weighted tables and
    estimate) after W warm-up ones; value = k * m / t as for the headline."""
    spec = graphgen.WORKLOADS[args.workload]
    g = graphgen.workload(args.workload)
    k, seed = spec["k"], spec["sample_seed"]
    beta = graphgen.node_weights(g.n, seed)
    log(f"workload {args.workload}: n={g.n} m={g.m} k={k}, {int((beta > 0).sum())} nodes of positive weight")
    ctx = cc.Context(0)
    gh = ctx.upload(g)
    for _ in range(args.warmup):
        cc.cc_estimate_weighted(ctx.handle, gh, beta, k, seed=seed)
    torch.cuda.synchronize()
    ms = []
    for _ in range(args.steps):
        a = time.perf_counter()
        res = cc.cc_estimate_weighted(ctx.handle, gh, beta, k, seed=seed)
        ms.append((time.perf_counter() - a) * 1e3)
    mean_ms = float(np.mean(ms))
    edges = k * g.m * (2 if g.directed else 1)
    line = {
        "metric": "node-weighted hybrid estimate (Sec. 5), GTEPS of the k-source traversal plus weighted epilogue",
        "value": round(edges / (mean_ms / 1e3) / 1e9, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(mean_ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64 bitmask / int32 dist / int64 weighted sums", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {g.name} n={g.n} m={g.m} k={k} node weights 1+floor(10 U^-0.7), "
                               "20% zero", "n": g.n, "m": g.m, "k": k, "sample_size": res["sample_size"],
                   "tau": res["tau"]},
        "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def reach_weighted_bench(args, graphgen, cc, torch):
    """Sec. 6.2 / Algorithm 5 for every node (priority ranks from heavy-tailed
    integer node weights, 20% zeros): K timed estimates after W warm-up ones."""
    spec = graphgen.WORKLOADS[args.workload]
    g = graphgen.workload(args.workload)
    k, seed = spec["k"], spec["sample_seed"]
    beta = graphgen.node_weights(g.n, seed)
    log(f"workload {args.workload}: n={g.n} arcs={g.arcs} k={k}, {int((beta > 0).sum())} nodes of positive weight")
    ctx = cc.Context(0)
    gh = ctx.upload(g)
    for _ in range(args.warmup):
        cc.cc_reach_weighted(ctx.handle, gh, beta, k, inbound=args.inbound, seed=seed)
    ms, t = [], None
    for _ in range(args.steps):
        a = time.perf_counter()
        res = cc.cc_reach_weighted(ctx.handle, gh, beta, k, inbound=args.inbound, seed=seed)
        ms.append((time.perf_counter() - a) * 1e3)
        t = cc.cc_last_timing(ctx.handle)
    mean_ms = float(np.mean(ms))
    line = {
        "metric": "node-weighted reachability sampling (Sec. 6.2, Algorithm 5), nodes estimated per second",
        "value": round(g.n / (mean_ms / 1e3), 1), "unit": "nodes/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(mean_ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 bitmask / u16 levels / int64 weighted sums" if g.w is None else "u64 distance words / int64 weighted sums",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {g.name} n={g.n} arcs={g.arcs} k={k} "
                               f"{'inbound' if args.inbound else 'outbound'}, node weights 1+floor(10 U^-0.7), 20% zero",
                   "n": g.n, "arcs": g.arcs, "k": k},
        "device_ms": round(t["total_ms"], 3), "levels": t["levels"], "launches": t["launches"],
        "full_samples": int((res["count"] == k).sum()), "cpu_baseline": None,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def reach_bench(args, graphgen, cc, torch):
    """Sec. 6.2 / Algorithm 4 for every node: K timed estimates after W
    warm-up ones on a resident graph; value = nodes estimated per second."""
    import oracle
    spec = graphgen.WORKLOADS[args.workload]
    t0 = time.time()
    g = graphgen.workload(args.workload)
    k, seed = spec["k"], spec["sample_seed"]
    log(f"workload {args.workload}: n={g.n} arcs={g.arcs} k={k} (generated in {time.time() - t0:.1f}s)")
    ctx = cc.Context(0)
    gh = ctx.upload(g)
    outs = ("count", "distsum", "T", "B", "R")
    for _ in range(args.warmup):
        cc.cc_reach_estimate(ctx.handle, gh, k, inbound=args.inbound, seed=seed, outputs=outs)
    torch.cuda.synchronize()
    ms, tims = [], []
    for _ in range(args.steps):
        a = time.perf_counter()
        res = cc.cc_reach_estimate(ctx.handle, gh, k, inbound=args.inbound, seed=seed, outputs=outs)
        ms.append((time.perf_counter() - a) * 1e3)
        tims.append(cc.cc_last_timing(ctx.handle))
    torch.cuda.synchronize()
    mean_ms = float(np.mean(ms))
    t = tims[-1]
    full = int((res["count"] == k).sum())
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle on a bounded sample of nodes (one search each), scaled to nodes per second
        order = oracle.draw_samples(g.n, g.n, seed)
        rg = graphgen.transpose(g) if args.inbound else None
        rng = np.random.default_rng(0)
        nodes, done, t_cpu, threads = [], 0, 0.0, os.cpu_count() or 1
        while t_cpu < 15.0 and done < g.n:
            batch = rng.integers(0, g.n, size=max(threads, 16)).astype(np.int32)
            a = time.perf_counter()
            oracle.reach_all(g, order, k, inbound=args.inbound, threads=threads, reverse_graph=rg, nodes=batch)
            t_cpu += time.perf_counter() - a
            done += len(batch)
        cpu = {"value": round(done / t_cpu, 3), "unit": "nodes/s", "cores": threads, "kind": "oracle",
               "sample": f"{done} random nodes, one search each, {t_cpu:.1f} s"}
        log(f"cpu baseline: {cpu}")
    line = {
        "metric": "reachability sampling (Sec. 6.2, Algorithm 4), nodes estimated per second",
        "value": round(g.n / (mean_ms / 1e3), 1), "unit": "nodes/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(mean_ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64 bitmask / u16 levels / int64 sums" if g.w is None else "u64 distance words / int64 sums",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {g.name} n={g.n} arcs={g.arcs} k={k} "
                               f"{'inbound' if args.inbound else 'outbound'}", "n": g.n, "arcs": g.arcs, "k": k,
                   "arc_lengths": g.w is not None},
        "device_ms": round(t["total_ms"], 3), "levels": t["levels"], "launches": t["launches"],
        "arcs_relaxed": t["arcs_scanned"] if g.w is not None else None,
        "full_samples": full, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def wsearch_roofline(timings, workload: str, n: int, arcs: int, k: int, tuning: dict) -> dict:
    """Per-launch algorithmic bytes / average launch duration of the weighted
    searches' kernel (one launch of one workgroup per sample).  Algorithmic
    bytes are those of a label-setting search that takes every node once and
    relaxes every arc once: 16 B per node (its distance word and its two row
    bounds) and 16 B per arc (its packed end and length, and the far end's
    8-byte word), k (n + arcs) x 16 per launch on a connected graph.  The
    device's own counts of nodes taken and arcs relaxed give the re-work of
    the Delta-stepping phases beside it."""
    launches = sum(t["kernel_launches"] for t in timings)
    ms = sum(t["kernel_ms"] for t in timings)
    if launches == 0 or ms <= 0:
        return {"bound": "hbm", "achieved": None, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": None,
                "traffic": None, "kernel": "k_wsearch"}
    per = 16 * k * (n + arcs) * len(timings) / launches
    achieved = per / (ms / launches / 1e3) / 1e9
    relaxed = sum(t["arcs_scanned"] for t in timings) / len(timings)
    taken = sum(t["nodes_visited"] for t in timings) / len(timings)
    return {"bound": "hbm", "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 5),
            "traffic": measured_traffic_kernel("k_wsearch", workload, "sssp_weighted.hip", f"delta={tuning['delta']}"),
            "kernel": "k_wsearch", "algorithmic_bytes_per_launch": int(per),
            "avg_launch_us": round(ms / launches * 1e3, 1), "launches_per_step": launches / len(timings),
            "bytes_per_node_and_arc": 16, "relaxations_per_arc": round(relaxed / (k * arcs), 4),
            "takes_per_node": round(taken / (k * n), 4),
            "relaxations_per_s": round(relaxed / (ms / len(timings) / 1e3) / 1e9, 3),
            # every relaxation is one atomic minimum and every take one atomic AND: against the device's
            # measured rate of random 64-bit atomics (profiles/atomic_rate_probe.md)
            "atomics_g_per_s": round((relaxed + taken) / (ms / len(timings) / 1e3) / 1e9, 3),
            "atomic_peak_g_per_s": ATOMIC_PEAK_GPS,
            "atomic_frac": round((relaxed + taken) / (ms / len(timings) / 1e3) / 1e9 / ATOMIC_PEAK_GPS, 4)}


def measured_traffic_kernel(kernel: str, workload: str, source: str, tuning: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    passes (profiles/<kernel>_<workload>_pmc.md), None once `source` has
    changed since or when the run's knobs (`tuning`) differ from the
    profiled ones."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_pmc.md")
    if not os.path.exists(path):
        return None
    with open(os.path.join(ROOT, "paper_1409_0035_amd", "csrc", source), "rb") as f:
        digest = hashlib.sha256(f.read()).hexdigest()[:16]
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ": " in line:
                key, _, val = line[2:].partition(": ")
                vals[key.strip()] = val.strip().strip("`")
    if vals.get(f"{source} sha256[:16]") != digest or vals.get("tuning") != tuning:
        return None
    try:
        return float(vals["scaled HBM bytes per launch"])
    except (KeyError, ValueError):
        return None


def run_config(name, cc, graphgen, torch, steps, warmup, plain_steps, autotune=True, fixed_tuning=None,
               outputs="hybrid", keep=False, graph=True):
    """One workload: K timed estimates into device memory after W warm-up ones
    (replays of the captured estimate where that applies), the dominant
    kernel's roofline from extra eager steps, and the plain one-source-at-a-
    time path.  Returns the summary (and, with keep, the context and graph)."""
    spec = graphgen.WORKLOADS[name]
    t0 = time.time()
    g = graphgen.workload(name)
    k, seed = spec["k"], spec["sample_seed"]
    edges = k * g.m * (2 if g.directed else 1)  # round trip: forward + reverse searches
    log(f"workload {name}: n={g.n} m={g.m} arcs={g.arcs} k={k} (generated in {time.time() - t0:.1f}s)")
    dev = torch.device("cuda:0")
    ctx = cc.Context(0)
    gh = ctx.upload(g)
    out = {f: torch.empty(g.n, dtype=dt, device=dev) for f, dt in
           (("S_hyb", torch.float64), ("S_samp", torch.float64), ("S_piv", torch.int64), ("S_pub", torch.int64),
            ("pivot", torch.int32), ("delta", torch.int32), ("sampsum", torch.int64))}
    extra = {"hybrid": (), "errors": ("S_err", "S_ad", "S_ad_err"), "sweep": ("S_sweep", "S_sweep_err")}
    for f in extra[outputs]:
        out[f] = torch.empty(g.n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()
    tuning = cc.cc_graph_get_tuning(gh)
    if fixed_tuning:
        tuning = cc.cc_graph_set_tuning(gh, **fixed_tuning)
    elif autotune:
        t0 = time.time()
        tuning, tuned_ms = cc.cc_autotune(ctx.handle, gh, k, seed=seed, reps=3 if g.w is None else 1)
        log(f"  autotune: {tuning} ({tuned_ms:.3f} ms) in {time.time() - t0:.1f}s")

    def step(mode):
        cc.cc_estimate_device(ctx.handle, gh, k, out, mode=mode, seed=seed, stream=stream)

    use_graph = graph and k <= 256
    main_mode = cc.CC_BATCHED | (cc.CC_GRAPH if use_graph else 0)
    for _ in range(warmup):
        step(main_mode)
    torch.cuda.synchronize()
    lat, timings = [], []
    t_start = time.perf_counter()
    for _ in range(steps):
        a = time.perf_counter()
        step(main_mode)
        lat.append((time.perf_counter() - a) * 1e3)
        timings.append(cc.cc_last_timing(ctx.handle))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = wall * 1e3 / steps
    gteps = edges / (ms_per_step / 1e3) / 1e9
    replayed = sum(1 for t in timings if t["launches"] == 1)
    log(f"  batched{' (graph replays: %d)' % replayed if use_graph else ''}: {ms_per_step:.3f} ms/step, "
        f"{gteps:.1f} GTEPS")
    if use_graph:  # replays carry no per-launch timing: take it from eager steps
        timings = []
        for _ in range(max(3, min(steps, 10))):
            step(cc.CC_BATCHED)
            timings.append(cc.cc_last_timing(ctx.handle))
    tm = timings[-1]
    if g.w is None:
        W = (min(k, 256) + 63) // 64
        roofline = scatter_roofline(timings, W, name, tuning)
    else:
        roofline = wsearch_roofline(timings, name, g.n, g.arcs, k, tuning)
    log(f"  roofline: {roofline}")
    plain = None
    if plain_steps > 0:
        a = time.perf_counter()
        step(cc.CC_PLAIN)
        torch.cuda.synchronize()
        first = time.perf_counter() - a
        reps = 1 if first > 2.0 else plain_steps
        a = time.perf_counter()
        for _ in range(reps):
            step(cc.CC_PLAIN)
        torch.cuda.synchronize()
        pms = (time.perf_counter() - a) * 1e3 / reps
        plain = {"ms_per_step": round(pms, 3), "gteps": round(edges / (pms / 1e3) / 1e9, 3), "steps": reps}
        log(f"  plain: {pms:.3f} ms/step, {plain['gteps']} GTEPS")
    summary = {
        "workload": f"{name}: {g.name} n={g.n} m={g.m} arcs={g.arcs} k={k}", "n": g.n, "m": g.m, "arcs": g.arcs,
        "k": k, "eps": f"1/{int(round(math.sqrt(k)))}", "round_trip": bool(g.directed), "weighted": g.w is not None,
        "steps": steps, "ms_per_step": round(ms_per_step, 4), "gteps": round(gteps, 3),
        "teps_edges_per_step": edges, "graph_replay": use_graph and replayed > 0,
        "latency_ms": {"p50": round(pct(lat, 50), 4), "p99": round(pct(lat, 99), 4)},
        "plain": plain, "speedup_vs_plain": None if plain is None else round(gteps / plain["gteps"], 2),
        "breakdown_ms": {"traverse": round(tm["traverse_ms"], 4), "epilogue": round(tm["epilogue_ms"], 4),
                         "level_kernels": round(float(np.median([t["kernel_ms"] for t in timings])), 4)},
        "levels": tm["levels"], "tuning": tuning, "roofline": roofline,
    }
    if keep:
        return summary, ctx, gh, g
    ctx.close()
    return summary


def serving_config(args, graphgen):
    """The serving mix: 512 Poisson-arriving BA / R-MAT jobs (n log-uniform in
    [1e3, 1e6], k in {16, 64, 256}) against resident graphs, at offered loads
    of 0.5, 0.8 and 1.0 times the measured burst capacity."""
    from paper_1409_0035_amd import serve
    t0 = time.time()
    jobs, graphs = serve.build_mix(args.serve_jobs, seed=5, n_lo=1e3, n_hi=1e6,
                                   threads=min(os.cpu_count() or 1, 16))
    log(f"serving mix: {len(jobs)} graphs generated in {time.time() - t0:.1f}s")
    res = serve.serve(jobs, graphs, load=[0.5, 0.8, 1.0], seed=5)
    res["workload"] = (f"serving mix: {len(jobs)} Poisson-arriving BA (4 edges per node) / R-MAT (edge factor 16) "
                       f"jobs, n log-uniform in [1e3, 1e6], k in {{16, 64, 256}}, eps = 1/round(sqrt(k))")
    res["alone_p99_ratio_at_0.8"] = round(res["loads"][1]["latency_ms"]["p99"] / res["service_alone_ms"]["p99"], 3)
    log(f"serving: {json.dumps(res)}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat22dir",
                    help="the headline workload (default: directed R-MAT scale 22, round trip, k = 128)")
    ap.add_argument("--only", action="store_true",
                    help="time the headline workload only (no other configurations, no serving mix)")
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--serve-jobs", type=int, default=512)
    ap.add_argument("--no-graph", action="store_true",
                    help="eager estimates only: no captured-graph replays (counter passes per launch)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="keep the default launch shapes instead of running the library's autotuner first")
    ap.add_argument("--tuning", default="",
                    help="fixed knobs instead of the autotuner, e.g. alpha=4,level_blocks=2048")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="after the run, launch one float32 copy kernel of MIB MiB (read MIB, write MIB) so "
                         "that counter passes can scale FETCH_SIZE / WRITE_SIZE")
    ap.add_argument("--outputs", choices=("hybrid", "errors", "sweep"), default="hybrid",
                    help="what each step computes besides the Sec. 2 estimates: nothing (default), the Sec. 4 "
                         "error estimates and adaptive estimate, or the threshold sweep of Algorithm 2")
    ap.add_argument("--reach", action="store_true",
                    help="time the outbound reachability sampling of Sec. 6.2 (Algorithm 4) on the workload "
                         "(default rmat20dir) instead of the hybrid estimate, and print its own JSON line")
    ap.add_argument("--inbound", action="store_true", help="with --reach: inbound instead of outbound")
    ap.add_argument("--beta", action="store_true",
                    help="time the node-weighted hybrid estimate of Sec. 5 (heavy-tailed integer node weights, "
                         "20%% zeros) on the workload and print its own JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU (asked for --gpus {args.gpus}): the estimate shards by sample "
              "across GPUs by design, but only its one-GPU path is implemented", file=sys.stderr)
        sys.exit(2)

    import torch

    import graphgen
    import paper_1409_0035_amd as cc

    if args.reach:
        if args.workload == "rmat22dir":
            args.workload = "rmat20dir"
        if args.beta:
            return reach_weighted_bench(args, graphgen, cc, torch)
        return reach_bench(args, graphgen, cc, torch)
    if args.beta:
        if args.workload == "rmat22dir":
            args.workload = "rmat20"
        return beta_bench(args, graphgen, cc, torch)

    fixed = {kv.split("=")[0]: int(kv.split("=")[1]) for kv in args.tuning.split(",") if kv} or None
    plain_steps = 0 if args.no_plain else args.plain_steps
    # ---- the headline workload
    head, hctx, hgh, hg = run_config(args.workload, cc, graphgen, torch, args.steps, args.warmup, plain_steps,
                                     autotune=not args.no_autotune, fixed_tuning=fixed, outputs=args.outputs,
                                     keep=True, graph=not args.no_graph)
    spec = graphgen.WORKLOADS[args.workload]
    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        rg = graphgen.transpose(hg) if hg.directed else None
        cpu, _ = cpu_baseline(hg, spec["k"], spec["sample_seed"], rg)
        log(f"cpu baseline: {cpu}")
    hctx.close()
    del hg
    # ---- the other configurations
    configs = {}
    if not args.only:
        for name, steps in (("ba10k", 50), ("rmat20", 20), ("grid2048w", 5)):
            if name == args.workload:
                continue
            keep = name == "ba10k"
            # the weighted searches keep the library's default bucket width (1.5 x the mean length):
            # the autotuner's one-shot timings of nearby widths differ by less than their noise
            r = run_config(name, cc, graphgen, torch, steps, 3 if name != "grid2048w" else 1, plain_steps,
                           keep=keep, autotune=name != "grid2048w")
            if keep:
                r, bctx, bgh, bg = r
                if not args.no_cpu_baseline:
                    spec1 = graphgen.WORKLOADS[name]
                    c1, exact = cpu_baseline(bg, spec1["k"], spec1["sample_seed"], budget_s=6.0,
                                             exact_all_pairs=True)
                    r["cpu_oracle"] = c1
                    r["estimator_error"] = estimator_error(bctx, bgh, bg, spec1["k"], spec1["sample_seed"], exact, cc)
                    log(f"  estimator error: {r['estimator_error']}")
                bctx.close()
            configs[name] = r
        if not args.no_serving:
            configs["serving"] = serving_config(args, graphgen)

    line = {
        "metric": METRIC, "value": head["gteps"], "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": head["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64 bitmask / int32 dist / int64 sums", "data": "synthetic",
        "config": {"workload": head["workload"] + (" round trip" if head["round_trip"] else "") + " batched",
                   "n": head["n"], "m": head["m"], "arcs": head["arcs"], "k": head["k"], "eps": head["eps"],
                   "graph_replay": head["graph_replay"], "outputs": args.outputs},
        "latency_ms": head["latency_ms"], "plain": head["plain"], "speedup_vs_plain": head["speedup_vs_plain"],
        "breakdown_ms": head["breakdown_ms"], "tuning": head["tuning"],
        "roofline": head["roofline"], "cpu_baseline": cpu, "configs": configs,
    }
    print(json.dumps(line), flush=True)
    if args.copy_calibration > 0:
        dev = torch.device("cuda:0")
        x = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + written by one elementwise kernel")


if __name__ == "__main__":
    main()
