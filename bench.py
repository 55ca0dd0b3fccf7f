"""Benchmark: k-source shortest-path traversal + hybrid closeness estimate on one MI355X.

One step = one full estimate (sample draw, all k traversals, every estimator
of Sec. 2 for every node, outputs left in device memory) on a resident graph.
Default workload: undirected R-MAT scale 20 (a,b,c,d = .57,.19,.19,.05, edge
factor 16, duplicates and self-loops removed, largest connected component),
k = 256 samples, batched 64-samples-per-word BFS.

Prints ONE JSON line.  `value` = GTEPS of the batched path = k * m / t with m
the undirected edge count (each edge once) and t the wall time of one step.
Also reported: the plain one-sample-at-a-time GPU path, per-step latency
percentiles, the roofline of the dominant kernel (the batched traversal
kernel: algorithmic bytes / its HIP-event-timed duration), and the CPU oracle
timed on a bounded sample of the same workload.
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
METRIC = "GTEPS of k-source SSSP + hybrid estimate, batched vs plain; p99 job latency"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(xs, q):
    return float(np.percentile(np.asarray(xs), q)) if len(xs) else None


SCATTER_KERNEL = "k_scatter_level"


def bytes_per_arc(W: int) -> int:
    """Algorithmic bytes per arc of the scatter kernel: 4 B for the arc's end
    id + 8W B for the far end's seen mask (a pull gathers the neighbour's
    mask; a push reads the target's mask to drop bits it already has).  The
    one atomic OR per hub chunk, and the pushes' atomics, are left out."""
    return 4 + 8 * W


def source_digest() -> str:
    import hashlib
    with open(os.path.join(ROOT, "paper_1409_0035_amd", "csrc", "bfs_batched.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(workload: str, tuning: dict, path: str | None = None):
    """HBM bytes per launch of the scatter kernel from the committed rocprofv3
    FETCH_SIZE / WRITE_SIZE passes, each scaled by the same counter on a copy
    of known size; None once the kernel source has changed since, or when
    the run's launch knobs differ from the profiled ones."""
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
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(workload, tuning),
            "kernel": SCATTER_KERNEL, "algorithmic_bytes_per_launch": int(per_launch),
            "avg_launch_us": round(avg_ms * 1e3, 2), "launches_per_step": launches / len(timings),
            "bytes_per_arc": bytes_per_arc(W),
            "pull_levels_gbs": round(pull_arcs * bytes_per_arc(W) / (pull_ms / 1e3) / 1e9, 1) if pull_ms > 0 else None}


def cpu_baseline(g, k, seed, rg=None, budget_s=20.0):
    """The CPU oracle, as it stands, on a bounded sample of the same workload:
    a prefix of the k sources' searches (all host threads, over sources) and
    the literal Eq. (6) walk for a set of random nodes (all host threads, over
    nodes), each grown until it has taken about half of `budget_s`, then
    extrapolated to k sources and all n nodes, as GTEPS."""
    import concurrent.futures as cf
    import ctypes

    import oracle

    threads = min(os.cpu_count() or 1, 16)
    samples = oracle.draw_samples(g.n, k, seed)
    half = budget_s / 2
    # searches: one batch of `threads` sources to size the rest
    ks = min(k, threads)
    t0 = time.perf_counter()
    oracle.sample_distances(g, samples[:ks], threads=threads, reverse_graph=rg)
    t_batch = time.perf_counter() - t0
    ks = min(k, max(ks, int(ks * half / max(t_batch, 1e-3))))
    t0 = time.perf_counter()
    D = oracle.sample_distances(g, samples[:ks], threads=threads, reverse_graph=rg)
    t_search = time.perf_counter() - t0
    per_source = t_search / ks  # wall time per source with all threads busy

    lib = oracle._load()
    sidx = oracle.sample_index(g.n, samples[:ks])
    Dc = np.ascontiguousarray(D)

    def one_node(v):
        row = np.ascontiguousarray(Dc[v])
        p = int(lib.orc_pivot(ks, oracle._p(row)))
        o = oracle.NodeOut()
        col = Dc[:, p:]
        lib.orc_node_estimates(g.n, ks, int(v), oracle._p(sidx), oracle._p(row),
                               ctypes.c_void_p(col.ctypes.data), ks, 1, 10, ctypes.byref(o))
        return o.S_hyb

    rng = np.random.default_rng(seed)
    nodes_done, t_walk = 0, 0.0
    with cf.ThreadPoolExecutor(threads) as ex:
        batch = min(threads, g.n)
        while t_walk < half and nodes_done < g.n:
            nodes = rng.integers(0, g.n, size=batch)
            t1 = time.perf_counter()
            list(ex.map(one_node, nodes))
            dt = time.perf_counter() - t1
            t_walk += dt
            nodes_done += batch
            batch = min(g.n - nodes_done, max(batch, int(batch * (half - t_walk) / max(dt, 1e-3))))
    per_node = t_walk / nodes_done  # wall time per node with all threads busy
    t_total = k * per_source + g.n * per_node
    m = g.m if not g.directed else 2 * g.arcs
    return {
        "value": k * m / t_total / 1e9, "unit": "GTEPS", "cores": threads, "kind": "oracle",
        "sample": (f"{ks} of {k} sources' searches ({t_search:.1f} s) + literal Eq.6 walk for {nodes_done} "
                   f"random nodes ({t_walk:.1f} s), {threads} threads; extrapolated to k={k} sources and "
                   f"n={g.n} nodes: {t_total:.1f} s per estimate"),
    }


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
        "vs_baseline": None, "dtype": "u64 bitmask / u16 levels / int64 weighted sums", "data": "synthetic",
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
        order = cc.cc_draw_samples(g.n, g.n, seed)
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
        "vs_baseline": None, "dtype": "u64 bitmask / u16 levels / int64 sums", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {g.name} n={g.n} arcs={g.arcs} k={k} "
                               f"{'inbound' if args.inbound else 'outbound'}", "n": g.n, "arcs": g.arcs, "k": k},
        "device_ms": round(t["total_ms"], 3), "levels": t["levels"], "launches": t["launches"],
        "full_samples": full, "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat20")
    ap.add_argument("--plain-steps", type=int, default=2)
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="time eager estimates instead of replays of the captured estimate (CC_GRAPH, used by "
                         "default where it applies; the roofline then comes from extra eager steps)")
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
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the path shards by sample "
              "across GPUs by design but no multi-GPU run is part of this build", file=sys.stderr)
        sys.exit(2)

    import torch

    import graphgen
    import paper_1409_0035_amd as cc

    if args.reach:
        if args.workload == "rmat20":
            args.workload = "rmat20dir"
        if args.beta:
            return reach_weighted_bench(args, graphgen, cc, torch)
        return reach_bench(args, graphgen, cc, torch)
    if args.beta:
        return beta_bench(args, graphgen, cc, torch)

    spec = graphgen.WORKLOADS[args.workload]
    t0 = time.time()
    g = graphgen.workload(args.workload)
    k, seed = spec["k"], spec["sample_seed"]
    rg = graphgen.transpose(g) if g.directed else None
    m = g.m
    teps_edges = k * m * (2 if g.directed else 1)  # round trip: forward + reverse searches
    log(f"workload {args.workload}: n={g.n} m={m} arcs={g.arcs} k={k} (generated in {time.time() - t0:.1f}s)")

    dev = torch.device("cuda:0")
    ctx = cc.Context(0)
    gh = ctx.upload(g)
    out = {
        "S_hyb": torch.empty(g.n, dtype=torch.float64, device=dev),
        "S_samp": torch.empty(g.n, dtype=torch.float64, device=dev),
        "S_piv": torch.empty(g.n, dtype=torch.int64, device=dev),
        "S_pub": torch.empty(g.n, dtype=torch.int64, device=dev),
        "pivot": torch.empty(g.n, dtype=torch.int32, device=dev),
        "delta": torch.empty(g.n, dtype=torch.int32, device=dev),
        "sampsum": torch.empty(g.n, dtype=torch.int64, device=dev),
    }
    extra = {"hybrid": (), "errors": ("S_err", "S_ad", "S_ad_err"), "sweep": ("S_sweep", "S_sweep_err")}
    for f in extra[args.outputs]:
        out[f] = torch.empty(g.n, dtype=torch.float64, device=dev)
    stream = torch.cuda.current_stream()

    tuning = cc.cc_graph_get_tuning(gh)
    if args.tuning:
        fixed = {kv.split("=")[0]: int(kv.split("=")[1]) for kv in args.tuning.split(",") if kv}
        tuning = cc.cc_graph_set_tuning(gh, **fixed)
        log(f"tuning fixed: {tuning}")
    elif not args.no_autotune:
        t0 = time.time()
        tuning, tuned_ms = cc.cc_autotune(ctx.handle, gh, k, seed=seed, reps=3)
        log(f"autotune: {tuning} ({tuned_ms:.3f} ms) in {time.time() - t0:.1f}s")

    def step(mode):
        cc.cc_estimate_device(ctx.handle, gh, k, out, mode=mode, seed=seed, stream=stream)

    use_graph = not args.no_graph and not g.directed and g.w is None and k <= 256
    main_mode = cc.CC_BATCHED | (cc.CC_GRAPH if use_graph else 0)
    for i in range(args.warmup):
        step(main_mode)
    log(f"warmup done ({args.warmup} steps)")
    torch.cuda.synchronize()
    lat, kern_ms, timings = [], [], []
    t_start = time.perf_counter()
    for i in range(args.steps):
        a = time.perf_counter()
        step(main_mode)
        lat.append((time.perf_counter() - a) * 1e3)
        tm = cc.cc_last_timing(ctx.handle)
        timings.append(tm)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_per_step = wall * 1e3 / args.steps
    gteps = teps_edges / (ms_per_step / 1e3) / 1e9
    replayed = sum(1 for t in timings if t["launches"] == 1)
    log(f"batched{' (graph replays: %d)' % replayed if use_graph else ''}: {ms_per_step:.3f} ms/step, "
        f"{gteps:.1f} GTEPS")
    if use_graph:  # replays carry no per-launch timing: take it from eager steps
        timings = []
        for i in range(max(3, min(args.steps, 10))):
            step(cc.CC_BATCHED)
            timings.append(cc.cc_last_timing(ctx.handle))

    # roofline of the dominant kernel (the per-level scatter kernel), timed
    # live with HIP events on the stream it is launched on
    tm = timings[-1]
    W = (min(k, 256) + 63) // 64
    roofline = scatter_roofline(timings, W, args.workload, tuning)
    level_ms = float(np.median([t["kernel_ms"] for t in timings]))
    log(f"roofline: {roofline}")

    plain = None
    if not args.no_plain and args.plain_steps > 0:
        step(cc.CC_PLAIN)
        torch.cuda.synchronize()
        a = time.perf_counter()
        for _ in range(args.plain_steps):
            step(cc.CC_PLAIN)
        torch.cuda.synchronize()
        pms = (time.perf_counter() - a) * 1e3 / args.plain_steps
        plain = {"ms_per_step": round(pms, 3), "gteps": round(teps_edges / (pms / 1e3) / 1e9, 3)}
        log(f"plain: {pms:.3f} ms/step, {plain['gteps']} GTEPS")

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(g, k, seed, rg)
        log(f"cpu baseline: {cpu['value']:.4f} GTEPS")

    line = {
        "metric": METRIC, "value": round(gteps, 3), "unit": "GTEPS", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u64 bitmask / int32 dist / int64 sums",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {g.name} n={g.n} m={m} k={k} batched", "n": g.n, "m": m,
                   "k": k, "eps": f"1/{int(round(math.sqrt(k)))}", "graph_replay": use_graph,
                   "outputs": args.outputs},
        "latency_ms": {"p50": round(pct(lat, 50), 4), "p99": round(pct(lat, 99), 4)},
        "plain": plain,
        "speedup_vs_plain": None if plain is None else round(gteps / plain["gteps"], 2),
        "breakdown_ms": {"traverse": round(tm["traverse_ms"], 4), "epilogue": round(tm["epilogue_ms"], 4),
                         "level_kernels": round(level_ms, 4),
                         "scatter_kernel": round(float(np.median([t["scatter_ms"] for t in timings])), 4)},
        "tuning": tuning,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    if args.copy_calibration > 0:
        x = torch.ones(args.copy_calibration << 18, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        torch.mul(x, 1.0, out=y)
        torch.cuda.synchronize()
        log(f"copy calibration: {args.copy_calibration} MiB read + written by one elementwise kernel")
    ctx.close()


if __name__ == "__main__":
    main()
