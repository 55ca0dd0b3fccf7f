"""Serving driver: closeness-estimate jobs arriving over time against graphs
kept resident on the device.

Each job names a resident graph, k and a sample seed.  Jobs arrive as a
Poisson process; the library's service admits a queued job as soon as a slot
(``max_inflight``) and its memory need (within ``mem_budget_bytes``) are free,
and runs admitted jobs concurrently, one stream each, so the work of a job
that arrives while others run overlaps theirs on the device.  Latency is the
library's own submit->done clock per job; p50/p99 are over all jobs.

Offered load is a fraction of the measured burst capacity: every job is
first run once on its own (this also warms every graph and gives each job's
service time alone), then all jobs are submitted at once, and the rate at
which that burst completes is the capacity; arrivals are then drawn at
``load x capacity`` jobs per second for each requested load.

    python -m paper_1409_0035_amd.serve --jobs 512 --load 0.8
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import paper_1409_0035_amd as cc  # noqa: E402

OUTPUTS = ("S_hyb", "S_samp", "pivot", "delta")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def percentile(xs, q):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q)) if len(xs) else None


def arrival_times(num_jobs: int, rate: float, seed: int) -> np.ndarray:
    """Poisson arrivals: exponential gaps with mean 1/rate seconds, first job at 0."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=num_jobs)
    gaps[0] = 0.0
    return np.cumsum(gaps)


def edges_traversed(g, k: int) -> int:
    """Edges counted for TEPS: k searches over m undirected edges, or over
    every arc twice (forward and reverse) for a digraph."""
    return k * (2 * g.arcs if g.directed else g.m)


def run_alone(ctx, handles, graphs, jobs, outputs=OUTPUTS):
    """Every job on its own through the synchronous call; returns the results
    and per-job service times (ms)."""
    res, times = [], []
    for j, job in enumerate(jobs):
        t0 = time.perf_counter()
        r = cc.cc_estimate(ctx.handle, handles[job["graph"]], job["k"], seed=job["sample_seed"], outputs=outputs)
        times.append((time.perf_counter() - t0) * 1e3)
        res.append(r)
    return res, times


def run_stream(ctx, handles, jobs, arrivals, outputs=OUTPUTS):
    """Submit each job at its arrival time (seconds from the start), then wait
    for all.  Returns results, per-job (queue_ms, total_ms) and the makespan."""
    pending = []
    t0 = time.perf_counter()
    for job, t_arr in zip(jobs, arrivals):
        while True:
            now = time.perf_counter() - t0
            if now >= t_arr:
                break
            time.sleep(min(t_arr - now, 0.002))
        pending.append(cc.cc_submit(ctx.handle, handles[job["graph"]], job["k"], seed=job["sample_seed"],
                                    outputs=outputs))
    results, lat = [], []
    for h in pending:
        results.append(cc.cc_wait(h))
        lat.append(cc.cc_job_times(h))
    makespan = time.perf_counter() - t0
    for h in pending:
        cc.cc_job_release(h)
    return results, lat, makespan


def same_result(a: dict, b: dict) -> bool:
    return all(np.array_equal(a[f], b[f]) for f in a)


def serve(jobs, graphs, load=0.8, seed: int = 5, max_inflight: int = 0, mem_budget_bytes: int = 0,
          check: bool = True, reference=None) -> dict:
    """Run a job list against pre-built graphs.  `jobs[i]["graph"]` indexes
    `graphs`; `load` is one fraction of the burst capacity or a list of them.
    Returns a summary dict (latencies in ms; one entry per load under
    "loads", the first load's figures also at the top level).  With check,
    every served result (paced and burst) must equal the job run alone;
    `reference`, if given, is a function i -> dict of expected arrays (the
    fields of OUTPUTS) that every result must equal as well."""
    loads = list(load) if isinstance(load, (list, tuple)) else [load]
    ctx = cc.Context(0, mem_budget_bytes=mem_budget_bytes, max_inflight=max_inflight)
    try:
        t0 = time.perf_counter()
        handles = [ctx.upload(g) for g in graphs]
        upload_s = time.perf_counter() - t0
        log(f"uploaded {len(graphs)} graphs ({sum(g.arcs for g in graphs)} arcs) in {upload_s:.1f}s")
        alone, service = run_alone(ctx, handles, graphs, jobs)
        # all jobs at once: the burst capacity, and how much the jobs overlap
        burst, blat, bspan = run_stream(ctx, handles, jobs, np.zeros(len(jobs)))
        cap = len(jobs) / bspan  # jobs/s the device sustains
        teps = sum(edges_traversed(graphs[j["graph"]], j["k"]) for j in jobs)
        mismatches = set()
        results = []
        for q, ld in enumerate(loads):
            rate = ld * cap
            arr = arrival_times(len(jobs), rate, seed + q)
            log(f"burst capacity {cap:.1f} jobs/s; load {ld}: offered {rate:.1f} jobs/s over {arr[-1]:.2f}s")
            mixed, lat, makespan = run_stream(ctx, handles, jobs, arr)
            if check:
                mismatches |= {i for i in range(len(jobs)) if not same_result(alone[i], mixed[i])}
            if reference is not None:
                for i in range(len(jobs)):
                    want = reference(i)
                    if not all(np.array_equal(mixed[i][f], np.asarray(want[f]).astype(mixed[i][f].dtype))
                               for f in OUTPUTS):
                        mismatches.add(i)
            total = [t for _, t in lat]
            queue = [qq for qq, _ in lat]
            results.append({
                "load": ld, "offered_jobs_per_s": round(rate, 2),
                "latency_ms": {"p50": round(percentile(total, 50), 4), "p99": round(percentile(total, 99), 4),
                               "max": round(max(total), 4)},
                "queue_ms": {"p50": round(percentile(queue, 50), 4), "p99": round(percentile(queue, 99), 4)},
                "throughput_jobs_per_s": round(len(jobs) / makespan, 2),
                "gteps": round(teps / makespan / 1e9, 3),
            })
        if check:
            mismatches |= {i for i in range(len(jobs)) if not same_result(alone[i], burst[i])}
        if reference is not None:
            for i in range(len(jobs)):
                want = reference(i)
                if not all(np.array_equal(r[f], np.asarray(want[f]).astype(r[f].dtype))
                           for r in (alone[i], burst[i]) for f in OUTPUTS):
                    mismatches.add(i)
        out = {
            "jobs": len(jobs), "burst_capacity_jobs_per_s": round(cap, 2),
            "service_alone_ms": {"p50": round(percentile(service, 50), 4),
                                 "p99": round(percentile(service, 99), 4)},
            "burst": {"makespan_s": round(bspan, 4), "jobs_per_s": round(cap, 2),
                      "gteps": round(teps / bspan / 1e9, 3),
                      "overlap": round(sum(service) / 1e3 / bspan, 3),
                      "latency_ms": {"p50": round(percentile([t for _, t in blat], 50), 4),
                                     "p99": round(percentile([t for _, t in blat], 99), 4)}},
            "loads": results, "max_inflight": max_inflight, "upload_s": round(upload_s, 2),
            "mismatches": sorted(mismatches),
        }
        out.update({kk: results[0][kk] for kk in ("load", "offered_jobs_per_s", "latency_ms", "queue_ms",
                                                  "throughput_jobs_per_s", "gteps")})
        return out
    finally:
        ctx.close()


def build_mix(num_jobs: int, seed: int, n_lo: float, n_hi: float, threads: int):
    """The serving mix's graphs (one per job), generated in parallel."""
    import graphgen
    jobs = graphgen.serving_mix(num_jobs, seed=seed, n_lo=n_lo, n_hi=n_hi)
    with cf.ThreadPoolExecutor(threads) as ex:
        graphs = list(ex.map(graphgen.make_job_graph, jobs))
    for i, j in enumerate(jobs):
        j["graph"] = i
    return jobs, graphs


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=512)
    ap.add_argument("--load", type=float, nargs="+", default=[0.5, 0.8, 1.0])
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--n-lo", type=float, default=1e3)
    ap.add_argument("--n-hi", type=float, default=1e6)
    ap.add_argument("--max-inflight", type=int, default=0)
    ap.add_argument("--mem-budget-gb", type=float, default=0.0)
    ap.add_argument("--threads", type=int, default=min(os.cpu_count() or 1, 16))
    args = ap.parse_args()
    t0 = time.time()
    jobs, graphs = build_mix(args.jobs, args.seed, args.n_lo, args.n_hi, args.threads)
    log(f"generated {len(graphs)} graphs in {time.time() - t0:.1f}s")
    out = serve(jobs, graphs, load=args.load, seed=args.seed, max_inflight=args.max_inflight,
                mem_budget_bytes=int(args.mem_budget_gb * (1 << 30)))
    out["workload"] = (f"serving mix: {args.jobs} Poisson-arriving BA/R-MAT jobs, n log-uniform in "
                       f"[{args.n_lo:g}, {args.n_hi:g}], k in {{16, 64, 256}}")
    print(json.dumps(out), flush=True)
    return 0 if not out["mismatches"] else 1


if __name__ == "__main__":
    sys.exit(main())
