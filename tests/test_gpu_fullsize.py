"""Parity at the full workload sizes, every node, against the oracle.

The oracle draws the samples itself (its own implementation of the draw),
runs all k searches (queue BFS / binary-heap Dijkstra, both directions for
round trip) and evaluates every estimator for every node with Algorithm 1's
accounting (``oracle.estimate_tails``, pinned against the literal per-node
walk).  The library draws from the same seed and must return the same
samples, the same distance matrix D and the same outputs, bit for bit:
  * test_fullsize_every_node: one eager estimate per workload, every output
    of Sec. 2 and Sec. 4 (S_err, S_ad) for every node, and the threshold
    sweep of Algorithm 2 on a few nodes from the node-level oracle;
  * test_timed_path_replays: exactly what the benchmark times on R-MAT scale
    20, k = 256 -- the autotuner first, then replays of the captured estimate
    (CC_BATCHED | CC_GRAPH) into device tensors, with two sample seeds, every
    replay checked against the oracle for every node."""
import sys

import numpy as np
import pytest

import graphgen
import oracle
import paper_1409_0035_amd as cc

pytestmark = pytest.mark.gpu
BENCH_OUT = ("S_hyb", "S_samp", "S_piv", "S_pub", "pivot", "delta", "sampsum")
ERR_OUT = ("S_err", "S_ad", "S_ad_err")
THREADS = 16
_REF = {}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = cc.Context(0)
    yield c
    c.close()


def _graph(name):
    if ("g", name) not in _REF:
        _say(f"  generating {name}")
        g = graphgen.workload(name)
        _REF[("g", name)] = (g, graphgen.transpose(g) if g.directed else None)
    return _REF[("g", name)]


def _reference(name, seed):
    """The oracle's samples, distances and every-node estimates (cached)."""
    key = (name, seed)
    if key not in _REF:
        g, rg = _graph(name)
        k = graphgen.WORKLOADS[name]["k"]
        samples = np.asarray(oracle.draw_samples(g.n, k, seed), dtype=np.int32)
        _say(f"  oracle: {k} searches on {name} (n={g.n}, arcs={g.arcs})")
        D = oracle.sample_distances(g, samples, threads=THREADS, reverse_graph=rg)
        _say("  oracle: every-node estimates")
        _REF[key] = oracle.estimate_tails(g, samples, D=D, threads=THREADS)
        assert not _REF[key]["overflow"]
    return _REF[key]


def _check(res, ref, fields, what):
    for f in fields:
        a, b = np.asarray(res[f]), ref[f]
        if a.dtype.kind == "f":
            # 1e-12 relative is the stated bar; both sides divide the same exact
            # integers once, so they are identical
            assert np.all(np.abs(a - b) <= 1e-12 * np.abs(b)), f"{what}: {f}"
        assert np.array_equal(a, b.astype(a.dtype)), f"{what}: {f} not bit-identical"


@pytest.mark.parametrize("name", ["rmat20", "grid2048w", "rmat22dir"])
def test_fullsize_every_node(ctx, name):
    spec = graphgen.WORKLOADS[name]
    k, seed = spec["k"], spec["sample_seed"]
    g, rg = _graph(name)
    ref = _reference(name, seed)
    _say(f"  gpu: {name} k={k}")
    gh = ctx.upload(g)
    try:
        res = cc.cc_estimate(ctx.handle, gh, k, seed=seed, outputs=BENCH_OUT + ("samples", "src_sum", "dmat"))
        res.update(cc.cc_estimate(ctx.handle, gh, k, seed=seed, outputs=("D",) + ERR_OUT))
        sweep = cc.cc_estimate(ctx.handle, gh, k, seed=seed, outputs=("S_sweep", "S_sweep_err"))
    finally:
        ctx.release(gh)
    assert np.array_equal(res["samples"], ref["samples"]), "the library's draw differs from the oracle's"
    assert np.array_equal(res["D"], ref["D"]), "D"
    del res["D"]
    _check(res, ref, BENCH_OUT + ("src_sum", "dmat") + ERR_OUT, name)
    # Algorithm 2's sweep on a few nodes from the node-level oracle (two
    # searches each plus a walk over V per threshold)
    rng = np.random.default_rng(seed)
    deg = np.diff(g.row_ptr)
    nodes = [int(x) for x in rng.integers(0, g.n, size=2)] + [int(np.argmax(deg)), int(ref["samples"][0])]
    for v in nodes:
        _say(f"  sweep at node {v}")
        a, ae = oracle.node_sweep(g, ref["samples"], v, reverse_graph=rg)
        assert sweep["S_sweep"][v] == a and sweep["S_sweep_err"][v] == ae, v
    if name in ("rmat22dir", "grid2048w"):
        # the benchmark's path (round trip, weighted): CC_GRAPH replays into device tensors
        import torch
        dt = {"S_hyb": torch.float64, "S_samp": torch.float64, "S_piv": torch.int64, "S_pub": torch.int64,
              "pivot": torch.int32, "delta": torch.int32, "sampsum": torch.int64}
        gh = ctx.upload(g)
        try:
            out = {f: torch.empty(g.n, dtype=dt[f], device="cuda") for f in BENCH_OUT}
            replays = 0
            for call in range(3):
                for t in out.values():
                    t.fill_(-1)
                cc.cc_estimate_device(ctx.handle, gh, k, out, mode=cc.CC_BATCHED | cc.CC_GRAPH, seed=seed)
                replays += cc.cc_last_timing(ctx.handle)["launches"] == 1
                torch.cuda.synchronize()
                _say(f"  {name} call {call}: checking every node")
                _check({f: t.cpu().numpy() for f, t in out.items()}, ref, BENCH_OUT, f"{name} replay {call}")
            assert replays >= 2, f"{name} was not replayed from the captured graph"
        finally:
            ctx.release(gh)
    if name != "rmat20":  # the replay test reuses rmat20's reference
        _REF.pop((name, seed), None)
        _REF.pop(("g", name), None)


def test_timed_path_replays(ctx):
    """The benchmark's path: autotuned launch shapes, then CC_GRAPH replays of
    the captured estimate into device tensors (rmat20, k = 256), two seeds."""
    import torch
    name = "rmat20"
    k = graphgen.WORKLOADS[name]["k"]
    g, _ = _graph(name)
    gh = ctx.upload(g)
    try:
        tuning, ms = cc.cc_autotune(ctx.handle, gh, k, seed=2, reps=1)
        _say(f"  autotune: {tuning} ({ms:.3f} ms)")
        dev = torch.device("cuda:0")
        dt = {"S_hyb": torch.float64, "S_samp": torch.float64, "S_piv": torch.int64, "S_pub": torch.int64,
              "pivot": torch.int32, "delta": torch.int32, "sampsum": torch.int64}
        out = {f: torch.empty(g.n, dtype=dt[f], device=dev) for f in BENCH_OUT}
        stream = torch.cuda.current_stream()
        replays = 0
        # the first call of a seed may capture (a capture is kept for the deepest
        # level its search reached); the calls after it replay
        for seed in (2, 2, 2, 12, 12, 12):
            ref = _reference(name, seed)
            for f in out.values():
                f.fill_(-1)
            cc.cc_estimate_device(ctx.handle, gh, k, out, mode=cc.CC_BATCHED | cc.CC_GRAPH, seed=seed,
                                  stream=stream)
            replays += cc.cc_last_timing(ctx.handle)["launches"] == 1
            torch.cuda.synchronize()
            got = {f: t.cpu().numpy() for f, t in out.items()}
            _say(f"  seed {seed}: checking every node")
            _check(got, ref, BENCH_OUT, f"replay seed {seed}")
        assert replays >= 4, "the estimates were not replayed from the captured graph"
    finally:
        ctx.release(gh)
