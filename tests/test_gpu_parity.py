"""GPU parity: the HIP library (through its C ABI) against the CPU oracle on
the same seeded inputs.  Integer outputs (distances, pivots, Delta, sums,
sample distance matrix) must be bit-exact; the two double estimates must agree
within a relative error of 1e-12 (both sides divide the same exact integer
numerator once, so they are expected to be identical)."""
import sys

import numpy as np
import pytest

import graphgen
import oracle
import paper_1409_0035_amd as cc

pytestmark = pytest.mark.gpu
RTOL = 1e-12
ALL = ("S_hyb", "S_samp", "S_piv", "S_pub", "pivot", "delta", "sampsum", "src_sum", "samples", "dmat", "D")


@pytest.fixture(scope="module")
def ctx():
    c = cc.Context(0)
    yield c
    c.close()


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(ctx, g, k, mode, samples=None, seed=0, eps=None, outputs=ALL):
    gh = ctx.upload(g)
    try:
        return cc.cc_estimate(ctx.handle, gh, k, mode=mode, seed=seed, samples=samples, eps=eps, outputs=outputs)
    finally:
        ctx.release(gh)


def check_all(res, ref, samples, with_D=True):
    if with_D:
        assert (res["D"] == ref["D"]).all(), "D"
    assert (res["samples"] == np.asarray(samples)).all()
    assert (res["pivot"] == ref["pivot"]).all(), "pivot"
    assert (res["delta"] == ref["delta"]).all(), "delta"
    assert (res["sampsum"] == ref["sampsum"]).all(), "sampsum"
    assert (res["src_sum"] == ref["src_sum"]).all(), "src_sum"
    assert (res["dmat"] == ref["dmat"]).all(), "dmat"
    assert (res["S_piv"] == ref["S_piv"]).all(), "S_piv"
    assert (res["S_pub"] == ref["S_pub"]).all(), "S_pub"
    for f in ("S_hyb", "S_samp"):
        a, b = res[f], ref[f]
        assert np.all(np.abs(a - b) <= RTOL * np.abs(b)), f
        assert (a == b).all(), f + " (not bit-identical)"


def parity(ctx, g, k, seed, eps=None, modes=(cc.CC_BATCHED, cc.CC_PLAIN)):
    samples = oracle.draw_samples(g.n, k, seed)
    rg = graphgen.transpose(g) if g.directed else None
    ref = oracle.estimate_all(g, samples, eps=eps, threads=8, reverse_graph=rg)
    out = {}
    for mode in modes:
        _say(f"  gpu {g.name} n={g.n} arcs={g.arcs} k={k} mode={mode} eps={eps}")
        res = run_gpu(ctx, g, k, mode, seed=seed, eps=eps)
        check_all(res, ref, samples)
        out[mode] = res
    return out


# ---------------------------------------------------------------- closed forms

@pytest.mark.parametrize("make,k", [(lambda: graphgen.path(50), 5), (lambda: graphgen.star(40), 7),
                                    (lambda: graphgen.cycle(33), 4), (lambda: graphgen.complete(20), 3),
                                    (lambda: graphgen.grid(13, 11, 4), 9), (lambda: graphgen.grid(12, 9, 8), 64)])
def test_closed_form_families(ctx, make, k):
    parity(ctx, make(), k, seed=7)


def test_worked_example_path9(ctx):
    g = graphgen.path(9)
    res = run_gpu(ctx, g, 3, cc.CC_BATCHED, samples=[0, 4, 8], eps=(1, 2))
    assert list(res["S_hyb"]) == [36, 33, 32, 18, 20, 18, 80 / 3, 33, 36]
    assert list(res["pivot"]) == [0, 0, 0, 1, 1, 1, 1, 2, 2]


# ---------------------------------------------------------------- random / ragged

@pytest.mark.parametrize("seed", range(8))
def test_random_small_graphs(ctx, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 200))
    directed = seed % 3 == 2
    g = graphgen.gnp(n, float(rng.uniform(0.01, 0.1)), seed, directed=directed)
    k = int(rng.integers(1, min(n, 130) + 1))
    eps = [(1, 1), (1, 3), (2, 5), None][seed % 4]
    parity(ctx, g, k, seed, eps=eps)


@pytest.mark.parametrize("k", [1, 63, 64, 65, 100, 192, 256, 257, 300])
def test_ragged_sample_counts(ctx, k):
    """k around the 64-bit word and 256-sample group boundaries."""
    g = graphgen.ba(3000, 3, seed=11)
    parity(ctx, g, k, seed=k)


def test_deep_graph_widens_distance_type(ctx):
    """More than 254 BFS levels: 8-bit distances overflow and the library
    reruns with 16-bit ones."""
    g = graphgen.path(700)
    parity(ctx, g, 6, seed=3)


# ---------------------------------------------------------------- workload shapes

def test_ba10k_k64_full(ctx):
    """Barabasi-Albert n=10,000, 4 edges per node, 64 samples: every output."""
    g = graphgen.workload("ba10k")
    out = parity(ctx, g, 64, seed=1)
    S = oracle.exact_sums(g, threads=8)
    err = np.abs(out[cc.CC_BATCHED]["S_hyb"] - S) / S
    _say(f"  ba10k hybrid mean rel err {err.mean():.4f}")
    assert err.mean() < 0.1


def test_rmat14_k256(ctx):
    g = graphgen.rmat(14, 16, seed=5)
    parity(ctx, g, 256, seed=5)


def test_directed_rmat_round_trip(ctx):
    g = graphgen.rmat(12, 16, seed=6, directed=True)
    parity(ctx, g, 128, seed=6)


@pytest.mark.parametrize("k", [16, 32, 64, 100, 128, 192, 256])
def test_round_trip_row_widths(ctx, k):
    """The round trip at every row width of the distance epilogue: k = 16
    (one 16-byte piece per node, the one-lane kernels), 32, 64, 128 and 256
    (2, 4, 8 and 16 lanes per node, byte-packed), 100 and 192 (rows that are
    not 16 * 2^j bytes); k = 64, 128, 192 and 256 sum both directions in one
    pass, k = 16, 32 and 100 (a partial mask word) write each direction's
    distances apart.  Eager, then captured and replayed, every output against
    the oracle's."""
    g = graphgen.rmat(11, 16, seed=60 + k, directed=True)
    seed = 70 + k
    samples = oracle.draw_samples(g.n, k, seed)
    ref = oracle.estimate_all(g, samples, threads=8, reverse_graph=graphgen.transpose(g))
    gh = ctx.upload(g)
    try:
        for mode, reps in ((cc.CC_BATCHED, 1), (cc.CC_BATCHED | cc.CC_GRAPH, 3)):
            for rep in range(reps):
                _say(f"  round trip n={g.n} arcs={g.arcs} k={k} mode={mode} call {rep}")
                res = cc.cc_estimate(ctx.handle, gh, k, mode=mode, seed=seed, outputs=ALL)
                check_all(res, ref, samples)
    finally:
        ctx.release(gh)


def test_symmetric_digraph_round_trip_is_twice(ctx):
    g = graphgen.ba(800, 3, seed=2)
    gd = graphgen.symmetric_digraph(g)
    a = run_gpu(ctx, g, 40, cc.CC_BATCHED, seed=9, eps=(1, 2))
    b = run_gpu(ctx, gd, 40, cc.CC_BATCHED, seed=9, eps=(1, 2))
    assert (a["pivot"] == b["pivot"]).all()
    assert (2 * a["S_hyb"] == b["S_hyb"]).all()


# ---------------------------------------------------------------- errors

def test_error_paths(ctx):
    g = graphgen.path(10)
    gh = ctx.upload(g)
    try:
        for kw in (dict(k=11), dict(k=0), dict(k=3, eps=(3, 2)), dict(k=3, eps=(0, 1)),
                   dict(k=3, samples=[1, 1, 2]), dict(k=2, samples=[0, 10])):
            with pytest.raises(cc.CCError) as e:
                cc.cc_estimate(ctx.handle, gh, **kw)
            assert e.value.status == cc.CC_EINVAL, kw
    finally:
        ctx.release(gh)
    # two components
    two = graphgen.csr_from_arcs(6, [0, 1, 3, 4], [1, 2, 4, 5])
    gh = ctx.upload(two)
    try:
        for mode in (cc.CC_BATCHED, cc.CC_PLAIN):
            with pytest.raises(cc.CCError) as e:
                cc.cc_estimate(ctx.handle, gh, 2, mode=mode, samples=[0, 1])
            assert e.value.status == cc.CC_EDISCONNECTED
    finally:
        ctx.release(gh)
    with pytest.raises(cc.CCError) as e:
        ctx.upload(graphgen.csr_from_arcs(3, [0], [1], symmetrize=False), validate=True)
    assert e.value.status == cc.CC_EINVAL


def test_device_outputs_on_torch_stream(ctx):
    import torch
    g = graphgen.ba(2000, 4, seed=3)
    gh = ctx.upload(g)
    try:
        n, k = g.n, 64
        out = {"S_hyb": torch.empty(n, dtype=torch.float64, device="cuda"),
               "pivot": torch.empty(n, dtype=torch.int32, device="cuda")}
        s = torch.cuda.Stream()
        cc.cc_estimate_device(ctx.handle, gh, k, out, seed=4, stream=s)
        s.synchronize()
        ref = cc.cc_estimate(ctx.handle, gh, k, seed=4, outputs=("S_hyb", "pivot"))
        assert (out["S_hyb"].cpu().numpy() == ref["S_hyb"]).all()
        assert (out["pivot"].cpu().numpy() == ref["pivot"]).all()
        t = cc.cc_last_timing(ctx.handle)
        assert t["total_ms"] > 0 and t["levels"] > 0
    finally:
        ctx.release(gh)


# ---------------------------------------------------------------- weighted

@pytest.mark.parametrize("seed", range(6))
def test_weighted_random_graphs(ctx, seed):
    rng = np.random.default_rng(50 + seed)
    n = int(rng.integers(2, 150))
    directed = seed % 3 == 2
    g = graphgen.gnp(n, float(rng.uniform(0.02, 0.1)), 50 + seed, directed=directed,
                     wmax=[3, 1000, 50][seed % 3])
    k = int(rng.integers(1, min(n, 70) + 1))
    parity(ctx, g, k, seed, eps=[(1, 2), None, (2, 3)][seed % 3])


def test_weighted_grid8(ctx):
    """8-neighbour grid, 10% of edges deleted, lengths in [1, 1000] -- the
    weighted workload's structure at 96 x 80."""
    g = graphgen.grid(96, 80, 8, 0.10, 1, 1000, seed=3)
    parity(ctx, g, 64, seed=3)


GRID_OUT = ("S_hyb", "S_samp", "S_piv", "S_pub", "pivot", "delta", "sampsum", "src_sum", "samples", "dmat", "D")


def _grid_check(got, ref, what):
    for f in GRID_OUT:
        assert np.array_equal(got[f], np.asarray(ref[f]).astype(got[f].dtype).reshape(got[f].shape)), (what, f)


@pytest.mark.parametrize("seed", [21, 22, 23])
def test_weighted_grid_seeds(ctx, seed):
    """The weighted workload's structure at 256 x 256 (65,536 nodes) with 64
    samples: 64 workgroups relax crowded neighbourhoods at once, so a lost
    update in the atomic relaxation would leave some distance above the
    oracle's.  Every output against the oracle (its Algorithm 1 accounting,
    which the pins tie to the literal Eq. (6))."""
    g = graphgen.grid(256, 256, 8, 0.10, 1, 1000, seed=seed)
    samples = np.asarray(oracle.draw_samples(g.n, 64, seed), dtype=np.int32)
    ref = oracle.estimate_tails(g, samples, threads=8, adaptive_eps=())
    _say(f"  grid256 seed={seed}")
    _grid_check(run_gpu(ctx, g, 64, cc.CC_BATCHED, seed=seed), ref, seed)


def test_weighted_grid_bucket_widths(ctx):
    """The same grid under bucket widths far below and far above the default
    (1, and 40 times the largest arc length): identical outputs, three runs
    each."""
    g = graphgen.grid(256, 256, 8, 0.10, 1, 1000, seed=25)
    samples = np.asarray(oracle.draw_samples(g.n, 64, 25), dtype=np.int32)
    ref = oracle.estimate_tails(g, samples, threads=8, adaptive_eps=())
    gh = ctx.upload(g)
    try:
        default = cc.cc_graph_get_tuning(gh)
        for delta in (1, 40_000, default["delta"]):
            cc.cc_graph_set_tuning(gh, **{**default, "delta": delta})
            for rep in range(3):
                _say(f"  grid256 delta={delta} run {rep}")
                got = cc.cc_estimate(ctx.handle, gh, 64, seed=25, outputs=GRID_OUT)
                _grid_check(got, ref, (delta, rep))
    finally:
        ctx.release(gh)


def test_weighted_unit_lengths_match_bfs(ctx):
    g = graphgen.ba(1500, 3, seed=8)
    gw = graphgen.Graph(g.n, g.row_ptr, g.col_idx, np.ones(g.arcs, np.int32), name="ba-unit-w")
    a = run_gpu(ctx, g, 40, cc.CC_BATCHED, seed=5)
    b = run_gpu(ctx, gw, 40, cc.CC_BATCHED, seed=5)
    for f in ("D", "pivot", "delta", "sampsum", "dmat", "src_sum", "S_piv", "S_pub"):
        assert (a[f] == b[f]).all(), f
    assert (a["S_hyb"] == b["S_hyb"]).all()


def test_weighted_deep_path(ctx):
    """Long path with lengths up to 1000: many delta-stepping buckets."""
    n = 900
    i = np.arange(n - 1, dtype=np.int32)
    w = (np.arange(n - 1) * 7919 % 1000 + 1).astype(np.int32)
    g = graphgen.csr_from_arcs(n, i, i + 1, w, name="wpath900")
    parity(ctx, g, 5, seed=2)


# ---------------------------------------------------------------- degenerate inputs

DEGENERATE = [
    ("single-node", lambda: graphgen.csr_from_arcs(1, [], [])),
    ("one-edge", lambda: graphgen.csr_from_arcs(2, [0], [1])),
    ("path3", lambda: graphgen.csr_from_arcs(3, [0, 1], [1, 2])),
    ("two-cycle-directed", lambda: graphgen.csr_from_arcs(2, [0, 1], [1, 0], symmetrize=False, directed=True)),
    ("one-edge-weighted", lambda: graphgen.csr_from_arcs(2, [0], [1], [7])),
    ("triangle-directed-weighted", lambda: graphgen.csr_from_arcs(3, [0, 1, 2], [1, 2, 0], [2, 3, 5], symmetrize=False,
                                                                  directed=True)),
]


@pytest.mark.parametrize("name,make", DEGENERATE, ids=[d[0] for d in DEGENERATE])
def test_degenerate_graphs(ctx, name, make):
    """One, two and three nodes, every k from 1 to n, on every path (batched,
    plain, captured replays): the estimates against the oracle."""
    import torch
    g = make()
    for k in range(1, g.n + 1):
        parity(ctx, g, k, seed=k)
        samples = oracle.draw_samples(g.n, k, k)
        rg = graphgen.transpose(g) if g.directed else None
        ref = oracle.estimate_all(g, samples, threads=1, reverse_graph=rg)
        gh = ctx.upload(g)
        try:
            out = {"S_hyb": torch.empty(g.n, dtype=torch.float64, device="cuda"),
                   "pivot": torch.empty(g.n, dtype=torch.int32, device="cuda")}
            for _ in range(3):
                cc.cc_estimate_device(ctx.handle, gh, k, out, mode=cc.CC_BATCHED | cc.CC_GRAPH, seed=k)
                torch.cuda.synchronize()
                assert np.array_equal(out["S_hyb"].cpu().numpy(), ref["S_hyb"]), (name, k)
                assert np.array_equal(out["pivot"].cpu().numpy(), ref["pivot"]), (name, k)
        finally:
            ctx.release(gh)


# ---------------------------------------------------------------- randomised sweep

def _random_case(rng):
    kind = rng.choice(["gnp", "ba", "rmat", "grid", "gnp-dir", "rmat-dir"])
    weighted = bool(rng.random() < 0.35)
    if kind == "gnp":
        g = graphgen.gnp(int(rng.integers(5, 400)), float(rng.uniform(0.01, 0.2)), int(rng.integers(1 << 30)),
                         wmax=int(rng.integers(2, 60)) if weighted else 1)
    elif kind == "gnp-dir":
        g = graphgen.gnp(int(rng.integers(5, 300)), float(rng.uniform(0.01, 0.2)), int(rng.integers(1 << 30)),
                         directed=True, wmax=int(rng.integers(2, 60)) if weighted else 1)
    elif kind == "ba":
        g = graphgen.ba(int(rng.integers(10, 3000)), int(rng.integers(1, 5)), seed=int(rng.integers(1 << 30)))
        if weighted:
            g = graphgen.with_lengths(g, 1, int(rng.integers(2, 500)), int(rng.integers(1 << 30)))
    elif kind == "grid":
        g = graphgen.grid(int(rng.integers(2, 40)), int(rng.integers(2, 40)), int(rng.choice([4, 8])),
                          float(rng.uniform(0, 0.15)), 1, int(rng.integers(2, 100)) if weighted else 1,
                          seed=int(rng.integers(1 << 30)))
    else:
        g = graphgen.rmat(int(rng.integers(6, 11)), int(rng.integers(4, 17)), seed=int(rng.integers(1 << 30)),
                          directed=kind == "rmat-dir")
        if weighted:
            g = graphgen.with_lengths(g, 1, int(rng.integers(2, 1000)), int(rng.integers(1 << 30)))
    k = int(min(g.n, rng.choice([1, 2, 7, 64, 65, 128, 200, 256, 300])))
    den = int(rng.integers(1, 12))
    eps = None if rng.random() < 0.4 else (int(rng.integers(1, den + 1)), den)
    mode = int(rng.choice([cc.CC_BATCHED, cc.CC_PLAIN, cc.CC_BATCHED | cc.CC_GRAPH]))
    return g, k, eps, mode


@pytest.mark.parametrize("case", range(24))
def test_random_configurations(ctx, case):
    """Seeded random graph family, direction, arc lengths, k, eps and mode
    (eager, plain, captured), every output against the oracle."""
    rng = np.random.default_rng(9000 + case)
    g, k, eps, mode = _random_case(rng)
    seed = int(rng.integers(1 << 20))
    samples = oracle.draw_samples(g.n, k, seed)
    rg = graphgen.transpose(g) if g.directed else None
    ref = oracle.estimate_all(g, samples, eps=eps, threads=8, reverse_graph=rg)
    _say(f"  case {case}: {g.name} n={g.n} arcs={g.arcs} weighted={g.w is not None} k={k} eps={eps} mode={mode}")
    gh = ctx.upload(g)
    try:
        for _ in range(2 if mode & cc.CC_GRAPH else 1):
            res = cc.cc_estimate(ctx.handle, gh, k, mode=mode, seed=seed, eps=eps, outputs=ALL)
            check_all(res, ref, samples)
    finally:
        ctx.release(gh)
