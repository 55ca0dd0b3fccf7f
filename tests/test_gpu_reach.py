"""GPU parity for the outbound / inbound reachability sampling of Sec. 6.2
(Algorithm 4): count, distsum and T bit-exact against the oracle's
definition (first k reached nodes in rank order), B and R bit-identical
(one IEEE division each, the same integers on both sides)."""
import sys

import numpy as np
import pytest

import graphgen
import oracle
import paper_1409_0035_amd as cc

pytestmark = pytest.mark.gpu
FIELDS = ("count", "distsum", "T", "B", "R")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = cc.Context(0)
    yield c
    c.close()


def h_n(h):
    return cc.cc_graph_info(h)[0]


def _same(got, ref, what):
    for f in FIELDS:
        assert np.array_equal(got[f], ref[f]), f"{what}: {f}"


def test_worked_example(ctx):
    src, dst = [0, 1, 2, 2, 3, 5], [1, 2, 0, 3, 4, 3]
    g = graphgen.csr_from_arcs(6, src, dst, symmetrize=False, directed=True)
    order = [3, 0, 5, 1, 4, 2]
    gh = ctx.upload(g)
    try:
        for inbound in (False, True):
            got = cc.cc_reach_estimate(ctx.handle, gh, 2, inbound=inbound, order=order)
            _same(got, oracle.reach_all(g, order, 2, inbound=inbound), f"inbound={inbound}")
    finally:
        ctx.release(gh)


CASES = [
    ("gnp-dir", lambda: graphgen.gnp(300, 0.01, 5, directed=True, connect=False), (1, 2, 7, 40, 400)),
    ("rmat-dir-s12", lambda: graphgen.rmat(12, 8, seed=3, directed=True, component=False), (1, 16, 100)),
    ("rmat-dir-s13-scc", lambda: graphgen.rmat(13, 16, seed=4, directed=True), (50, 257)),
    ("ba-undirected", lambda: graphgen.ba(3000, 3, seed=6), (3, 64)),
    ("path-dir", lambda: graphgen.csr_from_arcs(700, list(range(699)), list(range(1, 700)), symmetrize=False,
                                                directed=True), (1, 5, 1000)),
    ("star-dir", lambda: graphgen.csr_from_arcs(1025, [0] * 1024, list(range(1, 1025)), symmetrize=False,
                                                directed=True), (4, 300)),
    # no source has a propagation arc (the list of sources to pick batches from is empty), or one has
    ("no-arcs", lambda: graphgen.csr_from_arcs(50, [], [], symmetrize=False, directed=True), (1, 3)),
    ("one-arc", lambda: graphgen.csr_from_arcs(40, [7], [3], symmetrize=False, directed=True), (1, 2)),
]


@pytest.mark.parametrize("name,make,ks", CASES, ids=[c[0] for c in CASES])
def test_reach_matches_oracle(ctx, name, make, ks):
    g = make()
    rg = graphgen.transpose(g)
    gh = ctx.upload(g)
    try:
        for k in ks:
            for inbound in (False, True):
                seed = 11 + k
                _say(f"  {name}: n={g.n} arcs={g.arcs} k={k} inbound={inbound}")
                got = cc.cc_reach_estimate(ctx.handle, gh, k, inbound=inbound, seed=seed)
                order = oracle.draw_samples(g.n, g.n, seed)
                ref = oracle.reach_all(g, order, k, inbound=inbound, threads=8, reverse_graph=rg)
                _same(got, ref, f"{name} k={k} inbound={inbound}")
    finally:
        ctx.release(gh)


def test_explicit_order_equals_seeded(ctx):
    g = graphgen.rmat(11, 8, seed=8, directed=True, component=False)
    gh = ctx.upload(g)
    try:
        a = cc.cc_reach_estimate(ctx.handle, gh, 32, seed=77)
        b = cc.cc_reach_estimate(ctx.handle, gh, 32, order=oracle.draw_samples(g.n, g.n, 77))
        _same(a, b, "order")
        # another order gives another sample, same reach counts where the sample is not full
        c = cc.cc_reach_estimate(ctx.handle, gh, 32, seed=78)
        small = a["count"] < 32
        assert (c["count"][small] == a["count"][small]).all()
    finally:
        ctx.release(gh)


def test_invalid_arguments(ctx):
    g = graphgen.rmat(8, 8, seed=9, directed=True, component=False)
    gw = graphgen.grid(10, 10, 8, 0.1, 1, 10, seed=2)
    gh, ghw = ctx.upload(g), ctx.upload(gw)
    try:
        for h in (gh, ghw):
            for kw in (dict(k=0), dict(k=4, order=[0] * h_n(h))):
                with pytest.raises(cc.CCError) as e:
                    cc.cc_reach_estimate(ctx.handle, h, **kw)
                assert e.value.status == cc.CC_EINVAL
    finally:
        ctx.release(gh)
        ctx.release(ghw)


def test_fullsize_sampled_nodes(ctx):
    """Directed R-MAT scale 20, whole graph, k = 100, the benchmark's order:
    sampled nodes from the definition (one search each), identities for all."""
    spec = graphgen.WORKLOADS["rmat20dir"]
    k, seed = spec["k"], spec["sample_seed"]
    _say("  generating rmat20dir")
    g = graphgen.workload("rmat20dir")
    rg = graphgen.transpose(g)
    _say(f"  n={g.n} arcs={g.arcs}")
    gh = ctx.upload(g)
    try:
        res = {ib: cc.cc_reach_estimate(ctx.handle, gh, k, inbound=ib, seed=seed) for ib in (False, True)}
        t = cc.cc_last_timing(ctx.handle)
        _say(f"  inbound estimate: {t['total_ms']:.1f} ms, {t['levels']} levels, {t['launches']} launches")
    finally:
        ctx.release(gh)
    order = oracle.draw_samples(g.n, g.n, seed)
    rng = np.random.default_rng(seed)
    deg = np.diff(g.row_ptr)
    nodes = np.unique(np.concatenate([rng.integers(0, g.n, size=6), [int(np.argmax(deg)), 0, g.n - 1],
                                      order[:2], order[-2:]])).astype(np.int32)
    for ib in (False, True):
        r = res[ib]
        assert ((r["count"] >= 0) & (r["count"] <= k)).all()
        full = r["count"] == k
        assert (r["T"][full] >= k).all() and (r["T"][~full] == 0).all()
        nz = r["count"] > 0
        assert (r["B"][nz] == r["distsum"][nz] / r["count"][nz]).all()
        _say(f"  inbound={ib}: {int(full.sum())} full samples, checking {len(nodes)} nodes")
        ref = oracle.reach_all(g, order, k, inbound=ib, threads=8, reverse_graph=rg, nodes=nodes)
        for j, v in enumerate(nodes):
            for f in FIELDS:
                assert r[f][v] == ref[f][j], (ib, int(v), f)


# ---------------------------------------------------------------- Algorithm 5 (node weights)

WFIELDS = ("count", "kth", "S", "R")

WCASES = [
    ("gnp-dir", lambda: graphgen.gnp(300, 0.01, 5, directed=True, connect=False), (1, 2, 9, 60)),
    ("rmat-dir-s12", lambda: graphgen.rmat(12, 8, seed=3, directed=True, component=False), (1, 16, 100)),
    ("ba-undirected", lambda: graphgen.ba(3000, 3, seed=6), (5, 64)),
    ("path-dir", lambda: graphgen.csr_from_arcs(500, list(range(499)), list(range(1, 500)), symmetrize=False,
                                                directed=True), (3, 600)),
]


@pytest.mark.parametrize("name,make,ks", WCASES, ids=[c[0] for c in WCASES])
def test_reach_weighted_matches_oracle(ctx, name, make, ks):
    g = make()
    rg = graphgen.transpose(g)
    beta = graphgen.node_weights(g.n, 17, zero_frac=0.3)
    gh = ctx.upload(g)
    try:
        for k in ks:
            for inbound in (False, True):
                seed = 31 + k
                _say(f"  {name}: n={g.n} k={k} inbound={inbound}")
                got = cc.cc_reach_weighted(ctx.handle, gh, beta, k, inbound=inbound, seed=seed)
                ref = oracle.reach_weighted(g, beta, k, seed, inbound=inbound, threads=8, reverse_graph=rg)
                for f in WFIELDS:
                    assert np.array_equal(got[f], ref[f]), f"{name} k={k} inbound={inbound}: {f}"
    finally:
        ctx.release(gh)


def test_reach_weighted_fullsize_sampled_nodes(ctx):
    spec = graphgen.WORKLOADS["rmat20dir"]
    k, seed = spec["k"], spec["sample_seed"]
    g = graphgen.workload("rmat20dir")
    beta = graphgen.node_weights(g.n, seed)
    gh = ctx.upload(g)
    try:
        got = cc.cc_reach_weighted(ctx.handle, gh, beta, k, seed=seed)
        t = cc.cc_last_timing(ctx.handle)
        _say(f"  weighted outbound: {t['total_ms']:.1f} ms, {t['levels']} levels")
        with pytest.raises(cc.CCError) as e:
            cc.cc_reach_weighted(ctx.handle, gh, np.zeros(g.n, np.uint32), k)
        assert e.value.status == cc.CC_EINVAL
    finally:
        ctx.release(gh)
    rng = np.random.default_rng(seed)
    deg = np.diff(g.row_ptr)
    nodes = np.unique(np.concatenate([rng.integers(0, g.n, size=8), [int(np.argmax(deg)), 0]])).astype(np.int32)
    ref = oracle.reach_weighted(g, beta, k, seed, threads=8, nodes=nodes)
    for j, v in enumerate(nodes):
        for f in WFIELDS:
            assert got[f][v] == ref[f][j], (int(v), f)


# ---------------------------------------------------------------- arc lengths (the listing's Dijkstra)


def _with_lengths(g, hi, seed, lo=1):
    return graphgen.with_lengths(g, lo, hi, seed)


LCASES = [
    ("gnp-dir", lambda: graphgen.gnp(300, 0.01, 5, directed=True, wmax=50, connect=False), (1, 2, 7, 40, 400)),
    ("rmat-dir-s12", lambda: _with_lengths(graphgen.rmat(12, 8, seed=3, directed=True, component=False), 1000, 21),
     (1, 16, 100)),
    ("rmat-dir-s13-scc", lambda: _with_lengths(graphgen.rmat(13, 16, seed=4, directed=True), 100, 22), (50, 257)),
    ("grid-undirected", lambda: graphgen.grid(40, 30, 8, 0.1, 1, 1000, seed=4), (3, 64)),
    ("path-dir", lambda: _with_lengths(graphgen.csr_from_arcs(700, list(range(699)), list(range(1, 700)),
                                                              symmetrize=False, directed=True), 9, 23), (1, 5, 1000)),
    # every length 3: many equal distances
    ("rmat-dir-equal", lambda: _with_lengths(graphgen.rmat(11, 8, seed=5, directed=True, component=False), 3, 24,
                                             lo=3), (2, 33)),
    ("one-arc", lambda: graphgen.csr_from_arcs(40, [7], [3], [5], symmetrize=False, directed=True), (1, 2)),
]


@pytest.mark.parametrize("name,make,ks", LCASES, ids=[c[0] for c in LCASES])
def test_reach_lengths_matches_oracle(ctx, name, make, ks):
    """Algorithm 4 with arc lengths: count, distsum, T, B and R bit-exact
    against the oracle's definition (one Dijkstra per node)."""
    g = make()
    assert g.w is not None
    rg = graphgen.transpose(g)
    gh = ctx.upload(g)
    try:
        for k in ks:
            for inbound in (False, True):
                seed = 41 + k
                _say(f"  {name}: n={g.n} arcs={g.arcs} k={k} inbound={inbound}")
                got = cc.cc_reach_estimate(ctx.handle, gh, k, inbound=inbound, seed=seed)
                order = oracle.draw_samples(g.n, g.n, seed)
                ref = oracle.reach_all(g, order, k, inbound=inbound, threads=8, reverse_graph=rg)
                _same(got, ref, f"{name} k={k} inbound={inbound}")
    finally:
        ctx.release(gh)


def test_reach_lengths_unit_equals_bfs(ctx):
    """Lengths all 1 through the arc-length searches give what the BFS path gives."""
    g = graphgen.rmat(12, 8, seed=7, directed=True, component=False)
    gw = graphgen.Graph(n=g.n, row_ptr=g.row_ptr.copy(), col_idx=g.col_idx.copy(), w=np.ones(g.arcs, np.int32),
                        directed=True, name="unit-lengths")
    gh, ghw = ctx.upload(g), ctx.upload(gw)
    try:
        for k in (1, 10, 64):
            a = cc.cc_reach_estimate(ctx.handle, gh, k, seed=k)
            b = cc.cc_reach_estimate(ctx.handle, ghw, k, seed=k)
            _same(a, b, f"k={k}")
    finally:
        ctx.release(gh)
        ctx.release(ghw)


@pytest.mark.parametrize("name,make,ks", [c for c in LCASES if c[0] in ("gnp-dir", "rmat-dir-s12", "grid-undirected",
                                                                          "path-dir")],
                         ids=["gnp-dir", "rmat-dir-s12", "grid-undirected", "path-dir"])
def test_reach_weighted_lengths_matches_oracle(ctx, name, make, ks):
    """Algorithm 5 with arc lengths: count, the k-th member, S and R against
    the oracle's definition."""
    g = make()
    rg = graphgen.transpose(g)
    beta = graphgen.node_weights(g.n, 19, zero_frac=0.3)
    gh = ctx.upload(g)
    try:
        for k in ks:
            for inbound in (False, True):
                seed = 51 + k
                _say(f"  {name}: n={g.n} k={k} inbound={inbound} (node weights)")
                got = cc.cc_reach_weighted(ctx.handle, gh, beta, k, inbound=inbound, seed=seed)
                ref = oracle.reach_weighted(g, beta, k, seed, inbound=inbound, threads=8, reverse_graph=rg)
                for f in WFIELDS:
                    assert np.array_equal(got[f], ref[f]), f"{name} k={k} inbound={inbound}: {f}"
    finally:
        ctx.release(gh)


def test_reach_lengths_fullsize_sampled_nodes(ctx):
    """Directed R-MAT scale 20 with lengths uniform in [1, 1000], k = 100:
    sampled nodes from the definition (one Dijkstra each), identities for all."""
    spec = graphgen.WORKLOADS["rmat20dirw"]
    k, seed = spec["k"], spec["sample_seed"]
    _say("  generating rmat20dirw")
    g = graphgen.workload("rmat20dirw")
    rg = graphgen.transpose(g)
    order = oracle.draw_samples(g.n, g.n, seed)
    gh = ctx.upload(g)
    try:
        res = {}
        for ib in (False, True):
            res[ib] = cc.cc_reach_estimate(ctx.handle, gh, k, inbound=ib, seed=seed)
            t = cc.cc_last_timing(ctx.handle)
            _say(f"  inbound={ib}: {t['total_ms']:.1f} ms, {t['levels']} phases")
    finally:
        ctx.release(gh)
    rng = np.random.default_rng(seed)
    for ib in (False, True):
        r = res[ib]
        assert (r["count"] <= k).all() and (r["count"] >= 0).all()
        full = r["count"] == k
        assert (r["T"][full] >= k).all() and (r["T"][~full] == 0).all()
        nz = r["count"] > 0
        assert (r["B"][nz] == r["distsum"][nz] / r["count"][nz]).all()
        deg = np.diff(g.row_ptr if ib else rg.row_ptr)
        nodes = np.unique(np.concatenate([rng.integers(0, g.n, size=6), [int(np.argmax(deg))],
                                          np.flatnonzero(full)[:2], np.flatnonzero(~full & nz)[:2]])).astype(np.int32)
        _say(f"  inbound={ib}: {int(full.sum())} full samples, checking {len(nodes)} nodes")
        ref = oracle.reach_all(g, order, k, inbound=ib, threads=8, reverse_graph=rg, nodes=nodes)
        for j, v in enumerate(nodes):
            for f in FIELDS:
                assert r[f][v] == ref[f][j], (ib, int(v), f)


def test_reach_weighted_lengths_fullsize_sampled_nodes(ctx):
    """Algorithm 5 on the directed R-MAT scale 20 with arc lengths, k = 100:
    sampled nodes from the definition (one Dijkstra each)."""
    spec = graphgen.WORKLOADS["rmat20dirw"]
    k, seed = spec["k"], spec["sample_seed"]
    g = graphgen.workload("rmat20dirw")
    beta = graphgen.node_weights(g.n, seed)
    gh = ctx.upload(g)
    try:
        got = cc.cc_reach_weighted(ctx.handle, gh, beta, k, seed=seed)
        t = cc.cc_last_timing(ctx.handle)
        _say(f"  weighted outbound with lengths: {t['total_ms']:.1f} ms, {t['levels']} phases")
    finally:
        ctx.release(gh)
    rng = np.random.default_rng(seed + 1)
    deg = np.diff(g.row_ptr)
    full = np.flatnonzero(got["count"] == k)
    nodes = np.unique(np.concatenate([rng.integers(0, g.n, size=6), [int(np.argmax(deg))], full[:2]])).astype(np.int32)
    ref = oracle.reach_weighted(g, beta, k, seed, threads=8, nodes=nodes)
    for j, v in enumerate(nodes):
        for f in WFIELDS:
            assert got[f][v] == ref[f][j], (int(v), f)
