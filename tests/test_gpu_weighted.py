"""GPU parity for the node-weighted estimate of Sec. 5 (Algorithm 3): the
sample, tau and adjusted weights equal the oracle's; S_beta, its variance
estimate and its error estimate are bit-identical (both sides: the same exact integers, one
division for the estimate and the same order of double operations for the
variance; the bar is a relative error of 1e-12)."""
import sys

import numpy as np
import pytest

import graphgen
import oracle
import paper_1409_0035_amd as cc

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = cc.Context(0)
    yield c
    c.close()


def _check(got, ref):
    assert (got["samples"] == ref["samples"]).all()
    assert got["tau"] == ref["tau"]
    assert (got["adjusted"] == ref["adjusted"]).all()
    for f in ("S_beta", "S_beta_var", "S_beta_err"):
        a, b = got[f], ref[f]
        assert np.all(np.abs(a - b) <= 1e-12 * np.maximum(np.abs(b), 1.0)), f
        assert (a == b).all(), f + " (not bit-identical)"


CASES = [
    ("ba-bits", lambda: graphgen.ba(3000, 3, seed=1), 64, cc.CC_BATCHED, None, 0.2),
    ("rmat-bits", lambda: graphgen.rmat(12, 16, seed=2), 200, cc.CC_BATCHED, (2, 7), 0.5),
    ("grid-weighted", lambda: graphgen.grid(40, 30, 8, 0.1, 1, 1000, seed=4), 48, cc.CC_BATCHED, None, 0.0),
    ("rmat-dir-rt", lambda: graphgen.rmat(10, 16, seed=3, directed=True), 96, cc.CC_BATCHED, None, 0.3),
    ("ba-plain", lambda: graphgen.ba(2000, 3, seed=5), 20, cc.CC_PLAIN, (1, 3), 0.2),
    ("ba-k300", lambda: graphgen.ba(2500, 4, seed=6), 300, cc.CC_BATCHED, None, 0.1),
    ("grid-ones", lambda: graphgen.grid(30, 25, 4), 37, cc.CC_BATCHED, (1, 1), -1.0),
]


@pytest.mark.parametrize("name,make,k,mode,eps,zero", CASES, ids=[c[0] for c in CASES])
def test_weighted_matches_oracle(ctx, name, make, k, mode, eps, zero):
    g = make()
    rg = graphgen.transpose(g) if g.directed else None
    beta = (graphgen.node_weights(g.n, 11, zero_frac=zero) if zero >= 0 else
            (np.random.default_rng(3).random(g.n) < 0.5).astype(np.uint32))  # 0/1 weights
    _say(f"  {name}: n={g.n} k={k}")
    ref = oracle.estimate_weighted(g, beta, k, 7, eps=eps, threads=8, reverse_graph=rg)
    gh = ctx.upload(g)
    try:
        got = cc.cc_estimate_weighted(ctx.handle, gh, beta, k, seed=7, mode=mode, eps=eps)
    finally:
        ctx.release(gh)
    _check(got, ref)


@pytest.mark.parametrize("k,front,extra,seed", [(16, 64, {150: 3, 299: 1}, 7), (64, 128, {299: 1}, 8),
                                                (15, 32, {299: 1}, 8)])
def test_weighted_error_with_empty_hc(ctx, k, front, extra, seed):
    """A path of 300 nodes whose positive weights sit at the front (plus a
    few far nodes the sample leaves out): for the nodes past the samples every
    sample lies within Delta/eps of the pivot, so HC is empty while H still
    has weight, and the error estimate takes Sec. 4.1's mean over the samples
    farthest from the pivot (16 and 64 samples: rows of 4 and 16 pieces; 15
    samples: one lane per node)."""
    g = graphgen.path(300)
    beta = np.zeros(g.n, np.uint32)
    beta[:front] = 1
    for u, b in extra.items():
        beta[u] = b
    ref = oracle.estimate_weighted(g, beta, k, seed, eps=(1, 2), threads=8)
    assert 299 not in set(np.asarray(ref["samples"]).tolist())  # a weighted node beyond every sample
    gh = ctx.upload(g)
    try:
        got = cc.cc_estimate_weighted(ctx.handle, gh, beta, k, seed=seed, eps=(1, 2))
    finally:
        ctx.release(gh)
    _check(got, ref)


def test_weighted_exact_when_all_positive_nodes_sampled(ctx):
    g = graphgen.ba(1500, 3, seed=9)
    beta = graphgen.node_weights(g.n, 4, zero_frac=0.9)
    k = int((beta > 0).sum()) + 5
    gh = ctx.upload(g)
    try:
        got = cc.cc_estimate_weighted(ctx.handle, gh, beta, k, seed=1)
    finally:
        ctx.release(gh)
    assert got["sample_size"] == int((beta > 0).sum()) and got["tau"] == 0.0
    D = oracle.sample_distances(g, np.arange(g.n, dtype=np.int32), threads=8)
    exact = (D * beta.astype(np.int64)[:, None]).sum(axis=0)
    assert (got["S_beta"] == exact.astype(np.float64)).all() and (got["S_beta_var"] == 0).all()


def test_weighted_rejects_bad_input(ctx):
    g = graphgen.ba(300, 3, seed=2)
    gh = ctx.upload(g)
    try:
        with pytest.raises(cc.CCError) as e:
            cc.cc_estimate_weighted(ctx.handle, gh, np.zeros(g.n, np.uint32), 8)
        assert e.value.status == cc.CC_EINVAL
    finally:
        ctx.release(gh)


def test_weighted_fullsize_sampled_nodes(ctx):
    """R-MAT scale 20 (k = 256, heavy-tailed weights with 20% zeros), the
    configuration `bench.py --beta` times: sampled nodes from the oracle's
    walk over the sample distances."""
    spec = graphgen.WORKLOADS["rmat20"]
    k, seed = spec["k"], spec["sample_seed"]
    _say("  generating rmat20")
    g = graphgen.workload("rmat20")
    beta = graphgen.node_weights(g.n, seed)
    gh = ctx.upload(g)
    try:
        got = cc.cc_estimate_weighted(ctx.handle, gh, beta, k, seed=seed)
        t = cc.cc_last_timing(ctx.handle)
        _say(f"  estimate: {t['total_ms']:.2f} ms traversal")
    finally:
        ctx.release(gh)
    ids, light, R, m = oracle.draw_weighted([int(b) for b in beta], k, seed)
    assert (got["samples"] == np.array(ids)).all() and got["tau"] == R / m
    _say("  oracle distances")
    D = oracle.sample_distances(g, np.array(ids, np.int32), threads=8)
    rng = np.random.default_rng(seed)
    nodes = np.unique(np.concatenate([rng.integers(0, g.n, size=8), ids[:2], [0, g.n - 1]])).astype(np.int32)
    ref = oracle.estimate_weighted(g, beta, k, seed, threads=8, D=D, sample=(ids, light, R, m), nodes=nodes)
    for j, v in enumerate(nodes):
        assert got["S_beta"][v] == ref["S_beta"][j], int(v)
        assert got["S_beta_var"][v] == ref["S_beta_var"][j], int(v)
        assert got["S_beta_err"][v] == ref["S_beta_err"][j], int(v)
