"""GPU parity for the estimated errors, the adaptive estimate (Sec. 4) and
the threshold sweep (Algorithm 2, Sec. 4.2): S_err, S_ad, S_ad_err, S_sweep
and S_sweep_err against the oracle on every code path (snapshot epilogue,
round trip, weighted, one source at a time, more than 256 samples, batches),
bit-identical (both sides evaluate the same exact integers in the same order
of double operations; the bar is a relative error of 1e-12)."""
import sys

import numpy as np
import pytest

import graphgen
import oracle
import paper_1409_0035_amd as cc

pytestmark = pytest.mark.gpu
ERR = ("S_err", "S_ad", "S_ad_err", "S_sweep", "S_sweep_err", "S_hyb", "pivot")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    c = cc.Context(0)
    yield c
    c.close()


def _check(res, ref):
    assert (res["pivot"] == ref["pivot"]).all()
    for f in ("S_err", "S_ad", "S_ad_err", "S_sweep", "S_sweep_err", "S_hyb"):
        a, b = res[f], ref[f]
        assert np.all(np.abs(a - b) <= 1e-12 * np.maximum(np.abs(b), 1.0)), f
        assert (a == b).all(), f + " (not bit-identical)"


CASES = [
    ("ba-bits", lambda: graphgen.ba(3000, 3, seed=1), 64, cc.CC_BATCHED, None),
    ("rmat-bits-eps", lambda: graphgen.rmat(12, 16, seed=2), 200, cc.CC_BATCHED, (2, 7)),
    ("grid-bits-ragged", lambda: graphgen.grid(30, 25, 4), 37, cc.CC_BATCHED, (1, 1)),
    ("rmat-dir-rt", lambda: graphgen.rmat(10, 16, seed=3, directed=True), 96, cc.CC_BATCHED, None),
    ("grid-weighted", lambda: graphgen.grid(40, 30, 8, 0.1, 1, 1000, seed=4), 48, cc.CC_BATCHED, None),
    ("ba-plain", lambda: graphgen.ba(2000, 3, seed=5), 20, cc.CC_PLAIN, (1, 3)),
    ("ba-k300", lambda: graphgen.ba(2500, 4, seed=6), 300, cc.CC_BATCHED, None),
    ("deep-path", lambda: graphgen.path(600), 5, cc.CC_BATCHED, None),
    ("single-sample", lambda: graphgen.ba(800, 3, seed=8), 1, cc.CC_BATCHED, None),
    ("weighted-k130", lambda: graphgen.grid(25, 20, 8, 0.1, 1, 60, seed=9), 130, cc.CC_BATCHED, None),
]


@pytest.mark.parametrize("name,make,k,mode,eps", CASES, ids=[c[0] for c in CASES])
def test_error_estimates_match_oracle(ctx, name, make, k, mode, eps):
    g = make()
    samples = oracle.draw_samples(g.n, k, 7)
    rg = graphgen.transpose(g) if g.directed else None
    _say(f"  {name}: n={g.n} k={k}")
    ref = oracle.estimate_all(g, samples, eps=eps, threads=8, reverse_graph=rg, sweep=True)
    gh = ctx.upload(g)
    try:
        res = cc.cc_estimate(ctx.handle, gh, k, mode=mode, seed=7, eps=eps, outputs=ERR)
    finally:
        ctx.release(gh)
    _check(res, ref)


def test_error_estimates_in_a_batch(ctx):
    graphs = [graphgen.ba(1500, 3, seed=11), graphgen.rmat(10, 16, seed=12), graphgen.grid(20, 20, 8)]
    ks = [16, 100, 40]
    hs = [ctx.upload(g) for g in graphs]
    try:
        res, sts = cc.cc_estimate_batch(ctx.handle, [(h, k, 20 + j) for j, (h, k) in enumerate(zip(hs, ks))],
                                        outputs=ERR)
        assert sts == [cc.CC_OK] * 3
        for j, g in enumerate(graphs):
            ref = oracle.estimate_all(g, oracle.draw_samples(g.n, ks[j], 20 + j), threads=8, sweep=True)
            _check(res[j], ref)
    finally:
        for h in hs:
            ctx.release(h)


def test_sweep_only_outputs(ctx):
    """The sweep alone (no other Sec. 4 output) on the snapshot and the row
    paths."""
    for g, k in ((graphgen.rmat(11, 16, seed=13), 150), (graphgen.grid(30, 30, 8, 0.1, 1, 100, seed=14), 40)):
        samples = oracle.draw_samples(g.n, k, 3)
        ref = oracle.estimate_all(g, samples, threads=8, sweep=True)
        gh = ctx.upload(g)
        try:
            res = cc.cc_estimate(ctx.handle, gh, k, seed=3, outputs=("S_sweep", "S_sweep_err"))
        finally:
            ctx.release(gh)
        assert (res["S_sweep"] == ref["S_sweep"]).all() and (res["S_sweep_err"] == ref["S_sweep_err"]).all()
