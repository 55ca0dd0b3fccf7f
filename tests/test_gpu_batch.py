"""Several small graphs in one traversal (cc_estimate_batch, and the serving
slots that batch queued small jobs): every output of every job is identical
to that job run alone, whatever the mix of sizes, sample counts and word
positions; jobs that cannot be batched, or whose graph turns out
disconnected, come back with their own result or status."""
import sys

import numpy as np
import pytest

import graphgen
import oracle
import paper_1409_0035_amd as cc

pytestmark = pytest.mark.gpu
ALL = ("S_hyb", "S_samp", "S_piv", "S_pub", "pivot", "delta", "sampsum", "src_sum", "samples", "dmat", "D")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(a, b, what):
    for f in b:
        assert np.array_equal(a[f], b[f]), f"{what}: {f}"


@pytest.fixture(scope="module")
def ctx():
    c = cc.Context(0)
    yield c
    c.close()


def test_batch_matches_single_runs(ctx):
    # uneven sizes and degree skews; k of 1..3 words; ragged k
    graphs = [graphgen.ba(3000, 3, seed=1), graphgen.rmat(11, 16, seed=2), graphgen.grid(40, 30, 4),
              graphgen.ba(9000, 4, seed=3), graphgen.rmat(13, 16, seed=4), graphgen.path(300),
              graphgen.star(500), graphgen.ba(700, 2, seed=5)]
    ks = [16, 64, 33, 100, 64, 7, 130, 50]
    eps = [None, (1, 3), None, (2, 5), None, (1, 2), None, (1, 1)]
    hs = [ctx.upload(g) for g in graphs]
    try:
        jobs = [(h, k, 10 + j, e) for j, (h, k, e) in enumerate(zip(hs, ks, eps))]
        res, sts = cc.cc_estimate_batch(ctx.handle, jobs, outputs=ALL)
        assert sts == [cc.CC_OK] * len(jobs)
        for j, (h, k, seed, e) in enumerate(jobs):
            _say(f"  job {j}: {graphs[j].name} n={graphs[j].n} k={k}")
            alone = cc.cc_estimate(ctx.handle, h, k, seed=seed, eps=e, outputs=ALL)
            _same(res[j], alone, f"job {j}")
        # and against the oracle for two of them
        for j in (1, 3):
            samples = oracle.draw_samples(graphs[j].n, ks[j], 10 + j)
            ref = oracle.estimate_all(graphs[j], samples, eps=eps[j], threads=8)
            assert np.array_equal(res[j]["D"], ref["D"])
            assert np.array_equal(res[j]["S_hyb"], ref["S_hyb"])
            assert np.array_equal(res[j]["pivot"], ref["pivot"])
    finally:
        for h in hs:
            ctx.release(h)


def test_batch_with_jobs_that_run_alone_or_fail(ctx):
    """A digraph and a weighted graph run alone; a disconnected graph makes
    its batch fall back to single runs, where only that job fails."""
    gd = graphgen.rmat(10, 16, seed=6, directed=True)
    gw = graphgen.grid(30, 20, 8, 0.1, 1, 1000, seed=7)
    two = graphgen.csr_from_arcs(8, [0, 1, 2, 4, 5, 6], [1, 2, 3, 5, 6, 7])  # two paths
    gb = graphgen.ba(2000, 3, seed=8)
    gs = [gd, gb, two, gw, graphgen.ba(1500, 2, seed=9)]
    ks = [32, 40, 2, 20, 64]
    hs = [ctx.upload(g) for g in gs]
    try:
        jobs = [(h, k, 3 + j) for j, (h, k) in enumerate(zip(hs, ks))]
        res, sts = cc.cc_estimate_batch(ctx.handle, jobs, outputs=("S_hyb", "pivot", "dmat"))
        assert sts[2] == cc.CC_EDISCONNECTED
        for j in (0, 1, 3, 4):
            assert sts[j] == cc.CC_OK, j
            alone = cc.cc_estimate(ctx.handle, hs[j], ks[j], seed=3 + j, outputs=("S_hyb", "pivot", "dmat"))
            _same(res[j], alone, f"job {j}")
    finally:
        for h in hs:
            ctx.release(h)


def test_serving_batches_small_jobs(ctx):
    """One serving slot, many small queued jobs: the slot takes them in
    batches; every result equals the job alone."""
    graphs = [graphgen.ba(1000 + 300 * j, 3, seed=20 + j) if j % 2 else graphgen.rmat(10, 16, seed=20 + j)
              for j in range(12)]
    ks = [16, 64, 32, 48, 16, 100, 64, 8, 20, 64, 130, 16]
    with cc.Context(0, max_inflight=1) as sctx:
        hs = [sctx.upload(g) for g in graphs]
        alone = [cc.cc_estimate(sctx.handle, h, k, seed=j, outputs=ALL) for j, (h, k) in enumerate(zip(hs, ks))]
        sub = [cc.cc_submit(sctx.handle, h, k, seed=j, outputs=ALL) for j, (h, k) in enumerate(zip(hs, ks))]
        for j, job in enumerate(sub):
            _same(cc.cc_wait(job), alone[j], f"served job {j}")
            cc.cc_job_release(job)
