"""Serving on the GPU: jobs submitted while others run are admitted as slots
and memory free up, overlap on the device, and return exactly what the same
job returns when run alone and what the oracle computes for it from its own
draw of the samples (every output bit-identical, which is within the 1e-12
relative tolerance of the estimates)."""
import sys
import time

import numpy as np
import pytest

import graphgen
import oracle
import paper_1409_0035_amd as cc
from paper_1409_0035_amd import serve

pytestmark = pytest.mark.gpu
ALL = ("S_hyb", "S_samp", "S_piv", "S_pub", "pivot", "delta", "sampsum", "src_sum", "samples", "dmat", "D")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _mix():
    """A small mix of the serving workload's kinds and a few others: BA and
    R-MAT of uneven sizes, every k of the mix, a weighted grid, a digraph
    (round trip) and a plain-mode job."""
    jobs = graphgen.serving_mix(24, seed=11, n_lo=1e3, n_hi=3e4)
    graphs = [graphgen.make_job_graph(j) for j in jobs]
    for i, j in enumerate(jobs):
        j["graph"], j["mode"] = i, cc.CC_BATCHED
    extra = [(graphgen.grid(60, 50, 8, 0.1, 1, 1000, seed=3), 64, cc.CC_BATCHED),
             (graphgen.rmat(11, 16, seed=6, directed=True), 128, cc.CC_BATCHED),
             (graphgen.ba(4000, 3, seed=9), 16, cc.CC_PLAIN),
             (graphgen.ba(2500, 4, seed=10), 300, cc.CC_BATCHED)]
    for g, k, mode in extra:
        jobs.append(dict(job=len(jobs), graph=len(graphs), k=k, sample_seed=len(jobs), mode=mode))
        graphs.append(g)
    return jobs, graphs


def _check_same(a, b, what):
    for f in a:
        assert np.array_equal(a[f], b[f]), f"{what}: {f}"


def _oracle_ref(g, k, seed):
    """Every output of a job from the oracle: its own draw of the samples,
    all k searches, every node by Algorithm 1's accounting."""
    samples = np.asarray(oracle.draw_samples(g.n, k, seed), dtype=np.int32)
    rg = graphgen.transpose(g) if g.directed else None
    ref = oracle.estimate_tails(g, samples, threads=8, reverse_graph=rg, adaptive_eps=())
    return ref


def _check_oracle(res, ref, what):
    for f in res:
        want = ref[f]
        assert np.array_equal(res[f], np.asarray(want).astype(res[f].dtype).reshape(res[f].shape)), f"{what}: {f}"


def test_alone_vs_mix():
    jobs, graphs = _mix()
    # a budget well below the sum of the jobs' needs forces admission waits;
    # six slots let admitted jobs overlap
    with cc.Context(0, mem_budget_bytes=48 << 20, max_inflight=6) as ctx:
        hs = [ctx.upload(g) for g in graphs]
        alone = []
        for j in jobs:
            g = graphs[j["graph"]]
            _say(f"  alone job {j['job']} n={g.n} k={j['k']} mode={j['mode']}")
            alone.append(cc.cc_estimate(ctx.handle, hs[j["graph"]], j["k"], mode=j["mode"],
                                        seed=j["sample_seed"], outputs=ALL))
            # the job alone equals the oracle; the served ones must equal it
            _check_oracle(alone[-1], _oracle_ref(g, j["k"], j["sample_seed"]), f"job {j['job']} vs oracle")
        for rep in range(2):
            _say(f"  mix, burst {rep}")
            sub = [cc.cc_submit(ctx.handle, hs[j["graph"]], j["k"], mode=j["mode"], seed=j["sample_seed"],
                                outputs=ALL) for j in jobs]
            for i, h in enumerate(sub):
                _check_same(alone[i], cc.cc_wait(h), f"job {i}")
                q, t = cc.cc_job_times(h)
                assert 0 <= q <= t
                cc.cc_job_release(h)
        _say("  mix, staggered arrivals")
        sub = []
        for j in jobs:
            sub.append(cc.cc_submit(ctx.handle, hs[j["graph"]], j["k"], mode=j["mode"], seed=j["sample_seed"],
                                    outputs=ALL))
            time.sleep(0.0005)
        for i, h in enumerate(sub):
            _check_same(alone[i], cc.cc_wait(h), f"job {i} (staggered)")
            cc.cc_job_release(h)


def test_cancel_queued_job():
    g = graphgen.ba(20000, 4, seed=3)
    with cc.Context(0, max_inflight=1) as ctx:
        gh = ctx.upload(g)
        sub = [cc.cc_submit(ctx.handle, gh, 256, seed=s) for s in range(12)]
        st = cc.cc_cancel(sub[-1])
        assert st in (cc.CC_OK, cc.CC_EBUSY)
        for h in sub[:-1]:
            cc.cc_wait(h)
        if st == cc.CC_OK:
            assert cc.cc_poll(sub[-1]) == cc.CC_ECANCELLED
            with pytest.raises(cc.CCError) as e:
                cc.cc_wait(sub[-1])
            assert e.value.status == cc.CC_ECANCELLED
        else:
            cc.cc_wait(sub[-1])
        for h in sub:
            cc.cc_job_release(h)


def test_graph_release_while_jobs_queued():
    """A graph released by the caller stays alive until its queued jobs end."""
    g = graphgen.rmat(12, 16, seed=8)
    with cc.Context(0, max_inflight=2) as ctx:
        gh = ctx.upload(g)
        ref = cc.cc_estimate(ctx.handle, gh, 64, seed=1, outputs=("S_hyb", "pivot"))
        sub = [cc.cc_submit(ctx.handle, gh, 64, seed=1, outputs=("S_hyb", "pivot")) for _ in range(6)]
        ctx.release(gh)
        for h in sub:
            _check_same(ref, cc.cc_wait(h), "after release")
            cc.cc_job_release(h)


def test_serving_driver_small_mix():
    jobs, graphs = serve.build_mix(32, seed=7, n_lo=1e3, n_hi=5e4, threads=8)
    refs = {}

    def reference(i):  # what the oracle computes for job i
        if i not in refs:
            j = jobs[i]
            refs[i] = _oracle_ref(graphs[j["graph"]], j["k"], j["sample_seed"])
        return refs[i]

    out = serve.serve(jobs, graphs, load=0.8, seed=7, max_inflight=8, reference=reference)
    _say(f"  serving summary: {out}")
    assert out["mismatches"] == []
    assert out["jobs"] == 32
    assert 0 < out["latency_ms"]["p50"] <= out["latency_ms"]["p99"]
    assert out["burst"]["overlap"] > 0
