"""Launch shapes and thresholds change speed, never results: estimates under
extreme settings of every knob, and after the autotuner has picked its own,
are bit-identical to those under the defaults (and so to the oracle's, which
the parity tests establish for the defaults)."""
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


@pytest.fixture(scope="module")
def ctx():
    c = cc.Context(0)
    yield c
    c.close()


def _same(a, b, what):
    for f in a:
        assert np.array_equal(a[f], b[f]), f"{what}: {f}"


BFS_SETTINGS = [dict(alpha=1), dict(alpha=1024), dict(level_blocks=1), dict(scatter_blocks=1),
                dict(level_blocks=1, scatter_blocks=3, alpha=2), dict(level_blocks=65535, scatter_blocks=65535)]


@pytest.mark.parametrize("make,k", [(lambda: graphgen.ba(3000, 3, seed=4), 100),
                                    (lambda: graphgen.rmat(12, 16, seed=7), 256),
                                    (lambda: graphgen.rmat(11, 16, seed=9, directed=True), 64)])
def test_bfs_knobs_do_not_change_results(ctx, make, k):
    g = make()
    gh = ctx.upload(g)
    try:
        ref = cc.cc_estimate(ctx.handle, gh, k, seed=3, outputs=ALL)
        default = cc.cc_graph_get_tuning(gh)
        for setting in BFS_SETTINGS:
            _say(f"  {g.name} k={k} {setting}")
            cc.cc_graph_set_tuning(gh, **{**default, **setting})
            _same(ref, cc.cc_estimate(ctx.handle, gh, k, seed=3, outputs=ALL), str(setting))
    finally:
        ctx.release(gh)


def test_weighted_knobs_do_not_change_results(ctx):
    g = graphgen.grid(70, 60, 8, 0.1, 1, 1000, seed=5)
    gh = ctx.upload(g)
    try:
        samples = oracle.draw_samples(g.n, 48, 6)
        ref = cc.cc_estimate(ctx.handle, gh, 48, seed=6, outputs=ALL)
        orc = oracle.estimate_all(g, samples, threads=8)
        assert np.array_equal(ref["D"], orc["D"])
        default = cc.cc_graph_get_tuning(gh)
        assert default["delta"] >= 1
        for setting in [dict(delta=1), dict(delta=1 << 30), dict(local_passes=0), dict(local_passes=1024),
                        dict(round_blocks=1), dict(round_blocks=7, local_passes=3, delta=17)]:
            _say(f"  weighted grid {setting}")
            cc.cc_graph_set_tuning(gh, **{**default, **setting})
            _same(ref, cc.cc_estimate(ctx.handle, gh, 48, seed=6, outputs=ALL), str(setting))
    finally:
        ctx.release(gh)


def test_invalid_tuning_rejected(ctx):
    gh = ctx.upload(graphgen.path(20))
    try:
        before = cc.cc_graph_get_tuning(gh)
        for bad in (dict(alpha=0), dict(alpha=2000), dict(level_blocks=0), dict(scatter_blocks=70000),
                    dict(delta=0), dict(round_blocks=0), dict(local_passes=-1), dict(local_passes=5000)):
            with pytest.raises(cc.CCError) as e:
                cc.cc_graph_set_tuning(gh, **bad)
            assert e.value.status == cc.CC_EINVAL, bad
        assert cc.cc_graph_get_tuning(gh) == before
    finally:
        ctx.release(gh)


@pytest.mark.parametrize("make,k", [(lambda: graphgen.rmat(13, 16, seed=11), 128),
                                    (lambda: graphgen.grid(40, 40, 8, 0.1, 1, 1000, seed=2), 32)])
def test_autotune_keeps_results(ctx, make, k):
    g = make()
    gh = ctx.upload(g)
    try:
        ref = cc.cc_estimate(ctx.handle, gh, k, seed=1, outputs=ALL)
        best, ms = cc.cc_autotune(ctx.handle, gh, k, seed=1, reps=1)
        _say(f"  autotune {g.name}: {best} {ms:.3f} ms")
        assert ms > 0
        assert cc.cc_graph_get_tuning(gh) == best
        _same(ref, cc.cc_estimate(ctx.handle, gh, k, seed=1, outputs=ALL), "autotuned")
        # another sample set under the tuned setting still matches the oracle
        samples = oracle.draw_samples(g.n, k, 2)
        got = cc.cc_estimate(ctx.handle, gh, k, seed=2, outputs=("D", "pivot", "S_hyb"))
        orc = oracle.estimate_all(g, samples, threads=8)
        assert np.array_equal(got["D"], orc["D"]) and np.array_equal(got["pivot"], orc["pivot"])
        assert np.array_equal(got["S_hyb"], orc["S_hyb"])
    finally:
        ctx.release(gh)


@pytest.mark.parametrize("level_blocks", [1024, 100, 65])
def test_merge_grid_not_a_multiple_of_64(ctx, level_blocks):
    """R-MAT scale 16 (46,754 nodes, 731 64-node groups): the merge launch
    takes min(ceil(731 / 4), level_blocks) = 183, 100 or 65 blocks, more than
    the 64 counter slots and not a multiple of 64, so the slots of the level
    decision's two-step ticket hold different numbers of blocks.  Every output
    against the oracle, for every node."""
    g = graphgen.rmat(16, 16, seed=21)
    k = 192
    gh = ctx.upload(g)
    try:
        cc.cc_graph_set_tuning(gh, level_blocks=level_blocks)
        got = cc.cc_estimate(ctx.handle, gh, k, seed=4, outputs=ALL)
    finally:
        ctx.release(gh)
    samples = np.asarray(oracle.draw_samples(g.n, k, 4), dtype=np.int32)
    ref = oracle.estimate_tails(g, samples, threads=8, adaptive_eps=())
    assert np.array_equal(got["samples"], samples)
    for f in ALL:
        assert np.array_equal(got[f], np.asarray(ref[f]).astype(got[f].dtype).reshape(got[f].shape)), f
