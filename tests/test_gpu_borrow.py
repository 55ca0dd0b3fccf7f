"""cc_graph_borrow_device: a CSR that already sits in device memory (torch
tensors) is used in place.  Every output must equal what the same graph gives
after cc_graph_upload, bit for bit, and what the oracle computes from its own
draw of the samples; bad arrays are rejected before any search runs."""
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


def _tensors(g):
    import torch
    rp = torch.from_numpy(np.ascontiguousarray(g.row_ptr, dtype=np.int64)).cuda()
    col = torch.from_numpy(np.ascontiguousarray(g.col_idx, dtype=np.int32)).cuda()
    w = None if g.w is None else torch.from_numpy(np.ascontiguousarray(g.w, dtype=np.int32)).cuda()
    return rp, col, w


CASES = [
    ("rmat14", lambda: graphgen.rmat(14, 16, seed=31), 200, cc.CC_BATCHED),
    ("ba-hubs", lambda: graphgen.ba(20000, 4, seed=32), 64, cc.CC_BATCHED),
    ("rmat12-dir", lambda: graphgen.rmat(12, 16, seed=33, directed=True), 128, cc.CC_BATCHED),
    ("grid-weighted", lambda: graphgen.grid(60, 40, 8, 0.1, 1, 1000, seed=34), 48, cc.CC_BATCHED),
    ("gnp-dir-weighted", lambda: graphgen.gnp(400, 0.02, 35, directed=True, wmax=50), 32, cc.CC_BATCHED),
    ("rmat12-plain", lambda: graphgen.rmat(12, 16, seed=36), 20, cc.CC_PLAIN),
    ("ba-k300", lambda: graphgen.ba(3000, 3, seed=37), 300, cc.CC_BATCHED),
]


@pytest.mark.parametrize("name,make,k,mode", CASES, ids=[c[0] for c in CASES])
def test_borrowed_equals_uploaded_and_oracle(ctx, name, make, k, mode):
    g = make()
    seed = 5
    flags = cc.CC_DIRECTED if g.directed else 0
    rp, col, w = _tensors(g)
    _say(f"  {name}: n={g.n} arcs={g.arcs} k={k} mode={mode}")
    gb = cc.cc_graph_borrow_device(ctx.handle, g.n, g.arcs, rp, col, w, flags | cc.CC_VALIDATE)
    try:
        got = cc.cc_estimate(ctx.handle, gb, k, mode=mode, seed=seed, outputs=ALL)
        again = cc.cc_estimate(ctx.handle, gb, k, mode=mode, seed=seed, outputs=ALL)
    finally:
        cc.cc_graph_release(gb)
    gu = ctx.upload(g)
    try:
        ref = cc.cc_estimate(ctx.handle, gu, k, mode=mode, seed=seed, outputs=ALL)
    finally:
        ctx.release(gu)
    samples = np.asarray(oracle.draw_samples(g.n, k, seed), dtype=np.int32)
    orc = oracle.estimate_tails(g, samples, threads=8, adaptive_eps=(),
                                reverse_graph=graphgen.transpose(g) if g.directed else None)
    for f in ALL:
        assert np.array_equal(got[f], ref[f]), f"{name}: {f} differs from the uploaded graph"
        assert np.array_equal(got[f], again[f]), f"{name}: {f} differs between calls"
        assert np.array_equal(got[f], np.asarray(orc[f]).astype(got[f].dtype).reshape(got[f].shape)), \
            f"{name}: {f} differs from the oracle"
    # the caller's tensors are untouched
    assert np.array_equal(col.cpu().numpy(), g.col_idx) and np.array_equal(rp.cpu().numpy(), g.row_ptr)


def test_borrowed_device_outputs_and_replays(ctx):
    """Device outputs and CC_GRAPH replays on a borrowed graph."""
    import torch
    g = graphgen.rmat(13, 16, seed=38)
    k = 128
    rp, col, _ = _tensors(g)
    gb = cc.cc_graph_borrow_device(ctx.handle, g.n, g.arcs, rp, col)
    try:
        out = {"S_hyb": torch.empty(g.n, dtype=torch.float64, device="cuda"),
               "pivot": torch.empty(g.n, dtype=torch.int32, device="cuda")}
        ref = cc.cc_estimate(ctx.handle, gb, k, seed=3, outputs=("S_hyb", "pivot"))
        for _ in range(3):
            cc.cc_estimate_device(ctx.handle, gb, k, out, mode=cc.CC_BATCHED | cc.CC_GRAPH, seed=3)
            torch.cuda.synchronize()
            assert np.array_equal(out["S_hyb"].cpu().numpy(), ref["S_hyb"])
            assert np.array_equal(out["pivot"].cpu().numpy(), ref["pivot"])
    finally:
        cc.cc_graph_release(gb)


def test_borrowed_reach_and_serving(ctx):
    """Reachability sampling and a served job on a borrowed digraph."""
    g = graphgen.rmat(11, 8, seed=39, directed=True, component=False)
    rp, col, _ = _tensors(g)
    gb = cc.cc_graph_borrow_device(ctx.handle, g.n, g.arcs, rp, col, None, cc.CC_DIRECTED)
    gu = ctx.upload(g)
    try:
        a = cc.cc_reach_estimate(ctx.handle, gb, 16, seed=4)
        b = cc.cc_reach_estimate(ctx.handle, gu, 16, seed=4)
        for f in a:
            assert np.array_equal(a[f], b[f]), f
    finally:
        cc.cc_graph_release(gb)
        ctx.release(gu)
    h = graphgen.ba(5000, 3, seed=40)
    rp, col, _ = _tensors(h)
    with cc.Context(0, max_inflight=2) as sctx:
        gb = cc.cc_graph_borrow_device(sctx.handle, h.n, h.arcs, rp, col)
        alone = cc.cc_estimate(sctx.handle, gb, 64, seed=9, outputs=("S_hyb", "pivot"))
        jobs = [cc.cc_submit(sctx.handle, gb, 64, seed=9, outputs=("S_hyb", "pivot")) for _ in range(4)]
        cc.cc_graph_release(gb)  # stays alive while the jobs run
        for j in jobs:
            r = cc.cc_wait(j)
            assert np.array_equal(r["S_hyb"], alone["S_hyb"]) and np.array_equal(r["pivot"], alone["pivot"])
            cc.cc_job_release(j)


def test_borrow_rejects_bad_arrays(ctx):
    import torch
    g = graphgen.path(50)
    rp, col, _ = _tensors(g)
    bad_col = col.clone()
    bad_col[7] = g.n  # out of range
    bad_rp = rp.clone()
    bad_rp[3] = bad_rp[4] + 1  # decreasing
    w0 = torch.zeros(g.arcs, dtype=torch.int32, device="cuda")  # length 0
    lib = cc.load_library()
    import ctypes
    for args, what in (((rp, bad_col, None, 0), "id range"), ((bad_rp, col, None, 0), "row bounds"),
                       ((rp, col, w0, 0), "lengths")):
        with pytest.raises(cc.CCError) as e:
            cc.cc_graph_borrow_device(ctx.handle, g.n, g.arcs, *args)
        assert e.value.status == cc.CC_EINVAL, what
    # host memory is not device memory
    host_rp = np.ascontiguousarray(g.row_ptr, dtype=np.int64)
    host_col = np.ascontiguousarray(g.col_idx, dtype=np.int32)
    out = ctypes.c_void_p()
    st = lib.cc_graph_borrow_device(ctx.handle, g.n, g.arcs, ctypes.c_void_p(host_rp.ctypes.data),
                                    ctypes.c_void_p(host_col.ctypes.data), None, 0, ctypes.byref(out))
    assert st == cc.CC_EINVAL
    # an undirected CSR that is not symmetric, with CC_VALIDATE
    a = graphgen.csr_from_arcs(4, [0, 1, 2], [1, 2, 3], symmetrize=False, directed=True)
    rp, col, _ = _tensors(a)
    with pytest.raises(cc.CCError) as e:
        cc.cc_graph_borrow_device(ctx.handle, a.n, a.arcs, rp, col, None, cc.CC_VALIDATE)
    assert e.value.status == cc.CC_EINVAL
