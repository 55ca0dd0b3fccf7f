"""Captured estimates (CC_GRAPH): the first call runs eagerly and captures a
HIP graph; later calls with the same graph, k, eps, outputs and stream
replay it.  Every replay is checked against an eager estimate of the same
samples, with the program's own eager GPU work and synchronisations between
replays, and samples that change from call to call."""
import sys

import numpy as np
import pytest

import graphgen
import paper_1409_0035_amd as cc

pytestmark = pytest.mark.gpu
FIELDS = {"S_hyb": "float64", "S_samp": "float64", "S_piv": "int64", "S_pub": "int64", "pivot": "int32",
          "delta": "int32", "sampsum": "int64"}


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


ERR_FIELDS = {"S_err": "float64", "S_ad": "float64", "S_ad_err": "float64", "S_sweep": "float64",
              "S_sweep_err": "float64"}


def _outputs(torch, n, fields=FIELDS):
    return {f: torch.empty(n, dtype=getattr(torch, dt), device="cuda") for f, dt in fields.items()}


@pytest.mark.parametrize("make,k", [(lambda: graphgen.ba(5000, 4, seed=3), 64),
                                    (lambda: graphgen.rmat(12, 16, seed=5), 200),
                                    (lambda: graphgen.rmat(12, 16, seed=6, directed=True), 128),
                                    (lambda: graphgen.rmat(11, 8, seed=7, directed=True), 40)],
                         ids=["ba5000-k64", "rmat12-k200", "rmat12dir-k128-round-trip", "rmat11dir-k40-round-trip"])
def test_replays_match_eager(make, k):
    import torch
    g = make()
    with cc.Context(0) as ctx:
        gh = ctx.upload(g)
        s = torch.cuda.Stream()
        cap_out = _outputs(torch, g.n)   # the captured graph writes these
        ref_out = _outputs(torch, g.n)   # eager estimates to compare with
        x = torch.randn(256, 256, device="cuda")
        replays = 0
        for it, seed in enumerate([1, 1, 1, 2, 2, 1, 3, 3]):
            _say(f"  {g.name} k={k} call {it} seed {seed}")
            cc.cc_estimate_device(ctx.handle, gh, k, cap_out, mode=cc.CC_BATCHED | cc.CC_GRAPH, seed=seed,
                                  stream=s)
            t = cc.cc_last_timing(ctx.handle)
            replays += t["launches"] == 1
            # the program's own work on the same stream and a sync between calls
            with torch.cuda.stream(s):
                y = (x @ x).sum()
            s.synchronize()
            assert torch.isfinite(y)
            cc.cc_estimate_device(ctx.handle, gh, k, ref_out, mode=cc.CC_BATCHED, seed=seed, stream=s)
            s.synchronize()
            for f in FIELDS:
                assert torch.equal(cap_out[f], ref_out[f]), (it, seed, f)
        _say(f"  replays: {replays}")
        assert replays >= 4  # the repeated calls after the first of each level count replay
        ctx.release(gh)


def test_host_outputs_accept_graph_flag():
    """With host outputs the staging buffers differ per call, so each call is
    eager; the flag must not change results."""
    g = graphgen.ba(2000, 3, seed=8)
    with cc.Context(0) as ctx:
        gh = ctx.upload(g)
        a = cc.cc_estimate(ctx.handle, gh, 40, mode=cc.CC_BATCHED | cc.CC_GRAPH, seed=4)
        b = cc.cc_estimate(ctx.handle, gh, 40, mode=cc.CC_BATCHED, seed=4)
        for f in a:
            assert np.array_equal(a[f], b[f]), f
        with pytest.raises(cc.CCError) as e:
            cc.cc_estimate(ctx.handle, gh, 40, mode=cc.CC_PLAIN | cc.CC_GRAPH, seed=4)
        assert e.value.status == cc.CC_EINVAL
        ctx.release(gh)


def test_replays_with_error_outputs():
    """Calls that alternate between two output sets -- with and without the
    Sec. 4 and threshold-sweep outputs -- replay their own captures: each
    set is keyed separately and every replay matches an eager estimate."""
    import torch
    g = graphgen.rmat(12, 16, seed=6)
    k = 96
    both = {**FIELDS, **ERR_FIELDS}
    with cc.Context(0) as ctx:
        gh = ctx.upload(g)
        s = torch.cuda.Stream()
        plain_out, err_out = _outputs(torch, g.n), _outputs(torch, g.n, both)
        ref_plain, ref_err = _outputs(torch, g.n), _outputs(torch, g.n, both)
        replays = 0
        for it, (seed, which) in enumerate([(1, 0), (1, 1), (1, 0), (1, 1), (2, 1), (2, 0), (2, 1)]):
            out, ref, fields = (plain_out, ref_plain, FIELDS) if which == 0 else (err_out, ref_err, both)
            _say(f"  call {it} seed {seed} {'errors' if which else 'plain'}")
            for t in out.values():
                t.fill_(-1)
            cc.cc_estimate_device(ctx.handle, gh, k, out, mode=cc.CC_BATCHED | cc.CC_GRAPH, seed=seed, stream=s)
            replays += cc.cc_last_timing(ctx.handle)["launches"] == 1
            cc.cc_estimate_device(ctx.handle, gh, k, ref, mode=cc.CC_BATCHED, seed=seed, stream=s)
            s.synchronize()
            for f in fields:
                assert torch.equal(out[f], ref[f]), (it, seed, f)
        _say(f"  replays: {replays}")
        assert replays >= 3
        ctx.release(gh)


def test_replays_write_samples():
    """A captured estimate takes its samples from the lane's pinned staging
    buffer in its first launch, which also writes the `samples` output: every
    replay's samples and estimates match an eager batched estimate, and the
    samples match the plain path's (copied from the host) for the same seed."""
    import torch
    g = graphgen.rmat(12, 16, seed=9)
    k = 128
    fields = {**FIELDS}
    with cc.Context(0) as ctx:
        gh = ctx.upload(g)
        s = torch.cuda.Stream()
        out, ref = _outputs(torch, g.n), _outputs(torch, g.n)
        for d in (out, ref):
            d["samples"] = torch.empty(k, dtype=torch.int32, device="cuda")
        plain = {"samples": torch.empty(k, dtype=torch.int32, device="cuda")}
        replays = 0
        for it, seed in enumerate([5, 5, 6, 6, 6, 5, 7, 7]):
            _say(f"  call {it} seed {seed}")
            for t in out.values():
                t.fill_(-1)
            cc.cc_estimate_device(ctx.handle, gh, k, out, mode=cc.CC_BATCHED | cc.CC_GRAPH, seed=seed, stream=s)
            replays += cc.cc_last_timing(ctx.handle)["launches"] == 1
            cc.cc_estimate_device(ctx.handle, gh, k, ref, mode=cc.CC_BATCHED, seed=seed, stream=s)
            cc.cc_estimate_device(ctx.handle, gh, k, plain, mode=cc.CC_PLAIN, seed=seed, stream=s)
            s.synchronize()
            assert torch.equal(out["samples"], plain["samples"]), (it, seed)
            for f in (*fields, "samples"):
                assert torch.equal(out[f], ref[f]), (it, seed, f)
        _say(f"  replays: {replays}")
        assert replays >= 4
        ctx.release(gh)


@pytest.mark.parametrize("k", [40, 128, 256])
def test_round_trip_replays_match_oracle(k):
    """Round-trip estimates (Sec. 6.1) replayed from a captured graph: both
    searches, the distances and the D-based epilogue, with the Sec. 4
    outputs, against the oracle's every-node accounting for each seed."""
    import torch
    import oracle
    g = graphgen.rmat(11, 16, seed=6, directed=True)
    rg = graphgen.transpose(g)
    fields = {**FIELDS, "S_err": "float64", "S_ad": "float64", "S_ad_err": "float64"}
    refs = {}
    with cc.Context(0) as ctx:
        gh = ctx.upload(g)
        out = _outputs(torch, g.n, fields)
        replays = 0
        for it, seed in enumerate([4, 4, 4, 9, 9, 4]):
            if seed not in refs:
                samples = np.asarray(oracle.draw_samples(g.n, k, seed), dtype=np.int32)
                refs[seed] = oracle.estimate_tails(g, samples, threads=8, reverse_graph=rg)
            for t in out.values():
                t.fill_(-1)
            cc.cc_estimate_device(ctx.handle, gh, k, out, mode=cc.CC_BATCHED | cc.CC_GRAPH, seed=seed)
            replays += cc.cc_last_timing(ctx.handle)["launches"] == 1
            torch.cuda.synchronize()
            ref = refs[seed]
            for f in fields:
                got = out[f].cpu().numpy()
                assert np.array_equal(got, np.asarray(ref[f]).astype(got.dtype)), (it, seed, f)
        _say(f"  k={k}: {replays} replays")
        assert replays >= 3
        ctx.release(gh)


@pytest.mark.parametrize("make,k", [(lambda: graphgen.grid(60, 50, 8, 0.1, 1, 1000, seed=3), 64),
                                    (lambda: graphgen.gnp(400, 0.02, 35, directed=True, wmax=50), 32)],
                         ids=["grid-weighted-k64", "gnp-dir-weighted-k32-round-trip"])
def test_weighted_replays_match_oracle(make, k):
    """Weighted estimates replayed from a captured graph (the searches, the
    distances and the D-based epilogue), against the oracle for each seed,
    with seeds whose searches reach further than the captured ones."""
    import torch
    import oracle
    g = make()
    rg = graphgen.transpose(g) if g.directed else None
    fields = {**FIELDS, "S_err": "float64", "S_ad": "float64", "S_ad_err": "float64"}
    refs = {}
    with cc.Context(0) as ctx:
        gh = ctx.upload(g)
        out = _outputs(torch, g.n, fields)
        replays = 0
        for it, seed in enumerate([4, 4, 4, 9, 9, 9, 4]):
            if seed not in refs:
                samples = np.asarray(oracle.draw_samples(g.n, k, seed), dtype=np.int32)
                refs[seed] = oracle.estimate_tails(g, samples, threads=8, reverse_graph=rg)
            for t in out.values():
                t.fill_(-1)
            cc.cc_estimate_device(ctx.handle, gh, k, out, mode=cc.CC_BATCHED | cc.CC_GRAPH, seed=seed)
            replays += cc.cc_last_timing(ctx.handle)["launches"] == 1
            torch.cuda.synchronize()
            ref = refs[seed]
            for f in fields:
                got = out[f].cpu().numpy()
                assert np.array_equal(got, np.asarray(ref[f]).astype(got.dtype)), (it, seed, f)
        _say(f"  {g.name} k={k}: {replays} replays")
        assert replays >= 3
        ctx.release(gh)
