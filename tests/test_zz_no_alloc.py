"""cc_estimate_device_noalloc: the allocation-free variant of
cc_estimate_device, called through the C ABI, must return exactly what
cc_estimate_device returns (bit for bit, which is within the 1e-12 relative
bar of the estimates), on two calls in a row, the second on a smaller graph
(the static scratch keeps the first call's contents), and refuse what its
static scratch cannot hold or what it does not run."""
import ctypes
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


def _outputs(n, k, torch):
    out = {f: torch.full((n,), -7, dtype=getattr(torch, dt), device="cuda") for f, dt in FIELDS.items()}
    out["src_sum"] = torch.full((k,), -7, dtype=torch.int64, device="cuda")
    out["samples"] = torch.full((k,), -7, dtype=torch.int32, device="cuda")
    out["dmat"] = torch.full((k * k,), -7, dtype=torch.int32, device="cuda")
    out["D"] = torch.full((n * k,), -7, dtype=torch.int32, device="cuda")
    out["S_err"] = torch.full((n,), -7, dtype=torch.float64, device="cuda")
    return out


def _run(ctx, gh, n, k, seed, noalloc, torch):
    out = _outputs(n, k, torch)
    cc.cc_estimate_device(ctx.handle, gh, k, out, seed=seed, noalloc=noalloc)
    torch.cuda.synchronize()
    return {f: t.cpu().numpy() for f, t in out.items()}


def test_noalloc_matches_estimate_device():
    import torch
    cases = [(graphgen.rmat(14, 16, seed=51), 200, 3), (graphgen.ba(3000, 3, seed=52), 64, 4)]
    with cc.Context(0) as ctx:
        for g, k, seed in cases:  # the second call is on a smaller graph
            _say(f"  {g.name}: n={g.n} arcs={g.arcs} k={k}")
            gh = ctx.upload(g)
            try:
                a = _run(ctx, gh, g.n, k, seed, True, torch)
                b = _run(ctx, gh, g.n, k, seed, False, torch)
            finally:
                ctx.release(gh)
            for f in a:
                if a[f].dtype.kind == "f":
                    assert np.all(np.abs(a[f] - b[f]) <= 1e-12 * np.abs(b[f])), f
                assert np.array_equal(a[f], b[f]), f"{g.name}: {f}"


def test_noalloc_refuses_what_it_cannot_run():
    import torch
    with cc.Context(0) as ctx:
        # too large for the static scratch: 64 MiB of level masks alone
        big = graphgen.rmat(18, 16, seed=53)
        gh = ctx.upload(big)
        try:
            out = {"S_hyb": torch.empty(big.n, dtype=torch.float64, device="cuda"),
                   "D": torch.empty(big.n * 256, dtype=torch.int32, device="cuda")}
            with pytest.raises(cc.CCError) as e:
                cc.cc_estimate_device(ctx.handle, gh, 256, out, seed=1, noalloc=True)
            assert e.value.status == cc.CC_ENOMEM
        finally:
            ctx.release(gh)
        # a digraph, a weighted graph, plain mode: not run
        for g, kw in ((graphgen.rmat(10, 8, seed=54, directed=True), {}), (graphgen.grid(10, 10, 8, 0.1, 1, 9), {}),
                      (graphgen.ba(500, 3, seed=55), {"mode": cc.CC_PLAIN})):
            gh = ctx.upload(g)
            try:
                out = {"S_hyb": torch.empty(g.n, dtype=torch.float64, device="cuda")}
                with pytest.raises(cc.CCError) as e:
                    cc.cc_estimate_device(ctx.handle, gh, 8, out, seed=1, noalloc=True, **kw)
                assert e.value.status == cc.CC_EINVAL
            finally:
                ctx.release(gh)
        # after the refusals the array still serves a call
        g = graphgen.ba(2000, 4, seed=56)
        gh = ctx.upload(g)
        try:
            a = _run(ctx, gh, g.n, 64, 9, True, torch)
            b = _run(ctx, gh, g.n, 64, 9, False, torch)
            for f in a:
                assert np.array_equal(a[f], b[f]), f
        finally:
            ctx.release(gh)
