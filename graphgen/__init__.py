"""Seeded synthetic input graphs, shared by the CPU oracle tests and the GPU tests.

This module holds only input construction: graph generators, component
extraction, relabelling, CSR building and transposition.  It computes no
shortest-path distance and no estimate, so it can serve both sides of a parity
test without making them share any of the method's arithmetic.

Large generators (Barabasi-Albert, R-MAT, grids) run in ``gen.c`` through
ctypes; the closed-form families (path, star, cycle, complete graph) are built
here directly.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c into libgraphgen.so next to it (plain gcc, -O2)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64, i32, u64, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    lib.gg_ba.restype = i64
    lib.gg_ba.argtypes = [i64, i32, u64, P, P]
    lib.gg_rmat.restype = None
    lib.gg_rmat.argtypes = [i32, i64, dbl, dbl, dbl, u64, P, P]
    lib.gg_grid_capacity.restype = i64
    lib.gg_grid_capacity.argtypes = [i32, i32, i32]
    lib.gg_grid.restype = i64
    lib.gg_grid.argtypes = [i32, i32, i32, dbl, i32, i32, u64, P, P, P]
    lib.gg_csr_build.restype = i64
    lib.gg_csr_build.argtypes = [i64, i64, P, P, P, i32, P, P, P]
    lib.gg_lcc.restype = i64
    lib.gg_lcc.argtypes = [i64, P, P, P]
    lib.gg_lscc.restype = i64
    lib.gg_lscc.argtypes = [i64, P, P, P]
    lib.gg_induce.restype = i64
    lib.gg_induce.argtypes = [i64, P, P, P, P, P, P, P]
    lib.gg_transpose.restype = None
    lib.gg_transpose.argtypes = [i64, P, P, P, P, P, P]
    _lib = lib
    return lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


@dataclass
class Graph:
    """CSR graph.  Undirected graphs store both arcs of every edge.

    row_ptr int64[n+1], col_idx int32[arcs] (sorted per row), w int32[arcs]
    (None = unit lengths).  For directed graphs the arcs are u -> col_idx.
    """
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    w: Optional[np.ndarray] = None
    directed: bool = False
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def arcs(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def m(self) -> int:
        """Edges as the paper counts them: undirected edges once, arcs for digraphs."""
        return self.arcs if self.directed else self.arcs // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def csr_from_arcs(n: int, src, dst, w=None, symmetrize: bool = True, directed: bool = False,
                  name: str = "") -> Graph:
    lib = _load()
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = int(src.shape[0])
    cap = 2 * m if symmetrize else m
    rp = np.zeros(n + 1, dtype=np.int64)
    col = np.empty(max(cap, 1), dtype=np.int32)
    wi = None if w is None else np.ascontiguousarray(w, dtype=np.int32)
    wo = None if w is None else np.empty(max(cap, 1), dtype=np.int32)
    arcs = lib.gg_csr_build(n, m, _ptr(src), _ptr(dst), _ptr(wi), 1 if symmetrize else 0,
                            _ptr(rp), _ptr(col), _ptr(wo))
    if arcs < 0:
        raise MemoryError("gg_csr_build failed")
    col = col[:arcs].copy()
    wo = None if wo is None else wo[:arcs].copy()
    return Graph(n=n, row_ptr=rp, col_idx=col, w=wo, directed=directed, name=name)


def largest_component(g: Graph) -> Graph:
    """Largest connected component (undirected) or largest strongly connected
    component (directed), relabelled in increasing original-id order."""
    lib = _load()
    newid = np.empty(max(g.n, 1), dtype=np.int32)
    fn = lib.gg_lscc if g.directed else lib.gg_lcc
    nn = fn(g.n, _ptr(g.row_ptr), _ptr(g.col_idx), _ptr(newid))
    if nn < 0:
        raise MemoryError("component extraction failed")
    rp2 = np.zeros(nn + 1, dtype=np.int64)
    col2 = np.empty(max(g.arcs, 1), dtype=np.int32)
    w2 = None if g.w is None else np.empty(max(g.arcs, 1), dtype=np.int32)
    arcs = lib.gg_induce(g.n, _ptr(g.row_ptr), _ptr(g.col_idx), _ptr(g.w), _ptr(newid),
                         _ptr(rp2), _ptr(col2), _ptr(w2))
    meta = dict(g.meta)
    meta.update(n_before_component=g.n, arcs_before_component=g.arcs)
    return Graph(n=int(nn), row_ptr=rp2, col_idx=col2[:arcs].copy(),
                 w=None if w2 is None else w2[:arcs].copy(), directed=g.directed, name=g.name, meta=meta)


def transpose(g: Graph) -> Graph:
    lib = _load()
    rp2 = np.zeros(g.n + 1, dtype=np.int64)
    col2 = np.empty(max(g.arcs, 1), dtype=np.int32)
    w2 = None if g.w is None else np.empty(max(g.arcs, 1), dtype=np.int32)
    lib.gg_transpose(g.n, _ptr(g.row_ptr), _ptr(g.col_idx), _ptr(g.w), _ptr(rp2), _ptr(col2), _ptr(w2))
    return Graph(n=g.n, row_ptr=rp2, col_idx=col2[:g.arcs].copy(),
                 w=None if w2 is None else w2[:g.arcs].copy(), directed=g.directed, name=g.name + "^T",
                 meta=dict(g.meta))


# ---------------------------------------------------------------------------
# generators

def ba(n: int, m: int = 4, seed: int = 1) -> Graph:
    """Barabasi-Albert preferential attachment, m edges per new node, seed
    clique on m+1 nodes.  Connected by construction."""
    lib = _load()
    cap = m * (m + 1) // 2 + (n - m - 1) * m
    src = np.empty(cap, dtype=np.int32)
    dst = np.empty(cap, dtype=np.int32)
    e = lib.gg_ba(n, m, seed, _ptr(src), _ptr(dst))
    if e < 0:
        raise ValueError("bad BA parameters")
    g = csr_from_arcs(n, src[:e], dst[:e], name=f"ba-n{n}-m{m}-s{seed}")
    g.meta.update(kind="ba", m_per_node=m, seed=seed)
    return g


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 2, directed: bool = False, component: bool = True) -> Graph:
    """R-MAT with 2^scale ids and edge_factor * 2^scale tuples; self-loops and
    duplicates removed; undirected graphs are symmetrised; then the largest
    (strongly) connected component, relabelled."""
    lib = _load()
    n = 1 << scale
    ne = edge_factor * n
    src = np.empty(ne, dtype=np.int32)
    dst = np.empty(ne, dtype=np.int32)
    lib.gg_rmat(scale, ne, a, b, c, seed, _ptr(src), _ptr(dst))
    g = csr_from_arcs(n, src, dst, symmetrize=not directed, directed=directed,
                      name=f"rmat{'-dir' if directed else ''}-s{scale}-ef{edge_factor}-seed{seed}")
    del src, dst
    g.meta.update(kind="rmat", scale=scale, edge_factor=edge_factor, abcd=(a, b, c, 1 - a - b - c), seed=seed)
    return largest_component(g) if component else g


def grid(rows: int, cols: int, nbr: int = 8, pdel: float = 0.0, wlo: int = 1, whi: int = 1,
         seed: int = 3, component: bool = True) -> Graph:
    """rows x cols grid with 4 or 8 neighbours; each edge deleted with
    probability pdel; integer weights uniform in [wlo, whi] (unit if both 1)."""
    lib = _load()
    cap = lib.gg_grid_capacity(rows, cols, nbr)
    src = np.empty(max(cap, 1), dtype=np.int32)
    dst = np.empty(max(cap, 1), dtype=np.int32)
    weighted = not (wlo == 1 and whi == 1)
    w = np.empty(max(cap, 1), dtype=np.int32) if weighted else None
    e = lib.gg_grid(rows, cols, nbr, pdel, wlo, whi, seed, _ptr(src), _ptr(dst), _ptr(w))
    g = csr_from_arcs(rows * cols, src[:e], dst[:e], None if w is None else w[:e],
                      name=f"grid{nbr}-{rows}x{cols}-del{pdel}-w{wlo}_{whi}-s{seed}")
    g.meta.update(kind="grid", rows=rows, cols=cols, nbr=nbr, pdel=pdel, wlo=wlo, whi=whi, seed=seed)
    return largest_component(g) if component and pdel > 0 else g


def with_lengths(g: Graph, wlo: int, whi: int, seed: int) -> Graph:
    """The same arcs with integer lengths uniform in [wlo, whi] (numpy
    PCG64); an undirected graph gets one length per edge, on both of its arcs."""
    rng = np.random.default_rng(seed)
    if g.directed:
        w = rng.integers(wlo, whi + 1, size=g.arcs).astype(np.int32)
        out = Graph(n=g.n, row_ptr=g.row_ptr.copy(), col_idx=g.col_idx.copy(), w=w, directed=True,
                    name=f"{g.name}-w{wlo}_{whi}-s{seed}")
    else:
        src = np.repeat(np.arange(g.n, dtype=np.int32), np.diff(g.row_ptr))
        keep = src < g.col_idx
        s, d = src[keep], g.col_idx[keep]
        w = rng.integers(wlo, whi + 1, size=s.shape[0]).astype(np.int32)
        out = csr_from_arcs(g.n, s, d, w, symmetrize=True, directed=False, name=f"{g.name}-w{wlo}_{whi}-s{seed}")
    out.meta.update(g.meta)
    return out


def path(n: int) -> Graph:
    i = np.arange(n - 1, dtype=np.int32)
    return csr_from_arcs(n, i, i + 1, name=f"path{n}")


def cycle(n: int) -> Graph:
    i = np.arange(n, dtype=np.int32)
    return csr_from_arcs(n, i, (i + 1) % n, name=f"cycle{n}")


def star(n: int) -> Graph:
    """Node 0 is the centre, 1..n-1 the leaves."""
    i = np.arange(1, n, dtype=np.int32)
    return csr_from_arcs(n, np.zeros(n - 1, dtype=np.int32), i, name=f"star{n}")


def complete(n: int) -> Graph:
    s, d = np.triu_indices(n, 1)
    return csr_from_arcs(n, s.astype(np.int32), d.astype(np.int32), name=f"K{n}")


def directed_cycle(n: int) -> Graph:
    i = np.arange(n, dtype=np.int32)
    return csr_from_arcs(n, i, (i + 1) % n, symmetrize=False, directed=True, name=f"dcycle{n}")


def symmetric_digraph(g: Graph) -> Graph:
    """The undirected graph g viewed as a digraph with both arcs of every edge."""
    return Graph(n=g.n, row_ptr=g.row_ptr.copy(), col_idx=g.col_idx.copy(),
                 w=None if g.w is None else g.w.copy(), directed=True, name=g.name + "-as-digraph")


def gnp(n: int, p: float, seed: int, directed: bool = False, wmax: int = 1,
        connect: bool = True) -> Graph:
    """Small random graph G(n, p) (numpy PCG64).  With connect=True a random
    spanning path (undirected) or Hamiltonian cycle (directed) is added so the
    graph is connected / strongly connected.  wmax > 1 draws weights in [1, wmax]."""
    rng = np.random.default_rng(seed)
    if directed:
        mask = rng.random((n, n)) < p
        np.fill_diagonal(mask, False)
        s, d = np.nonzero(mask)
    else:
        s, d = np.triu_indices(n, 1)
        keep = rng.random(s.shape[0]) < p
        s, d = s[keep], d[keep]
    s = list(s)
    d = list(d)
    if connect and n > 1:
        perm = rng.permutation(n)
        for i in range(n - 1):
            s.append(perm[i]); d.append(perm[i + 1])
        if directed:
            s.append(perm[n - 1]); d.append(perm[0])
    s = np.asarray(s, dtype=np.int32)
    d = np.asarray(d, dtype=np.int32)
    w = rng.integers(1, wmax + 1, size=s.shape[0]).astype(np.int32) if wmax > 1 else None
    return csr_from_arcs(n, s, d, w, symmetrize=not directed, directed=directed,
                         name=f"gnp{'-dir' if directed else ''}-n{n}-p{p}-s{seed}")


# ---------------------------------------------------------------------------
# named workloads (sizes and structure of the paper's instance families)

def node_weights(n: int, seed: int, zero_frac: float = 0.2, cap: int = 1 << 20) -> np.ndarray:
    """Integer node weights for the node-weighted estimate (Sec. 5): a
    fraction zero_frac of the nodes weigh 0, the others 1 + floor(10 * U^-0.7)
    (heavy-tailed, U uniform in (0, 1]), capped at `cap` (numpy PCG64)."""
    rng = np.random.default_rng(seed)
    u = 1.0 - rng.random(n)
    w = 1 + np.floor(10.0 * u ** -0.7)
    w = np.minimum(w, cap).astype(np.uint32)
    w[rng.random(n) < zero_frac] = 0
    return w


WORKLOADS = {
    # Barabasi-Albert, 10,000 nodes, 4 edges per new node (~40k edges); 64 samples
    "ba10k": dict(make=lambda: ba(10_000, 4, seed=1), k=64, sample_seed=1),
    # undirected R-MAT scale 20 (a,b,c,d = .57,.19,.19,.05), largest component; 256 samples
    "rmat20": dict(make=lambda: rmat(20, 16, seed=2), k=256, sample_seed=2),
    # 2048 x 2048 8-neighbour grid, 10% of edges deleted, weights U{1..1000}, largest component; 64 samples
    "grid2048w": dict(make=lambda: grid(2048, 2048, 8, 0.10, 1, 1000, seed=3), k=64, sample_seed=3),
    # directed R-MAT scale 22, largest strongly connected component; 128 samples, round-trip distances
    "rmat22dir": dict(make=lambda: rmat(22, 16, seed=4, directed=True), k=128, sample_seed=4),
    # directed R-MAT scale 20, the whole graph (not strongly connected); reachability
    # sampling (Sec. 6.2) with k = 100 as in the paper's directed experiments
    "rmat20dir": dict(make=lambda: rmat(20, 16, seed=6, directed=True, component=False), k=100, sample_seed=6),
    # the same digraph with arc lengths uniform in [1, 1000] (the listing's Dijkstra searches)
    "rmat20dirw": dict(make=lambda: with_lengths(rmat(20, 16, seed=6, directed=True, component=False), 1, 1000, 7),
                       k=100, sample_seed=7),
}


def workload(name: str) -> Graph:
    spec = WORKLOADS[name]
    g = spec["make"]()
    g.meta.update(workload=name, k=spec["k"], sample_seed=spec["sample_seed"])
    return g


def serving_mix(num_jobs: int = 512, seed: int = 5, n_lo: float = 1e3, n_hi: float = 1e6,
                ks=(16, 64, 256)):
    """Job list for the serving workload: each job is a BA (m=4) or R-MAT
    (edge factor 16, scale = round(log2 n)) graph with n log-uniform in
    [n_lo, n_hi], k uniform over `ks`.  Returns dicts with the graph recipe;
    arrival times are drawn by the caller (they depend on the offered load)."""
    rng = np.random.default_rng(seed)
    jobs = []
    for j in range(num_jobs):
        n = int(10 ** rng.uniform(math.log10(n_lo), math.log10(n_hi)))
        kind = "ba" if rng.random() < 0.5 else "rmat"
        k = int(ks[rng.integers(0, len(ks))])
        jobs.append(dict(job=j, kind=kind, n=n, k=k, graph_seed=5000 + j, sample_seed=j))
    return jobs


def make_job_graph(job: dict) -> Graph:
    if job["kind"] == "ba":
        return ba(max(job["n"], 6), 4, seed=job["graph_seed"])
    scale = max(4, int(round(math.log2(job["n"]))))
    return rmat(scale, 16, seed=job["graph_seed"])
