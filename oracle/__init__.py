"""CPU ORACLE for the sample-based closeness estimators -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import, build, load or call anything in this package.  The
GPU library (``paper_1409_0035_amd``) never imports it and shares no code with
it; the only module both sides use is ``graphgen`` (input construction).

What it computes (Cohen, Delling, Pajor & Werneck 2014):
  * distances from each sampled node by plain BFS / binary-heap Dijkstra
    (Sec. 3), round-trip distances on strongly connected digraphs (Sec. 6.1);
  * the pivot c(v) and Delta(v) (Sec. 2), the sample average Eq. (5), the
    pivot estimate, the pivoting upper bound (Sec. 1), and the hybrid
    estimate Eq. (6), by an explicit walk over all nodes per estimated node;
  * the estimated squared error of the hybrid estimate (Sec. 4.1), the
    adaptive estimate that picks, per node, the eps of a list with the
    smallest estimated error (Sec. 4, eps list of Sec. 8), and the threshold
    sweep of Algorithm 2 (Sec. 4.2);
  * the outbound / inbound reachability sampling of Sec. 6.2 (Algorithm 4)
    from its definition;
  * exact S(v) for every node (Eq. (1)) by one search per node.

Pins (closed forms, special cases, worked examples, brute force) live in
``tests/test_oracle_pins.py``; every function here is pinned by them.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

from .sampler import draw_samples, draw_weighted  # noqa: F401  (re-export)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c (gcc -O2, no fast-math, no FP contraction)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread",
                               "-ffp-contract=off", "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class NodeOut(ctypes.Structure):
    _fields_ = [("pivot", ctypes.c_int32), ("delta", ctypes.c_int64), ("sampsum", ctypes.c_int64),
                ("S_piv", ctypes.c_int64), ("S_pub", ctypes.c_int64), ("S_samp", ctypes.c_double),
                ("S_hyb", ctypes.c_double), ("L_num", ctypes.c_int64), ("LC_num", ctypes.c_int64),
                ("HC_num", ctypes.c_int64), ("H_num", ctypes.c_int64), ("LC_sum", ctypes.c_int64),
                ("HC_sum", ctypes.c_int64), ("H_sum", ctypes.c_int64), ("N", ctypes.c_int64),
                ("overflow", ctypes.c_int32), ("sampled", ctypes.c_int32), ("LC_sumsq", ctypes.c_int64),
                ("HC_sqerr", ctypes.c_int64), ("S_err", ctypes.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=True)
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64, i32 = ctypes.c_int64, ctypes.c_int32
    lib.orc_bfs.restype = i64
    lib.orc_bfs.argtypes = [i64, P, P, i32, P]
    lib.orc_dijkstra.restype = i64
    lib.orc_dijkstra.argtypes = [i64, P, P, P, i32, P]
    lib.orc_sample_distances.restype = ctypes.c_int
    lib.orc_sample_distances.argtypes = [i64, P, P, P, P, P, P, i32, P, i32, P]
    lib.orc_pivot.restype = i32
    lib.orc_pivot.argtypes = [i32, P]
    lib.orc_node_estimates.restype = ctypes.c_int
    lib.orc_node_estimates.argtypes = [i64, i32, i64, P, P, P, i64, i64, i64, ctypes.POINTER(NodeOut)]
    lib.orc_estimate_all.restype = ctypes.c_int
    lib.orc_estimate_all.argtypes = [i64, i32, P, P, i64, i64, i32, P, P, P, P, P, P, P, P, P, P, i32, P, P, P, P]
    lib.orc_node_sweep.restype = ctypes.c_int
    lib.orc_node_sweep.argtypes = [i64, i32, i64, P, P, P, i64, ctypes.POINTER(ctypes.c_double),
                                   ctypes.POINTER(ctypes.c_double)]
    lib.orc_node_adaptive.restype = ctypes.c_int
    lib.orc_node_adaptive.argtypes = [i64, i32, i64, P, P, P, i64, P, P, i32, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]
    lib.orc_estimate_tails.restype = ctypes.c_int
    lib.orc_estimate_tails.argtypes = [i64, i32, P, P, P, P, i32, i32, P, P, P, P, P, P, P, P, P, P, P, P]
    lib.orc_exact_sums.restype = ctypes.c_int
    lib.orc_exact_sums.argtypes = [i64, P, P, P, P, P, P, i32, P]
    lib.orc_beta_all.restype = ctypes.c_int
    lib.orc_beta_all.argtypes = [i64, i32, P, P, P, i64, i32, P, i64, i64, P, i64, i32, P, P, P]
    lib.orc_reach_beta.restype = ctypes.c_int
    lib.orc_reach_beta.argtypes = [i64, P, P, P, P, P, P, i64, i32, P, i64, i32, P, P, P, P]
    lib.orc_reach_all.restype = ctypes.c_int
    lib.orc_reach_all.argtypes = [i64, P, P, P, P, i32, P, i64, i32, P, P, P, P, P]
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


def default_eps(k: int) -> tuple[int, int]:
    """eps = 1/round(sqrt(k)) as num/den (the paper's eps = sqrt(1/k), Sec. 8)."""
    return 1, max(1, int(round(math.sqrt(k))))


class OracleError(RuntimeError):
    pass


def sssp(g, src: int, reverse_graph=None) -> np.ndarray:
    """Distances from src (int64, -1 = unreachable).  With reverse_graph (the
    transpose of a digraph) the result is the round-trip distance."""
    lib = _load()
    out = np.empty(g.n, dtype=np.int64)
    rp, col, w = _c(g.row_ptr, np.int64), _c(g.col_idx, np.int32), _c(g.w, np.int32)
    if w is None:
        lib.orc_bfs(g.n, _p(rp), _p(col), int(src), _p(out))
    else:
        lib.orc_dijkstra(g.n, _p(rp), _p(col), _p(w), int(src), _p(out))
    if reverse_graph is not None:
        back = sssp(reverse_graph, src)
        bad = (out < 0) | (back < 0)
        out = out + back
        out[bad] = -1
    return out


def sample_distances(g, samples, threads: int = 1, reverse_graph=None) -> np.ndarray:
    """Node-major D[v, i] = d(c_i, v) (int64), round-trip when reverse_graph is given."""
    lib = _load()
    samples = np.ascontiguousarray(samples, dtype=np.int32)
    k = int(samples.shape[0])
    D = np.empty((g.n, k), dtype=np.int64)
    rg = reverse_graph
    st = lib.orc_sample_distances(
        g.n, _p(_c(g.row_ptr, np.int64)), _p(_c(g.col_idx, np.int32)), _p(_c(g.w, np.int32)),
        None if rg is None else _p(_c(rg.row_ptr, np.int64)),
        None if rg is None else _p(_c(rg.col_idx, np.int32)),
        None if rg is None else _p(_c(rg.w, np.int32)),
        k, _p(samples), int(threads), _p(D))
    if st == 2:
        raise OracleError("graph is not (strongly) connected: a node is unreachable from a sample")
    if st != 0:
        raise OracleError(f"orc_sample_distances failed ({st})")
    return D


def sample_index(n: int, samples) -> np.ndarray:
    sidx = np.full(n, -1, dtype=np.int32)
    for i, c in enumerate(samples):
        sidx[int(c)] = i
    return sidx


# The eps values the experiments of Sec. 8 choose from per node for the
# adaptive hybrid estimate, as exact fractions.
ADAPTIVE_EPS = ((1, 1000), (1, 40), (1, 20), (1, 10), (1, 5), (1, 2), (99, 100))


def estimate_all(g, samples, eps=None, D=None, threads: int = 1, reverse_graph=None,
                 adaptive_eps=ADAPTIVE_EPS, sweep: bool = False) -> dict:
    """Every estimator for every node (O(n^2) hybrid walk: small graphs only).
    Also returns D, the per-sample sums S(c_i) and the sample distance matrix
    dmat[i, j] = d(c_i, c_j)."""
    lib = _load()
    samples = np.ascontiguousarray(samples, dtype=np.int32)
    k = int(samples.shape[0])
    en, ed = eps if eps is not None else default_eps(k)
    if D is None:
        D = sample_distances(g, samples, threads=threads, reverse_graph=reverse_graph)
    D = np.ascontiguousarray(D, dtype=np.int64)
    n = g.n
    sidx = sample_index(n, samples)
    out = dict(pivot=np.empty(n, np.int32), delta=np.empty(n, np.int64), sampsum=np.empty(n, np.int64),
               S_piv=np.empty(n, np.int64), S_pub=np.empty(n, np.int64), S_samp=np.empty(n, np.float64),
               S_hyb=np.empty(n, np.float64), S_err=np.empty(n, np.float64), S_ad=np.empty(n, np.float64),
               S_ad_err=np.empty(n, np.float64), S_sweep=np.empty(n, np.float64),
               S_sweep_err=np.empty(n, np.float64))
    ad = list(adaptive_eps or ())
    ad_n = np.array([a for a, _ in ad] or [1], dtype=np.int64)
    ad_d = np.array([b for _, b in ad] or [1], dtype=np.int64)
    st = lib.orc_estimate_all(n, k, _p(sidx), _p(D), int(en), int(ed), int(threads),
                              _p(out["pivot"]), _p(out["delta"]), _p(out["sampsum"]), _p(out["S_piv"]),
                              _p(out["S_pub"]), _p(out["S_samp"]), _p(out["S_hyb"]), _p(out["S_err"]),
                              _p(ad_n), _p(ad_d), len(ad), _p(out["S_ad"]) if ad else None,
                              _p(out["S_ad_err"]) if ad else None, _p(out["S_sweep"]) if sweep else None,
                              _p(out["S_sweep_err"]) if sweep else None)
    if not sweep:
        del out["S_sweep"], out["S_sweep_err"]
    if not ad:
        del out["S_ad"], out["S_ad_err"]
    if st != 0:
        raise OracleError(f"orc_estimate_all failed ({st})")
    out["D"] = D
    out["src_sum"] = D.sum(axis=0)               # S(c_i) = sum_v d(c_i, v)
    out["dmat"] = D[samples, :].T.copy()         # dmat[i, j] = D[c_j, i] = d(c_i, c_j)
    out["samples"] = samples
    out["eps"] = (en, ed)
    return out


def estimate_tails(g, samples, eps=None, D=None, threads: int = 1, reverse_graph=None,
                   adaptive_eps=ADAPTIVE_EPS) -> dict:
    """Every node at any size, with Algorithm 1's accounting (Sec. 3): the
    sums over H(v) from each pivot sample's sorted distances and suffix sums,
    the samples split by their distance from the pivot.  Gives the same values
    as estimate_all (pinned against it), without its O(n^2) walk: pivot,
    delta, sampsum, src_sum, dmat, S_piv, S_pub, S_samp, S_hyb, S_err, and
    S_ad / S_ad_err over adaptive_eps."""
    lib = _load()
    samples = np.ascontiguousarray(samples, dtype=np.int32)
    k = int(samples.shape[0])
    en, ed = eps if eps is not None else default_eps(k)
    if D is None:
        D = sample_distances(g, samples, threads=threads, reverse_graph=reverse_graph)
    D = np.ascontiguousarray(D, dtype=np.int64)
    n = g.n
    sidx = sample_index(n, samples)
    ad = list(adaptive_eps or ())
    nums = np.array([en] + [a for a, _ in ad], dtype=np.int64)
    dens = np.array([ed] + [b for _, b in ad], dtype=np.int64)
    out = dict(pivot=np.empty(n, np.int32), delta=np.empty(n, np.int64), sampsum=np.empty(n, np.int64),
               src_sum=np.empty(k, np.int64), dmat=np.empty((k, k), np.int64), S_piv=np.empty(n, np.int64),
               S_pub=np.empty(n, np.int64), S_samp=np.empty(n, np.float64), S_hyb=np.empty(n, np.float64),
               S_err=np.empty(n, np.float64), S_ad=np.empty(n, np.float64), S_ad_err=np.empty(n, np.float64))
    st = lib.orc_estimate_tails(n, k, _p(sidx), _p(D), _p(nums), _p(dens), len(nums), int(threads),
                                *[_p(out[f]) for f in ("pivot", "delta", "sampsum", "src_sum", "dmat", "S_piv",
                                                       "S_pub", "S_samp", "S_hyb", "S_err", "S_ad", "S_ad_err")])
    if not ad:
        del out["S_ad"], out["S_ad_err"]
    if st == 3:
        raise OracleError("out of memory")
    if st not in (0, 4):
        raise OracleError(f"orc_estimate_tails failed ({st})")
    out["overflow"] = st == 4
    out["D"] = D
    out["samples"] = samples
    out["eps"] = (en, ed)
    return out


def node_estimates(g, samples, v: int, eps=None, reverse_graph=None, row=None) -> NodeOut:
    """Estimators for one node v straight from the definitions, with two
    searches: one from v (its distances to the samples) and one from its
    pivot c_p (the column d(c_p, .)).  Works at any graph size."""
    lib = _load()
    samples = np.ascontiguousarray(samples, dtype=np.int32)
    k = int(samples.shape[0])
    en, ed = eps if eps is not None else default_eps(k)
    if row is None:
        # undirected: d(c_i, v) = d(v, c_i); round trip is symmetric as well
        dv = sssp(g, v, reverse_graph)
        row = dv[samples]
    row = np.ascontiguousarray(row, dtype=np.int64)
    if (row < 0).any():
        raise OracleError("unreachable sample")
    p = int(lib.orc_pivot(k, _p(row)))
    colp = sssp(g, int(samples[p]), reverse_graph)
    if (colp < 0).any():
        raise OracleError("unreachable node")
    sidx = sample_index(g.n, samples)
    o = NodeOut()
    st = lib.orc_node_estimates(g.n, k, int(v), _p(sidx), _p(row), _p(colp), 1, int(en), int(ed),
                                ctypes.byref(o))
    if st not in (0, 4):
        raise OracleError(f"orc_node_estimates failed ({st})")
    return o


def node_adaptive(g, samples, v: int, adaptive_eps=ADAPTIVE_EPS, reverse_graph=None):
    """The adaptive hybrid estimate of one node (Sec. 4 / Sec. 8): the eps of
    the list whose estimate has the smallest estimated squared error.
    Returns (S_ad, S_ad_err, index of the chosen eps)."""
    lib = _load()
    samples = np.ascontiguousarray(samples, dtype=np.int32)
    k = int(samples.shape[0])
    row = np.ascontiguousarray(sssp(g, v, reverse_graph)[samples], dtype=np.int64)
    p = int(lib.orc_pivot(k, _p(row)))
    colp = sssp(g, int(samples[p]), reverse_graph)
    sidx = sample_index(g.n, samples)
    ad_n = np.array([a for a, _ in adaptive_eps], dtype=np.int64)
    ad_d = np.array([b for _, b in adaptive_eps], dtype=np.int64)
    a, e, w = ctypes.c_double(), ctypes.c_double(), ctypes.c_int32()
    st = lib.orc_node_adaptive(g.n, k, int(v), _p(sidx), _p(row), _p(colp), 1, _p(ad_n), _p(ad_d),
                               len(adaptive_eps), ctypes.byref(a), ctypes.byref(e), ctypes.byref(w))
    if st not in (0, 4):
        raise OracleError(f"orc_node_adaptive failed ({st})")
    return a.value, e.value, w.value


def node_sweep(g, samples, v: int, reverse_graph=None):
    """The threshold-sweep estimate of one node (Algorithm 2 / Sec. 4.2) and
    its estimated squared error, with two searches (from v and its pivot)."""
    lib = _load()
    samples = np.ascontiguousarray(samples, dtype=np.int32)
    k = int(samples.shape[0])
    row = np.ascontiguousarray(sssp(g, v, reverse_graph)[samples], dtype=np.int64)
    p = int(lib.orc_pivot(k, _p(row)))
    colp = sssp(g, int(samples[p]), reverse_graph)
    sidx = sample_index(g.n, samples)
    a, e = ctypes.c_double(), ctypes.c_double()
    st = lib.orc_node_sweep(g.n, k, int(v), _p(sidx), _p(row), _p(colp), 1, ctypes.byref(a), ctypes.byref(e))
    if st not in (0, 4):
        raise OracleError(f"orc_node_sweep failed ({st})")
    return a.value, e.value


def exact_sums(g, threads: int = 1, reverse_graph=None) -> np.ndarray:
    """S(v) for every node, n searches (round-trip with reverse_graph)."""
    lib = _load()
    S = np.empty(g.n, dtype=np.int64)
    rg = reverse_graph
    st = lib.orc_exact_sums(g.n, _p(_c(g.row_ptr, np.int64)), _p(_c(g.col_idx, np.int32)),
                            _p(_c(g.w, np.int32)),
                            None if rg is None else _p(_c(rg.row_ptr, np.int64)),
                            None if rg is None else _p(_c(rg.col_idx, np.int32)),
                            None if rg is None else _p(_c(rg.w, np.int32)), int(threads), _p(S))
    if st != 0:
        raise OracleError(f"orc_exact_sums failed ({st})")
    return S


def rank_of(order) -> np.ndarray:
    """rank[u] = position of u in the order (a permutation of the nodes)."""
    order = np.asarray(order, dtype=np.int64)
    rank = np.empty(order.shape[0], dtype=np.int32)
    rank[order] = np.arange(order.shape[0], dtype=np.int32)
    return rank


def reach_all(g, order, k: int, inbound: bool = False, threads: int = 1, reverse_graph=None, nodes=None) -> dict:
    """Sec. 6.2 / Algorithm 4 from its definition: for every node (or for the
    listed nodes, one search each, outputs in list order) the bottom-k sample
    (first k in `order`) of the nodes it reaches (outbound) or that reach it
    (inbound, searching the transpose), with count, distsum, T and the
    estimates B (average distance) and R (reachability)."""
    lib = _load()
    h = g
    if inbound:
        if reverse_graph is None:
            from graphgen import transpose
            reverse_graph = transpose(g)
        h = reverse_graph
    n = g.n
    rank = rank_of(order)
    sel = None if nodes is None else np.ascontiguousarray(nodes, dtype=np.int32)
    m = n if sel is None else sel.shape[0]
    out = dict(count=np.empty(m, np.int32), distsum=np.empty(m, np.int64), T=np.empty(m, np.int64),
               B=np.empty(m, np.float64), R=np.empty(m, np.float64))
    st = lib.orc_reach_all(n, _p(_c(h.row_ptr, np.int64)), _p(_c(h.col_idx, np.int32)), _p(_c(h.w, np.int32)),
                           _p(rank), int(k), _p(sel), int(m), int(threads), _p(out["count"]), _p(out["distsum"]),
                           _p(out["T"]), _p(out["B"]), _p(out["R"]))
    if st != 0:
        raise OracleError(f"orc_reach_all failed ({st})")
    return out


def estimate_weighted(g, beta, k: int, seed: int, eps=None, threads: int = 1, reverse_graph=None, D=None,
                      sample=None, nodes=None) -> dict:
    """Sec. 5: the node-weighted hybrid estimate of S_beta(v) = sum_u beta(u)
    d(v,u) for every node (O(n^2) walk: small graphs) or for the listed nodes
    (outputs in list order), from the sample of draw_weighted (or `sample` =
    (ids, light flags, R, m)), with its variance estimate; also the sample,
    tau = R/m and the adjusted weights."""
    lib = _load()
    beta = np.ascontiguousarray(beta, dtype=np.uint32)
    ids, light, R, m = sample if sample is not None else draw_weighted([int(b) for b in beta], k, seed)
    ids = np.ascontiguousarray(ids, dtype=np.int32)
    kk = int(ids.shape[0])
    if eps is None:
        r = int(round(math.sqrt(kk)))
        eps = (1, max(r, 1))
    if D is None:
        D = sample_distances(g, ids, threads=threads, reverse_graph=reverse_graph)
    D = np.ascontiguousarray(D, dtype=np.int64)
    sidx = sample_index(g.n, ids)
    lf = np.ascontiguousarray(light, dtype=np.uint8)
    sel = None if nodes is None else np.ascontiguousarray(nodes, dtype=np.int32)
    cnt = g.n if sel is None else sel.shape[0]
    out = dict(S_beta=np.empty(cnt, np.float64), S_beta_var=np.empty(cnt, np.float64),
               S_beta_err=np.empty(cnt, np.float64))
    st = lib.orc_beta_all(g.n, kk, _p(sidx), _p(lf), _p(beta), int(R), int(m), _p(D), int(eps[0]), int(eps[1]),
                          _p(sel), int(cnt), int(threads), _p(out["S_beta"]), _p(out["S_beta_var"]),
                          _p(out["S_beta_err"]))
    if st not in (0, 4):
        raise OracleError(f"orc_beta_all failed ({st})")
    tau = R / m
    out.update(samples=ids, light=np.asarray(light, bool), R=int(R), m=int(m), tau=float(tau),
               adjusted=np.array([tau if lt else float(beta[v]) for v, lt in zip(ids, light)]), D=D,
               status=st)
    return out


def priority_numerators(n: int, seed: int) -> np.ndarray:
    """U(u) in [1, 2^53] for the priority ranks of Sec. 6.2 / Algorithm 5:
    (x >> 11) + 1 for the u-th output x of SplitMix64(seed), u = 0..n-1."""
    from .sampler import SplitMix64
    rng = SplitMix64(seed)
    return np.array([(rng.next() >> 11) + 1 for _ in range(n)], dtype=np.uint64)


def priority_order(beta, U) -> np.ndarray:
    """The nodes with beta > 0 by increasing rank U/beta (exact), ties by id."""
    from functools import cmp_to_key
    pos = [u for u in range(len(beta)) if beta[u] > 0]

    def cmp(a, b):
        x, y = int(U[a]) * int(beta[b]), int(U[b]) * int(beta[a])
        return -1 if x < y or (x == y and a < b) else (1 if (x, a) != (y, b) else 0)
    return np.array(sorted(pos, key=cmp_to_key(cmp)), dtype=np.int32)


def reach_weighted(g, beta, k: int, seed: int, inbound: bool = False, threads: int = 1, reverse_graph=None,
                   nodes=None, U=None) -> dict:
    """Sec. 6.2 / Algorithm 5 from its definition: per node the k members of
    its reachability set with beta > 0 first in priority-rank order, count,
    the k-th member (-1 if fewer), and the estimates S (weighted distance sum)
    and R (weighted reach)."""
    lib = _load()
    h = g
    if inbound:
        if reverse_graph is None:
            from graphgen import transpose
            reverse_graph = transpose(g)
        h = reverse_graph
    beta = np.ascontiguousarray(beta, dtype=np.uint32)
    U = priority_numerators(g.n, seed) if U is None else np.ascontiguousarray(U, dtype=np.uint64)
    by_rank = priority_order(beta, U)
    sel = None if nodes is None else np.ascontiguousarray(nodes, dtype=np.int32)
    m = g.n if sel is None else sel.shape[0]
    out = dict(count=np.empty(m, np.int32), kth=np.empty(m, np.int32), S=np.empty(m, np.float64),
               R=np.empty(m, np.float64))
    st = lib.orc_reach_beta(g.n, _p(_c(h.row_ptr, np.int64)), _p(_c(h.col_idx, np.int32)), _p(_c(h.w, np.int32)),
                            _p(beta), _p(U), _p(by_rank), int(by_rank.shape[0]), int(k), _p(sel), int(m), int(threads),
                            _p(out["count"]), _p(out["kth"]), _p(out["S"]), _p(out["R"]))
    if st != 0:
        raise OracleError(f"orc_reach_beta failed ({st})")
    out["order"] = by_rank
    return out
