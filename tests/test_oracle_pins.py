"""Pins for the CPU oracle: it is checked against things other than itself --
closed forms, special cases where Eq. (6) collapses to a known value, hand
derivations (tests/golden), deterministic inequalities from Sec. 1, and an
all-pairs brute force that shares no search code with it."""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import graphgen
import oracle
from oracle import tiny

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(x) for x in line.split()])
    return np.array(rows, dtype=np.int64)


# ---------------------------------------------------------------- distances

def _s_path(n, v):
    return v * (v + 1) // 2 + (n - 1 - v) * (n - v) // 2


@pytest.mark.parametrize("n", [1, 2, 7, 50])
def test_bfs_path_closed_form(n):
    g = graphgen.path(n) if n > 1 else graphgen.Graph(1, np.zeros(2, np.int64), np.zeros(0, np.int32))
    for s in {0, n // 2, n - 1}:
        d = oracle.sssp(g, s)
        assert (d == np.abs(np.arange(n) - s)).all()


@pytest.mark.parametrize("n", [3, 8, 33])
def test_bfs_cycle_star_complete(n):
    d = oracle.sssp(graphgen.cycle(n), 0)
    i = np.arange(n)
    assert (d == np.minimum(i, n - i)).all()
    d = oracle.sssp(graphgen.star(n), 0)
    assert d[0] == 0 and (d[1:] == 1).all()
    d = oracle.sssp(graphgen.star(n), 1)
    assert d[0] == 1 and d[1] == 0 and (d[2:] == 2).all()
    d = oracle.sssp(graphgen.complete(n), n - 1)
    assert (d[:-1] == 1).all() and d[-1] == 0


@pytest.mark.parametrize("rows,cols", [(5, 7), (9, 4)])
def test_bfs_grids_closed_form(rows, cols):
    g4 = graphgen.grid(rows, cols, 4)
    g8 = graphgen.grid(rows, cols, 8)
    y, x = np.divmod(np.arange(rows * cols), cols)
    for s in (0, rows * cols // 2 + 1, rows * cols - 1):
        sy, sx = divmod(s, cols)
        assert (oracle.sssp(g4, s) == np.abs(y - sy) + np.abs(x - sx)).all()           # L1
        assert (oracle.sssp(g8, s) == np.maximum(np.abs(y - sy), np.abs(x - sx))).all()  # Chebyshev


@pytest.mark.parametrize("seed", range(12))
def test_sssp_vs_floyd_warshall(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(2, 24))
    directed = seed % 3 == 2
    wmax = 1 if seed % 2 == 0 else 9
    g = graphgen.gnp(n, float(rng.uniform(0.05, 0.4)), seed, directed=directed, wmax=wmax)
    fw = tiny.floyd_warshall(g.n, g.row_ptr, g.col_idx, g.w)
    for s in range(n):
        d = oracle.sssp(g, s)
        assert list(d) == [int(x) for x in fw[s]]
    if directed:
        gt = graphgen.transpose(g)
        rt = tiny.round_trip(fw)
        for s in range(n):
            assert list(oracle.sssp(g, s, gt)) == [int(x) for x in rt[s]]


def test_dijkstra_unit_weights_equals_bfs():
    g = graphgen.rmat(10, 8, seed=7)
    gw = graphgen.Graph(g.n, g.row_ptr, g.col_idx, np.ones(g.arcs, np.int32))
    for s in (0, 5, g.n - 1):
        assert (oracle.sssp(g, s) == oracle.sssp(gw, s)).all()


def test_directed_cycle_round_trip():
    n = 11
    g = graphgen.directed_cycle(n)
    gt = graphgen.transpose(g)
    for s in range(n):
        d = oracle.sssp(g, s, gt)
        assert d[s] == 0 and (np.delete(d, s) == n).all()


# ---------------------------------------------------------------- exact sums

def test_exact_sums_closed_forms():
    n = 13
    assert (oracle.exact_sums(graphgen.path(n)) == [_s_path(n, v) for v in range(n)]).all()
    assert (oracle.exact_sums(graphgen.cycle(n)) == n * n // 4).all()
    assert (oracle.exact_sums(graphgen.cycle(12)) == 12 * 12 // 4).all()
    s = oracle.exact_sums(graphgen.star(n))
    assert s[0] == n - 1 and (s[1:] == 2 * n - 3).all()
    assert (oracle.exact_sums(graphgen.complete(n)) == n - 1).all()
    R, C = 6, 5
    g = graphgen.grid(R, C, 4)
    y, x = np.divmod(np.arange(R * C), C)
    want = [C * _s_path(R, yy) + R * _s_path(C, xx) for yy, xx in zip(y, x)]
    assert (oracle.exact_sums(g) == want).all()
    gd = graphgen.directed_cycle(9)
    assert (oracle.exact_sums(gd, reverse_graph=graphgen.transpose(gd)) == 9 * 8).all()


# ---------------------------------------------------------------- estimators

@pytest.mark.parametrize("name,C,n", [("path9_C048_eps1_2.txt", [0, 4, 8], 9),
                                      ("path5_C04_eps1_2.txt", [0, 4], 5)])
def test_worked_examples(name, C, n):
    gold = _read_golden(name)
    r = oracle.estimate_all(graphgen.path(n), C, eps=(1, 2))
    assert (r["pivot"] == gold[:, 1]).all()
    assert (r["delta"] == gold[:, 2]).all()
    assert (r["S_hyb"] == gold[:, 4] / gold[:, 5]).all()      # one rounding of an exact rational
    assert (r["S_samp"] == gold[:, 6] / gold[:, 7]).all()
    sampled = np.isin(np.arange(n), C)
    assert (r["S_hyb"][sampled] == gold[sampled, 3]).all()


def test_tie_break_changes_result():
    """Pivot ties go to the lowest sample index: listing the samples in the
    other order moves node 2 of P_9 to the 80/3 value (and node 6 to 32)."""
    r = oracle.estimate_all(graphgen.path(9), [8, 4, 0], eps=(1, 2))
    assert r["S_hyb"][2] == 80 / 3 and r["S_hyb"][6] == 32.0


@pytest.mark.parametrize("n", [6, 17])
def test_all_sampled_gives_exact(n):
    g = graphgen.gnp(n, 0.3, n, wmax=5)
    S = oracle.exact_sums(g)
    r = oracle.estimate_all(g, list(np.random.default_rng(n).permutation(n)), eps=(1, 3))
    for key in ("S_hyb", "S_samp", "S_piv", "S_pub"):
        assert (r[key] == S).all(), key
    assert (r["delta"] == 0).all()


@pytest.mark.parametrize("k", [1, 3, 10])
def test_complete_graph_exact(k):
    n = 12
    r = oracle.estimate_all(graphgen.complete(n), list(range(2, 2 + k)), eps=(1, 4))
    assert (r["S_hyb"] == n - 1).all()


def test_star_closed_forms():
    n, k = 15, 4
    g = graphgen.star(n)
    # centre sampled (listed second), eps <= 1: an unsampled leaf gets (n-1)(2k-1)/k
    C = [3, 0, 7, 9]
    r = oracle.estimate_all(g, C, eps=(1, 1))
    leaves = [v for v in range(1, n) if v not in C]
    assert (r["S_hyb"][leaves] == (n - 1) * (2 * k - 1) / k).all()
    assert (r["pivot"][leaves] == 1).all()
    # centre unsampled: eps <= 1/2 -> exact n-1 ; 1/2 < eps <= 1 -> 2n-2-k
    C = [3, 5, 7, 9]
    assert oracle.estimate_all(g, C, eps=(1, 2))["S_hyb"][0] == n - 1
    assert oracle.estimate_all(g, C, eps=(2, 3))["S_hyb"][0] == 2 * n - 2 - k
    assert oracle.estimate_all(g, C, eps=(1, 1))["S_hyb"][0] == 2 * n - 2 - k
    # unsampled leaf, centre unsampled: 2(n-1) for every eps <= 1
    for eps in ((1, 1), (1, 2), (1, 10)):
        r = oracle.estimate_all(g, C, eps=eps)
        assert r["S_hyb"][1] == 2 * (n - 1) and r["S_hyb"][2] == 2 * (n - 1)


@pytest.mark.parametrize("seed", range(4))
def test_tiny_eps_reduces_to_sample_average(seed):
    """Delta/eps beyond every distance puts all of V \\ {v} in L(v): Eq. (6)
    becomes (n-1)/k times the sum of the sampled distances, Eq. (5)."""
    g = graphgen.gnp(30, 0.1, 200 + seed, wmax=4)
    C = oracle.draw_samples(g.n, 7, seed)
    D = oracle.sample_distances(g, C)
    r = oracle.estimate_all(g, C, eps=(1, int(D.max()) + 1), D=D)
    assert (r["S_hyb"] == r["S_samp"]).all()


@pytest.mark.parametrize("seed", range(6))
def test_pivot_bounds(seed):
    """Sec. 1 triangle-inequality facts, deterministic for every node:
    S(v) <= S(c(v)) + (n-1) Delta(v)  and  S(c(v)) <= S(v) + (n-1) Delta(v)."""
    g = graphgen.gnp(40, 0.08, 300 + seed, wmax=1 + 5 * (seed % 2))
    C = oracle.draw_samples(g.n, 5, seed)
    S = oracle.exact_sums(g)
    r = oracle.estimate_all(g, C)
    assert (S <= r["S_pub"]).all()
    assert (r["S_piv"] <= S + (g.n - 1) * r["delta"]).all()
    D = r["D"]
    assert (r["delta"] == D.min(axis=1)).all()
    assert (D[np.arange(g.n), r["pivot"]] == r["delta"]).all()
    # lowest index among ties
    first = np.argmax(D == D.min(axis=1, keepdims=True), axis=1)
    assert (r["pivot"] == first).all()


def test_symmetric_digraph_round_trip_doubles():
    g = graphgen.gnp(25, 0.15, 9, wmax=3)
    gd = graphgen.symmetric_digraph(g)
    C = oracle.draw_samples(g.n, 6, 3)
    a = oracle.estimate_all(g, C, eps=(1, 2))
    b = oracle.estimate_all(gd, C, eps=(1, 2), reverse_graph=graphgen.transpose(gd))
    assert (b["pivot"] == a["pivot"]).all()
    assert (b["S_hyb"] == 2 * a["S_hyb"]).all()


@pytest.mark.parametrize("seed", range(40))
def test_oracle_vs_set_brute_force(seed):
    """Random tiny graphs, all eps kinds: the C oracle equals the Fraction /
    Python-set evaluation of Eq. (6) on Floyd-Warshall distances."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 20))
    directed = seed % 4 == 3
    g = graphgen.gnp(n, float(rng.uniform(0.05, 0.5)), seed, directed=directed,
                     wmax=1 if seed % 2 else 6)
    k = int(rng.integers(1, n + 1))
    C = oracle.draw_samples(n, k, seed)
    eps = [(1, 1), (1, 2), (2, 3), (1, 3), (1, 10), (3, 7)][seed % 6]
    fw = tiny.floyd_warshall(g.n, g.row_ptr, g.col_idx, g.w)
    rg = None
    if directed:
        fw = tiny.round_trip(fw)
        rg = graphgen.transpose(g)
    t = tiny.estimates(fw, C, Fraction(*eps))
    r = oracle.estimate_all(g, C, eps=eps, reverse_graph=rg)
    assert list(r["pivot"]) == t["pivot"]
    for key in ("S_hyb", "S_samp", "S_piv", "S_pub"):
        assert [float(x) for x in t[key]] == list(r[key].astype(float)), key


def test_node_estimates_match_all_nodes():
    g = graphgen.ba(300, 3, seed=4)
    C = oracle.draw_samples(g.n, 16, 8)
    r = oracle.estimate_all(g, C)
    for v in (0, 5, 77, 299, int(C[3])):
        o = oracle.node_estimates(g, C, v)
        assert o.pivot == r["pivot"][v] and o.delta == r["delta"][v]
        assert o.S_hyb == r["S_hyb"][v] and o.S_samp == r["S_samp"][v]
        assert o.S_pub == r["S_pub"][v] and o.sampsum == r["sampsum"][v]
        if v not in C:
            assert o.L_num + o.HC_num + o.H_num == g.n - 1
            assert o.LC_num + o.HC_num == len(C)
            assert o.LC_num >= 1


@pytest.mark.parametrize("seed", range(16))
def test_tails_form_equals_definition_walk(seed):
    """Algorithm 1's accounting (tail sums per pivot, estimate_tails) gives
    exactly the values of the literal walk over V per node (estimate_all) on
    random undirected, weighted and round-trip graphs, several eps."""
    rng = np.random.default_rng(1300 + seed)
    n = int(rng.integers(2, 160))
    directed = seed % 4 == 3
    g = graphgen.gnp(n, float(rng.uniform(0.02, 0.2)), 1300 + seed, directed=directed,
                     wmax=[1, 1, 30, 1][seed % 4])
    rg = graphgen.transpose(g) if directed else None
    k = int(rng.integers(1, g.n + 1))
    samples = oracle.draw_samples(g.n, k, seed)
    eps = [(1, 1), (1, 3), (2, 5), None][seed % 4]
    a = oracle.estimate_all(g, samples, eps=eps, reverse_graph=rg)
    b = oracle.estimate_tails(g, samples, eps=eps, D=a["D"], threads=1 + seed % 3)
    for f in ("pivot", "delta", "sampsum", "src_sum", "dmat", "S_piv", "S_pub", "S_samp", "S_hyb", "S_err",
              "S_ad", "S_ad_err"):
        assert np.array_equal(a[f], b[f]), f


def test_tails_form_worked_examples():
    """The hand-derived fixtures through the tails form as well."""
    rows = _read_golden("path7_C01_eps1_suffix.txt")
    out = oracle.estimate_tails(graphgen.path(7), [0, 1], eps=(1, 1))
    for node, hn, hd, en, ed, *_ in rows:
        assert out["S_hyb"][node] == hn / hd and out["S_err"][node] == en / ed, node
    out = oracle.estimate_tails(graphgen.path(9), [0, 4, 8], eps=(1, 2))
    assert list(out["S_hyb"]) == [36, 33, 32, 18, 20, 18, 80 / 3, 33, 36]


def test_sum_invariant_per_sample():
    """S(c_i) = sum over non-sampled u of d(c_i,u) + sum_j dmat[i][j]."""
    g = graphgen.grid(20, 20, 8, 0.1, 1, 50, seed=5)
    C = oracle.draw_samples(g.n, 9, 2)
    r = oracle.estimate_all(g, C)
    D = r["D"]
    mask = np.ones(g.n, bool)
    mask[C] = False
    assert (r["src_sum"] == D[mask].sum(axis=0) + r["dmat"].sum(axis=1)).all()
    assert (r["dmat"] == r["dmat"].T).all() and (np.diag(r["dmat"]) == 0).all()


# ---------------------------------------------------------------- sampler

def test_sampler_properties():
    for n, k, seed in [(10, 10, 1), (1000, 64, 2), (1 << 22, 256, 3), (5, 1, 4)]:
        s = oracle.draw_samples(n, k, seed)
        assert len(s) == k and len(set(s)) == k and min(s) >= 0 and max(s) < n
        assert s == oracle.draw_samples(n, k, seed)
    assert oracle.draw_samples(1000, 64, 2) != oracle.draw_samples(1000, 64, 3)
    # k = n is a permutation
    assert sorted(oracle.draw_samples(50, 50, 9)) == list(range(50))


def test_sampler_uniformity():
    """First draw over n=10 from 20,000 seeds: chi-square well below the
    0.999 quantile for 9 degrees of freedom (27.9)."""
    counts = np.zeros(10)
    for seed in range(20000):
        counts[oracle.draw_samples(10, 1, seed)[0]] += 1
    chi2 = ((counts - 2000) ** 2 / 2000).sum()
    assert chi2 < 27.9


def test_splitmix_bounded_is_exact_on_small_ranges():
    """below(s) is a deterministic function of the 64-bit draws; check its
    range and that s = 1 always yields 0 and s = 2^k uses the top bits."""
    from oracle.sampler import SplitMix64
    r1, r2 = SplitMix64(42), SplitMix64(42)
    for _ in range(1000):
        x = r2.next()
        assert r1.below(8) == x >> 61           # power of two: never rejects
    r = SplitMix64(7)
    assert all(r.below(1) == 0 for _ in range(100))


# ---------------------------------------------------------------- Sec. 4 error estimates

def test_error_estimate_worked_example():
    """Sec. 4.1 on the hand-derived path example (fixture with derivation)."""
    rows = [list(map(int, ln.split())) for ln in open(os.path.join(GOLDEN, "path9_C048_eps1_2_err.txt"))
            if ln.strip() and not ln.startswith("#")]
    g = graphgen.path(9)
    out = oracle.estimate_all(g, [0, 4, 8], eps=(1, 2))
    for node, num, den in rows:
        assert abs(out["S_err"][node] - num / den) <= 1e-15 * max(1.0, num / den), node
    t = tiny.estimates(tiny.floyd_warshall(g.n, g.row_ptr, g.col_idx), [0, 4, 8], Fraction(1, 2))
    assert [x for x in t["S_err"]] == [Fraction(num, den) for _, num, den in rows]


@pytest.mark.parametrize("seed", range(24))
def test_error_and_adaptive_vs_bruteforce(seed):
    rng = np.random.default_rng(900 + seed)
    n = int(rng.integers(3, 26))
    directed = seed % 4 == 3
    g = graphgen.gnp(n, float(rng.uniform(0.15, 0.5)), 900 + seed, directed=directed,
                     wmax=[1, 9, 1, 4][seed % 4])
    if g.n < 3:
        pytest.skip("component too small")
    d = tiny.floyd_warshall(g.n, g.row_ptr, g.col_idx, g.w)
    rg = None
    if directed:
        d = tiny.round_trip(d)
        rg = graphgen.transpose(g)
    if any(x == tiny.INF for r in d for x in r):
        pytest.skip("not connected")
    k = int(rng.integers(1, g.n + 1))
    samples = [int(x) for x in rng.permutation(g.n)[:k]]
    eps = [(1, 1), (1, 2), (2, 7), (1, 5)][seed % 4]
    out = oracle.estimate_all(g, samples, eps=eps, reverse_graph=rg)
    t = tiny.estimates(d, samples, Fraction(*eps))
    for v in range(g.n):
        exact = t["S_err"][v]
        assert abs(out["S_err"][v] - float(exact)) <= 1e-12 * max(1.0, float(exact)), (v, exact)
    eps_list = [Fraction(a, b) for a, b in oracle.ADAPTIVE_EPS]
    per = [tiny.estimates(d, samples, e) for e in eps_list]
    S_ad, S_ad_err, which = tiny.adaptive(d, samples, eps_list)
    for v in range(g.n):
        # the oracle's pick must be one of the exact minimisers (exact ties may
        # be broken differently by rounded errors) and return that eps's estimate
        best = min(p["S_err"][v] for p in per)
        assert S_ad_err[v] == best
        assert abs(out["S_ad_err"][v] - float(best)) <= 1e-12 * max(1.0, float(best)), v
        assert any(p["S_err"][v] == best and abs(out["S_ad"][v] - float(p["S_hyb"][v])) <=
                   1e-12 * float(p["S_hyb"][v]) for p in per), v


def test_error_special_cases():
    # K_n: every distance 1, H and HC empty -> 0
    g = graphgen.complete(12)
    out = oracle.estimate_all(g, [3, 7, 1], eps=(1, 2))
    assert (out["S_err"] == 0).all()
    # k = n: every node sampled -> 0, adaptive = exact
    g = graphgen.ba(40, 2, seed=3)
    out = oracle.estimate_all(g, list(range(g.n)))
    assert (out["S_err"] == 0).all() and (out["S_ad_err"] == 0).all()
    assert (out["S_ad"] == oracle.exact_sums(g)).all()
    # tiny eps: H and HC empty, L = V \ {v}: (n-1)/k times the population
    # variance of the k sample distances
    g = graphgen.grid(9, 7, 4)
    samples = [0, 10, 33, 50, 62]
    out = oracle.estimate_all(g, samples, eps=(1, 1000))
    D = out["D"]
    sampled = set(samples)
    for v in range(g.n):
        if v in sampled:
            continue
        want = np.var(D[v].astype(np.float64)) * (g.n - 1) / len(samples)
        assert abs(out["S_err"][v] - want) <= 1e-9 * max(1.0, want), v


def test_adaptive_properties():
    g = graphgen.rmat(8, 8, seed=4)
    samples = oracle.draw_samples(g.n, 16, 2)
    full = oracle.estimate_all(g, samples)
    per = [oracle.estimate_all(g, samples, eps=e, D=full["D"], adaptive_eps=()) for e in oracle.ADAPTIVE_EPS]
    errs = np.stack([p["S_err"] for p in per])
    hyb = np.stack([p["S_hyb"] for p in per])
    first_min = np.argmin(errs, axis=0)   # numpy: first index among equal minima
    idx = np.arange(g.n)
    assert (full["S_ad_err"] == errs[first_min, idx]).all()
    assert (full["S_ad"] == hyb[first_min, idx]).all()
    # a one-element list is the fixed-eps estimate
    one = oracle.estimate_all(g, samples, eps=(1, 2), D=full["D"], adaptive_eps=((1, 2),))
    assert (one["S_ad"] == one["S_hyb"]).all() and (one["S_ad_err"] == one["S_err"]).all()


# ---------------------------------------------------------------- Algorithm 2 threshold sweep

def test_sweep_worked_example():
    """Algorithm 2 on the hand-derived path example (fixture with derivation)."""
    rows = _read_golden("path9_C048_sweep.txt")
    g = graphgen.path(9)
    out = oracle.estimate_all(g, [0, 4, 8], sweep=True)
    t_est, t_err = tiny.sweep(tiny.floyd_warshall(g.n, g.row_ptr, g.col_idx), [0, 4, 8])
    for node, en, ed, rn, rd in rows:
        assert out["S_sweep"][node] == en / ed, node
        assert abs(out["S_sweep_err"][node] - rn / rd) <= 1e-15 * max(1.0, rn / rd), node
        assert t_est[node] == Fraction(int(en), int(ed)) and t_err[node] == Fraction(int(rn), int(rd)), node
    for node in range(g.n):  # the single-node entry point agrees
        a, e = oracle.node_sweep(g, [0, 4, 8], node)
        assert a == out["S_sweep"][node] and e == out["S_sweep_err"][node]


@pytest.mark.parametrize("seed", range(24))
def test_sweep_vs_bruteforce(seed):
    """Against explicit-set exact arithmetic on small graphs of every kind
    (distance ties included): the chosen error is the exact minimum over the
    candidates and the estimate is that of a candidate attaining it."""
    rng = np.random.default_rng(1700 + seed)
    n = int(rng.integers(3, 24))
    directed = seed % 4 == 3
    g = graphgen.gnp(n, float(rng.uniform(0.15, 0.5)), 1700 + seed, directed=directed,
                     wmax=[1, 9, 1, 5][seed % 4])
    if g.n < 3:
        pytest.skip("component too small")
    d = tiny.floyd_warshall(g.n, g.row_ptr, g.col_idx, g.w)
    rg = None
    if directed:
        d = tiny.round_trip(d)
        rg = graphgen.transpose(g)
    if any(x == tiny.INF for r in d for x in r):
        pytest.skip("not connected")
    k = int(rng.integers(1, g.n + 1))
    samples = [int(x) for x in rng.permutation(g.n)[:k]]
    out = oracle.estimate_all(g, samples, reverse_graph=rg, sweep=True)
    S = [sum(r) for r in d]
    for v in range(g.n):
        if v in samples:
            assert out["S_sweep"][v] == S[v] and out["S_sweep_err"][v] == 0.0
            continue
        cand = tiny.sweep_candidates(d, samples, v)
        best = min(e for _, e in cand)
        assert abs(out["S_sweep_err"][v] - float(best)) <= 1e-12 * max(1.0, float(best)), v
        assert any(e == best and abs(out["S_sweep"][v] - float(s)) <= 1e-12 * float(s) for s, e in cand), v


def test_sweep_single_sample_is_pivoting():
    """k = 1: the threshold T = 0 puts only the sample in L and nothing in HC,
    and its estimate sums d(c,u) over u != v plus d(v,c), which is S(c) on an
    undirected graph.  With HC empty, Sec. 4.1 averages the pivot error over
    the farthest samples, here the pivot itself: Delta^2 per node of H, which
    is the n - 2 other nodes, the same as pure pivoting's Delta^2 (n - 1 - k).
    The tie keeps pure pivoting: S_piv with error Delta^2 (n - 2)."""
    for g in (graphgen.ba(60, 2, seed=5), graphgen.grid(8, 6, 4), graphgen.grid(7, 7, 8, 0.1, 1, 50, seed=3)):
        for s in (0, g.n // 2):
            out = oracle.estimate_all(g, [s], sweep=True)
            un = np.arange(g.n) != s
            assert (out["S_sweep"][un] == out["S_piv"][un].astype(np.float64)).all()
            want = out["delta"][un].astype(np.float64) ** 2 * (g.n - 2)
            assert (out["S_sweep_err"][un] == want).all()


def test_empty_hc_suffix_worked_example():
    """Sec. 4.1's fallback for an empty HC, on a hand-derived fixture where
    HC is empty and H is not (the samples sit at one end of a path): S_hyb,
    S_err and the threshold sweep of Algorithm 2, node by node."""
    rows = _read_golden("path7_C01_eps1_suffix.txt")
    g = graphgen.path(7)
    out = oracle.estimate_all(g, [0, 1], eps=(1, 1), sweep=True)
    d = tiny.floyd_warshall(g.n, g.row_ptr, g.col_idx)
    t = tiny.estimates(d, [0, 1], Fraction(1, 1))
    sw, swe = tiny.sweep(d, [0, 1])
    for node, hn, hd, en, ed, sn, sd, sen, sed in rows:
        assert out["S_hyb"][node] == hn / hd and t["S_hyb"][node] == Fraction(hn, hd), node
        assert out["S_err"][node] == en / ed and t["S_err"][node] == Fraction(en, ed), node
        assert out["S_sweep"][node] == sn / sd and sw[node] == Fraction(sn, sd), node
        assert out["S_sweep_err"][node] == sen / sed and swe[node] == Fraction(sen, sed), node
    # the node-level oracle agrees at every node
    for v in range(2, 7):
        o = oracle.node_estimates(g, [0, 1], v, eps=(1, 1))
        assert o.S_err == out["S_err"][v]


def test_sweep_special_cases():
    # K_n: T = 0 leaves HC with no pivot error and |L| = 1: the exact n - 1
    g = graphgen.complete(10)
    out = oracle.estimate_all(g, [2, 5, 9], sweep=True)
    assert (out["S_sweep"] == 9.0).all() and (out["S_sweep_err"] == 0).all()
    # k = n: every node sampled -> exact, error 0
    g = graphgen.ba(40, 2, seed=3)
    out = oracle.estimate_all(g, list(range(g.n)), sweep=True)
    assert (out["S_sweep"] == oracle.exact_sums(g)).all() and (out["S_sweep_err"] == 0).all()


def test_sweep_never_worse_than_pivoting():
    """Pure pivoting is a candidate: the chosen error never exceeds its error,
    (sum_i (d(v,c_i) - d(c,c_i))^2 / k) * (n-1-k), evaluated here from D."""
    g = graphgen.rmat(8, 8, seed=6)
    samples = oracle.draw_samples(g.n, 20, 4)
    out = oracle.estimate_all(g, samples, sweep=True)
    D, dmat, piv = out["D"].astype(np.int64), out["dmat"].astype(np.int64), out["pivot"]
    k, n = len(samples), g.n
    pure = ((D - dmat[piv]) ** 2).sum(axis=1) / k * (n - 1 - k)
    un = np.ones(n, bool)
    un[samples] = False
    assert (out["S_sweep_err"][un] <= pure[un] * (1 + 1e-12)).all()
    assert (out["S_sweep_err"] >= 0).all()


# ---------------------------------------------------------------- Sec. 6.2 / Algorithm 4

DIGRAPH6 = [(0, 1), (1, 2), (2, 0), (2, 3), (3, 4), (5, 3)]
ORDER6 = [3, 0, 5, 1, 4, 2]


def _reach_tuple_ok(got, j, want):
    # B is one correctly rounded division of exact integers; R adds 1 to a
    # rounded quotient, so it is within one rounding of the exact value
    cnt, ds, T, B, R = want
    return (got["count"][j] == cnt and got["distsum"][j] == ds and got["T"][j] == T
            and got["B"][j] == float(B) and abs(got["R"][j] - float(R)) <= 4e-16 * float(R))


def test_reach_worked_example():
    """Algorithm 4 on the hand-derived 6-node digraph (fixture with derivation),
    outbound and inbound, from the definition and from the literal algorithm."""
    rows = _read_golden("digraph6_reach_k2.txt")
    g = graphgen.csr_from_arcs(6, [a for a, _ in DIGRAPH6], [b for _, b in DIGRAPH6], symmetrize=False,
                               directed=True)
    out = oracle.reach_all(g, ORDER6, 2)
    inn = oracle.reach_all(g, ORDER6, 2, inbound=True)
    arcs = [(a, b, 1) for a, b in DIGRAPH6]
    alg_out = tiny.reach_algorithm4(6, arcs, ORDER6, 2, corrected=True)
    alg_in = tiny.reach_algorithm4(6, [(b, a, w) for a, b, w in arcs], ORDER6, 2, corrected=True)
    for d, v, cnt, ds, T, bn, bd, rn, rd in rows:
        want = (cnt, ds, T, Fraction(int(bn), int(bd)), Fraction(int(rn), int(rd)))
        got, alg = (out, alg_out) if d == 0 else (inn, alg_in)
        assert _reach_tuple_ok(got, v, want), (d, v)
        assert alg[v] == want, (d, v, alg[v])
    # the printed pruning rule loses node 1 from outbound node 0's sample
    printed = tiny.reach_algorithm4(6, arcs, ORDER6, 2)
    assert printed[0][:2] == (1, 3) and out["count"][0] == 2


@pytest.mark.parametrize("seed", range(24))
def test_reach_definition_vs_algorithm4(seed):
    """The definition-level oracle equals the pruned sequential searches of
    Algorithm 4 (with the corrected pruning rule) and an exact-rational
    restatement of the definition on random digraphs, weighted or not, not
    strongly connected."""
    rng = np.random.default_rng(2400 + seed)
    n = int(rng.integers(2, 30))
    wmax = [1, 7, 1, 3][seed % 4]
    g = graphgen.gnp(n, float(rng.uniform(0.03, 0.3)), 2400 + seed, directed=True, wmax=wmax, connect=False)
    order = [int(x) for x in oracle.draw_samples(g.n, g.n, 50 + seed)]
    k = int(rng.integers(1, g.n + 2))
    arcs = []
    for a in range(g.n):
        for e in range(g.row_ptr[a], g.row_ptr[a + 1]):
            arcs.append((a, int(g.col_idx[e]), 1 if g.w is None else int(g.w[e])))
    d = tiny.floyd_warshall(g.n, g.row_ptr, g.col_idx, g.w)
    dT = [[d[u][v] for u in range(g.n)] for v in range(g.n)]
    for inbound, dist, arcs_dir in ((False, d, arcs), (True, dT, [(b, a, w) for a, b, w in arcs])):
        got = oracle.reach_all(g, order, k, inbound=inbound)
        defn = tiny.reach_definition(dist, order, k)
        alg = tiny.reach_algorithm4(g.n, arcs_dir, order, k, corrected=True)
        assert defn == alg
        for v in range(g.n):
            assert _reach_tuple_ok(got, v, defn[v]), (inbound, v, defn[v])


def test_reach_closed_forms():
    # directed cycle: every node reaches the other n-1 at distances 1..n-1
    n = 9
    g = graphgen.csr_from_arcs(n, list(range(n)), [(i + 1) % n for i in range(n)], symmetrize=False, directed=True)
    order = [int(x) for x in oracle.draw_samples(n, n, 3)]
    big = oracle.reach_all(g, order, n + 3)
    assert (big["count"] == n - 1).all() and (big["distsum"] == n * (n - 1) // 2).all()
    assert (big["B"] == n / 2).all() and (big["R"] == n - 1).all() and (big["T"] == 0).all()
    # k = n-1 on a node reaching everything: the k-th is the last other node, T = n-1, R exact
    full = oracle.reach_all(g, order, n - 1)
    assert (full["T"] == n - 1).all() and (full["R"] == n - 1).all()
    # path 0 -> 1 -> ... -> n-1: outbound reach of v is v+1..n-1, inbound 0..v-1
    g = graphgen.csr_from_arcs(n, list(range(n - 1)), list(range(1, n)), symmetrize=False, directed=True)
    o = oracle.reach_all(g, order, n)
    i = oracle.reach_all(g, order, n, inbound=True)
    for v in range(n):
        a, b = n - 1 - v, v
        assert o["count"][v] == a and o["distsum"][v] == a * (a + 1) // 2
        assert i["count"][v] == b and i["distsum"][v] == b * (b + 1) // 2
    # complete digraph: the k-th member is the k-th other node in the order, T = k, R = n-1 exactly
    n = 12
    src = [a for a in range(n) for b in range(n) if a != b]
    dst = [b for a in range(n) for b in range(n) if a != b]
    g = graphgen.csr_from_arcs(n, src, dst, symmetrize=False, directed=True)
    for k in (2, 5, 11):
        r = oracle.reach_all(g, [int(x) for x in oracle.draw_samples(n, n, k)], k)
        assert (r["T"] == k).all() and (r["R"] == n - 1).all() and (r["B"] == 1.0).all()


# ---------------------------------------------------------------- Sec. 5 node-weighted centrality

def test_weighted_worked_example():
    rows = _read_golden("path7_beta_C135.txt")
    g = graphgen.path(7)
    beta = [1, 2, 1, 3, 1, 1, 2]
    out = oracle.estimate_weighted(g, beta, 3, 0, eps=(1, 2), sample=([1, 3, 5], [True, False, True], 5, 2))
    d = tiny.floyd_warshall(g.n, g.row_ptr, g.col_idx)
    est, var = tiny.weighted_estimates(d, beta, [1, 3, 5], [True, False, True], Fraction(5, 2), Fraction(1, 2))
    for v, en, ed, vn, vd in rows:
        assert out["S_beta"][v] == en / ed and abs(out["S_beta_var"][v] - vn / vd) <= 1e-15 * max(1, vn / vd)
        assert est[v] == Fraction(int(en), int(ed)) and var[v] == Fraction(int(vn), int(vd))


def _exact_weighted(d, beta):
    n = len(d)
    return [sum(beta[u] * d[v][u] for u in range(n)) for v in range(n)]


def test_weighted_sampler_threshold_and_size():
    rng = np.random.default_rng(31)
    for trial in range(40):
        n = int(rng.integers(2, 60))
        beta = [int(x) for x in rng.integers(0, [2, 10, 1000, 5][trial % 4], size=n)]
        if trial % 5 == 0:
            beta[int(rng.integers(0, n))] = 10 ** 6  # one very heavy node
        pos = [v for v in range(n) if beta[v] > 0]
        k = int(rng.integers(1, n + 1))
        ids, light, R, m = oracle.draw_weighted(beta, k, 100 + trial)
        assert ids == sorted(set(ids)) and all(beta[v] > 0 for v in ids)
        if len(pos) <= k:
            assert ids == pos and R == 0 and m == 1 and not any(light)
            continue
        assert len(ids) == k
        tau = Fraction(R, m)
        # tau is VarOpt's threshold: sum of min(1, beta/tau) over the nodes is k
        assert sum(min(Fraction(1), Fraction(beta[v]) / tau) for v in pos) == k
        # every node at or above the threshold is taken, as heavy
        heavy = {v for v in pos if beta[v] >= tau}
        assert heavy <= set(ids)
        assert {v for v, lt in zip(ids, light) if not lt} == heavy


def test_weighted_sampler_inclusion_frequencies():
    """Inclusion frequency of each node over many seeds is min(1, beta/tau)
    (within 5 standard deviations); 0/1 weights sample uniformly among the
    ones; pairs are never positively correlated beyond noise."""
    beta = [3, 1, 4, 1, 5, 9, 2, 6, 5, 3, 5, 8, 9, 7, 9, 3, 0, 0, 20]
    k, T = 6, 4000
    _, _, R, m = oracle.draw_weighted(beta, k, 0)
    tau = R / m
    hits = np.zeros(len(beta))
    pair = np.zeros((len(beta), len(beta)))
    for sd in range(T):
        ids, _, _, _ = oracle.draw_weighted(beta, k, sd)
        x = np.zeros(len(beta))
        x[ids] = 1
        hits += x
        pair += np.outer(x, x)
    for v, b in enumerate(beta):
        p = min(1.0, b / tau)
        sd = math.sqrt(max(p * (1 - p), 1e-12) / T)
        assert abs(hits[v] / T - p) <= 5 * sd + 1e-12, (v, b, hits[v] / T, p)
    light = [v for v, b in enumerate(beta) if 0 < b < tau]
    for i in light:
        for j in light:
            if i < j:
                pi, pj = min(1, beta[i] / tau), min(1, beta[j] / tau)
                assert pair[i, j] / T <= pi * pj + 5 * math.sqrt(pi * pj / T), (i, j)
    ones = [0, 1, 1, 0, 1, 1, 1, 0, 1, 1]
    h = np.zeros(len(ones))
    for sd in range(2000):
        ids, light_, R1, m1 = oracle.draw_weighted(ones, 3, sd)
        assert all(ones[v] for v in ids) and all(light_) and Fraction(R1, m1) == Fraction(7, 3)
        h[ids] += 1
    p = 3 / 7
    for v in range(len(ones)):
        want = p if ones[v] else 0.0
        assert abs(h[v] / 2000 - want) <= 5 * math.sqrt(p * (1 - p) / 2000)


@pytest.mark.parametrize("seed", range(24))
def test_weighted_vs_bruteforce(seed):
    rng = np.random.default_rng(3100 + seed)
    n = int(rng.integers(3, 26))
    directed = seed % 4 == 3
    g = graphgen.gnp(n, float(rng.uniform(0.15, 0.5)), 3100 + seed, directed=directed, wmax=[1, 9, 1, 4][seed % 4])
    d = tiny.floyd_warshall(g.n, g.row_ptr, g.col_idx, g.w)
    rg = None
    if directed:
        d = tiny.round_trip(d)
        rg = graphgen.transpose(g)
    beta = [int(x) for x in rng.integers(0, [3, 20, 1000, 2][seed % 4], size=g.n)]
    beta[0] = max(beta[0], 1)
    k = int(rng.integers(1, g.n + 1))
    eps = [(1, 1), (1, 2), (2, 7), (1, 5)][seed % 4]
    out = oracle.estimate_weighted(g, beta, k, 77 + seed, eps=eps, reverse_graph=rg)
    tau = Fraction(out["R"], out["m"])
    est, var = tiny.weighted_estimates(d, beta, list(out["samples"]), list(out["light"]), tau, Fraction(*eps))
    err = tiny.weighted_errors(d, beta, list(out["samples"]), list(out["light"]), tau, Fraction(*eps))
    for v in range(g.n):
        assert out["S_beta"][v] == float(est[v]), v  # one correctly rounded division of exact integers
        assert abs(out["S_beta_var"][v] - float(var[v])) <= 1e-12 * max(1.0, abs(float(var[v]))), v
        assert abs(out["S_beta_err"][v] - float(err[v])) <= 1e-12 * max(1.0, abs(float(err[v]))), v


def test_weighted_exact_when_every_positive_node_is_sampled():
    g = graphgen.grid(7, 6, 8)
    d = tiny.floyd_warshall(g.n, g.row_ptr, g.col_idx)
    rng = np.random.default_rng(5)
    beta = [int(x) if x > 2 else 0 for x in rng.integers(0, 9, size=g.n)]
    k = sum(1 for b in beta if b > 0)
    out = oracle.estimate_weighted(g, beta, k, 1)
    assert out["R"] == 0 and not out["light"].any()
    assert (out["S_beta"] == np.array(_exact_weighted(d, beta), dtype=np.float64)).all()
    assert (out["S_beta_var"] == 0).all()


# ---------------------------------------------------------------- Sec. 6.2 / Algorithm 5

def _reach_beta_ok(got, j, want):
    cnt, kth, S, R = want
    return (got["count"][j] == cnt and got["kth"][j] == kth
            and abs(got["S"][j] - float(S)) <= 1e-12 * max(1.0, float(S))
            and abs(got["R"][j] - float(R)) <= 1e-12 * max(1.0, float(R)))


@pytest.mark.parametrize("seed", range(20))
def test_reach_weighted_vs_definition_and_algorithm5(seed):
    """The oracle equals an exact-rational restatement of the definition, and
    the sequential pruned searches of Algorithm 5 find the same members."""
    rng = np.random.default_rng(4200 + seed)
    n = int(rng.integers(2, 28))
    g = graphgen.gnp(n, float(rng.uniform(0.03, 0.3)), 4200 + seed, directed=True, wmax=[1, 6][seed % 2],
                     connect=False)
    beta = rng.integers(0, [3, 50, 1000, 2][seed % 4], size=g.n).astype(np.uint32)
    beta[0] = max(int(beta[0]), 1)
    k = int(rng.integers(1, g.n + 2))
    U = oracle.priority_numerators(g.n, 60 + seed)
    arcs = []
    for a in range(g.n):
        for e in range(g.row_ptr[a], g.row_ptr[a + 1]):
            arcs.append((a, int(g.col_idx[e]), 1 if g.w is None else int(g.w[e])))
    d = tiny.floyd_warshall(g.n, g.row_ptr, g.col_idx, g.w)
    dT = [[d[u][v] for u in range(g.n)] for v in range(g.n)]
    for inbound, dist, arcs_dir in ((False, d, arcs), (True, dT, [(b, a, w) for a, b, w in arcs])):
        got = oracle.reach_weighted(g, beta, k, 60 + seed, inbound=inbound)
        defn = tiny.reach_weighted_definition(dist, beta, U, k)
        alg = tiny.reach_weighted_algorithm5(g.n, arcs_dir, beta, U, k)
        for v in range(g.n):
            assert _reach_beta_ok(got, v, defn[v]), (inbound, v, defn[v])
            mem = sorted((u for u in range(g.n) if beta[u] > 0 and u != v and dist[v][u] != tiny.INF),
                         key=lambda u: (Fraction(int(U[u]), int(beta[u])), u))[:k]
            assert [u for u, _ in alg[v]] == mem and all(dd == dist[v][u] for u, dd in alg[v]), (inbound, v)


def test_reach_weighted_unbiased():
    """Priority sampling is unbiased: over many rank draws the mean estimates
    approach the exact weighted reach and weighted distance sum (4 standard
    errors); the printed S = sum beta d / T would be off for unequal weights."""
    g = graphgen.gnp(14, 0.25, 7, directed=True, wmax=3, connect=False)
    rng = np.random.default_rng(8)
    beta = rng.integers(1, 30, size=g.n).astype(np.uint32)
    beta[3] = 200  # one heavy node
    d = tiny.floyd_warshall(g.n, g.row_ptr, g.col_idx, g.w)
    k, T = 4, 3000
    S = np.zeros((T, g.n))
    R = np.zeros((T, g.n))
    for t in range(T):
        o = oracle.reach_weighted(g, beta, k, 1000 + t)
        S[t], R[t] = o["S"], o["R"]
    for v in range(g.n):
        reach = [u for u in range(g.n) if u != v and d[v][u] != tiny.INF]
        exR = sum(int(beta[u]) for u in reach)
        exS = sum(int(beta[u]) * d[v][u] for u in reach)
        for est, ex in ((R[:, v], exR), (S[:, v], exS)):
            se = est.std() / math.sqrt(T) + 1e-9
            assert abs(est.mean() - ex) <= 4 * se + 1e-9 * max(1, ex), (v, est.mean(), ex)


def test_reach_weighted_unit_weights_and_small_sets():
    # beta = 1: R = (k-1)/T and S = (sum of the first k-1 distances)/T, Algorithm 5's own final step
    g = graphgen.csr_from_arcs(9, list(range(9)), [(i + 1) % 9 for i in range(9)], symmetrize=False, directed=True)
    beta = np.ones(9, np.uint32)
    U = oracle.priority_numerators(9, 5)
    o = oracle.reach_weighted(g, beta, 3, 5)
    d = tiny.floyd_warshall(g.n, g.row_ptr, g.col_idx)
    order = list(oracle.priority_order(beta, U))
    for v in range(9):
        mem = [u for u in order if u != v][:3]
        Tk = Fraction(int(U[mem[-1]]), 1 << 53)
        assert abs(o["R"][v] - float(2 / Tk)) <= 1e-12 * float(2 / Tk)
        s = sum(d[v][u] for u in mem[:2])
        assert abs(o["S"][v] - float(s / Tk)) <= 1e-12 * float(s / Tk)
    # fewer than k members: exact weighted sums
    o = oracle.reach_weighted(g, beta, 20, 5)
    assert (o["count"] == 8).all() and (o["R"] == 8).all() and (o["S"] == 36).all() and (o["kth"] == -1).all()



def test_weighted_error_reduces_to_unit_weights():
    """With every weight 1 the H term of the weighted error estimate is the
    one of Sec. 4.1: |H| times the mean squared pivot error over HC."""
    g = graphgen.grid(8, 7, 8)
    d = tiny.floyd_warshall(g.n, g.row_ptr, g.col_idx)
    beta = [1] * g.n
    samples = [3, 17, 30, 44, 51]
    out = oracle.estimate_weighted(g, beta, 5, 0, eps=(1, 2), sample=(samples, [True] * 5, g.n, 5))
    _, var = tiny.weighted_estimates(d, beta, samples, [True] * 5, Fraction(g.n, 5), Fraction(1, 2))
    ref = oracle.estimate_all(g, samples, eps=(1, 2))
    for v in range(g.n):
        if v in samples:
            continue
        # the unweighted S_err is the L variance term (ratio form) plus the same H term
        hterm = float(out["S_beta_err"][v] - out["S_beta_var"][v])
        row = ref["D"][v]
        p = int(np.argmin(row))
        thr = Fraction(int(row[p]) * 2)
        far = [u for u in range(g.n) if u != v and d[samples[p]][u] > thr]
        hc = [u for u in far if u in samples]
        h = [u for u in far if u not in samples]
        want = (sum((d[v][u] - d[samples[p]][u]) ** 2 for u in hc) / len(hc)) * len(h) if hc else 0
        assert abs(hterm - float(want)) <= 1e-9 * max(1.0, float(want)), v
