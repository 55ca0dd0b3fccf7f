"""Input generators: structure checks against scipy's component routines and
the generator recipes (edge counts, symmetry, no self-loops, sorted rows)."""
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components

import graphgen


def _csr(g):
    return sp.csr_matrix((np.ones(g.arcs), g.col_idx, g.row_ptr), shape=(g.n, g.n))


def _check_basic(g):
    assert g.row_ptr[0] == 0 and (np.diff(g.row_ptr) >= 0).all()
    assert g.col_idx.min() >= 0 and g.col_idx.max() < g.n
    src = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    assert (src != g.col_idx).all()                           # no self-loops
    for v in range(0, g.n, max(1, g.n // 50)):                # sorted, no duplicates
        row = g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]
        assert (np.diff(row) > 0).all()
    if not g.directed:
        A = _csr(g)
        assert (A != A.T).nnz == 0


def test_ba_counts():
    g = graphgen.ba(2000, 4, seed=1)
    _check_basic(g)
    assert g.m == 4 * 5 // 2 + (2000 - 5) * 4
    assert connected_components(_csr(g), directed=False)[0] == 1
    assert g.degrees().min() >= 4


def test_rmat_lcc_matches_scipy():
    full = graphgen.rmat(12, 8, seed=3, component=False)
    _check_basic(full)
    nc, lab = connected_components(_csr(full), directed=False)
    sizes = np.bincount(lab)
    g = graphgen.largest_component(full)
    _check_basic(g)
    assert g.n == sizes.max()
    assert connected_components(_csr(g), directed=False)[0] == 1


def test_directed_rmat_scc_matches_scipy():
    full = graphgen.rmat(12, 8, seed=4, directed=True, component=False)
    _check_basic(full)
    nc, lab = connected_components(_csr(full), directed=True, connection="strong")
    g = graphgen.largest_component(full)
    assert g.n == np.bincount(lab).max()
    assert connected_components(_csr(g), directed=True, connection="strong")[0] == 1
    gt = graphgen.transpose(g)
    assert (_csr(gt) != _csr(g).T).nnz == 0


def test_grid8_edges_and_weights():
    g = graphgen.grid(40, 30, 8, 0.0, 1, 1000, seed=5)
    _check_basic(g)
    assert g.m == 40 * 29 + 39 * 30 + 2 * 39 * 29
    assert g.w.min() >= 1 and g.w.max() <= 1000
    A = sp.csr_matrix((g.w, g.col_idx, g.row_ptr), shape=(g.n, g.n))
    assert (A != A.T).nnz == 0                                 # symmetric weights
    h = graphgen.grid(40, 30, 8, 0.1, 1, 1000, seed=5)
    assert 0.85 * g.m < h.m < 0.95 * g.m
    assert connected_components(_csr(h), directed=False)[0] == 1


def test_parallel_arcs_keep_min_weight():
    g = graphgen.csr_from_arcs(3, [0, 0, 1, 1], [1, 1, 2, 2], [5, 3, 9, 4])
    assert list(g.col_idx) == [1, 0, 2, 1] and list(g.w) == [3, 3, 4, 4]


def test_serving_mix_recipe():
    jobs = graphgen.serving_mix(512, seed=5)
    assert len(jobs) == 512
    ns = np.array([j["n"] for j in jobs])
    assert ns.min() >= 1000 and ns.max() <= 1_000_000
    assert {j["k"] for j in jobs} == {16, 64, 256}
    assert {j["kind"] for j in jobs} == {"ba", "rmat"}
