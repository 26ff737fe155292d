"""Pins of the oracle's graph properties (Preliminaries) against library
routines, closed forms and hand-worked cases:

  - triangles lambda_i = diag(A^3)_i / 2 (numpy matrix products), clustering
    c_i = lambda_i / (d_i (d_i - 1) / 2) and C_G over d_i > 1 (Eq. cc);
  - closed forms on K_n, cycles and stars;
  - components equal scipy's connected_components (labels as the smallest
    vertex of each component);
  - Spearman by the stated formula: scipy's value on tie-free scores, +1 and
    -1, and a hand-worked case with ties (mean ranks);
  - the sparsified subgraph keeps exactly the kept edges, renumbered in
    order.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1601_05527_amd import graphs as G


def _dense(g):
    A = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    A[rows, g.col] = 1.0
    return A


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_triangles_and_clustering_match_matrix_powers(seed):
    g = G.gnm(150, 900 + 300 * seed, seed=seed)
    A = _dense(g)
    lam_ref = np.rint(np.diag(A @ A @ A) / 2).astype(np.int64)
    pr = oracle.properties(g.n, g.row_ptr, g.col)
    np.testing.assert_array_equal(pr["lambda"], lam_ref)
    d = A.sum(axis=1)
    live = d > 1
    c_ref = np.zeros(g.n)
    c_ref[live] = lam_ref[live] / (d[live] * (d[live] - 1) / 2)
    np.testing.assert_allclose(pr["c"], c_ref, rtol=1e-15, atol=0)
    assert pr["C_G"] == pytest.approx(c_ref[live].mean(), rel=1e-13)


def _complete(n):
    u, v = np.triu_indices(n, 1)
    return G.from_edges(n, u, v)


def test_closed_forms():
    k = oracle.properties(7, _complete(7).row_ptr, _complete(7).col)
    assert np.all(k["lambda"] == math.comb(6, 2)) and np.all(k["c"] == 1.0) and k["C_G"] == 1.0
    assert k["n_components"] == 1
    cyc = G.from_edges(9, np.arange(9), (np.arange(9) + 1) % 9)
    pc = oracle.properties(9, cyc.row_ptr, cyc.col)
    assert np.all(pc["lambda"] == 0) and pc["C_G"] == 0.0
    star = G.from_edges(6, np.zeros(5, int), np.arange(1, 6))
    ps = oracle.properties(6, star.row_ptr, star.col)
    assert ps["C_G"] == 0.0 and ps["n_components"] == 1
    # a triangle {0,1,2} with a pendant 3 on vertex 2: c = 1, 1, 1/3; vertex 3 left out
    tp = G.from_edges(4, [0, 1, 0, 2], [1, 2, 2, 3])
    pt = oracle.properties(4, tp.row_ptr, tp.col)
    assert pt["lambda"].tolist() == [1, 1, 1, 0]
    np.testing.assert_allclose(pt["c"], [1.0, 1.0, 1.0 / 3.0, 0.0], rtol=1e-15)
    assert pt["C_G"] == pytest.approx((1 + 1 + 1 / 3) / 3, rel=1e-15)


def test_components_match_scipy():
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components
    rng = np.random.default_rng(4)
    for n, m in [(500, 300), (2000, 1500), (3000, 6000)]:
        g = G.gnm(n, m, seed=int(rng.integers(1 << 30)))
        pr = oracle.properties(g.n, g.row_ptr, g.col)
        A = csr_matrix((np.ones(len(g.col)), g.col, g.row_ptr), shape=(g.n, g.n))
        nc, lab = connected_components(A, directed=False)
        assert pr["n_components"] == nc
        first = {}
        for i, l in enumerate(lab):
            first.setdefault(l, i)
        np.testing.assert_array_equal(pr["comp"], [first[l] for l in lab])
    # three disjoint K4 and two isolated vertices
    blocks = [_complete(4)]
    u = np.concatenate([blocks[0].edge_u + 4 * b for b in range(3)])
    v = np.concatenate([blocks[0].edge_v + 4 * b for b in range(3)])
    g = G.from_edges(14, u, v)
    pr = oracle.properties(14, g.row_ptr, g.col)
    assert pr["n_components"] == 5
    assert pr["comp"].tolist() == [0] * 4 + [4] * 4 + [8] * 4 + [12, 13]


def test_spearman_formula():
    from scipy.stats import spearmanr
    rng = np.random.default_rng(5)
    x = rng.permutation(1000).astype(float)
    y = x + rng.normal(0, 200, 1000)
    assert oracle.spearman(x, y) == pytest.approx(spearmanr(x, y).statistic, rel=1e-12)
    assert oracle.spearman(x, x) == 1.0
    assert oracle.spearman(x, -x) == pytest.approx(-1.0, rel=1e-15)
    # ties share mean ranks: x ranks 1, 2.5, 2.5, 4 against 1, 2, 3, 4
    assert oracle.spearman([1, 2, 2, 3], [1, 2, 3, 4]) == pytest.approx(1 - 6 * 0.5 / (4 * 15), rel=1e-15)


def test_subgraph_keeps_exactly_the_kept_edges():
    g = G.chung_lu(2000, 12_000, seed=6)
    keep = (np.random.default_rng(7).random(g.m) < 0.4).astype(np.uint8)
    rp, col, w, eid, oe, ms = oracle.subgraph(g, keep)
    kept = np.nonzero(keep)[0]
    assert ms == kept.size
    h = G.from_edges(g.n, g.edge_u[kept], g.edge_v[kept], g.edge_w[kept], orig_id=g.orig_id)
    np.testing.assert_array_equal(rp, h.row_ptr)
    np.testing.assert_array_equal(col, h.col)
    np.testing.assert_array_equal(w, h.w)
    np.testing.assert_array_equal(eid, h.eid)
    np.testing.assert_array_equal(oe, kept[eid])
    full = oracle.subgraph(g, np.ones(g.m, np.uint8))
    np.testing.assert_array_equal(full[1], g.col)
    np.testing.assert_array_equal(full[3], g.eid)
    none = oracle.subgraph(g, np.zeros(g.m, np.uint8))
    assert none[5] == 0 and np.all(none[0] == 0)
