"""Pins of the oracle's multilevel sparsification (Algorithm 6) by what the
paper fixes and by its parts:

  - seeds: no two seeds are strongly coupled, every other vertex is strongly
    coupled to a seed, and a set-based Python traversal of the vertices in
    the stated order (degree, then the hashed name) picks the same seeds;
  - P (Eq. P): seeds are their own aggregates, numbered in id order; every
    other vertex joins a seed neighbour of largest strength;
  - the coarse graph built by merging aggregate pairs is the Galerkin
    product P^T L P (dense numpy);
  - one level is SparsifyB; exponent 1 everywhere keeps every edge;
  - two levels compose as the algorithm states: the coarse level's result
    is inherited, distances are recomputed on what is left, and SparsifyB
    chooses among it; the ratio vector lists the coarsest level first;
  - the level-span vectors equal the ones the paper prints (6 levels,
    span 2; tests/golden/ml_level_span.txt); a negative entry skips
    SparsifyB at its level; with `fit` an entry is the level's retention
    target;
  - results do not depend on vertex labels.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1601_05527_amd import graphs as G

EPS, THETA = 1e-12, 0.5


def _case(n=600, m=4000, seed=3, weighted=True):
    g = G.chung_lu(n, m, seed=seed)
    if not weighted:
        g = G.from_edges(g.n, g.edge_u, g.edge_v, orig_id=g.orig_id)
    rho = oracle.algebraic_distance(g, 8, 10, 0.5, seed=1)
    return g, rho


def _strengths(g, rho):
    d = 1.0 / np.sqrt(rho[g.eid] ** 2 + EPS)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    smax = np.zeros(g.n)
    np.maximum.at(smax, rows, d)
    strong = (d >= THETA * smax[rows]) | (d >= THETA * smax[g.col])
    return rows, d, smax, strong


def test_seed_rule_by_sets():
    g, rho = _case()
    seeds = oracle.ml_seeds(g, rho, EPS, THETA)
    rows, d, smax, strong = _strengths(g, rho)
    nbr = [set() for _ in range(g.n)]
    for p in np.nonzero(strong)[0]:
        nbr[rows[p]].add(int(g.col[p]))
    deg = np.diff(g.row_ptr)
    hashed = [oracle.bin_priority(0, int(g.orig_id[i])) for i in range(g.n)]     # fmix32 of the name
    order = sorted(range(g.n), key=lambda i: (-deg[i], hashed[i], g.orig_id[i]))
    chosen = set()
    for i in order:
        if not (nbr[i] & chosen):
            chosen.add(i)
    assert set(np.nonzero(seeds)[0].tolist()) == chosen
    # independent and dominating in the strong relation
    for i in range(g.n):
        if seeds[i]:
            assert not any(seeds[j] for j in nbr[i])
        else:
            assert any(seeds[j] for j in nbr[i])


def test_aggregates_follow_eq_p():
    g, rho = _case(seed=4)
    seeds = oracle.ml_seeds(g, rho, EPS, THETA)
    agg, nc = oracle.ml_aggregates(g, rho, seeds, EPS)
    assert nc == int(seeds.sum())
    sid = np.nonzero(seeds)[0]
    np.testing.assert_array_equal(agg[sid], np.arange(nc))
    rows, d, _, _ = _strengths(g, rho)
    for i in np.nonzero(seeds == 0)[0]:
        ps = range(g.row_ptr[i], g.row_ptr[i + 1])
        cand = [(d[p], -g.orig_id[g.col[p]], g.col[p]) for p in ps if seeds[g.col[p]]]
        best = max(cand)
        assert agg[i] == agg[best[2]]


def test_coarse_graph_is_the_galerkin_product():
    g, rho = _case(n=300, m=1500, seed=5)
    seeds = oracle.ml_seeds(g, rho, EPS, THETA)
    agg, nc = oracle.ml_aggregates(g, rho, seeds, EPS)
    rp, col, wc, eid, orig, mc, _ = oracle.ingest(nc, agg[g.edge_u], agg[g.edge_v], g.edge_w, order=0)
    A = np.zeros((g.n, g.n))
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    A[rows, g.col] = g.w
    L = np.diag(A.sum(1)) - A
    P = np.zeros((g.n, nc))
    P[np.arange(g.n), agg] = 1.0
    Lc = P.T @ L @ P
    Ac = np.zeros((nc, nc))
    crows = np.repeat(np.arange(nc), np.diff(rp))
    Ac[crows, col] = wc
    np.testing.assert_allclose(-(Lc - np.diag(np.diag(Lc))), Ac, rtol=1e-6, atol=0)
    np.testing.assert_allclose(np.diag(Lc), Ac.sum(1), rtol=1e-6)


def test_one_level_is_sparsify_b_and_exponent_one_keeps_all():
    g, _ = _case(seed=6)
    keep, kept, depth = oracle.ml_sparsify(g, 8, 10, [0.5], seed=1, levels=1, bin_seed=4)
    rho = oracle.algebraic_distance(g, 8, 10, 0.5, seed=1)
    kb, nb = oracle.sparsify_binned(g, rho, 0.5, 4)
    assert depth == 0 and kept == nb and np.array_equal(keep, kb)
    keep, kept, depth = oracle.ml_sparsify(g, 8, 10, [1.0], seed=1, levels=5, n_min=50, bin_seed=4)
    assert depth > 0 and kept == g.m


def _two_level_parts(g, rho, x_coarse, bin_seed):
    """The coarse graph of g and the keep of its SparsifyB at exponent x_coarse."""
    seeds = oracle.ml_seeds(g, rho, EPS, THETA)
    agg, nc = oracle.ml_aggregates(g, rho, seeds, EPS)
    names = g.orig_id[np.nonzero(seeds)[0]]
    rp, col, wc, ceid, corig, mc, _ = oracle.ingest(nc, agg[g.edge_u], agg[g.edge_v], g.edge_w, orig_id=names,
                                                    order=0)
    cg = G.Graph(n=nc, row_ptr=rp, col=col, w=wc, eid=ceid, orig_id=corig, edge_u=None, edge_v=None, edge_w=None)
    crow = np.repeat(np.arange(nc), np.diff(rp))
    cg.edge_u = crow[col > crow].astype(np.int32)     # coarse edges in id order
    cg.edge_v = col[col > crow]
    rho_c = oracle.algebraic_distance(cg, 8, 10, 0.5, seed=1, graph_id=1)
    if x_coarse < 0:
        keep_c = np.ones(mc, dtype=np.uint8)
    else:
        keep_c, _ = oracle.sparsify_binned(cg, rho_c, x_coarse, bin_seed, graph_id=1)
    # inherit: an edge between aggregates takes its coarse edge's state
    a, b = agg[g.edge_u], agg[g.edge_v]
    inh = np.ones(g.m, dtype=np.uint8)
    for q in np.nonzero(a != b)[0]:
        x, y = min(a[q], b[q]), max(a[q], b[q])
        lo, hi = rp[x], rp[x + 1]
        p = lo + np.searchsorted(col[lo:hi], y)
        inh[q] = keep_c[ceid[p]]
    return inh


def _fine_select(g, inh, x_fine, bin_seed):
    srp, scol, sw, seid, soe, ms = oracle.subgraph(g, inh)
    sg = G.Graph(n=g.n, row_ptr=srp, col=scol, w=sw, eid=seid, orig_id=g.orig_id, edge_u=None, edge_v=None,
                 edge_w=None)
    srow = np.repeat(np.arange(g.n), np.diff(srp))
    sg.edge_u = srow[scol > srow].astype(np.int32)
    sg.edge_v = scol[scol > srow]
    rho_s = oracle.algebraic_distance(sg, 8, 10, 0.5, seed=1, graph_id=0)
    keep_s, _ = oracle.sparsify_binned(sg, rho_s, x_fine, bin_seed, graph_id=0)
    want = np.zeros(g.m, dtype=np.uint8)
    want[soe[keep_s[seid] == 1]] = 1
    return want


def test_two_levels_compose_as_stated():
    g, rho = _case(n=2000, m=14000, seed=7)
    e = [0.6, 0.4]              # coarsest level first
    keep, kept, depth = oracle.ml_sparsify(g, 8, 10, e, seed=1, levels=2, n_min=100, bin_seed=9)
    assert depth == 1
    inh = _two_level_parts(g, rho, e[0], 9)
    want = _fine_select(g, inh, e[1], 9)
    np.testing.assert_array_equal(keep, want)
    assert np.all(keep <= inh)
    # -1 at the finest level: the coarse result is inherited and nothing more is dropped
    keep, kept, _ = oracle.ml_sparsify(g, 8, 10, [0.6, -1], seed=1, levels=2, n_min=100, bin_seed=9)
    np.testing.assert_array_equal(keep, inh)
    # -1 at the coarsest level: the fine level selects among all its edges
    keep, kept, _ = oracle.ml_sparsify(g, 8, 10, [-1, 0.4], seed=1, levels=2, n_min=100, bin_seed=9)
    kb, _ = oracle.sparsify_binned(g, rho, 0.4, 9)
    np.testing.assert_array_equal(keep, kb)
    # -1 everywhere keeps the graph
    keep, kept, depth = oracle.ml_sparsify(g, 8, 10, [-1], seed=1, levels=4, n_min=100, bin_seed=9)
    assert depth >= 2 and kept == g.m


def _golden_span():
    path = os.path.join(os.path.dirname(__file__), "golden", "ml_level_span.txt")
    rows = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#"):
            name, *vals = line.split()
            rows[name] = [float(v) for v in vals]
    return rows


def test_level_span_vectors_are_the_papers():
    rows = _golden_span()
    for s, name in enumerate(["coarsest", "middle", "finest"]):
        np.testing.assert_array_equal(oracle.ml_level_span(6, 2, s, 0.3), rows[name])
    # nine levels, span 3: three whole thirds; a span beyond a segment stays inside it
    np.testing.assert_array_equal(oracle.ml_level_span(9, 3, 1, 0.5), [-1] * 3 + [0.5] * 3 + [-1] * 3)
    np.testing.assert_array_equal(oracle.ml_level_span(6, 5, 2, 0.2), [-1] * 4 + [0.2] * 2)
    np.testing.assert_array_equal(oracle.ml_level_span(6, 1, 0, 0.2), [0.2] + [-1] * 5)


def test_level_span_follows_the_levels_reached():
    g, rho = _case(n=2000, m=14000, seed=7)
    k1, n1, d1 = oracle.ml_sparsify(g, 8, 10, None, seed=1, levels=6, n_min=100, bin_seed=9, span=1, segment=2,
                                    span_value=0.5)
    vec = oracle.ml_level_span(d1 + 1, 1, 2, 0.5)
    k2, n2, d2 = oracle.ml_sparsify(g, 8, 10, vec, seed=1, levels=d1 + 1, n_min=100, bin_seed=9)
    assert d1 == d2 and n1 == n2
    np.testing.assert_array_equal(k1, k2)


def test_fit_takes_the_entry_as_a_retention_target():
    g, rho = _case(seed=6)
    keep, kept, depth = oracle.ml_sparsify(g, 8, 10, [0.3], seed=1, levels=1, bin_seed=4, fit=True)
    e_f, kb, nb = oracle.fit_exponent_binned(g, rho, 0.3, 4)
    assert depth == 0 and kept == nb and np.array_equal(keep, kb)
    assert kept >= 0.3 * g.m


def test_multilevel_does_not_depend_on_labels():
    g, _ = _case(n=3000, m=20000, seed=8, weighted=False)
    h = G.relabel(g, np.random.default_rng(1).permutation(g.n))
    k1, n1, d1 = oracle.ml_sparsify(g, 8, 10, [0.5, 0.7], seed=2, levels=3, n_min=100, bin_seed=5)
    k2, n2, d2 = oracle.ml_sparsify(h, 8, 10, [0.5, 0.7], seed=2, levels=3, n_min=100, bin_seed=5)
    assert d1 == d2 == 2 and n1 == n2
    np.testing.assert_array_equal(k2, k1[h.edge_perm])
