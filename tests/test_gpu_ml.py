"""Multilevel sparsification (Algorithm 6) on the GPU against the oracle,
through the C ABI.

  - ad_ml_aggregate on the oracle's own distances: seeds and aggregates are
    integer decisions taken from the same values in the same precision
    (strengths in double), so they must match bit for bit, in FP64 and on
    FP32-rounded distances;
  - ad_ml_sparsify with FP64 relaxation against oracle.ml_sparsify: the
    kept set, its size and the depth reached must match exactly.  The two
    relaxations agree to about 1e-12 (relative), far below the gaps the
    strength, aggregation and bin decisions compare, so on these seeded
    cases no decision flips;
  - the per-level ratio vector (coarsest level first), negative entries
    that skip a level, retention targets (fit) and the level-span rule,
    against the oracle in FP64;
  - properties that hold at any size: one level is SparsifyB on the
    library's own distances, exponent 1 keeps every edge, an empty graph
    keeps nothing.
"""
import numpy as np
import pytest

import oracle
from paper_1601_05527_amd import graphs as G

from gpu_helpers import announce
from test_gpu_parity import _mixed_degree_graph

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

EPS, THETA = 1e-12, 0.5


@pytest.fixture(scope="module")
def api():
    from paper_1601_05527_amd import api as _api
    return _api


def _np(t):
    return t.detach().cpu().numpy()


def _graph(kind):
    if kind == "chung_lu":
        return G.chung_lu(20_000, 200_000, seed=21)
    if kind == "chung_lu_unweighted":
        g = G.chung_lu(20_000, 150_000, seed=22)
        return G.from_edges(g.n, g.edge_u, g.edge_v, orig_id=g.orig_id)
    if kind == "mixed":
        return _mixed_degree_graph()
    if kind == "grid":
        return G.grid_long_range(80, 30, seed=4)
    if kind == "degree_ordered":
        g0 = G.chung_lu(30_000, 250_000, seed=23)
        return G.relabel(g0, G.degree_descending_order(g0))
    raise ValueError(kind)


@pytest.mark.parametrize("kind", ["chung_lu", "chung_lu_unweighted", "mixed", "grid", "degree_ordered"])
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_aggregates_match_oracle(api, kind, prec):
    announce(f"ml aggregate {kind} {prec}")
    g = _graph(kind)
    rho = oracle.algebraic_distance(g, 8, 10, 0.5, seed=5)
    if prec == "f32":
        rho = rho.astype(np.float32)
    dg = api.DeviceGraph.from_host(g, "cuda")
    agg, is_seed, nc = api.ml_aggregate(dg, torch.from_numpy(rho).cuda(), EPS, THETA)
    seeds_o = oracle.ml_seeds(g, rho.astype(np.float64), EPS, THETA)
    agg_o, nc_o = oracle.ml_aggregates(g, rho.astype(np.float64), seeds_o, EPS)
    assert nc == nc_o
    np.testing.assert_array_equal(_np(is_seed), seeds_o)
    np.testing.assert_array_equal(_np(agg), agg_o)


def test_aggregates_other_theta_and_ties(api):
    """theta = 0 (every edge strong: a maximal independent set in the
    traversal order), theta = 1, and equal distances everywhere (every
    choice decided by the tie rules)."""
    announce("ml aggregate theta and ties")
    g = G.chung_lu(8000, 60_000, seed=24)
    dg = api.DeviceGraph.from_host(g, "cuda")
    rho = oracle.algebraic_distance(g, 8, 10, 0.5, seed=6)
    for theta, r in [(0.0, rho), (1.0, rho), (0.5, np.full(g.m, 0.25)), (0.5, np.zeros(g.m))]:
        agg, is_seed, nc = api.ml_aggregate(dg, torch.from_numpy(r).cuda(), EPS, theta)
        seeds_o = oracle.ml_seeds(g, r, EPS, theta)
        agg_o, nc_o = oracle.ml_aggregates(g, r, seeds_o, EPS)
        assert nc == nc_o, theta
        np.testing.assert_array_equal(_np(is_seed), seeds_o)
        np.testing.assert_array_equal(_np(agg), agg_o)


@pytest.mark.parametrize("case", [
    ("chung_lu", [0.5, 0.6, 0.7], 3, 300),
    ("chung_lu_unweighted", [0.4], 4, 200),
    ("mixed", [0.5, 0.3], 3, 500),
    ("grid", [0.6, 0.5], 5, 100),
])
def test_ml_sparsify_matches_oracle(api, case):
    kind, e, levels, n_min = case
    announce(f"ml sparsify {kind} levels={levels}")
    g = _graph(kind)
    dg = api.DeviceGraph.from_host(g, "cuda")
    e = (list(e) + [e[-1]] * levels)[:levels]
    keep, kept, depth = api.ml_sparsify(dg, 8, 10, e, seed=3, graph_id=2, levels=levels, n_min=n_min,
                                        store="f64", bin_seed=11)
    keep_o, kept_o, depth_o = oracle.ml_sparsify(g, 8, 10, e, seed=3, graph_id=2, levels=levels, n_min=n_min,
                                                 bin_seed=11)
    print(f"{kind}: m={g.m} kept={kept} depth={depth}")
    assert depth == depth_o and depth >= 1
    assert kept == kept_o
    np.testing.assert_array_equal(_np(keep), keep_o)


def test_ml_sparsify_fp32_against_oracle(api):
    """FP32 relaxation (each component centred apart, the last two sweeps
    in FP64; every level's distances within 1e-5 of the FP64 oracle's):
    the same depth and kept edges as the FP64 oracle, edge for edge -- on
    these seeded inputs no seed, aggregate or selection decision lies within
    that tolerance of its threshold."""
    announce("ml sparsify f32")
    g = _graph("chung_lu")
    dg = api.DeviceGraph.from_host(g, "cuda")
    keep, kept, depth = api.ml_sparsify(dg, 8, 10, [0.5] * 3, seed=3, levels=3, n_min=300, store="f32", bin_seed=11)
    keep_o, kept_o, depth_o = oracle.ml_sparsify(g, 8, 10, [0.5] * 3, seed=3, levels=3, n_min=300, bin_seed=11)
    print(f"f32: kept {kept} oracle {kept_o}, depth {depth} oracle {depth_o}, "
          f"{int((_np(keep) != keep_o).sum())} edges differ")
    assert depth == depth_o
    assert int(_np(keep).sum()) == kept
    assert kept == kept_o
    np.testing.assert_array_equal(_np(keep), keep_o)


def test_one_level_is_binned_and_exponent_one_keeps_all(api):
    announce("ml sparsify one level / e = 1")
    g = _graph("degree_ordered")
    dg = api.DeviceGraph.from_host(g, "cuda")
    keep, kept, depth = api.ml_sparsify(dg, 8, 10, [0.5], seed=4, levels=1, store="f32", bin_seed=7)
    res = api.relax(dg, 8, 10, seed=4, store="f32")
    rho = api.edge_dist(dg, res.x, res.minmax)
    kb, nb, _ = api.sparsify_binned(dg, rho, 7, e=0.5)
    assert depth == 0 and kept == int(_np(nb)[0])
    np.testing.assert_array_equal(_np(keep), _np(kb))
    keep, kept, depth = api.ml_sparsify(dg, 8, 10, [1.0] * 6, seed=4, levels=6, n_min=100, store="f32", bin_seed=7)
    assert depth >= 2 and kept == g.m and bool(np.all(_np(keep) == 1))


def test_small_and_empty_graphs(api):
    announce("ml sparsify small and empty")
    g = G.from_edges(5, np.zeros(0, int), np.zeros(0, int))
    dg = api.DeviceGraph.from_host(g, "cuda")
    keep, kept, depth = api.ml_sparsify(dg, 8, 10, [0.5] * 3, levels=3, n_min=0, store="f64")
    assert kept == 0 and depth == 0
    # a graph below n_min is one SparsifyB level
    g = G.clusters_with_bridges(4, 8)
    dg = api.DeviceGraph.from_host(g, "cuda")
    keep, kept, depth = api.ml_sparsify(dg, 8, 10, [0.5] * 4, seed=1, levels=4, n_min=1000, store="f64", bin_seed=2)
    keep_o, kept_o, depth_o = oracle.ml_sparsify(g, 8, 10, [0.5] * 4, seed=1, levels=4, n_min=1000, bin_seed=2)
    assert depth == depth_o == 0 and kept == kept_o
    np.testing.assert_array_equal(_np(keep), keep_o)
    # n_min = 0 coarsens a small graph until the 90% rule or the level cap stops it
    keep, kept, depth = api.ml_sparsify(dg, 8, 10, [0.5] * 6, seed=1, levels=6, n_min=0, store="f64", bin_seed=2)
    keep_o, kept_o, depth_o = oracle.ml_sparsify(g, 8, 10, [0.5] * 6, seed=1, levels=6, n_min=0, bin_seed=2)
    assert depth == depth_o and kept == kept_o
    np.testing.assert_array_equal(_np(keep), keep_o)


@pytest.mark.parametrize("variant", ["skip_finest", "skip_coarsest", "fit", "span_coarsest", "span_middle",
                                     "span_finest", "all_skipped"])
def test_ratio_vector_variants_match_oracle(api, variant):
    announce(f"ml sparsify ratio vector {variant}")
    g = _graph("chung_lu")
    dg = api.DeviceGraph.from_host(g, "cuda")
    kw = dict(seed=5, graph_id=1, levels=4, n_min=200, bin_seed=13)
    if variant == "skip_finest":
        kw.update(e_levels=[0.5, 0.5, 0.6, -1])
    elif variant == "skip_coarsest":
        kw.update(e_levels=[-1, 0.4, 0.6, 0.7])
    elif variant == "fit":
        kw.update(e_levels=[0.5, -1, 0.35, 0.3], fit=True)
    elif variant.startswith("span"):
        kw.update(span=1, segment=["span_coarsest", "span_middle", "span_finest"].index(variant), span_value=0.4)
    else:
        kw.update(e_levels=[-1] * 4)
    keep, kept, depth = api.ml_sparsify(dg, 8, 10, store="f64", **kw)
    keep_o, kept_o, depth_o = oracle.ml_sparsify(g, 8, 10, **kw)
    print(f"{variant}: kept {kept} of {g.m}, depth {depth}")
    assert depth == depth_o and kept == kept_o
    np.testing.assert_array_equal(_np(keep), keep_o)
    if variant == "all_skipped":
        assert kept == g.m


@pytest.mark.parametrize("shape", ["single_edge", "star", "path", "triangles_and_isolated", "complete"])
def test_degenerate_graphs_match_oracle(api, shape):
    """Coarsening down to one vertex (n_min = 0), stars (one seed takes
    everything), paths (long chains of equal degree), isolated vertices and
    a complete graph (every distance tied at the fixed point)."""
    announce(f"ml sparsify degenerate {shape}")
    if shape == "single_edge":
        g = G.from_edges(2, [0], [1])
    elif shape == "star":
        g = G.from_edges(51, np.zeros(50, int), np.arange(1, 51))
    elif shape == "path":
        g = G.from_edges(100, np.arange(99), np.arange(1, 100))
    elif shape == "triangles_and_isolated":
        g = G.from_edges(9, [0, 1, 0, 3, 4, 3], [1, 2, 2, 4, 5, 5])
    else:
        u, v = np.triu_indices(12, 1)
        g = G.from_edges(12, u, v)
    dg = api.DeviceGraph.from_host(g, "cuda")
    for e in ([0.5] * 5, [0.0] * 5, [-1.0, 0.7, 0.7, 0.7, 0.7]):
        keep, kept, depth = api.ml_sparsify(dg, 8, 10, e, seed=2, levels=5, n_min=0, store="f64", bin_seed=3)
        keep_o, kept_o, depth_o = oracle.ml_sparsify(g, 8, 10, e, seed=2, levels=5, n_min=0, bin_seed=3)
        assert depth == depth_o and kept == kept_o, (shape, e)
        np.testing.assert_array_equal(_np(keep), keep_o)
