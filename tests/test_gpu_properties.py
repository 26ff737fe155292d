"""Property checks (ad_subgraph, ad_graph_properties, ad_spearman) against
the oracle through the C ABI: subgraphs, triangle counts, per-vertex
clustering and component labels are integer (or identically computed)
results and must match bit for bit; C_G (a mean summed in another order)
and Spearman's rho agree to 1e-12.
"""
import numpy as np
import pytest

import oracle
from paper_1601_05527_amd import graphs as G

from gpu_helpers import announce
from test_gpu_parity import _mixed_degree_graph

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    from paper_1601_05527_amd import api as _api
    return _api


def _np(t):
    return t.detach().cpu().numpy()


def _check_props(api, dg, g_rp, g_col):
    pr = api.graph_properties(dg)
    ref = oracle.properties(dg.n, g_rp, g_col)
    np.testing.assert_array_equal(_np(pr["lambda"]), ref["lambda"])
    np.testing.assert_array_equal(_np(pr["c"]), ref["c"])
    np.testing.assert_array_equal(_np(pr["comp"]), ref["comp"])
    assert pr["n_components"] == ref["n_components"]
    assert pr["C_G"] == pytest.approx(ref["C_G"], rel=1e-12, abs=1e-15)
    return pr, ref


@pytest.mark.parametrize("kind", ["mixed", "chung_lu", "clusters", "grid"])
def test_properties_match_oracle(api, kind):
    announce(f"properties {kind}")
    if kind == "mixed":
        g = _mixed_degree_graph()
    elif kind == "chung_lu":
        g = G.chung_lu(30_000, 400_000, seed=9)
    elif kind == "clusters":
        g = G.clusters_with_bridges(6, 12)
    else:
        g = G.grid_long_range(64, 20, seed=3)
    _check_props(api, api.DeviceGraph.from_host(g, "cuda"), g.row_ptr, g.col)


def test_properties_beyond_the_bitmap_range(api):
    """More than 2^20 vertices: long rows are searched as sorted arrays (the
    id-range bitmap covers at most 2^20 ids).  A dense Chung-Lu core of
    4,000 vertices is spread over the whole id range; the rest is isolated."""
    announce("properties n > 2^20")
    core = G.chung_lu(4000, 120_000, seed=12)
    n = (1 << 20) + 5000
    ids = np.sort(np.random.default_rng(13).choice(n, size=core.n, replace=False))
    g = G.from_edges(n, ids[core.edge_u], ids[core.edge_v])
    assert int(np.diff(g.row_ptr).max()) > 64
    _check_props(api, api.DeviceGraph.from_host(g, "cuda"), g.row_ptr, g.col)


@pytest.mark.parametrize("frac", [0.0, 0.05, 0.4, 1.0])
def test_subgraph_matches_oracle(api, frac):
    announce(f"subgraph frac={frac}")
    g = _mixed_degree_graph()
    keep = (np.random.default_rng(11).random(g.m) < frac).astype(np.uint8)
    dg = api.DeviceGraph.from_host(g, "cuda")
    sg = api.subgraph(dg, torch.from_numpy(keep).cuda())
    rp, col, w, eid, oe, ms = oracle.subgraph(g, keep)
    assert sg.m == ms
    np.testing.assert_array_equal(_np(sg.row_ptr), rp)
    np.testing.assert_array_equal(_np(sg.col), col)
    np.testing.assert_array_equal(_np(sg.w), w)
    np.testing.assert_array_equal(_np(sg.eid), eid)
    np.testing.assert_array_equal(_np(sg.orig_edge), oe)
    if ms:
        _check_props(api, sg, rp, col)


def test_long_paths_and_many_components(api):
    """A path of 300,000 vertices (one component, a long hook chain), 5,000
    disjoint triangles and isolated vertices."""
    announce("properties long path and many components")
    n_path = 300_000
    u = [np.arange(n_path - 1)]
    v = [np.arange(1, n_path)]
    base = n_path
    for t in range(5000):
        a = base + 3 * t
        u.append(np.array([a, a + 1, a]))
        v.append(np.array([a + 1, a + 2, a + 2]))
    n = base + 3 * 5000 + 7
    g = G.from_edges(n, np.concatenate(u), np.concatenate(v))
    perm = np.random.default_rng(2).permutation(n)
    h = G.relabel(g, perm)
    for gg in (g, h):
        pr, ref = _check_props(api, api.DeviceGraph.from_host(gg, "cuda"), gg.row_ptr, gg.col)
        assert ref["n_components"] == 1 + 5000 + 7


def test_spearman_matches_oracle(api):
    announce("spearman")
    rng = np.random.default_rng(3)
    for n, ties in [(2, False), (1000, False), (100_000, True), (1_000_003, True)]:
        x = rng.integers(0, 50, n).astype(np.float64) if ties else rng.normal(size=n)
        y = x + rng.normal(0, 5.0 if ties else 0.7, n)
        if ties:
            y = np.round(y)
        got = api.spearman(torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda())
        assert got == pytest.approx(oracle.spearman(x, y), rel=1e-12, abs=1e-14)
    x = torch.arange(10, dtype=torch.float64, device="cuda")
    assert api.spearman(x, x) == 1.0
    assert api.spearman(x, -x) == pytest.approx(-1.0, rel=1e-15)


def test_comparison_of_a_sparsified_graph(api):
    """compare_properties on a real sparsification (LOCAL, e = 1/2, on the
    oracle's distances) against the same comparisons from the oracle."""
    announce("compare properties")
    g = G.chung_lu(20_000, 200_000, seed=12)
    rho = oracle.algebraic_distance(g, 8, 12, 0.5, seed=2)
    keep, _ = oracle.sparsify(g, rho, 0, 0.5)
    dg = api.DeviceGraph.from_host(g, "cuda")
    cmp = api.compare_properties(dg, torch.from_numpy(keep).cuda())
    po = oracle.properties(g.n, g.row_ptr, g.col)
    rp, col, _, _, _, ms = oracle.subgraph(g, keep)
    ps = oracle.properties(g.n, rp, col)
    assert cmp["m_kept"] == ms
    assert cmp["components"] == po["n_components"] and cmp["components_sparse"] == ps["n_components"]
    assert cmp["C_G_sparse"] == pytest.approx(ps["C_G"], rel=1e-12)
    assert cmp["degree_spearman"] == pytest.approx(
        oracle.spearman(np.diff(g.row_ptr).astype(float), np.diff(rp).astype(float)), rel=1e-12)
    assert cmp["clustering_spearman"] == pytest.approx(oracle.spearman(po["c"], ps["c"]), rel=1e-12)


def test_empty_and_edgeless_graphs(api):
    announce("properties empty graphs")
    g = G.from_edges(6, np.zeros(0, int), np.zeros(0, int))
    dg = api.DeviceGraph.from_host(g, "cuda")
    pr = api.graph_properties(dg)
    assert pr["n_components"] == 6 and pr["C_G"] == 0.0
    assert _np(pr["comp"]).tolist() == list(range(6))
    sg = api.subgraph(dg, torch.zeros(0, dtype=torch.uint8, device="cuda"))
    assert sg.m == 0 and _np(sg.row_ptr).tolist() == [0] * 7
