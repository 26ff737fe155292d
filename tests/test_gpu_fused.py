"""Distances and selection in one call (ad_edge_dist_sparsify,
ad_edge_dist_fit_both) against the separate calls and the oracle.

The fused calls compute every CSR entry's distance from whole rows and rank
from those values; they must return the same distances as ad_edge_dist,
bit for bit, and the same masks, counts and fitted exponents as ad_sparsify
and ad_sparsify_fit_both on them, which in turn equal the oracle's
selection on the same distances.
"""
import numpy as np
import pytest

import oracle
from paper_1601_05527_amd import graphs as G
from paper_1601_05527_amd.workloads import FP64_TAIL

from gpu_helpers import announce
from test_gpu_parity import _long_row_graph, _mixed_degree_graph

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    from paper_1601_05527_amd import api as _api
    return _api


def _np(t):
    return t.detach().cpu().numpy()


_GRAPHS = {}


def _graph(case):
    if case not in _GRAPHS:
        if case == "mixed":        # degrees across every ranking path, one isolated vertex
            g = _mixed_degree_graph()
        elif case == "long":       # rows up to 70,000 (bucket partition; distance work items)
            g0 = _long_row_graph()
            g = G.with_weights(g0, G.random_weights(g0.m, 46))
        elif case == "chung_lu":   # power-law rows in degree order
            g = G.chung_lu(1 << 14, 240_000, seed=8)
        else:                      # isolated vertices and two-vertex components
            g = G.from_edges(40, np.array([0, 2, 4, 4, 5, 9]), np.array([1, 3, 5, 6, 6, 30]),
                             G.random_weights(6, 3))
        _GRAPHS[case] = g
    return _GRAPHS[case]


@pytest.mark.parametrize("case", ["mixed", "long", "chung_lu", "tiny"])
@pytest.mark.parametrize("store", ["f32", "f32_fp64_tail"])
def test_fused_equals_separate_and_oracle(api, case, store):
    announce(f"fused distance + selection {case} {store}")
    g = _graph(case)
    assert g.m == g.edge_u.size
    dg = api.DeviceGraph.from_host(g, "cuda")
    tail = FP64_TAIL if store == "f32_fp64_tail" else 0
    res = api.relax(dg, 8, 10, seed=5, fp64_tail=tail)
    assert res.x.dtype == (torch.float64 if tail else torch.float32)
    rho_s = api.distances(dg, res)
    rho_s_np = _np(rho_s)
    rho64 = rho_s_np.astype(np.float64)
    for orient in (0, 1):
        for e in (0.0, 0.3, 0.7, 1.0):
            rho_f, keep_f, n_f = api.edge_dist_sparsify(dg, res, orient, e)
            keep_s, n_s = api.sparsify(dg, rho_s, orient, e)
            assert np.array_equal(_np(rho_f).view(np.uint32), rho_s_np.view(np.uint32)), (orient, e)
            assert np.array_equal(_np(keep_f), _np(keep_s)), (orient, e)
            assert int(_np(n_f)[0]) == int(_np(n_s)[0])
            keep_o, kept_o = oracle.sparsify(g, rho64, orient, e)
            assert np.array_equal(_np(keep_f), keep_o), (orient, e)
            assert int(_np(n_f)[0]) == kept_o
    for target in (0.1, 0.3, 0.8):
        rho_f, kl, kg, nk, (el, eg) = api.edge_dist_fit_both(dg, res, target)
        assert np.array_equal(_np(rho_f).view(np.uint32), rho_s_np.view(np.uint32))
        kl_s, kg_s, nk_s, (el_s, eg_s) = api.sparsify_fit_both(dg, rho_s, target)
        assert (el, eg) == (el_s, eg_s)
        assert np.array_equal(_np(kl), _np(kl_s)) and np.array_equal(_np(kg), _np(kg_s))
        assert np.array_equal(_np(nk), _np(nk_s))
        for o, (keep, e) in enumerate([(kl, el), (kg, eg)]):
            e_o, keep_o, kept_o = oracle.fit_exponent(g, rho64, o, target)
            assert e == e_o
            assert np.array_equal(_np(keep), keep_o)
            assert int(_np(nk)[o]) == kept_o


def test_fused_edgeless_graph(api):
    announce("fused distance + selection, no edges")
    g = G.from_edges(7, np.zeros(0, int), np.zeros(0, int))
    dg = api.DeviceGraph.from_host(g, "cuda")
    res = api.relax(dg, 4, 3, seed=1)
    rho, kl, kg, nk, (el, eg) = api.edge_dist_fit_both(dg, res, 0.3)
    assert rho.numel() == 0 and el == 0.0 and eg == 0.0
    assert _np(nk).tolist() == [0, 0]
    rho, keep, n_kept = api.edge_dist_sparsify(dg, res, 1, 0.5)
    assert int(_np(n_kept)[0]) == 0
