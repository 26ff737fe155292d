"""Selection with binning (Algorithm 4, ad_sparsify_binned) against the FP64
oracle, through the C ABI.  Both sides bin the same distances (the oracle's,
rounded to the precision handed to the library), so bins, random orders,
rounds and kept sets are integer results and must agree bit for bit; the
fitted exponent must equal the oracle's bisection end point exactly.
"""
import numpy as np
import pytest

import oracle
from paper_1601_05527_amd import graphs as G

from gpu_helpers import announce
from test_gpu_parity import _long_row_graph, _mixed_degree_graph

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

SEED = 29


@pytest.fixture(scope="module")
def api():
    from paper_1601_05527_amd import api as _api
    return _api


@pytest.fixture(scope="module")
def mixed():
    """Degrees on both sides of every ranking path boundary (64 .. 8193),
    an isolated vertex, and the oracle's distances."""
    g = _mixed_degree_graph()
    rho = oracle.algebraic_distance(g, 8, 12, 0.5, seed=3)
    return g, rho


def _dg(api, g):
    return api.DeviceGraph.from_host(g, "cuda")


def _np(t):
    return t.detach().cpu().numpy()


def _cast(rho, prec):
    r = rho.astype(np.float32 if prec == "f32" else np.float64)
    return r, r.astype(np.float64)


def _check_fixed(api, g, rho_in, rho_ref, e, seed=SEED, graph_id=0, dg=None):
    dg = dg or _dg(api, g)
    keep, nk, e_used = api.sparsify_binned(dg, torch.from_numpy(rho_in).cuda(), seed, e=e, graph_id=graph_id)
    keep_o, kept_o = oracle.sparsify_binned(g, rho_ref, e, seed, graph_id)
    got = _np(keep)
    bad = np.nonzero(got != keep_o)[0]
    assert bad.size == 0, f"{bad.size} edges differ, first {bad[:8].tolist()}"
    assert int(_np(nk)[0]) == kept_o
    assert e_used == e
    return got


@pytest.mark.parametrize("prec", ["f32", "f64"])
@pytest.mark.parametrize("e", [0.0, 0.3, 0.5, 0.8, 1.0])
def test_binned_selection_bit_exact(api, mixed, prec, e):
    announce(f"binned {prec} e={e}")
    g, rho = mixed
    rho_in, rho_ref = _cast(rho, prec)
    _check_fixed(api, g, rho_in, rho_ref, e)


@pytest.mark.parametrize("kind", ["quantised", "equal_rows", "two_values"])
def test_binned_degenerate_distances(api, mixed, kind):
    """Ties in the distances, rows whose distances are all equal (one bin,
    sigma = 0) and rows with two distinct values."""
    announce(f"binned degenerate {kind}")
    g, rho = mixed
    r = rho.astype(np.float32)
    if kind == "quantised":
        r = np.round(r, 1).astype(np.float32)
    elif kind == "equal_rows":
        r = np.full(g.m, 0.375, dtype=np.float32)
    else:
        r = np.where(np.arange(g.m) % 3 == 0, 0.25, 0.75).astype(np.float32)
    _check_fixed(api, g, r, r.astype(np.float64), 0.5)


def test_binned_rows_beyond_the_in_lds_sort(api):
    """Rows of degree 8193 .. 70000 take the bucket-partition ranking."""
    announce("binned long rows")
    g = _long_row_graph()
    rho = np.random.default_rng(47).lognormal(0.0, 0.6, g.m).astype(np.float32)
    for e in (0.4, 0.7):
        _check_fixed(api, g, rho, rho.astype(np.float64), e)


@pytest.mark.parametrize("target", [0.15, 0.3, 0.6])
def test_binned_fit_matches_oracle(api, mixed, target):
    announce(f"binned fit target={target}")
    g, rho = mixed
    rho32 = rho.astype(np.float32)
    dg = _dg(api, g)
    keep, nk, e = api.sparsify_binned(dg, torch.from_numpy(rho32).cuda(), SEED, target=target)
    e_o, keep_o, kept_o = oracle.fit_exponent_binned(g, rho32.astype(np.float64), target, SEED)
    assert e == e_o
    assert np.array_equal(_np(keep), keep_o)
    assert int(_np(nk)[0]) == kept_o
    # the same exponent, fixed, gives the same set
    keep2, _, _ = api.sparsify_binned(dg, torch.from_numpy(rho32).cuda(), SEED, e=e)
    assert np.array_equal(_np(keep2), keep_o)


def test_binned_on_normalised_distances(api, mixed):
    announce("binned normalised")
    g, rho = mixed
    rn = oracle.normalize_dist(g, rho, by_strength=True).astype(np.float32)
    _check_fixed(api, g, rn, rn.astype(np.float64), 0.5)


def test_binned_seed_and_graph_id(api, mixed):
    announce("binned seed / graph id")
    g, rho = mixed
    r = rho.astype(np.float32)
    dg = _dg(api, g)
    a = _check_fixed(api, g, r, r.astype(np.float64), 0.5, seed=SEED, dg=dg)
    b = _check_fixed(api, g, r, r.astype(np.float64), 0.5, seed=SEED + 1, dg=dg)
    c = _check_fixed(api, g, r, r.astype(np.float64), 0.5, seed=SEED, graph_id=5, dg=dg)
    assert (a != b).any() and (a != c).any()
    again, _, _ = api.sparsify_binned(dg, torch.from_numpy(r).cuda(), SEED, e=0.5)
    assert np.array_equal(_np(again), a)


def test_binned_relabelled_graph_keeps_the_same_edges(api):
    """Priorities and the Philox key follow orig_id: a relabelled copy keeps
    the same undirected edges."""
    announce("binned relabelled")
    g = G.chung_lu(6000, 60_000, seed=5)
    rho = np.random.default_rng(3).lognormal(0.0, 0.5, g.m).astype(np.float32)
    h = G.relabel(g, G.degree_descending_order(g))
    k1 = _check_fixed(api, g, rho, rho.astype(np.float64), 0.5)
    rh = rho[h.edge_perm]
    k2 = _check_fixed(api, h, rh, rh.astype(np.float64), 0.5)
    assert np.array_equal(k2, k1[h.edge_perm])


def test_binned_tiny_and_empty_graphs(api):
    announce("binned tiny and empty")
    one = G.from_edges(2, np.array([0]), np.array([1]))
    _check_fixed(api, one, np.array([0.5], dtype=np.float32), np.array([0.5]), 0.0)
    path = G.from_edges(5, np.arange(4), np.arange(1, 5))
    r = np.array([0.1, 0.2, 0.3, 0.4], dtype=np.float32)
    _check_fixed(api, path, r, r.astype(np.float64), 0.5)
    empty = G.from_edges(4, np.array([], dtype=np.int64), np.array([], dtype=np.int64))
    dg = _dg(api, empty)
    keep, nk, e = api.sparsify_binned(dg, torch.zeros(0, dtype=torch.float32, device="cuda"), SEED, e=0.5)
    assert keep.numel() == 0 and int(_np(nk)[0]) == 0 and e == 0.5
