"""Batched form: each graph of a batch gets, bit for bit, the distances and
kept edges of running it alone, and agrees with the FP64 oracle (FP32
storage with its last sweeps in FP64: 1e-5 relative on every edge)."""
import numpy as np
import pytest

import oracle
from paper_1601_05527_amd import graphs as G
from paper_1601_05527_amd.workloads import FP64_TAIL

from gpu_helpers import announce, rel_stats

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    from paper_1601_05527_amd import api as _api
    return _api


def _graphs():
    out = [
        G.chung_lu(3000, 30_000, seed=21),
        G.chung_lu(700, 4_000, seed=22),
        G.grid_long_range(40, 20, seed=23),
        G.gnm(1500, 9_000, 24),
        G.from_edges(50, np.zeros(0, int), np.zeros(0, int)),       # no edges
        G.rmat(11, 12_000, seed=25),
        G.chung_lu(12_000, 200_000, seed=26),                         # has hub rows
    ]
    # a graph with isolated vertices and unit weights
    g = G.gnm(990, 3000, 27)
    out.append(G.from_edges(1000, g.edge_u, g.edge_v))
    return out


@pytest.mark.parametrize("orient", [0, 1])
def test_batch_equals_standalone_and_oracle(api, orient):
    announce(f"batch vs standalone orient={orient}")
    gs = _graphs()
    dgs = [api.DeviceGraph.from_host(g, "cuda") for g in gs]
    R, k, seed, gid, e = 8, 20, 5, 100, 0.5
    b = api.Batch(dgs, R, k, seed=seed, graph_id=gid, orient=orient, e=e, autotune=True, fp64_tail=FP64_TAIL)
    b.run()
    rho, keep, n_kept, mm = [t.cpu().numpy() for t in b.fetch()]
    torch.cuda.synchronize()
    for q, (g, dg) in enumerate(zip(gs, dgs)):
        e0, e1 = b.edge_off[q], b.edge_off[q + 1]
        res = api.relax(dg, R, k, seed=seed, graph_id=gid + q, rows_per_wave=b.rows_per_wave, fp64_tail=FP64_TAIL)
        rho_s = api.distances(dg, res)
        if g.m:
            keep_s, nk_s = api.sparsify(dg, rho_s, orient, e)
            assert np.array_equal(rho[e0:e1], rho_s.cpu().numpy()), q
            assert np.array_equal(keep[e0:e1], keep_s.cpu().numpy()), q
            assert int(n_kept[q]) == int(nk_s.item()), q
            rho_o = oracle.algebraic_distance(g, R, k, 0.5, seed=seed, graph_id=gid + q)
            assert rel_stats(rho[e0:e1], rho_o)["max"] <= 1e-5, q
        else:
            assert int(n_kept[q]) == 0
        assert np.array_equal(mm[q], res.minmax.cpu().numpy()), q
    b.close()


def test_batch_replays_are_identical(api):
    announce("batch graph replays")
    gs = _graphs()[:4]
    dgs = [api.DeviceGraph.from_host(g, "cuda") for g in gs]
    b = api.Batch(dgs, 8, 20, seed=1, orient=0, e=0.5, autotune=False)
    b.run(captured=False)
    ref = [t.clone() for t in b.fetch()]
    for rep in range(3):
        b.run()
        # eager work and a synchronisation between replays
        scratch = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        got = b.fetch()
        for a, c in zip(ref, got):
            assert torch.equal(a, c), rep
        del scratch
    b.close()
