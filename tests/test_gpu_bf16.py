"""BF16 storage of the test vectors (FP32 arithmetic, FP32 degree
normalisation and distances) against the FP64 oracle.

Bound: 2e-2 relative on rho, over edges whose oracle distance is at least
a tenth of the median (smaller distances are measured against that floor:
BF16 keeps 8 significant bits of x_i and x_j, so the error of x_i - x_j is
absolute, on the scale of the vectors, not of their difference), with the
last 8 sweeps stored in FP32 (they damp the rounding noise of the BF16
sweeps, which is mostly high-frequency).  Kept-edge sets agree except on
edges within 2e-2 of a deciding endpoint's cut.
"""
import numpy as np
import pytest

import oracle
from paper_1601_05527_amd import graphs as G

from gpu_helpers import announce, check_fp32, near_cut_mismatches, rel_stats

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

TOL = 2e-2
TAIL = 8          # sweeps stored in FP32 at the end of the relaxation


@pytest.fixture(scope="module")
def api():
    from paper_1601_05527_amd import api as _api
    return _api


def _np(t):
    return t.detach().cpu().numpy()


def _case(kind):
    if kind == "rmat":
        return G.rmat(15, 16 << 15, seed=31), 16, 30
    if kind == "chung_lu":
        return G.chung_lu(1 << 15, 400_000, seed=32), 16, 20
    return G.grid_long_range(128, 400, seed=33), 8, 20


def _stats(rho, rho_o):
    floor = 0.1 * float(np.median(rho_o))
    st = rel_stats(rho, rho_o, floor)
    rel = st["rel"]
    return {"max": st["max"], "p999": st["p999"], "p99": float(np.quantile(rel, 0.99)),
            "median": float(np.median(rel)), "floor": floor}


@pytest.mark.parametrize("kind", ["rmat", "chung_lu", "grid"])
def test_bf16_distances_against_oracle(api, kind):
    announce(f"BF16 storage {kind}")
    g, R, k = _case(kind)
    dg = api.DeviceGraph.from_host(g, "cuda")
    rho_o, xk_o, _, mm_o = oracle.algebraic_distance(g, R, k, 0.5, seed=9, want_vectors=True)
    x0 = oracle.start_vectors(g.n, R, 9, 0, g.orig_id)
    res16 = api.relax(dg, R, k, seed=9, store="bf16", fp32_tail=TAIL)
    rho16 = _np(api.edge_dist(dg, res16.x, res16.minmax))
    res32 = api.relax(dg, R, k, seed=9, store="f32")
    rho32 = _np(api.edge_dist(dg, res32.x, res32.minmax))
    s16 = _stats(rho16, rho_o)
    ratio32, s32 = check_fp32(g, x0, xk_o, mm_o, rho32, rho_o, k)
    print(f"{kind}: n={g.n} m={g.m} R={R} k={k}  BF16 rel err max {s16['max']:.2e} p99.9 {s16['p999']:.2e} "
          f"p99 {s16['p99']:.2e} median {s16['median']:.2e}  |  FP32 {s32}, worst/bound {ratio32:.2f}")
    assert ratio32 <= 1.0
    assert s16["max"] <= TOL
    # kept edges: BF16 distances against the oracle's, both orientations
    for orient in (0, 1):
        e = 0.5
        keep, _ = api.sparsify(dg, torch.from_numpy(rho16).cuda(), orient, e)
        keep_o, _ = oracle.sparsify(g, rho_o, orient, e)
        bad = near_cut_mismatches(g, rho_o, _np(keep), keep_o, orient, e, TOL)
        assert not bad, bad[:10]


@pytest.mark.parametrize("tail", [1, 2, 4, 8, 12])
def test_bf16_fp32_tail(api, tail):
    """Every split between BF16 and FP32 sweeps runs; the error falls as
    the FP32 tail (the last sweeps stored in FP32) grows, and from 8 tail
    sweeps on it is within the bound."""
    announce(f"BF16 tail={tail}")
    g, R, k = _case("rmat")
    dg = api.DeviceGraph.from_host(g, "cuda")
    rho_o = oracle.algebraic_distance(g, R, k, 0.5, seed=9)
    res = api.relax(dg, R, k, seed=9, store="bf16", fp32_tail=tail)
    rho = _np(api.edge_dist(dg, res.x, res.minmax))
    st = _stats(rho, rho_o)
    print(f"tail {tail}: max {st['max']:.2e} p99.9 {st['p999']:.2e} p99 {st['p99']:.2e} median {st['median']:.2e}")
    assert st["median"] <= TOL
    if tail >= TAIL:
        assert st["max"] <= TOL
