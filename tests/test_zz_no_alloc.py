"""The allocation-free distance entry point (ad_edge_dist_noalloc) against
ad_edge_dist, through the C ABI: two calls in a row on one GPU, the second
on a smaller graph (the fixed scratch array keeps the first call's plan),
each equal to the workspace call bit for bit, for FP32 and FP64 vectors."""
import ctypes

import numpy as np
import pytest

from paper_1601_05527_amd import graphs as G
from paper_1601_05527_amd.workloads import FP64_TAIL

from gpu_helpers import announce

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    from paper_1601_05527_amd import api as _api
    return _api


def _noalloc(api, dg, x, minmax, rho_dtype):
    R = x.shape[1]
    out = torch.full((dg.m,), float("nan"), dtype=rho_dtype, device=x.device)
    g = dg.abi()
    xt = api.AD_F64 if x.dtype == torch.float64 else api.AD_F32
    rt = api.AD_F64 if rho_dtype == torch.float64 else api.AD_F32
    st = api.lib.ad_edge_dist_noalloc(ctypes.byref(g), R, xt, ctypes.c_void_p(x.data_ptr()),
                                      ctypes.c_void_p(minmax.data_ptr()), rt, ctypes.c_void_p(out.data_ptr()),
                                      api._stream())
    api._check(st)
    return out


def test_noalloc_equals_edge_dist(api):
    big = G.chung_lu(200_000, 3_000_000, seed=51)          # hub rows beyond the distance pass's hub degree
    small = G.rmat(12, 30_000, seed=52)
    for name, g in (("chung-lu 200k", big), ("r-mat 4k", small)):
        announce(f"noalloc distances {name}")
        dg = api.DeviceGraph.from_host(g, "cuda")
        for store, tail in (("f32", 0), ("f32", FP64_TAIL), ("f64", 0)):
            res = api.relax(dg, 16, 12, seed=3, store=store, fp64_tail=tail)
            want = api.distances(dg, res)
            got = _noalloc(api, dg, res.x, res.minmax, want.dtype)
            torch.cuda.synchronize()
            assert torch.equal(got, want), (name, store, tail)


def test_noalloc_refuses_a_plan_beyond_the_array(api):
    announce("noalloc refuses an oversized plan")
    n = 1 << 24
    g = api.ADGraph(n, 1, 0x1000, 0x2000, None, 0x3000, None, 1, None)
    p = ctypes.c_void_p(0x4000)
    assert api.lib.ad_edge_dist_workspace_size(ctypes.byref(g)) > api.lib.ad_edge_dist_noalloc_max_bytes()
    st = api.lib.ad_edge_dist_noalloc(ctypes.byref(g), 16, api.AD_F32, p, p, api.AD_F32, p, None)
    assert st == 2 and "scratch" in api.lib.ad_last_error().decode()
