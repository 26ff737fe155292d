"""Host-side checks of the C ABI that need no GPU: the library loads, every
function declared in include/ad.h is exported, and argument validation
rejects bad input before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ad.h")
LIB = os.environ.get("AD_LIBRARY") or os.path.join(ROOT, "paper_1601_05527_amd", "libad.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(ad_[a-z_0-9]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libad.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_four_calls():
    names = _declared()
    for n in ["ad_relax", "ad_edge_dist", "ad_sparsify", "ad_relax_backward"]:
        assert n in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    from paper_1601_05527_amd import api
    for name in _declared():
        assert hasattr(api.lib, name)


def _graph_struct(api, n=4, m=3):
    return api.ADGraph(n, m, 0x1000, 0x2000, None, 0x3000, None, 3, None)


def test_status_strings(lib):
    lib.ad_status_string.restype = ctypes.c_char_p
    assert lib.ad_status_string(0) == b"AD_OK"
    assert lib.ad_status_string(3) == b"AD_ERR_WORKSPACE"


def test_relax_rejects_bad_arguments():
    from paper_1601_05527_amd import api
    L = api.lib
    g = _graph_struct(api)
    ws = ctypes.c_void_p(0x10000)
    out = ctypes.c_void_p(0x20000)
    mm = ctypes.c_void_p(0x30000)

    def call(opts, gp=ctypes.byref(g), ws_=ws, nbytes=1 << 30):
        return L.ad_relax(gp, ctypes.byref(opts), None, out, mm, None, None, ws_, nbytes, None)

    assert L.ad_relax(None, ctypes.byref(api.relax_opts(4, 2)), None, out, mm, None, None, ws,
                      1 << 30, None) == 1
    assert call(api.relax_opts(0, 2)) == 1          # R = 0
    assert call(api.relax_opts(65, 2)) == 1         # R > 64
    assert call(api.relax_opts(4, -1)) == 1         # k < 0
    assert call(api.relax_opts(4, 2, omega=0.0)) == 1
    assert call(api.relax_opts(4, 2, omega=1.5)) == 1
    assert call(api.relax_opts(4, 2, store="bf16", fp32_tail=0)) == 1
    assert call(api.relax_opts(4, 2, store="bf16", ckpt_every=2)) == 2
    assert call(api.relax_opts(4, 2, fp64_tail=-1)) == 1
    assert call(api.relax_opts(4, 2, fp64_tail=1, ckpt_every=1)) == 2     # checkpoints need no FP64 tail
    assert call(api.relax_opts(4, 8, store="bf16", fp32_tail=2, fp64_tail=2)) == 1
    bad_comp = api.Components(2, 1, *[__import__("torch").zeros(1)] * 4)  # fewer chunks than components
    assert call(api.relax_opts(4, 2, comp=bad_comp)) == 1
    assert call(api.relax_opts(4, 2), ws_=ctypes.c_void_p(0x10001)) == 3   # misaligned
    assert call(api.relax_opts(4, 2), nbytes=16) == 3                     # too small
    msg = L.ad_last_error().decode()
    assert "workspace" in msg
    bad = api.ADGraph(4, 3, None, 0x2000, None, 0x3000, None, 3, None)
    assert call(api.relax_opts(4, 2), gp=ctypes.byref(bad)) == 1


def test_selection_rejects_bad_arguments():
    from paper_1601_05527_amd import api
    L = api.lib
    g = _graph_struct(api)
    p = ctypes.c_void_p(0x40000)
    ws = ctypes.c_void_p(0x10000)
    e = ctypes.c_double()
    assert L.ad_sparsify_fit(ctypes.byref(g), 1, p, 0, 0.0, p, p, ctypes.byref(e), ws, 1 << 30, None) == 1
    assert L.ad_sparsify_fit(ctypes.byref(g), 1, p, 0, 1.5, p, p, ctypes.byref(e), ws, 1 << 30, None) == 1
    assert L.ad_sparsify_fit(ctypes.byref(g), 2, p, 0, 0.3, p, p, ctypes.byref(e), ws, 1 << 30, None) == 1
    assert L.ad_sparsify(ctypes.byref(g), 1, p, 7, p, p, p, ws, 1 << 30, None) == 1
    assert L.ad_sparsify(ctypes.byref(g), 1, p, 0, None, p, p, ws, 1 << 30, None) == 1
    assert L.ad_edge_dist(ctypes.byref(g), 0, 1, p, p, 1, p, ws, 1 << 30, None) == 1
    assert L.ad_edge_dist(ctypes.byref(g), 4, 2, p, p, 1, p, ws, 1 << 30, None) == 1
    assert L.ad_edge_dist(ctypes.byref(g), 4, 1, p, p, 2, p, ws, 1 << 30, None) == 1     # BF16 rho
    assert L.ad_edge_dist(ctypes.byref(g), 4, 1, p, p, 0, p, ws, 1 << 30, None) == 2     # FP64 rho of FP32 x
    assert L.ad_edge_dist(ctypes.byref(g), 4, 1, p, p, 1, p, ws, 16, None) == 3
    # fit of both orientations: target and keep_global
    e2 = (ctypes.c_double * 2)()
    assert L.ad_sparsify_fit_both(ctypes.byref(g), 1, p, 0.0, p, p, p, e2, ws, 1 << 30, None) == 1
    assert L.ad_sparsify_fit_both(ctypes.byref(g), 1, p, 0.3, p, None, p, e2, ws, 1 << 30, None) == 1
    # selection with binning: target, exponent, e_used_host, dtype, workspace
    eb = ctypes.byref(e)
    assert L.ad_sparsify_binned(ctypes.byref(g), 1, p, 7, 0, 0.5, 1.5, p, p, eb, ws, 1 << 30, None) == 1
    assert L.ad_sparsify_binned(ctypes.byref(g), 1, p, 7, 0, 0.5, -0.1, p, p, eb, ws, 1 << 30, None) == 1
    assert L.ad_sparsify_binned(ctypes.byref(g), 1, p, 7, 0, 1.5, 0.0, p, p, eb, ws, 1 << 30, None) == 1
    assert L.ad_sparsify_binned(ctypes.byref(g), 1, p, 7, 0, 0.5, 0.3, p, p, None, ws, 1 << 30, None) == 1
    assert L.ad_sparsify_binned(ctypes.byref(g), 2, p, 7, 0, 0.5, 0.0, p, p, eb, ws, 1 << 30, None) == 1
    assert L.ad_sparsify_binned(ctypes.byref(g), 1, p, 7, 0, 0.5, 0.0, None, p, eb, ws, 1 << 30, None) == 1
    need = L.ad_sparsify_binned_workspace_size(ctypes.byref(g))
    assert need >= L.ad_sparsify_fit_both_workspace_size(ctypes.byref(g)) + 5 * 256   # keys, firsts, tables
    assert L.ad_sparsify_binned(ctypes.byref(g), 1, p, 7, 0, 0.5, 0.0, p, p, eb, ws, need - 256, None) == 3
    assert L.ad_sparsify_binned(ctypes.byref(g), 1, p, 7, 0, 0.5, 0.0, p, p, eb, ctypes.c_void_p(0x10008),
                                need, None) == 3
    # distances and selection in one call: R, x dtype, orientation, budget,
    # n_kept, target, keep_global, e_used_host, workspace size and alignment
    gb = ctypes.byref(g)
    need = L.ad_edge_dist_select_workspace_size(gb)
    assert need >= (L.ad_sparsify_fit_both_workspace_size(gb) + L.ad_edge_dist_workspace_size(gb)
                    + 4 * 2 * g.m)
    assert L.ad_edge_dist_sparsify(gb, 0, 1, p, p, p, 0, p, p, p, ws, need, None) == 1
    assert L.ad_edge_dist_sparsify(gb, 4, 2, p, p, p, 0, p, p, p, ws, need, None) == 1      # BF16 x
    assert L.ad_edge_dist_sparsify(gb, 4, 1, p, p, p, 7, p, p, p, ws, need, None) == 1
    assert L.ad_edge_dist_sparsify(gb, 4, 1, p, p, p, 0, None, p, p, ws, need, None) == 1
    assert L.ad_edge_dist_sparsify(gb, 4, 1, p, p, p, 0, p, p, None, ws, need, None) == 1
    assert L.ad_edge_dist_sparsify(gb, 4, 1, p, p, None, 0, p, p, p, ws, need, None) == 1    # rho
    assert L.ad_edge_dist_sparsify(gb, 4, 1, p, p, p, 0, p, p, p, ws, need - 1, None) == 3
    assert L.ad_edge_dist_sparsify(gb, 4, 1, p, p, p, 0, p, p, p, ctypes.c_void_p(0x10008), need, None) == 3
    assert L.ad_edge_dist_fit_both(gb, 4, 1, p, p, p, 0.0, p, p, p, e2, ws, need, None) == 1
    assert L.ad_edge_dist_fit_both(gb, 4, 1, p, p, p, 0.3, p, None, p, e2, ws, need, None) == 1
    assert L.ad_edge_dist_fit_both(gb, 4, 1, p, p, p, 0.3, p, p, p, None, ws, need, None) == 1
    assert L.ad_edge_dist_fit_both(gb, 65, 0, p, p, p, 0.3, p, p, p, e2, ws, need, None) == 1
    assert L.ad_edge_dist_fit_both(gb, 4, 0, p, p, p, 0.3, p, p, p, e2, ws, need - 256, None) == 3
    # normalization: dtype, eps, workspace
    assert L.ad_normalize_dist(ctypes.byref(g), 2, p, 1, 0.0, p, ws, 1 << 30, None) == 1
    assert L.ad_normalize_dist(ctypes.byref(g), 1, p, 1, -1.0, p, ws, 1 << 30, None) == 1
    assert L.ad_normalize_dist(ctypes.byref(g), 1, p, 1, 0.0, p, ws, 8, None) == 3


def test_budget_table_host():
    from paper_1601_05527_amd import api
    import math
    t = api.budget_table(20000, 0.5)
    assert t[0] == 0
    assert all(t[d] == math.isqrt(d) for d in range(1, 20001))
    assert np.all(api.budget_table(100, 0.0)[1:] == 1)
    assert np.all(api.budget_table(100, 1.0) == np.arange(101))
    with pytest.raises(api.ADError):
        api.budget_table(10, 1.5)


def test_workspace_sizes_are_positive():
    from paper_1601_05527_amd import api
    L = api.lib
    g = api.ADGraph(1000, 5000, 0x1000, 0x2000, None, 0x3000, None, 40, None)
    o = api.relax_opts(16, 20)
    assert L.ad_relax_workspace_size(ctypes.byref(g), ctypes.byref(o)) >= 2 * 1000 * 16 * 4
    assert L.ad_sparsify_workspace_size(ctypes.byref(g)) >= 5000 * 24
    assert L.ad_relax_num_checkpoints(ctypes.byref(api.relax_opts(16, 20, ckpt_every=5))) == 4
    assert L.ad_relax_num_checkpoints(ctypes.byref(api.relax_opts(16, 21, ckpt_every=5))) == 5
    assert L.ad_relax_num_checkpoints(ctypes.byref(api.relax_opts(16, 20))) == 0


def test_budget_table_matches_oracle_budget_everywhere():
    """The library fills budget tables step by step; every entry must equal
    the oracle's per-degree floor(d^e) (clamped to [1, d]), including
    exponents at which d^e hits integers (perfect squares, cubes, ...) and
    the fit's grid points k / 2^40."""
    import ctypes
    import oracle
    from paper_1601_05527_amd import api
    lib = oracle._load()
    lib.orc_budget.restype = ctypes.c_int64
    rng = np.random.default_rng(5)
    grid = [float(k) / 2.0 ** 40 for k in rng.integers(0, 1 << 40, 40)]
    exps = [0.0, 1e-12, 0.05, 0.1, 0.25, 1.0 / 3.0, 0.5, 2.0 / 3.0, 0.75, 0.9, 0.999999, 1.0] + grid
    exps += list(rng.uniform(0, 1, 20))
    for d_max in (1, 2, 7, 100, 7147, 70004):
        for e in exps:
            t = api.budget_table(d_max, e)
            want = np.array([0] + [lib.orc_budget(d, e) for d in range(1, d_max + 1)], dtype=np.int64)
            assert np.array_equal(t.astype(np.int64), want), (d_max, e)


def test_gather_probe_library_loads_and_rejects_bad_arguments():
    """The benchmark's gather probe (a measurement aid outside the method's
    library) is built, exports its two calls, and rejects bad arguments
    before launching anything."""
    path = os.path.join(ROOT, "paper_1601_05527_amd", "libad_probe.so")
    if not os.path.exists(path):
        pytest.fail("libad_probe.so is not built (run __graft_entry__.build())")
    probe = ctypes.CDLL(path)
    probe.ad_probe_threads.restype = ctypes.c_int64
    probe.ad_probe_threads.argtypes = [ctypes.c_int]
    assert probe.ad_probe_threads(2048) == 2048 * 256
    i64 = ctypes.c_int64
    probe.ad_probe_gather.argtypes = [ctypes.c_void_p, i64, ctypes.c_int, ctypes.c_void_p, i64, ctypes.c_void_p,
                                      ctypes.c_int, ctypes.c_void_p]
    fake = 0x1000
    assert probe.ad_probe_gather(None, 4, 64, fake, 8, fake, 1, None) == -1      # no rows
    assert probe.ad_probe_gather(fake, 4, 48, fake, 8, fake, 1, None) == -1      # row size
    assert probe.ad_probe_gather(fake, 0, 64, fake, 8, fake, 1, None) == -1      # empty array
    assert probe.ad_probe_gather(fake, 4, 64, fake, 8, fake, 0, None) == -1      # no blocks
    assert probe.ad_probe_gather(fake, 4, 64, fake, 0, fake, 1, None) == 0       # nothing to gather


def test_ingest_rejects_bad_arguments():
    from paper_1601_05527_amd import api
    L = api.lib
    p = ctypes.c_void_p(0x40000)
    ws = ctypes.c_void_p(0x10000)
    m, d, k = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int64()

    def call(n=10, m_in=5, u=p, v=p, w=None, order=1, rp=p, col=p, w_out=p, eid=p, orig=p, ws_=ws, nb=1 << 30):
        return L.ad_ingest(n, m_in, u, v, w, None, order, rp, col, w_out, eid, orig, ctypes.byref(m),
                           ctypes.byref(d), ctypes.byref(k), ws_, nb, None)

    assert call(n=-1) == 1
    assert call(m_in=-2) == 1
    assert call(n=1 << 31) == 2
    assert call(order=3) == 1
    assert call(order=-1) == 1
    assert call(u=None) == 1
    assert call(rp=None) == 1
    assert call(col=None) == 1
    assert call(orig=None) == 1
    assert call(w=p, w_out=None) == 1
    need = L.ad_ingest_workspace_size(10, 5)
    assert need > 0
    assert call(nb=need - 256) == 3
    assert call(ws_=ctypes.c_void_p(0x10010), nb=need) == 3
    assert L.ad_ingest_workspace_size(-1, 5) == 0
    assert L.ad_ingest_workspace_size(10, 1 << 31) == 0
    # the workspace grows with the list and the vertex count
    assert L.ad_ingest_workspace_size(1000, 100_000) > L.ad_ingest_workspace_size(1000, 1000)


def test_property_calls_reject_bad_arguments():
    from paper_1601_05527_amd import api
    L = api.lib
    g = _graph_struct(api)
    p = ctypes.c_void_p(0x40000)
    ws = ctypes.c_void_p(0x10000)
    ms = ctypes.c_int64()
    assert L.ad_subgraph(ctypes.byref(g), None, p, p, None, p, None, ctypes.byref(ms), ws, 1 << 30, None) == 1
    assert L.ad_subgraph(ctypes.byref(g), p, None, p, None, p, None, ctypes.byref(ms), ws, 1 << 30, None) == 1
    assert L.ad_subgraph(ctypes.byref(g), p, p, None, None, p, None, ctypes.byref(ms), ws, 1 << 30, None) == 1
    need = L.ad_subgraph_workspace_size(ctypes.byref(g))
    assert need > 0
    assert L.ad_subgraph(ctypes.byref(g), p, p, p, None, p, None, ctypes.byref(ms), ws, need - 256, None) == 3
    summ = (ctypes.c_double * 2)()
    assert L.ad_graph_properties(ctypes.byref(g), None, None, None, None, ws, 1 << 30, None) == 1
    needp = L.ad_graph_properties_workspace_size(ctypes.byref(g))
    assert L.ad_graph_properties(ctypes.byref(g), None, None, None, summ, ws, needp - 256, None) == 3
    assert L.ad_graph_properties(ctypes.byref(g), None, None, None, summ, ctypes.c_void_p(0x10010), needp,
                                 None) == 3
    rho = ctypes.c_double()
    assert L.ad_spearman(-1, p, p, ctypes.byref(rho), ws, 1 << 30, None) == 1
    assert L.ad_spearman(10, None, p, ctypes.byref(rho), ws, 1 << 30, None) == 1
    assert L.ad_spearman(10, p, p, None, ws, 1 << 30, None) == 1
    assert L.ad_spearman(1 << 31, p, p, ctypes.byref(rho), ws, 1 << 30, None) == 2
    assert L.ad_spearman_workspace_size(-3) == 0


def test_multilevel_calls_reject_bad_arguments():
    from paper_1601_05527_amd import api
    L = api.lib
    g = _graph_struct(api)
    p = ctypes.c_void_p(0x40000)
    ws = ctypes.c_void_p(0x10000)
    nc = ctypes.c_int64()
    need = L.ad_ml_aggregate_workspace_size(ctypes.byref(g))
    assert need > 0
    assert L.ad_ml_aggregate(ctypes.byref(g), 2, p, 1e-12, 0.5, p, None, ctypes.byref(nc), ws, need, None) == 1
    assert L.ad_ml_aggregate(ctypes.byref(g), 1, None, 1e-12, 0.5, p, None, ctypes.byref(nc), ws, need, None) == 1
    assert L.ad_ml_aggregate(ctypes.byref(g), 1, p, 1e-12, 0.5, None, None, ctypes.byref(nc), ws, need, None) == 1
    assert L.ad_ml_aggregate(ctypes.byref(g), 1, p, 1e-12, 0.5, p, None, None, ws, need, None) == 1
    assert L.ad_ml_aggregate(ctypes.byref(g), 1, p, -1.0, 0.5, p, None, ctypes.byref(nc), ws, need, None) == 1
    assert L.ad_ml_aggregate(ctypes.byref(g), 1, p, 1e-12, 1.5, p, None, ctypes.byref(nc), ws, need, None) == 1
    assert L.ad_ml_aggregate(ctypes.byref(g), 1, p, 1e-12, 0.5, p, None, ctypes.byref(nc), ws, need - 256,
                             None) == 3
    assert L.ad_ml_aggregate(ctypes.byref(g), 1, p, 1e-12, 0.5, p, None, ctypes.byref(nc),
                             ctypes.c_void_p(0x10010), need, None) == 3
    big = api.ADGraph(1 << 31, 3, 0x1000, 0x2000, None, 0x3000, None, 3, None)
    assert L.ad_ml_aggregate_workspace_size(ctypes.byref(big)) == 0

    e = (ctypes.c_double * 4)(0.5, 0.5, 0.5, 0.5)
    ep = ctypes.cast(e, ctypes.c_void_p).value

    def opts(**kw):
        base = dict(R=8, k=10, omega=0.5, seed=1, graph_id=0, store=1, levels=4, n_min=10, e_host=ep, eps=1e-12,
                    theta=0.5, bin_seed=3)
        base.update(kw)
        return api.ADMLOpts(**base)

    kept, depth = ctypes.c_int64(), ctypes.c_int32()

    def call(o, keep=p, kh=True):
        return L.ad_ml_sparsify(ctypes.byref(g), ctypes.byref(o), keep, ctypes.byref(kept) if kh else None,
                                ctypes.byref(depth), None)

    for bad in [dict(R=0), dict(R=65), dict(k=-1), dict(omega=0.0), dict(omega=1.5), dict(store=2),
                dict(levels=0), dict(levels=65), dict(n_min=-1), dict(e_host=None), dict(eps=-1.0),
                dict(theta=2.0), dict(fit=2), dict(span=-1), dict(span=1, segment=3), dict(span=1, segment=-1),
                dict(span=1, span_value=1.5), dict(span=1, span_value=float("nan"))]:
        assert call(opts(**bad)) == 1, bad
    e[2] = 1.5
    assert call(opts()) == 1
    e[2] = 0.5
    assert call(opts(), keep=None) == 1
    assert call(opts(), kh=False) == 1
    huge = api.ADGraph(4, 1 << 30, 0x1000, 0x2000, None, 0x3000, None, 3, None)
    assert L.ad_ml_sparsify(ctypes.byref(huge), ctypes.byref(opts()), p, ctypes.byref(kept), None, None) == 2


def test_level_span_helper_matches_oracle():
    import oracle
    from paper_1601_05527_amd import api
    for n in range(1, 13):
        for span in range(0, 5):
            for seg in range(3):
                np.testing.assert_array_equal(api.ml_level_span(n, span, seg, 0.3),
                                              oracle.ml_level_span(n, span, seg, 0.3))
    out = (ctypes.c_double * 4)()
    p = ctypes.cast(out, ctypes.c_void_p)
    assert api.lib.ad_ml_level_span(0, 1, 0, 0.3, p) == 1
    assert api.lib.ad_ml_level_span(4, 1, 3, 0.3, p) == 1
    assert api.lib.ad_ml_level_span(4, -1, 0, 0.3, p) == 1
    assert api.lib.ad_ml_level_span(4, 1, 0, 0.3, None) == 1
