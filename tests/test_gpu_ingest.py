"""Ingest (ad_ingest: an edge list into the symmetric CSR) against the oracle,
through the C ABI.  Integer work and a fixed summation order: every output
array must equal the oracle's bit for bit.
"""
import numpy as np
import pytest

import oracle
from paper_1601_05527_amd import graphs as G

from gpu_helpers import announce

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def api():
    from paper_1601_05527_amd import api as _api
    return _api


def _np(t):
    return t.detach().cpu().numpy()


def _list(n, m_in, seed, dup_frac=0.2, loop_frac=0.02):
    rng = np.random.default_rng(seed)
    u = rng.integers(0, n, m_in)
    v = rng.integers(0, n, m_in)
    k = int(m_in * dup_frac)
    pick = rng.integers(0, m_in, k)
    flip = rng.random(k) < 0.5
    u = np.concatenate([u, np.where(flip, v[pick], u[pick])])
    v = np.concatenate([v, np.where(flip, u[pick], v[pick])])
    loops = rng.integers(0, n, int(m_in * loop_frac))
    u = np.concatenate([u, loops])
    v = np.concatenate([v, loops])
    perm = rng.permutation(u.size)
    w = rng.lognormal(0.0, 1.0, u.size).astype(np.float32)
    return u[perm].astype(np.int32), v[perm].astype(np.int32), w


def _run(api, n, u, v, w=None, orig=None, by_degree=True, order=None):
    cu = lambda a: None if a is None else torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return api.ingest(n, cu(u), cu(v), cu(w), cu(orig), by_degree=by_degree, order=order)


def _compare(dg, ref):
    row_ptr, col, we, eid, orig, m, dropped = ref
    assert dg.m == m and dg.n_dropped == dropped
    assert dg.d_max == (int(np.diff(row_ptr).max()) if len(row_ptr) > 1 else 0)
    np.testing.assert_array_equal(_np(dg.row_ptr), row_ptr)
    np.testing.assert_array_equal(_np(dg.col), col)
    np.testing.assert_array_equal(_np(dg.eid), eid)
    np.testing.assert_array_equal(_np(dg.orig_id), orig)
    if we is None:
        assert dg.w is None
    else:
        np.testing.assert_array_equal(_np(dg.w), we)


@pytest.mark.parametrize("by_degree", [False, True])
@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("weighted", [False, True])
def test_ingest_bit_exact(api, by_degree, seed, weighted):
    announce(f"ingest seed={seed} by_degree={by_degree} weighted={weighted}")
    n = [300, 5000, 70_000][seed]
    u, v, w = _list(n, 8 * n, seed)
    w = w if weighted else None
    dg = _run(api, n, u, v, w, by_degree=by_degree)
    _compare(dg, oracle.ingest(n, u, v, w, order=1 if by_degree else 0))


def test_ingest_long_runs_and_hubs(api):
    """One pair listed 5,000 times (a long merge run, summed by a workgroup),
    a star of degree 20,000 and isolated vertices."""
    announce("ingest long runs and hubs")
    rng = np.random.default_rng(7)
    n = 40_000
    u = [np.full(5000, 3), np.full(20_000, 9), rng.integers(100, 30_000, 50_000)]
    v = [np.full(5000, 17), rng.permutation(np.arange(10, 40_000))[:20_000], rng.integers(100, 30_000, 50_000)]
    u = np.concatenate(u).astype(np.int32)
    v = np.concatenate(v).astype(np.int32)
    w = rng.uniform(0.01, 10.0, u.size).astype(np.float32)
    for by_degree in (False, True):
        dg = _run(api, n, u, v, w, by_degree=by_degree)
        _compare(dg, oracle.ingest(n, u, v, w, order=1 if by_degree else 0))


def test_ingest_run_lengths_at_the_wave_bounds(api):
    """Runs of 1 .. 1000 repeats around the one-thread / one-wave split and
    the 64-lane chunks, weights spread over many binades (so the order of
    the double additions shows), listed in shuffled order; a hub that is
    the larger endpoint of 30,000 edges and one that is the smaller."""
    announce("ingest run lengths at wave bounds")
    rng = np.random.default_rng(19)
    n = 50_000
    us, vs = [], []
    for r, L in enumerate([1, 2, 15, 16, 17, 63, 64, 65, 127, 128, 129, 1000]):
        us.append(np.full(L, 100 + r))
        vs.append(np.full(L, 200 + r))
    us.append(rng.integers(0, n - 1, 30_000))
    vs.append(np.full(30_000, n - 1))
    us.append(np.full(20_000, 5))
    vs.append(rng.integers(6, n, 20_000))
    u = np.concatenate(us).astype(np.int32)
    v = np.concatenate(vs).astype(np.int32)
    perm = rng.permutation(u.size)
    u, v = u[perm], v[perm]
    w = np.exp(rng.uniform(-20, 20, u.size)).astype(np.float32)
    for by_degree in (False, True):
        dg = _run(api, n, u, v, w, by_degree=by_degree)
        _compare(dg, oracle.ingest(n, u, v, w, order=1 if by_degree else 0))


def test_ingest_exact_weight_sums(api):
    """Merged weights are exact sums rounded once: ties to even, a value
    just above a tie, subnormals, runs whose values span more than 53 bits
    (the digit path) and less (the double path), short and long, in
    shuffled list order."""
    announce("ingest exact weight sums")
    f = np.float32
    rng = np.random.default_rng(29)
    runs = [[1.0, 2.0 ** -24], [1.0, 2.0 ** -24, 2.0 ** -60], [1.0 + 2.0 ** -23, 2.0 ** -24],
            [2.0 ** -149] * 3, [3.0], [2.0 ** 100, 2.0 ** -100, 2.0 ** -149]]
    runs.append(list(rng.uniform(1, 2, 40) * 2.0 ** rng.integers(-140, 100, 40)))      # short, digits
    runs.append(list(rng.uniform(1, 2, 900) * 2.0 ** rng.integers(-3, 3, 900)))        # long, double
    runs.append(list(rng.uniform(1, 2, 5000) * 2.0 ** rng.integers(-120, 120, 5000)))  # long, digits
    runs.append([1.0] + [2.0 ** -30] * 63 + [2.0 ** -90] * 200)                           # long, near a tie
    u, v, w = [], [], []
    for r, vals in enumerate(runs):
        u += [2 * r] * len(vals)
        v += [2 * r + 1] * len(vals)
        w += vals
    u, v = np.array(u, np.int32), np.array(v, np.int32)
    w = np.maximum(np.array(w, dtype=np.float32), f(2.0 ** -149))
    perm = rng.permutation(u.size)
    u, v, w = u[perm], v[perm], w[perm]
    n = 2 * len(runs)
    for by_degree in (False, True):
        dg = _run(api, n, u, v, w, by_degree=by_degree)
        _compare(dg, oracle.ingest(n, u, v, w, order=1 if by_degree else 0))
    dg = _run(api, n, u, v, w, by_degree=False)
    got = _np(dg.w)[_np(dg.row_ptr)[:-1:2]]          # row 2r holds the one edge of run r
    assert got[0] == f(1.0) and got[1] == f(1.0 + 2.0 ** -23) and got[2] == f(1.0 + 2.0 ** -22)
    assert got[3] == f(3 * 2.0 ** -149)
    for bad in (0.0, -2.0, np.inf, np.nan):
        with pytest.raises(api.ADError) as ex:
            _run(api, 3, np.array([0, 1], np.int32), np.array([1, 2], np.int32), np.array([1.0, bad], np.float32))
        assert ex.value.status == 4       # AD_ERR_GRAPH


def test_ingest_orig_ids_and_reuse(api):
    """Names pass through; the ingested graph relaxes exactly like the same
    CSR uploaded from the host."""
    announce("ingest names and use")
    g = G.chung_lu(8000, 60_000, seed=4)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    up = g.col > rows
    names = np.random.default_rng(3).permutation(g.n).astype(np.int32)
    dg = _run(api, g.n, rows[up].astype(np.int32), g.col[up], g.w[up], names)
    _compare(dg, oracle.ingest(g.n, rows[up], g.col[up], g.w[up], orig_id=names, order=1))
    h = G.relabel(G.from_edges(g.n, rows[up], g.col[up], g.w[up], orig_id=names),
                  G.degree_descending_order(g))
    dh = api.DeviceGraph.from_host(h, "cuda")
    a = api.relax(dg, 8, 10, seed=5)
    b = api.relax(dh, 8, 10, seed=5)
    assert torch.equal(a.x, b.x) and torch.equal(a.minmax, b.minmax)


@pytest.mark.parametrize("seed", [0, 1, 2])
@pytest.mark.parametrize("weighted", [False, True])
def test_ingest_rcm_bit_exact(api, seed, weighted):
    """Reverse Cuthill-McKee order (order 2) against the oracle on random
    lists with repeats and loops (one large component, isolated vertices)."""
    announce(f"ingest rcm seed={seed} weighted={weighted}")
    n = [300, 5000, 70_000][seed]
    u, v, w = _list(n, 8 * n, seed)
    w = w if weighted else None
    dg = _run(api, n, u, v, w, order="rcm")
    _compare(dg, oracle.ingest(n, u, v, w, order=2))


@pytest.mark.parametrize("kind", ["components", "grid", "path", "power_law"])
def test_ingest_rcm_shapes(api, kind):
    """Many components of different sizes searched at once; a grid (a few
    hundred levels, many degree ties); a path (one level per vertex); a
    power-law graph (hub rows, many equal degrees)."""
    announce(f"ingest rcm {kind}")
    rng = np.random.default_rng(7)
    if kind == "components":
        us, vs, base = [], [], 0
        for size in [1, 2, 3, 10, 50, 400, 2000, 1, 7, 300]:
            if size > 1:
                a = rng.integers(0, size, 3 * size)
                b = (a + rng.integers(1, size, 3 * size)) % size
                us.append(a + base)
                vs.append(b + base)
            base += size
        n = base + 100                                     # 100 isolated vertices at the end
        perm = rng.permutation(n)
        u, v = perm[np.concatenate(us)], perm[np.concatenate(vs)]
    elif kind == "grid":
        k = 120
        idx = np.arange(k * k).reshape(k, k)
        u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
        v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
        n = k * k
        perm = rng.permutation(n)
        u, v = perm[u], perm[v]
    elif kind == "path":
        n = 3000
        perm = rng.permutation(n)
        u, v = perm[:-1], perm[1:]
    else:
        g = G.chung_lu(20_000, 150_000, seed=5)
        rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
        up = g.col > rows
        n, u, v = g.n, rows[up], g.col[up]
    u, v = u.astype(np.int32), v.astype(np.int32)
    w = rng.uniform(0.5, 2.0, u.size).astype(np.float32)
    dg = _run(api, n, u, v, w, order="rcm")
    _compare(dg, oracle.ingest(n, u, v, w, order=2))


def test_ingest_edge_cases(api):
    announce("ingest edge cases")
    z = np.zeros(0, dtype=np.int32)
    dg = _run(api, 5, z, z)
    assert dg.m == 0 and dg.d_max == 0 and _np(dg.row_ptr).tolist() == [0] * 6
    assert _np(dg.orig_id).tolist() == list(range(5))
    only_loops = np.array([1, 2, 2], dtype=np.int32)
    dg = _run(api, 4, only_loops, only_loops)
    assert dg.m == 0 and dg.n_dropped == 3
    one = _run(api, 2, np.array([1], dtype=np.int32), np.array([0], dtype=np.int32),
               np.array([2.5], dtype=np.float32), by_degree=False)
    _compare(one, oracle.ingest(2, [1], [0], [2.5], order=0))
    # reverse Cuthill-McKee with no edges (every vertex a component of its own),
    # only loops, and one edge among isolated vertices
    for n, uu, vv in [(5, z, z), (4, only_loops, only_loops), (6, np.array([4], np.int32), np.array([1], np.int32))]:
        dg = _run(api, n, uu, vv, order="rcm")
        _compare(dg, oracle.ingest(n, uu, vv, order=2))
    with pytest.raises(api.ADError) as ex:
        _run(api, 4, np.array([0, 4], dtype=np.int32), np.array([1, 1], dtype=np.int32))
    assert ex.value.status == 4       # AD_ERR_GRAPH
    with pytest.raises(api.ADError):
        _run(api, 4, np.array([-1], dtype=np.int32), np.array([1], dtype=np.int32))
