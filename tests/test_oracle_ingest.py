"""Pins of the oracle's ingest (edge list -> the symmetric CSR of the graph
model of Section 2) by brute force on small lists and by invariants:

  - a Python dictionary build of the same reading (pairs unordered, loops
    dropped, repeats merged with the exact sum of their weights rounded once
    to single precision, by fractions.Fraction and an exact nearest-float
    search) gives the same arrays, entry for entry;
  - the exact sum itself against Fraction arithmetic over weights spanning
    the whole float range (subnormals included), and hand-worked ties;
  - the CSR is symmetric, rows ascending, edge ids paired and numbered in
    (smaller, larger) order; feeding its own edge list back is a fixed point;
  - the decreasing-degree order really is one, ties by listed id, and keeps
    the edge set (through orig_id);
  - the reverse Cuthill-McKee order: a hand-worked graph with a degree tie;
    bandwidth 1 on a scrambled path and at most 2k on a scrambled k x k
    grid; and on random graphs with several components, checked by brute
    force against breadth-first distances from scipy: components contiguous
    in increasing order of their smallest id, each starting at its vertex of
    least (degree, id), levels non-decreasing, and each level ordered by
    (place of the first-placed neighbour one level up, degree, id);
  - out-of-range endpoints are refused; the empty list gives an empty graph.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from paper_1601_05527_amd import graphs as G


def _random_list(n, m_in, seed, loops=True, dups=True):
    rng = np.random.default_rng(seed)
    u = rng.integers(0, n, m_in)
    v = rng.integers(0, n, m_in)
    if not loops:
        keep = u != v
        u, v = u[keep], v[keep]
    if dups and u.size > 4:
        # repeat some pairs, some flipped
        k = u.size // 5
        u = np.concatenate([u, v[:k], u[k:2 * k]])
        v = np.concatenate([v, u[:k], v[k:2 * k]])
    w = rng.uniform(0.1, 3.0, u.size).astype(np.float32)
    return u.astype(np.int32), v.astype(np.int32), w


def _round_f32(fr):
    """The float32 nearest to the rational fr (ties to the even mantissa),
    found by exact comparison among float32 neighbours."""
    # half an ulp above FLT_MAX is a tie, which goes to the even inf
    if fr >= Fraction(float(np.finfo(np.float32).max)) + Fraction(2) ** 103:
        return np.float32(np.inf)
    f = np.float32(float(fr))
    cands = {f, np.nextafter(f, np.float32(np.inf)), np.nextafter(f, np.float32(-np.inf))}
    cands = [c for c in cands if np.isfinite(c)]
    best = min(cands, key=lambda c: (abs(Fraction(float(c)) - fr), int(np.array(c).view(np.uint32)) & 1))
    return np.float32(best)


def _brute(n, u, v, w):
    sums = {}
    for q in range(len(u)):
        a, b = int(u[q]), int(v[q])
        if a == b:
            continue
        key = (min(a, b), max(a, b))
        sums[key] = sums.get(key, Fraction(0)) + Fraction(float(w[q]))     # exact
    edges = sorted(sums)
    eid = {e: i for i, e in enumerate(edges)}
    rows = [[] for _ in range(n)]
    for (a, b) in edges:
        rows[a].append(b)
        rows[b].append(a)
    row_ptr, col, ws, ids = [0], [], [], []
    for i in range(n):
        for j in sorted(rows[i]):
            e = (min(i, j), max(i, j))
            col.append(j)
            ws.append(_round_f32(sums[e]))
            ids.append(eid[e])
        row_ptr.append(len(col))
    return (np.array(row_ptr), np.array(col, dtype=np.int32), np.array(ws, dtype=np.float32),
            np.array(ids, dtype=np.int32), len(edges))


@pytest.mark.parametrize("seed", range(6))
def test_ingest_equals_dictionary_build(seed):
    n = 40 + 7 * seed
    u, v, w = _random_list(n, 300, seed)
    row_ptr, col, we, eid, orig, m, dropped = oracle.ingest(n, u, v, w)
    b_rp, b_col, b_w, b_eid, b_m = _brute(n, u, v, w)
    assert m == b_m and dropped == len(u) - m
    np.testing.assert_array_equal(row_ptr, b_rp)
    np.testing.assert_array_equal(col, b_col)
    np.testing.assert_array_equal(we, b_w)
    np.testing.assert_array_equal(eid, b_eid)
    np.testing.assert_array_equal(orig, np.arange(n))


def _check_csr(n, row_ptr, col, eid, m):
    assert row_ptr[0] == 0 and row_ptr[-1] == 2 * m
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    for i in range(n):
        r = col[row_ptr[i]:row_ptr[i + 1]]
        assert np.all(np.diff(r) > 0) and np.all(r != i)
    # each edge id appears exactly twice, as (a, b) and (b, a)
    first = {}
    for p in range(len(col)):
        first.setdefault(int(eid[p]), []).append((int(rows[p]), int(col[p])))
    assert sorted(first) == list(range(m))
    pairs = []
    for e in range(m):
        (a, b), (c, d) = first[e]
        assert (a, b) == (d, c)
        pairs.append((min(a, b), max(a, b)))
    assert pairs == sorted(pairs)          # ids follow (smaller, larger) order


@pytest.mark.parametrize("order", [0, 1, 2])
def test_ingest_structure_and_fixed_point(order):
    n = 200
    u, v, w = _random_list(n, 2000, 11)
    row_ptr, col, we, eid, orig, m, _ = oracle.ingest(n, u, v, w, order=order)
    _check_csr(n, row_ptr, col, eid, m)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    up = col > rows
    again = oracle.ingest(n, rows[up], col[up], we[up], orig_id=orig)
    np.testing.assert_array_equal(again[0], row_ptr)
    np.testing.assert_array_equal(again[1], col)
    np.testing.assert_array_equal(again[2], we)
    np.testing.assert_array_equal(again[3], eid)
    np.testing.assert_array_equal(again[4], orig)


def test_decreasing_degree_order():
    n = 300
    u, v, w = _random_list(n, 2500, 12)
    base = oracle.ingest(n, u, v, w)
    row_ptr, col, we, eid, orig, m, _ = oracle.ingest(n, u, v, w, order=1)
    deg = np.diff(row_ptr)
    assert np.all(np.diff(deg) <= 0)
    # ties keep the listed order
    for d in np.unique(deg):
        ids = orig[deg == d]
        assert np.all(np.diff(ids) > 0)
    assert sorted(orig.tolist()) == list(range(n))
    # the same weighted edge set, named by listed ids
    def edge_set(rp, cl, ww, oid):
        rows = np.repeat(np.arange(n), np.diff(rp))
        return {(int(min(oid[a], oid[b])), int(max(oid[a], oid[b]))): float(x)
                for a, b, x in zip(rows, cl, ww)}
    assert edge_set(row_ptr, col, we, orig) == edge_set(base[0], base[1], base[2], base[4])


def test_decreasing_degree_order_matches_relabel():
    g = G.chung_lu(3000, 20_000, seed=2)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    up = g.col > rows
    h = G.relabel(g, G.degree_descending_order(g))
    out = oracle.ingest(g.n, rows[up], g.col[up], g.w[up], order=1)
    np.testing.assert_array_equal(out[0], h.row_ptr)
    np.testing.assert_array_equal(out[1], h.col)
    np.testing.assert_array_equal(out[2], h.w)
    np.testing.assert_array_equal(out[3], h.eid)
    np.testing.assert_array_equal(out[4], h.orig_id)


def test_rcm_hand_worked():
    """Edges 0-1, 0-2, 0-3, 1-4, 2-4, 3-5 and the isolated vertex 6.
    Component {0..5} starts at 5 (the only degree-1 vertex): 5; 3; 0; then
    0's neighbours 1 and 2 (both degree 2: by id); then 4.  Component {6}
    follows.  Cuthill-McKee order 5 3 0 1 2 4 6, reversed: new ids
    6 <- 5, 5 <- 3, 4 <- 0, 3 <- 1, 2 <- 2, 1 <- 4, 0 <- 6."""
    u = np.array([0, 0, 0, 1, 2, 3], dtype=np.int32)
    v = np.array([1, 2, 3, 4, 4, 5], dtype=np.int32)
    row_ptr, col, _, eid, orig, m, _ = oracle.ingest(7, u, v, order=2)
    assert m == 6
    assert orig.tolist() == [6, 4, 2, 1, 0, 3, 5]
    _check_csr(7, row_ptr, col, eid, m)


def _bandwidth(row_ptr, col):
    rows = np.repeat(np.arange(row_ptr.size - 1), np.diff(row_ptr))
    return int(np.abs(rows - col).max()) if col.size else 0


def test_rcm_bandwidth_of_path_and_grid():
    rng = np.random.default_rng(21)
    n = 500
    perm = rng.permutation(n)
    u, v = perm[:-1], perm[1:]
    row_ptr, col, *_ = oracle.ingest(n, u, v, order=2)
    assert _bandwidth(row_ptr, col) == 1
    k = 30
    ii, jj = np.meshgrid(np.arange(k), np.arange(k), indexing="ij")
    idx = (ii * k + jj).ravel()
    right = np.stack([idx.reshape(k, k)[:, :-1].ravel(), idx.reshape(k, k)[:, 1:].ravel()])
    down = np.stack([idx.reshape(k, k)[:-1, :].ravel(), idx.reshape(k, k)[1:, :].ravel()])
    e = np.concatenate([right, down], axis=1)
    scr = rng.permutation(k * k)
    base = oracle.ingest(k * k, scr[e[0]], scr[e[1]])
    assert _bandwidth(base[0], base[1]) > 10 * k           # scrambled
    row_ptr, col, *_ = oracle.ingest(k * k, scr[e[0]], scr[e[1]], order=2)
    assert _bandwidth(row_ptr, col) <= 2 * k


@pytest.mark.parametrize("seed", [31, 32, 33])
def test_rcm_is_the_stated_breadth_first_order(seed):
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components, shortest_path
    rng = np.random.default_rng(seed)
    n = 400
    # a few dense blocks, sparse links, isolated vertices, repeated pairs
    u = rng.integers(0, 300, 700)
    v = (u + rng.integers(1, 12, 700)) % 300
    u = np.concatenate([u, rng.integers(300, 380, 90)])
    v = np.concatenate([v, rng.integers(300, 380, 90)])
    w = rng.uniform(0.5, 2.0, u.size).astype(np.float32)
    listed = oracle.ingest(n, u, v, w)                 # the graph under the listed ids
    lrp, lcol = listed[0], listed[1]
    deg = np.diff(lrp)
    a = sp.csr_matrix((np.ones(lcol.size), lcol, lrp), shape=(n, n))
    nc, lab = connected_components(a, directed=False)
    row_ptr, col, we, eid, orig, m, _ = oracle.ingest(n, u, v, w, order=2)
    _check_csr(n, row_ptr, col, eid, m)
    assert sorted(orig.tolist()) == list(range(n))
    cm = orig[::-1]                                    # listed vertex at each Cuthill-McKee place
    place = np.empty(n, dtype=np.int64)
    place[cm] = np.arange(n)
    # components contiguous, in increasing order of their smallest id
    comp_seq = lab[cm]
    runs = [comp_seq[0]] + [c for p, c in zip(comp_seq[:-1], comp_seq[1:]) if c != p]
    assert len(runs) == nc
    smallest = {c: int(np.nonzero(lab == c)[0].min()) for c in range(nc)}
    assert [smallest[c] for c in runs] == sorted(smallest[c] for c in runs)
    start = 0
    for c in runs:
        members = np.nonzero(lab == c)[0]
        seq = cm[start:start + members.size]
        s0 = min(members, key=lambda x: (deg[x], x))
        assert seq[0] == s0
        dist = shortest_path(a, unweighted=True, indices=[s0])[0]
        lev = dist[seq]
        assert np.all(np.diff(lev) >= 0)
        key = []
        for x in seq[1:]:
            ups = [y for y in lcol[lrp[x]:lrp[x + 1]] if dist[y] == dist[x] - 1]
            key.append((dist[x], min(place[y] for y in ups), deg[x], x))
        assert key == sorted(key)
        start += members.size
    # the same weighted edge set, named by listed ids
    def edge_set(rp, cl, ww, oid):
        rows = np.repeat(np.arange(n), np.diff(rp))
        return {(int(min(oid[p], oid[q])), int(max(oid[p], oid[q]))): float(x) for p, q, x in zip(rows, cl, ww)}
    assert edge_set(row_ptr, col, we, orig) == edge_set(listed[0], listed[1], listed[2], listed[4])


def test_orig_ids_pass_through():
    n = 50
    u, v, w = _random_list(n, 200, 13)
    names = np.random.default_rng(1).permutation(10_000)[:n].astype(np.int32)
    out = oracle.ingest(n, u, v, w, orig_id=names, order=1)
    ref = oracle.ingest(n, u, v, w, order=1)
    np.testing.assert_array_equal(out[4], names[ref[4]])


def test_unweighted_lists_and_edge_cases():
    out = oracle.ingest(5, [0, 1, 1], [1, 0, 1])
    assert out[2] is None and out[5] == 1 and out[6] == 2
    empty = oracle.ingest(3, [], [])
    assert empty[5] == 0 and np.all(empty[0] == 0)
    with pytest.raises(ValueError):
        oracle.ingest(3, [0, 3], [1, 1])
    with pytest.raises(ValueError):
        oracle.ingest(3, [-1], [1])


def test_exact_sum_against_fractions():
    rng = np.random.default_rng(21)
    tiny = np.float32(2.0 ** -149)
    for trial in range(40):
        k = int(rng.integers(1, 60))
        # magnitudes spread over the whole float range, subnormals included
        x = (rng.uniform(1, 2, k) * 2.0 ** rng.integers(-149, 100, k)).astype(np.float32)
        x = np.maximum(x, tiny)
        want = _round_f32(sum((Fraction(float(t)) for t in x), Fraction(0)))
        assert oracle.exact_sum_f32(x) == want, (trial, x)
    # the same order-free result for any permutation
    x = (rng.uniform(0.5, 2, 500) * 2.0 ** rng.integers(-40, 40, 500)).astype(np.float32)
    s0 = oracle.exact_sum_f32(x)
    for _ in range(3):
        assert oracle.exact_sum_f32(rng.permutation(x)) == s0


def test_exact_sum_hand_cases():
    f = np.float32
    e = lambda k: f(2.0 ** k)
    s = oracle.exact_sum_f32
    assert s([f(1.0), e(-24)]) == f(1.0)                              # a tie goes to the even 1.0
    assert s([f(1.0), e(-24), e(-60)]) == f(1.0 + 2.0 ** -23)         # just above the tie
    assert s([f(1.0 + 2.0 ** -23), e(-24)]) == f(1.0 + 2.0 ** -22)    # a tie with an odd mantissa
    assert s([e(-149), e(-149)]) == e(-148)                           # subnormals add exactly
    assert s([f(np.finfo(np.float32).max)] * 2) == np.inf
    assert s([f(3.0)]) == f(3.0) and s([]) == f(0.0)
    # summing in double in list order would give 1.0 here: the exact sum does not
    x = [f(1.0), e(-24), e(-60)]
    assert f(np.float64(1.0) + 2.0 ** -24 + 2.0 ** -60) == f(1.0)
    assert s(x) == f(1.0 + 2.0 ** -23)


def test_ingest_refuses_non_positive_weights():
    u, v = np.array([0, 1], np.int32), np.array([1, 2], np.int32)
    for bad in (0.0, -1.0, np.inf, np.nan):
        with pytest.raises(ValueError):
            oracle.ingest(3, u, v, np.array([1.0, bad], np.float32))
