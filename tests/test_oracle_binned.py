"""Pins of the oracle's SparsifyB (Algorithm 4, binned selection) against
what the paper and the mathematics fix, without reusing the oracle's code:

  - Scott's bin rule h = 3.5 sigma / d^(1/3) worked by hand on arithmetic
    progressions, where sigma has a closed form;
  - the random neighbour order: MurmurHash3's finalizer against the
    published empty-input vectors of MurmurHash3_x86_32, and distinctness;
  - special cases: one bin (all distances equal) is a uniform sample,
    e = 0 keeps the first neighbour of the random order, e = 1 keeps all;
  - invariants: every bin gives an edge before any gives a second (the
    "sample from all bins" of Section 4), the choices grow with e, counts
    are the budget, results do not depend on vertex labels, and the fit
    returns the smallest bisection point reaching the target.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1601_05527_amd import graphs as G

SEED = 11


def _star(values):
    """Star whose centre 0 has one edge per value; rho of edge (0, q+1) is
    values[q] (edge ids follow the CSR convention: edge q joins 0 and q+1)."""
    d = len(values)
    g = G.from_edges(d + 1, np.zeros(d, dtype=np.int64), np.arange(1, d + 1))
    rho = np.zeros(g.m)
    for e in range(g.m):
        rho[e] = values[int(g.edge_v[e]) - 1]
    return g, rho


def test_fmix32_matches_murmur3_empty_input_vectors():
    # MurmurHash3_x86_32 of the empty input with seed s is fmix32(s)
    assert oracle.bin_priority(0, 1) == 0x514E28B7
    assert oracle.bin_priority(0, -1) == 0x81F16F39
    assert oracle.bin_priority(0, 0) == 0


def test_priorities_are_a_permutation_of_neighbour_ids():
    K = oracle.bin_vertex_key(SEED, 12345)
    ids = np.random.default_rng(0).choice(1 << 30, size=20000, replace=False)
    pr = {oracle.bin_priority(K, int(i)) for i in ids}
    assert len(pr) == len(ids)


@pytest.mark.parametrize("c", [1.0, 0.37, 1e-3])
def test_scott_rule_on_eight_equally_spaced_values(c):
    # sigma = c sqrt(63/12) = 2.2913c, h = 3.5 sigma / 2 = 4.0098c, range 7c:
    # two bins, values 0..4 (below h) in the first, 5..7 in the second
    g, rho = _star([c * q for q in range(8)])
    bins, nb = oracle.bin_layout(g, rho)
    assert nb[0] == 2 and all(nb[1:] == 1)
    centre = bins[g.row_ptr[0]:g.row_ptr[1]]
    leaf = g.col[g.row_ptr[0]:g.row_ptr[1]] - 1
    np.testing.assert_array_equal(centre, (leaf >= 5).astype(np.int32))


def test_scott_rule_on_twenty_seven_equally_spaced_values():
    # sigma = sqrt(728/12) = 7.7889, h = 3.5 sigma / 3 = 9.0870, range 26:
    # three bins holding 0..9, 10..18 and 19..26
    g, rho = _star([float(q) for q in range(27)])
    bins, nb = oracle.bin_layout(g, rho)
    assert nb[0] == 3
    centre = bins[g.row_ptr[0]:g.row_ptr[1]]
    leaf = g.col[g.row_ptr[0]:g.row_ptr[1]] - 1
    np.testing.assert_array_equal(centre, np.where(leaf <= 9, 0, np.where(leaf <= 18, 1, 2)))
    assert np.bincount(centre).tolist() == [10, 9, 8]


def test_sigma_is_the_population_deviation():
    # 0..4: population sigma = sqrt(2) = 1.4142, h = 3.5 sigma / 5^(1/3) =
    # 2.8946, bins = ceil(4 / 2.8946) = 2 holding 0..2 and 3..4 (the sample
    # deviation, 1.5811, would put 3 in the first bin)
    g, rho = _star([float(q) for q in range(5)])
    bins, nb = oracle.bin_layout(g, rho)
    leaf = g.col[g.row_ptr[0]:g.row_ptr[1]] - 1
    assert nb[0] == 2
    np.testing.assert_array_equal(bins[g.row_ptr[0]:g.row_ptr[1]], (leaf >= 3).astype(np.int32))
    # 0..2: sigma = sqrt(2/3) = 0.8165, h = 1.9814 < range 2: two bins, the
    # top value alone (the sample deviation, 1, would give one bin)
    g, rho = _star([0.0, 1.0, 2.0])
    bins, nb = oracle.bin_layout(g, rho)
    leaf = g.col[g.row_ptr[0]:g.row_ptr[1]] - 1
    assert nb[0] == 2
    np.testing.assert_array_equal(bins[g.row_ptr[0]:g.row_ptr[1]], (leaf == 2).astype(np.int32))


def test_one_outlier_spreads_bins_over_the_range():
    # values 0 (63 times) and 64: mean 1, population variance (63 + 63^2) / 64
    # = 63, sigma = 7.937; h = 3.5 * 7.937 / 4 = 6.945, bins = ceil(64 / 6.945)
    # = 10; the zeros fill bin 0 and the outlier the last bin
    g, rho = _star([0.0] * 63 + [64.0])
    bins, nb = oracle.bin_layout(g, rho)
    sigma = math.sqrt(63.0)
    assert nb[0] == math.ceil(64.0 / (3.5 * sigma / 4.0)) == 10
    centre = bins[g.row_ptr[0]:g.row_ptr[1]]
    leaf = g.col[g.row_ptr[0]:g.row_ptr[1]] - 1
    assert all(centre[leaf < 63] == 0) and centre[leaf == 63][0] == 9


def _random_case(n=300, m=2400, seed=3):
    g = G.gnm(n, m, seed=seed)
    rho = np.random.default_rng(seed).lognormal(0.0, 0.7, g.m)
    return g, rho


def _rows(g):
    return np.repeat(np.arange(g.n), np.diff(g.row_ptr))


def _priorities(g, seed=SEED):
    rows = _rows(g)
    out = np.zeros(len(g.col), dtype=np.uint64)
    keys = {}
    for p in range(len(g.col)):
        i = int(rows[p])
        if i not in keys:
            keys[i] = oracle.bin_vertex_key(seed, int(g.orig_id[i]))
        out[p] = oracle.bin_priority(keys[i], int(g.orig_id[g.col[p]]))
    return out


def test_equal_distances_give_one_bin_and_a_uniform_sample():
    g, _ = _random_case(n=120, m=900, seed=4)
    rho = np.full(g.m, 0.25)
    _, nb = oracle.bin_layout(g, rho)
    assert all(nb[np.diff(g.row_ptr) > 0] == 1)
    ch = oracle.binned_choices(g, rho, 0.5, SEED)
    pr = _priorities(g)
    for i in range(g.n):
        b, e = g.row_ptr[i], g.row_ptr[i + 1]
        if e == b:
            continue
        c = oracle.budget(e - b, 0.5)
        want = np.zeros(e - b, dtype=np.uint8)
        want[np.argsort(pr[b:e])[:c]] = 1
        np.testing.assert_array_equal(ch[b:e], want)


def test_exponent_zero_and_one():
    g, rho = _random_case()
    ch0 = oracle.binned_choices(g, rho, 0.0, SEED)
    pr = _priorities(g)
    for i in range(g.n):
        b, e = g.row_ptr[i], g.row_ptr[i + 1]
        if e > b:
            assert ch0[b:e].sum() == 1 and ch0[b + int(np.argmin(pr[b:e]))] == 1
    keep1, kept1 = oracle.sparsify_binned(g, rho, 1.0, SEED)
    assert kept1 == g.m and keep1.all()


@pytest.mark.parametrize("e", [0.3, 0.5, 0.8])
def test_every_bin_gives_one_edge_before_any_gives_two(e):
    g, rho = _random_case(n=200, m=3000, seed=6)
    bins, nb = oracle.bin_layout(g, rho)
    ch = oracle.binned_choices(g, rho, e, SEED)
    checked = 0
    for i in range(g.n):
        b, en = g.row_ptr[i], g.row_ptr[i + 1]
        d = en - b
        if d == 0:
            continue
        assert ch[b:en].sum() == oracle.budget(d, e)
        size = np.bincount(bins[b:en], minlength=nb[i])
        took = np.bincount(bins[b:en], weights=ch[b:en], minlength=nb[i]).astype(int)
        open_bins = (size > took) & (size > 0)
        if open_bins.any():
            lo, hi = took[open_bins].min(), took[size > 0].max()
            assert hi - lo <= 1, (i, size, took)
            # a bin that ran out holds fewer edges than any open bin took, plus one
            assert all(took[(size == took) & (size > 0)] <= lo + 1)
        if oracle.budget(d, e) >= (size > 0).sum():
            assert all(took[size > 0] >= 1)
            checked += 1
    if e >= 0.5:      # budgets large enough to reach every bin somewhere
        assert checked > 20


def test_choices_grow_with_the_exponent():
    g, rho = _random_case(seed=8)
    prev = oracle.binned_choices(g, rho, 0.0, SEED)
    for e in np.linspace(0.05, 1.0, 12):
        cur = oracle.binned_choices(g, rho, float(e), SEED)
        assert np.all(cur >= prev)
        prev = cur


def test_keep_is_the_union_of_both_endpoints_choices():
    g, rho = _random_case(seed=9)
    ch = oracle.binned_choices(g, rho, 0.4, SEED)
    keep, kept = oracle.sparsify_binned(g, rho, 0.4, SEED)
    want = np.zeros(g.m, dtype=np.uint8)
    want[g.eid[ch == 1]] = 1
    np.testing.assert_array_equal(keep, want)
    assert kept == int(want.sum())


def test_binned_selection_does_not_depend_on_labels():
    g, rho = _random_case(n=250, m=2000, seed=10)
    perm = np.random.default_rng(2).permutation(g.n)
    h = G.relabel(g, perm)
    k1, n1 = oracle.sparsify_binned(g, rho, 0.5, SEED)
    k2, n2 = oracle.sparsify_binned(h, rho[h.edge_perm], 0.5, SEED)
    assert n1 == n2
    np.testing.assert_array_equal(k2, k1[h.edge_perm])


def test_seed_changes_the_sample_but_not_the_counts():
    g, rho = _random_case(seed=12)
    a = oracle.binned_choices(g, rho, 0.5, SEED)
    b = oracle.binned_choices(g, rho, 0.5, SEED + 1)
    assert (a != b).any()
    rows = _rows(g)
    np.testing.assert_array_equal(np.bincount(rows, weights=a, minlength=g.n),
                                  np.bincount(rows, weights=b, minlength=g.n))


def test_binned_fit_is_minimal_bisection_point():
    g, rho = _random_case(seed=13)
    target = 0.45
    e, keep, kept = oracle.fit_exponent_binned(g, rho, target, SEED)
    assert kept / g.m >= target
    _, below = oracle.sparsify_binned(g, rho, max(0.0, e - 2.0 ** -38), SEED)
    assert below / g.m < target
    np.testing.assert_array_equal(keep, oracle.sparsify_binned(g, rho, e, SEED)[0])
