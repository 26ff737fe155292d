"""Pins of the FP64 oracle against facts that do not come from the oracle.

Each test checks one oracle function against a library routine, a closed
form, an invariant of the method or a brute-force computation on a tiny
graph, chosen so that a plausible slip (a dropped term, a swapped sign, a
wrong index or normalisation) fails at least one of them.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from paper_1601_05527_amd import graphs as G

OMEGA = 0.5


# --------------------------------------------------------------------------
# Start vectors: Philox4x64-10 against numpy's implementation of the same
# published generator.  numpy advances its counter by one before producing
# a block, so block c comes from a numpy generator started at counter c - 1.

def _numpy_philox_block(counter, key):
    ctr = [int(x) for x in counter]
    # subtract one with borrow across the four 64-bit words
    for wi in range(4):
        if ctr[wi] > 0:
            ctr[wi] -= 1
            break
        ctr[wi] = (1 << 64) - 1
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(ctr, dtype=np.uint64))
    return bg.random_raw(4)


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (0, 0)),
    ((12345, 3, 0, 0), (7, 11)),
    ((2**31 - 1, 15, 0, 0), (2**64 - 1, 2**63 + 5)),
    ((0, 1, 0, 0), (42, 0)),
])
def test_philox_matches_numpy(counter, key):
    got = oracle.philox4x64_10(counter, key)
    want = _numpy_philox_block(counter, key)
    assert np.array_equal(got, want)


def test_start_vectors_layout_and_distribution():
    n, R, seed, gid = 5000, 10, 3, 9
    oid = np.random.default_rng(0).permutation(n).astype(np.int32)
    x0 = oracle.start_vectors(n, R, seed, gid, oid)
    # value = word_{r%4}(Philox(key=(seed,gid), ctr=(orig_id, r//4, 0, 0))) >> 40, / 2^24, - 1/2
    for i in [0, 17, 4999]:
        for r in range(R):
            words = _numpy_philox_block((int(oid[i]), r // 4, 0, 0), (seed, gid))
            want = float(int(words[r % 4]) >> 40) / 2**24 - 0.5
            assert x0[i, r] == want
    assert x0.min() >= -0.5 and x0.max() <= 0.5 - 2**-24
    assert np.all((x0 + 0.5) * 2**24 == np.round((x0 + 0.5) * 2**24))
    assert abs(x0.mean()) < 0.01
    assert abs(x0.var() - 1 / 12) < 0.005


# --------------------------------------------------------------------------
# Sweeps: the k JOR sweeps are the linear map H^k with
# H = (1-omega) I + omega S^-1 W (identity rows for isolated vertices).

def _dense_h(g, omega):
    n = g.n
    W = np.zeros((n, n))
    w = np.ones(g.nnz) if g.w is None else g.w.astype(np.float64)
    for i in range(n):
        for p in range(g.row_ptr[i], g.row_ptr[i + 1]):
            W[i, g.col[p]] = w[p]
    s = W.sum(axis=1)
    H = np.eye(n)
    nz = s > 0
    H[nz] = (1 - omega) * np.eye(n)[nz] + omega * W[nz] / s[nz, None]
    return H, W, s


def _tiny_weighted(n=40, m=90, seed=5, isolated=2):
    g = G.gnm(n - isolated, m, seed)
    u, v = g.edge_u, g.edge_v
    w = G.random_weights(m, seed + 1)
    return G.from_edges(n, u, v, w)


def test_sweeps_equal_matrix_power():
    g = _tiny_weighted()
    H, _, _ = _dense_h(g, OMEGA)
    x0 = np.random.default_rng(1).uniform(-0.5, 0.5, g.n)
    for k in [0, 1, 7, 20]:
        got = oracle.relax_vector(g, x0, k, OMEGA)
        want = np.linalg.matrix_power(H, k) @ x0
        np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


def test_sweeps_equal_symmetric_eigendecomposition():
    g = _tiny_weighted(n=50, m=200, seed=8, isolated=0)
    _, W, s = _dense_h(g, 0.7)
    Sh = np.diag(np.sqrt(s))
    Shi = np.diag(1 / np.sqrt(s))
    A = (1 - 0.7) * np.eye(g.n) + 0.7 * Shi @ W @ Shi   # similar to H, symmetric
    lam, U = np.linalg.eigh(A)
    x0 = np.random.default_rng(2).uniform(-0.5, 0.5, g.n)
    k = 13
    want = Shi @ U @ np.diag(lam**k) @ U.T @ Sh @ x0
    got = oracle.relax_vector(g, x0, k, 0.7)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_cycle_closed_form_fft():
    n = 64
    g = G.from_edges(n, np.arange(n), (np.arange(n) + 1) % n)
    x0 = np.random.default_rng(3).uniform(-0.5, 0.5, n)
    k = 25
    q = np.arange(n)
    mu = 1 - OMEGA + OMEGA * np.cos(2 * np.pi * q / n)
    want = np.real(np.fft.ifft(np.fft.fft(x0) * mu**k))
    got = oracle.relax_vector(g, x0, k, OMEGA)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13)


def test_complete_graph_distance_closed_form():
    n, R = 9, 6
    iu = np.array([(a, b) for a in range(n) for b in range(a + 1, n)])
    g = G.from_edges(n, iu[:, 0], iu[:, 1])
    lam = 1 - OMEGA * n / (n - 1)       # the only eigenvalue of H off the constants
    for k in [1, 5, 20]:
        rho = oracle.algebraic_distance(g, R, k, OMEGA, seed=4)
        x0 = oracle.start_vectors(n, R, 4, 0, g.orig_id)
        span = x0.max(axis=0) - x0.min(axis=0)
        xh = (x0 - x0.min(axis=0)) / span
        want = np.sqrt((((xh[g.edge_u] - xh[g.edge_v])) ** 2).sum(axis=1))
        # x^(k) - mean shrinks by lam^k, so FP64 rounding of x (about 1e-17
        # absolute) grows by 1/lam^k relative to the rescaled differences.
        np.testing.assert_allclose(rho, want, rtol=max(1e-13, 1e-15 / lam**k), atol=0)


def test_single_edge_collapses_to_zero():
    g = G.from_edges(2, [0], [1])
    rho = oracle.algebraic_distance(g, 4, 1, OMEGA, seed=1)
    assert rho.tolist() == [0.0]
    rho = oracle.algebraic_distance(g, 4, 6, OMEGA, seed=1)
    assert rho.tolist() == [0.0]


def test_constant_vector_is_a_fixed_point():
    g = _tiny_weighted(n=60, m=150, seed=9)
    x0 = np.full(g.n, 0.25)
    xk = oracle.relax_vector(g, x0, 30, OMEGA)
    assert np.all(xk == 0.25)
    rho = oracle.algebraic_distance(g, 3, 30, OMEGA, x0=np.full((g.n, 3), 0.25))
    assert np.all(rho == 0.0)


def test_weighted_mean_is_conserved():
    # s^T H = s^T, so sum_i s_i x_i^(t) is the same for every t.
    g = _tiny_weighted(n=300, m=1500, seed=11)
    w = g.w.astype(np.float64)
    s = np.bincount(np.repeat(np.arange(g.n), np.diff(g.row_ptr)), weights=w, minlength=g.n)
    x0 = np.random.default_rng(4).uniform(-0.5, 0.5, g.n)
    tr = oracle.relax_vector(g, x0, 20, 0.6, trace=True)
    tot = tr @ s
    np.testing.assert_allclose(tot, tot[0], rtol=0, atol=1e-12)


def test_rescale_maps_onto_half_interval():
    g = _tiny_weighted(n=80, m=200, seed=12, isolated=3)
    x = np.random.default_rng(5).normal(size=g.n)
    xh, lo, hi = oracle.rescale_vector(g, x)
    live = np.diff(g.row_ptr) > 0
    assert lo == x[live].min() and hi == x[live].max()
    assert xh[live].min() == -0.5 and xh[live].max() == 0.5
    assert np.all(xh[~live] == 0.0)


def test_distance_invariant_under_positive_affine_start():
    g = _tiny_weighted(n=120, m=500, seed=13)
    R = 5
    x0 = oracle.start_vectors(g.n, R, 1, 0, g.orig_id)
    rho = oracle.algebraic_distance(g, R, 20, OMEGA, x0=x0)
    rho2 = oracle.algebraic_distance(g, R, 20, OMEGA, x0=3.0 * x0 - 0.125)
    np.testing.assert_allclose(rho2, rho, rtol=1e-12, atol=1e-15)


def test_distance_invariant_under_relabelling():
    g = _tiny_weighted(n=150, m=600, seed=14)
    perm = np.random.default_rng(6).permutation(g.n)
    h = G.relabel(g, perm)
    rho = oracle.algebraic_distance(g, 4, 15, OMEGA, seed=2)
    rho_h = oracle.algebraic_distance(h, 4, 15, OMEGA, seed=2)
    np.testing.assert_allclose(rho_h, rho[h.edge_perm], rtol=1e-12, atol=1e-15)


def test_distance_matches_dense_pipeline():
    # Algorithm 1 end to end with dense numpy: H^k x0, min-max, sum of squares.
    g = _tiny_weighted(n=45, m=120, seed=15, isolated=1)
    R, k = 7, 11
    H, _, _ = _dense_h(g, OMEGA)
    x0 = oracle.start_vectors(g.n, R, 5, 2, g.orig_id)
    xk = np.linalg.matrix_power(H, k) @ x0
    live = np.diff(g.row_ptr) > 0
    lo = xk[live].min(axis=0)
    hi = xk[live].max(axis=0)
    xh = (xk - lo) / (hi - lo) - 0.5
    want = np.sqrt(((xh[g.edge_u] - xh[g.edge_v]) ** 2).sum(axis=1))
    rho, xk_o, xh_o, mm = oracle.algebraic_distance(g, R, k, OMEGA, seed=5, graph_id=2,
                                                    want_vectors=True)
    np.testing.assert_allclose(xk_o, xk, rtol=0, atol=1e-13)
    np.testing.assert_allclose(mm, np.concatenate([lo, hi]), rtol=0, atol=1e-13)
    np.testing.assert_allclose(rho, want, rtol=1e-11, atol=1e-13)


def test_strength_is_inverse_distance():
    rho = np.array([0.0, 1e-3, 0.5, 2.0])
    d = oracle.strength(rho, 1e-12)
    assert d[0] == 1 / math.sqrt(1e-12)
    np.testing.assert_allclose(d[1:], 1 / rho[1:], rtol=1e-6)


# --------------------------------------------------------------------------
# Budget and selection

def test_budget_closed_forms():
    for d in range(1, 20001):
        assert oracle.budget(d, 0.5) == math.isqrt(d)
    for d in [1, 2, 3, 10, 1000, 123457]:
        assert oracle.budget(d, 0.0) == 1
        assert oracle.budget(d, 1.0) == d
    assert oracle.budget(0, 0.5) == 0
    assert oracle.budget(16, 0.25) == 2 and oracle.budget(16, 0.75) == 8
    assert oracle.budget(27, 1 / 3) in (2, 3)   # 1/3 is not exact in binary


def _brute_sparsify(g, rho, orient, e):
    keep = set()
    for i in range(g.n):
        nb = []
        for p in range(g.row_ptr[i], g.row_ptr[i + 1]):
            j = int(g.col[p])
            r = float(rho[g.eid[p]])
            nb.append(((r if orient == oracle.LOCAL else -r), int(g.orig_id[j]), int(g.eid[p])))
        if not nb:
            continue
        nb.sort()
        d = len(nb)
        c = min(d, max(1, int(math.floor(d ** e))))
        keep.update(x[2] for x in nb[:c])
    return keep


@pytest.mark.parametrize("orient", [oracle.LOCAL, oracle.GLOBAL])
@pytest.mark.parametrize("e", [0.0, 0.25, 0.5, 0.75, 1.0])
def test_sparsify_brute_force(orient, e):
    g = _tiny_weighted(n=70, m=260, seed=16, isolated=2)
    rho = oracle.algebraic_distance(g, 6, 10, OMEGA, seed=3)
    rho = np.round(rho, 2)          # force many ties in rho
    keep, kept = oracle.sparsify(g, rho, orient, e)
    want = _brute_sparsify(g, rho, orient, e)
    assert set(np.nonzero(keep)[0].tolist()) == want
    assert kept == len(want)
    deg = np.diff(g.row_ptr)
    c = np.array([min(d, max(1, math.floor(d ** e))) if d else 0 for d in deg])
    assert c.sum() / 2 <= kept <= c.sum()
    if e == 1.0:
        assert kept == g.m
    # every non-isolated vertex keeps at least one edge
    kept_ids = np.nonzero(keep)[0]
    touched = set(g.edge_u[kept_ids].tolist()) | set(g.edge_v[kept_ids].tolist())
    assert touched == set(np.nonzero(deg)[0].tolist())


def test_sparsify_orientation_picks_extremes():
    g = _tiny_weighted(n=90, m=400, seed=17)
    rho = oracle.algebraic_distance(g, 8, 20, OMEGA, seed=6)
    kl, _ = oracle.sparsify(g, rho, oracle.LOCAL, 0.0)
    kg, _ = oracle.sparsify(g, rho, oracle.GLOBAL, 0.0)
    for i in range(g.n):
        ps = range(g.row_ptr[i], g.row_ptr[i + 1])
        ids = [int(g.eid[p]) for p in ps]
        if not ids:
            continue
        best = min(ids, key=lambda q: rho[q])
        worst = max(ids, key=lambda q: rho[q])
        assert kl[best] == 1 and kg[worst] == 1


def test_fit_is_minimal_bisection_point():
    g = _tiny_weighted(n=200, m=1600, seed=18)
    rho = oracle.algebraic_distance(g, 8, 20, OMEGA, seed=7)
    ratios = [len(_brute_sparsify(g, rho, oracle.LOCAL, e)) / g.m for e in np.linspace(0, 1, 21)]
    assert all(b >= a for a, b in zip(ratios, ratios[1:]))
    for orient in (oracle.LOCAL, oracle.GLOBAL):
        for target in (0.3, 0.55):
            e, keep, kept = oracle.fit_exponent(g, rho, orient, target)
            assert 0 < e <= 1
            assert e * 2**40 == round(e * 2**40)
            assert len(_brute_sparsify(g, rho, orient, e)) / g.m >= target
            assert len(_brute_sparsify(g, rho, orient, e - 2**-40)) / g.m < target
            assert kept == int(keep.sum()) == len(_brute_sparsify(g, rho, orient, e))


def test_three_clusters_local_drops_bridges_global_keeps_them():
    # The small network of the paper's Figure 1: dense clusters, sparse cuts.
    g = G.clusters_with_bridges(3, 10)
    bridges = [q for q in range(g.m) if g.edge_u[q] // 10 != g.edge_v[q] // 10]
    top_hits = 0
    local_drop = 0
    global_keep = 0
    seeds = range(100)
    for seed in seeds:
        rho = oracle.algebraic_distance(g, 10, 20, OMEGA, seed=seed)
        top = set(np.argsort(-rho)[:len(bridges)].tolist())
        top_hits += all(b in top for b in bridges)
        kl, _ = oracle.sparsify(g, rho, oracle.LOCAL, 0.0)
        kg, _ = oracle.sparsify(g, rho, oracle.GLOBAL, 0.0)
        local_drop += all(kl[b] == 0 for b in bridges)
        global_keep += all(kg[b] == 1 for b in bridges)
    assert top_hits >= 90
    assert local_drop >= 90
    assert global_keep >= 90


# --------------------------------------------------------------------------
# Gradient of L = sum_e c_e rho_e with respect to the edge weights.



def test_gradient_matches_central_differences():
    g = G.grid_long_range(8, 2, seed=3)
    R, k, seed = 4, 9, 2
    c = np.random.default_rng(9).normal(size=g.m)
    ew = g.edge_w.astype(np.float64)
    x0 = oracle.start_vectors(g.n, R, seed, 0, g.orig_id)
    grad = oracle.grad_weights(g, c, R, k, OMEGA, x0=x0)

    # Dense FP64 forward (independent of the oracle) for the differences.
    def loss(wv):
        n = g.n
        W = np.zeros((n, n))
        W[g.edge_u, g.edge_v] = wv
        W[g.edge_v, g.edge_u] = wv
        s = W.sum(axis=1)
        x = x0.copy()
        for _ in range(k):
            x = (1 - OMEGA) * x + OMEGA * (W @ x) / s[:, None]
        xh = (x - x.min(axis=0)) / (x.max(axis=0) - x.min(axis=0)) - 0.5
        rho = np.sqrt(((xh[g.edge_u] - xh[g.edge_v]) ** 2).sum(axis=1))
        return float(c @ rho)

    fd = np.zeros(g.m)
    for q in range(g.m):
        h = 1e-6 * ew[q]
        wp = ew.copy(); wp[q] += h
        wm = ew.copy(); wm[q] -= h
        fd[q] = (loss(wp) - loss(wm)) / (2 * h)
    err = np.linalg.norm(grad - fd) / np.linalg.norm(fd)
    assert err < 1e-6, err


def test_gradient_matches_central_differences_16x16():
    """The differentiation workload's own pin: on the 16 x 16 copy of the
    grid (480 grid edges + 2 long-range, lognormal weights), R = 8, k = 20,
    the oracle's reverse-mode gradient of sum_e c_e rho_e equals central
    differences of an independent dense FP64 forward, h = 1e-6 w_e, on
    every edge."""
    g = G.grid_long_range(16, 2, seed=0)
    assert g.m == 482
    R, k, seed = 8, 20, 1
    c = np.random.default_rng(10).normal(size=g.m)
    ew = g.edge_w.astype(np.float64)
    x0 = oracle.start_vectors(g.n, R, seed, 0, g.orig_id)
    grad = oracle.grad_weights(g, c, R, k, OMEGA, x0=x0)
    n = g.n

    def loss(wv):
        W = np.zeros((n, n))
        W[g.edge_u, g.edge_v] = wv
        W[g.edge_v, g.edge_u] = wv
        s = W.sum(axis=1)
        x = x0.copy()
        for _ in range(k):
            x = (1 - OMEGA) * x + OMEGA * (W @ x) / s[:, None]
        xh = (x - x.min(axis=0)) / (x.max(axis=0) - x.min(axis=0)) - 0.5
        return float(c @ np.sqrt(((xh[g.edge_u] - xh[g.edge_v]) ** 2).sum(axis=1)))

    fd = np.zeros(g.m)
    for q in range(g.m):
        h = 1e-6 * ew[q]
        wp = ew.copy(); wp[q] += h
        wm = ew.copy(); wm[q] -= h
        fd[q] = (loss(wp) - loss(wm)) / (2 * h)
    err = np.linalg.norm(grad - fd) / np.linalg.norm(fd)
    per = np.abs(grad - fd) / (np.abs(fd) + 1e-3 * np.abs(fd).max())
    assert err < 1e-6, err
    assert per.max() < 1e-5, per.max()


def test_gradient_matches_torch_autograd():
    torch = pytest.importorskip("torch")
    g = G.grid_long_range(16, 2, seed=0)
    R, k, seed = 8, 20, 1
    c = np.random.default_rng(10).normal(size=g.m)
    x0 = oracle.start_vectors(g.n, R, seed, 0, g.orig_id)
    grad = oracle.grad_weights(g, c, R, k, OMEGA, x0=x0)
    wv = torch.tensor(g.edge_w.astype(np.float64), requires_grad=True)
    u = torch.tensor(g.edge_u.astype(np.int64))
    v = torch.tensor(g.edge_v.astype(np.int64))
    n = g.n
    W = torch.zeros((n, n), dtype=torch.float64)
    W = W.index_put((u, v), wv).index_put((v, u), wv)
    s = W.sum(dim=1)
    x = torch.tensor(x0)
    for _ in range(k):
        x = (1 - OMEGA) * x + OMEGA * (W @ x) / s[:, None]
    xh = (x - x.min(dim=0).values) / (x.max(dim=0).values - x.min(dim=0).values) - 0.5
    rho = torch.sqrt(((xh[u] - xh[v]) ** 2).sum(dim=1))
    L = (torch.tensor(c) * rho).sum()
    L.backward()
    np.testing.assert_allclose(grad, wv.grad.numpy(), rtol=1e-9, atol=1e-12)


# --------------------------------------------------------------------------
# Optional normalization (Algorithm 1, last step): out_e = sqrt(rho^2 + eps)
# * sqrt(f_i f_j), the distance whose reciprocal is the normalized delta.

def test_normalization_on_complete_graph_closed_form():
    """On K_n every degree is n - 1: out = (n - 1) * rho, with rho from the
    closed form of the complete graph (independent of the oracle's sweeps)."""
    n, R, k = 9, 6, 5
    iu = np.array([(a, b) for a in range(n) for b in range(a + 1, n)])
    g = G.from_edges(n, iu[:, 0], iu[:, 1])
    x0 = oracle.start_vectors(n, R, 4, 0, g.orig_id)
    xh = (x0 - x0.min(axis=0)) / (x0.max(axis=0) - x0.min(axis=0))
    rho_cf = np.sqrt(((xh[g.edge_u] - xh[g.edge_v]) ** 2).sum(axis=1))
    rho = oracle.algebraic_distance(g, R, k, OMEGA, seed=4)
    for by_strength in (False, True):
        out = oracle.normalize_dist(g, rho, by_strength=by_strength)
        np.testing.assert_allclose(out, (n - 1) * rho_cf, rtol=1e-12)


def test_normalization_invariances():
    g = _tiny_weighted(n=80, m=300, seed=21)
    rho = oracle.algebraic_distance(g, 8, 10, OMEGA, seed=2)
    # unit weights: strength and degree normalizations coincide
    gu = G.with_weights(g, None)
    np.testing.assert_array_equal(oracle.normalize_dist(gu, rho, True), oracle.normalize_dist(gu, rho, False))
    # scaling every weight by c (a power of two, exact in FP32) leaves rho and
    # the degree form unchanged and scales the strength form by c
    c = 4.0
    gc = G.with_weights(g, g.edge_w * np.float32(c))
    rho_c = oracle.algebraic_distance(gc, 8, 10, OMEGA, seed=2)
    np.testing.assert_array_equal(rho_c, rho)
    np.testing.assert_allclose(oracle.normalize_dist(gc, rho, True), c * oracle.normalize_dist(g, rho, True),
                               rtol=1e-12)
    np.testing.assert_array_equal(oracle.normalize_dist(gc, rho, False), oracle.normalize_dist(g, rho, False))
    # eps only lifts the distance: sqrt(rho^2 + eps) >= rho, with equality at eps = 0
    assert np.all(oracle.normalize_dist(g, rho, True, 1e-3) >= oracle.normalize_dist(g, rho, True, 0.0))
    # a single edge collapses to rho = 0, and both ends have degree 1 and weight w
    g1 = G.from_edges(2, [0], [1], np.array([4.0], dtype=np.float32))
    rho1 = oracle.algebraic_distance(g1, 4, 3, OMEGA, seed=1)
    assert oracle.normalize_dist(g1, rho1, False, 0.25).tolist() == [0.5]
    assert oracle.normalize_dist(g1, rho1, True, 0.25).tolist() == [2.0]
    # relabelling the vertices leaves every edge's value unchanged
    perm = np.random.default_rng(3).permutation(g.n)
    gr = G.relabel(g, perm)
    rho_r = oracle.algebraic_distance(gr, 8, 10, OMEGA, seed=2)
    out_r = oracle.normalize_dist(gr, rho_r, True)
    np.testing.assert_allclose(out_r, oracle.normalize_dist(g, rho, True)[gr.edge_perm], rtol=1e-12)


def test_normalization_on_regular_graph_keeps_every_selection():
    """On a regular unweighted graph the factor sqrt(d_i d_j) is one
    constant, so every Algorithm 3 selection is unchanged."""
    n = 60
    u = np.arange(n)
    g = G.from_edges(n, np.concatenate([u, u]), np.concatenate([(u + 1) % n, (u + 7) % n]))
    rho = oracle.algebraic_distance(g, 6, 8, OMEGA, seed=5)
    out = oracle.normalize_dist(g, rho, False)
    np.testing.assert_allclose(out, 4.0 * rho, rtol=1e-15)
    for orient in (0, 1):
        for e in (0.3, 0.6):
            assert np.array_equal(oracle.sparsify(g, out, orient, e)[0], oracle.sparsify(g, rho, orient, e)[0])
