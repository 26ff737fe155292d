"""Graph containers and seeded synthetic generators.

This module only builds inputs: symmetric CSR arrays of an undirected simple
graph G = (V, E, w) (the graph model of the paper's Preliminaries section:
undirected, no self-loops, no multi-edges, non-negative weights) and seeded
random graphs with the structure of the paper's workloads.  It holds none of
the method's arithmetic (no degrees-as-weights, no relaxation, no distances);
both the FP64 oracle and the HIP library consume the arrays it returns.

CSR conventions (shared by every consumer):

* ``row_ptr`` int64[n+1], ``col`` int32[2m] sorted ascending inside each row.
* ``w`` float32[2m] (``w[ij] == w[ji]``) or ``None`` for unit weights.
* ``eid`` int32[2m]: undirected edge id of each stored entry.  Both mirror
  entries (i, j) and (j, i) carry the same id.  Edges are numbered in
  lexicographic order of (min(i, j), max(i, j)), so the upper entries
  (j > i) of the CSR enumerate 0, 1, 2, ... in storage order.
* ``orig_id`` int32[n]: the vertex id before any relabelling; it keys the
  random start vectors and breaks ranking ties, so results do not depend on
  the storage order of the vertices.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np


@dataclasses.dataclass
class Graph:
    """Symmetric CSR of an undirected simple weighted graph (host arrays)."""

    n: int
    row_ptr: np.ndarray          # int64 [n+1]
    col: np.ndarray              # int32 [2m]
    w: Optional[np.ndarray]      # float32 [2m] or None (unit weights)
    eid: np.ndarray              # int32 [2m]
    orig_id: np.ndarray          # int32 [n]
    edge_u: np.ndarray           # int32 [m], edge_u < edge_v
    edge_v: np.ndarray           # int32 [m]
    edge_w: Optional[np.ndarray]  # float32 [m] or None

    @property
    def m(self) -> int:
        return int(self.edge_u.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def degree(self) -> np.ndarray:
        return np.diff(self.row_ptr)

    @property
    def d_max(self) -> int:
        return int(self.degree.max()) if self.n else 0

    def degree_values(self) -> np.ndarray:
        """Sorted distinct degrees present (int32)."""
        return np.unique(self.degree).astype(np.int32)


def from_edges(n: int, u, v, w=None, orig_id=None) -> Graph:
    """Build the symmetric CSR from an undirected edge list.

    ``u``/``v`` may be in any order and orientation; self-loops and repeated
    pairs are rejected (the graph model excludes them).  ``w`` holds one
    weight per listed edge.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if u.shape != v.shape:
        raise ValueError("u and v differ in length")
    if u.size and (min(u.min(), v.min()) < 0 or max(u.max(), v.max()) >= n):
        raise ValueError("vertex id out of range")
    if np.any(u == v):
        raise ValueError("self-loops are not allowed")
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = lo * n + hi
    order = np.argsort(key, kind="stable")
    key_s = key[order]
    if key_s.size > 1 and np.any(key_s[1:] == key_s[:-1]):
        raise ValueError("repeated edges are not allowed")
    lo = lo[order]
    hi = hi[order]
    m = lo.size
    ew = None
    if w is not None:
        ew = np.asarray(w, dtype=np.float32)[order]
        if not np.all(np.isfinite(ew)) or np.any(ew <= 0):
            raise ValueError("weights must be finite and > 0")
    # Directed entries: (lo, hi) and (hi, lo); sort by (row, col).
    rows = np.concatenate([lo, hi])
    cols = np.concatenate([hi, lo])
    ids = np.concatenate([np.arange(m, dtype=np.int64)] * 2)
    dkey = rows * n + cols
    dorder = np.argsort(dkey, kind="stable")
    rows = rows[dorder]
    cols = cols[dorder]
    ids = ids[dorder]
    counts = np.bincount(rows, minlength=n) if n else np.zeros(0, np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    cw = None
    if ew is not None:
        cw = ew[ids].astype(np.float32)
    if orig_id is None:
        orig_id = np.arange(n, dtype=np.int32)
    return Graph(
        n=int(n),
        row_ptr=row_ptr,
        col=cols.astype(np.int32),
        w=cw,
        eid=ids.astype(np.int32),
        orig_id=np.asarray(orig_id, dtype=np.int32),
        edge_u=lo.astype(np.int32),
        edge_v=hi.astype(np.int32),
        edge_w=ew,
    )


def relabel(g: Graph, perm_new_of_old: np.ndarray) -> Graph:
    """Store vertex ``i`` under the new id ``perm_new_of_old[i]``.

    The undirected edge set, weights and ``orig_id`` travel with the
    vertices, so every result keyed by ``orig_id`` is unchanged.  Edge ids
    are renumbered by the CSR convention of the new labels; ``edge_perm`` on
    the result maps new edge id -> old edge id.
    """
    p = np.asarray(perm_new_of_old, dtype=np.int64)
    nu = p[g.edge_u]
    nv = p[g.edge_v]
    new_orig = np.empty(g.n, dtype=np.int32)
    new_orig[p] = g.orig_id
    lo = np.minimum(nu, nv)
    hi = np.maximum(nu, nv)
    order = np.argsort(lo * g.n + hi, kind="stable")
    h = from_edges(g.n, lo[order], hi[order],
                   None if g.edge_w is None else g.edge_w[order],
                   orig_id=new_orig)
    h.edge_perm = order.astype(np.int64)  # type: ignore[attr-defined]
    return h


def degree_descending_order(g: Graph) -> np.ndarray:
    """New id of every vertex when vertices are stored by decreasing degree
    (ties by current id).  A storage layout, not part of the method."""
    deg = g.degree
    order_old = np.lexsort((np.arange(g.n), -deg))
    new_of_old = np.empty(g.n, dtype=np.int64)
    new_of_old[order_old] = np.arange(g.n)
    return new_of_old


# ---------------------------------------------------------------------------
# Seeded generators
# ---------------------------------------------------------------------------

def gnm(n: int, m: int, seed: int = 0) -> Graph:
    """Erdos-Renyi G(n, m): m distinct unordered non-loop pairs, rejection
    sampled with ``numpy.random.default_rng(seed)``.  Unit weights."""
    if m > n * (n - 1) // 2:
        raise ValueError("too many edges")
    rng = np.random.default_rng(seed)
    keys = np.zeros(0, dtype=np.int64)
    while keys.size < m:
        need = m - keys.size
        a = rng.integers(0, n, size=2 * need + 16)
        b = rng.integers(0, n, size=2 * need + 16)
        ok = a != b
        a, b = a[ok], b[ok]
        lo = np.minimum(a, b)
        hi = np.maximum(a, b)
        new = lo * n + hi
        # keep the first occurrence order-independently: sorted unique merge
        cand = np.setdiff1d(np.unique(new), keys, assume_unique=True)
        if cand.size > need:
            cand = rng.permutation(cand)[:need]
        keys = np.union1d(keys, cand)
    return from_edges(n, keys // n, keys % n)


def chung_lu(n: int, m: int, gamma: float = 2.1, seed: int = 0,
             weights: str = "lognormal", permute: bool = True) -> Graph:
    """Chung-Lu power-law graph with exactly ``m`` distinct edges.

    Expected-degree weights theta_i = ((i + 1/2) / n)^(-1/(gamma-1)), capped
    at sqrt(sum theta) (so that no pair is forced above probability one),
    endpoint pairs drawn i.i.d. proportionally to theta, loops and repeats
    dropped, drawing repeated until ``m`` distinct pairs exist.  Vertex ids
    are then randomly permuted.  Weights: lognormal(0, 1) per undirected
    edge, or unit.
    """
    rng = np.random.default_rng(seed)
    i = np.arange(n, dtype=np.float64)
    theta = ((i + 0.5) / n) ** (-1.0 / (gamma - 1.0))
    theta *= (2.0 * m / n) / theta.mean()        # expected degrees, mean 2m/n
    theta = np.minimum(theta, math.sqrt(theta.sum()))
    cdf = np.cumsum(theta)
    cdf /= cdf[-1]
    keys = np.zeros(0, dtype=np.int64)
    while keys.size < m:
        need = m - keys.size
        k = int(need * 1.15) + 1024
        a = np.searchsorted(cdf, rng.random(k), side="right")
        b = np.searchsorted(cdf, rng.random(k), side="right")
        a = np.minimum(a, n - 1)
        b = np.minimum(b, n - 1)
        ok = a != b
        a, b = a[ok], b[ok]
        lo = np.minimum(a, b).astype(np.int64)
        hi = np.maximum(a, b).astype(np.int64)
        new = np.unique(lo * n + hi)
        new = new[~np.isin(new, keys, assume_unique=True)]
        if new.size > need:
            new = np.sort(rng.choice(new, size=need, replace=False))
        keys = np.union1d(keys, new)
    lo = keys // n
    hi = keys % n
    if permute:
        perm = rng.permutation(n)
        lo, hi = perm[lo], perm[hi]
    w = None
    if weights == "lognormal":
        w = rng.lognormal(0.0, 1.0, size=m).astype(np.float32)
    elif weights == "uniform":
        w = rng.uniform(0.5, 2.0, size=m).astype(np.float32)
    return from_edges(n, lo, hi, w)


def rmat(scale: int, m: int, a=0.57, b=0.19, c=0.19, seed: int = 0,
         weights: str = "uniform", permute: bool = True,
         chunk: int = 1 << 24) -> Graph:
    """R-MAT graph on n = 2^scale vertices with ``m`` distinct undirected
    non-loop edges (quadrant probabilities a, b, c, d = 1-a-b-c), drawn in
    chunks until ``m`` distinct pairs exist, then randomly permuted.
    Weights uniform(0.5, 2) per undirected edge by default."""
    n = 1 << scale
    rng = np.random.default_rng(seed)
    keys = np.zeros(0, dtype=np.int64)
    ab = a + b
    abc = a + b + c
    while keys.size < m:
        need = m - keys.size
        k = min(chunk, int(need * 1.3) + 1024)
        src = np.zeros(k, dtype=np.int64)
        dst = np.zeros(k, dtype=np.int64)
        for lvl in range(scale):
            r = rng.random(k, dtype=np.float32)
            bit = np.int64(1) << (scale - 1 - lvl)
            right = ((r >= a) & (r < ab)) | (r >= abc)
            down = r >= ab
            src += np.where(down, bit, 0)
            dst += np.where(right, bit, 0)
        ok = src != dst
        lo = np.minimum(src[ok], dst[ok])
        hi = np.maximum(src[ok], dst[ok])
        new = np.unique(lo * n + hi)
        new = new[~np.isin(new, keys, assume_unique=True)]
        if new.size > need:
            new = np.sort(rng.choice(new, size=need, replace=False))
        keys = np.union1d(keys, new)
    lo = keys // n
    hi = keys % n
    if permute:
        perm = rng.permutation(n)
        lo, hi = perm[lo], perm[hi]
    w = None
    if weights == "uniform":
        w = rng.uniform(0.5, 2.0, size=m).astype(np.float32)
    elif weights == "lognormal":
        w = rng.lognormal(0.0, 1.0, size=m).astype(np.float32)
    return from_edges(n, lo, hi, w)


def grid_long_range(side: int, n_long: int, seed: int = 0,
                    weights: str = "lognormal") -> Graph:
    """side x side 4-neighbour grid plus ``n_long`` uniformly random extra
    edges between distinct non-adjacent vertex pairs.  Row-major vertex ids
    (the natural, banded order of a mesh)."""
    n = side * side
    rng = np.random.default_rng(seed)
    idx = np.arange(n, dtype=np.int64).reshape(side, side)
    h_u = idx[:, :-1].ravel()
    h_v = idx[:, 1:].ravel()
    v_u = idx[:-1, :].ravel()
    v_v = idx[1:, :].ravel()
    base = np.union1d(np.concatenate([h_u, v_u]) * n + np.concatenate([h_v, v_v]),
                      np.zeros(0, np.int64))
    extra = np.zeros(0, dtype=np.int64)
    while extra.size < n_long:
        need = n_long - extra.size
        a = rng.integers(0, n, size=2 * need + 8)
        b = rng.integers(0, n, size=2 * need + 8)
        ok = a != b
        lo = np.minimum(a[ok], b[ok])
        hi = np.maximum(a[ok], b[ok])
        cand = np.unique(lo * n + hi)
        cand = cand[~np.isin(cand, base)]
        cand = cand[~np.isin(cand, extra)]
        if cand.size > need:
            cand = np.sort(rng.choice(cand, size=need, replace=False))
        extra = np.union1d(extra, cand)
    keys = np.union1d(base, extra)
    w = None
    if weights == "lognormal":
        w = rng.lognormal(0.0, 1.0, size=keys.size).astype(np.float32)
    return from_edges(n, keys // n, keys % n, w)


def clusters_with_bridges(n_clusters: int = 3, size: int = 10) -> Graph:
    """Disjoint complete graphs K_size joined in a ring by single bridge
    edges (the small three-cluster network of the paper's Figure 1)."""
    us, vs = [], []
    for c in range(n_clusters):
        base = c * size
        for a_ in range(size):
            for b_ in range(a_ + 1, size):
                us.append(base + a_)
                vs.append(base + b_)
    for c in range(n_clusters):
        us.append(c * size)
        vs.append(((c + 1) % n_clusters) * size + 1)
    return from_edges(n_clusters * size, us, vs)


def random_weights(m: int, seed: int, kind: str = "lognormal") -> np.ndarray:
    rng = np.random.default_rng(seed)
    if kind == "lognormal":
        return rng.lognormal(0.0, 1.0, size=m).astype(np.float32)
    return rng.uniform(0.5, 2.0, size=m).astype(np.float32)


def with_weights(g: Graph, edge_w) -> Graph:
    """Same structure, new per-edge weights (one per undirected edge id)."""
    ew = None if edge_w is None else np.asarray(edge_w, dtype=np.float32)
    return Graph(n=g.n, row_ptr=g.row_ptr, col=g.col,
                 w=None if ew is None else ew[g.eid],
                 eid=g.eid, orig_id=g.orig_id, edge_u=g.edge_u,
                 edge_v=g.edge_v, edge_w=ew)


# ---------------------------------------------------------------------------
# Device-side generators for graphs too large to build quickly on the host.
# Same constructions as above, drawn with torch on a GPU (seeded torch
# generator, so a device and seed give the same graph); the result is a dict
# of device tensors in the CSR conventions of this module.
# ---------------------------------------------------------------------------

def _csr_from_keys_torch(n: int, keys, w, orig_id):
    """Symmetric CSR (dict of tensors) from sorted unique keys lo * n + hi."""
    import torch
    dev = keys.device
    m = keys.numel()
    lo = keys // n
    hi = keys % n
    rows = torch.cat([lo, hi])
    cols = torch.cat([hi, lo])
    ids = torch.cat([torch.arange(m, device=dev), torch.arange(m, device=dev)])
    order = torch.argsort(rows * n + cols)
    rows, cols, ids = rows[order], cols[order], ids[order]
    counts = torch.bincount(rows, minlength=n)
    row_ptr = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    row_ptr[1:] = torch.cumsum(counts, 0)
    out = {"n": n, "m": m, "row_ptr": row_ptr, "col": cols.to(torch.int32), "eid": ids.to(torch.int32),
           "w": None if w is None else w[ids].contiguous(), "edge_w": w,
           "orig_id": orig_id.to(torch.int32), "edge_u": lo, "edge_v": hi,
           "d_max": int(counts.max().item()) if n else 0}
    return out


def _dedup_draws_torch(draw, m: int, n: int, gen):
    """Draw endpoint pairs with draw(k) until m distinct non-loop pairs."""
    import torch
    keys = None
    while keys is None or keys.numel() < m:
        have = 0 if keys is None else keys.numel()
        need = m - have
        a, b = draw(int(need * 1.2) + 4096)
        ok = a != b
        lo = torch.minimum(a[ok], b[ok])
        hi = torch.maximum(a[ok], b[ok])
        new = torch.unique(lo * n + hi)
        if keys is not None:
            new = new[~torch.isin(new, keys)]
        if new.numel() > need:
            pick = torch.randperm(new.numel(), generator=gen, device=new.device)[:need]
            new = new[pick]
        keys = new if keys is None else torch.cat([keys, new])
        keys = torch.sort(keys).values
    return keys


def _relabel_torch(n: int, keys, gen, perm=None):
    import torch
    if perm is None:
        perm = torch.randperm(n, generator=gen, device=keys.device)
    lo = perm[keys // n]
    hi = perm[keys % n]
    a = torch.minimum(lo, hi)
    b = torch.maximum(lo, hi)
    k2 = a * n + b
    order = torch.argsort(k2)
    return k2[order], order, perm


def chung_lu_device(n: int, m: int, gamma: float = 2.1, seed: int = 0, weights: str = "lognormal",
                    device="cuda", degree_order: bool = True):
    """Chung-Lu graph (the construction of `chung_lu`) drawn on a GPU.  With
    degree_order the vertices are stored by decreasing degree afterwards
    (orig_id keeps the randomly permuted ids)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    i = torch.arange(n, dtype=torch.float64, device=device)
    theta = ((i + 0.5) / n) ** (-1.0 / (gamma - 1.0))
    theta = theta * ((2.0 * m / n) / theta.mean())
    theta = torch.minimum(theta, torch.sqrt(theta.sum()))
    cdf = torch.cumsum(theta, 0)
    cdf = cdf / cdf[-1]

    def draw(k):
        a = torch.searchsorted(cdf, torch.rand(k, generator=gen, device=device, dtype=torch.float64), right=True)
        b = torch.searchsorted(cdf, torch.rand(k, generator=gen, device=device, dtype=torch.float64), right=True)
        return torch.clamp(a, max=n - 1), torch.clamp(b, max=n - 1)

    keys = _dedup_draws_torch(draw, m, n, gen)
    keys, _, perm = _relabel_torch(n, keys, gen)          # random vertex permutation
    orig = torch.arange(n, device=device)
    w = None
    if weights == "lognormal":
        w = torch.exp(torch.randn(m, generator=gen, device=device)).float()
    elif weights == "uniform":
        w = (0.5 + 1.5 * torch.rand(m, generator=gen, device=device)).float()
    if degree_order:
        keys, w, orig = _degree_order_torch(n, keys, w, orig)
    return _csr_from_keys_torch(n, keys, w, orig)


def rmat_device(scale: int, m: int, a=0.57, b=0.19, c=0.19, seed: int = 0, weights: str = "uniform",
                device="cuda", degree_order: bool = True):
    """R-MAT graph (the construction of `rmat`) drawn on a GPU."""
    import torch
    n = 1 << scale
    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    ab, abc = a + b, a + b + c

    def draw(k):
        src = torch.zeros(k, dtype=torch.int64, device=device)
        dst = torch.zeros(k, dtype=torch.int64, device=device)
        for lvl in range(scale):
            r = torch.rand(k, generator=gen, device=device)
            bit = 1 << (scale - 1 - lvl)
            right = ((r >= a) & (r < ab)) | (r >= abc)
            down = r >= ab
            src += down.to(torch.int64) * bit
            dst += right.to(torch.int64) * bit
        return src, dst

    keys = _dedup_draws_torch(draw, m, n, gen)
    keys, _, perm = _relabel_torch(n, keys, gen)
    orig = torch.arange(n, device=device)
    w = None
    if weights == "uniform":
        w = (0.5 + 1.5 * torch.rand(m, generator=gen, device=device)).float()
    elif weights == "lognormal":
        w = torch.exp(torch.randn(m, generator=gen, device=device)).float()
    if degree_order:
        keys, w, orig = _degree_order_torch(n, keys, w, orig)
    return _csr_from_keys_torch(n, keys, w, orig)


def _degree_order_torch(n: int, keys, w, orig):
    """Relabel so that vertices are stored by decreasing degree (ties by id);
    edge weights and original ids travel with the edges and vertices."""
    import torch
    dev = keys.device
    lo = keys // n
    hi = keys % n
    deg = torch.bincount(torch.cat([lo, hi]), minlength=n)
    ids = torch.arange(n, device=dev)
    order = torch.argsort(-deg * n + ids)                  # decreasing degree, ties by id
    new_of_old = torch.empty(n, dtype=torch.int64, device=dev)
    new_of_old[order] = ids
    a = new_of_old[lo]
    b = new_of_old[hi]
    k2 = torch.minimum(a, b) * n + torch.maximum(a, b)
    o2 = torch.argsort(k2)
    new_orig = torch.empty_like(orig)
    new_orig[new_of_old] = orig
    return k2[o2], (None if w is None else w[o2]), new_orig


def device_to_host(d) -> Graph:
    """Copy a device graph dict back to a host Graph (for the oracle)."""
    def c(t, dt):
        return None if t is None else t.detach().cpu().numpy().astype(dt)
    return Graph(n=d["n"], row_ptr=c(d["row_ptr"], np.int64), col=c(d["col"], np.int32), w=c(d["w"], np.float32),
                 eid=c(d["eid"], np.int32), orig_id=c(d["orig_id"], np.int32), edge_u=c(d["edge_u"], np.int32),
                 edge_v=c(d["edge_v"], np.int32), edge_w=c(d["edge_w"], np.float32))
