"""Python access to the plain FP64 CPU oracle (``oracle.c``).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg import this package; the library never does, and this
package imports nothing from the library.  Every function here is a thin
ctypes wrapper around the C oracle, which follows the paper's Algorithm 1
(ComputeAlgDist), Algorithm 3 (Sparsify), Algorithm 4 (SparsifyB), the binary-search
fitting of Section 6.2, Algorithm 6 (MLSparsify) and the graph properties of the
Preliminaries in double precision.

Parity status: every function is pinned by tests that do not reuse its own
formulas (closed forms, library routines, brute force); the one reading
that no test can pin is recorded in ``PINS`` below.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# Readings that only this spec fixes (the paper does not): the value of eps,
# min-max (rather than max-abs) rescaling, floor (rather than ceil/round)
# in the per-vertex budget, the Philox stream layout, and for SparsifyB the
# random neighbour order, the round-robin reading of its selection step and
# the single-precision sigma.  Tests pin what follows from these readings
# (closed forms, invariants, special cases), not the readings themselves.
PINS = {"parity_unpinned": ["eps value", "min-max rescale", "floor in d^e", "start-vector stream layout",
                            "SparsifyB random order (vertex key stream, priority hash)",
                            "SparsifyB round-robin reading of 'randomly select bins and edges'",
                            "SparsifyB single-precision sigma",
                            "multilevel strength threshold theta, eps and the seed traversal's tie order",
                            "multilevel ratio-vector alignment when fewer levels are reached than entries",
                            "level-span segment bounds when the level count is not a multiple of 3"]}

LOCAL = 0
GLOBAL = 1


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (-O2, OpenMP).  With ``sanitize``
    compile ``liboracle_san.so`` instead: -O1 with AddressSanitizer and
    UndefinedBehaviorSanitizer (gcc's runtimes, to be preloaded into the
    process), no OpenMP, so that the checks see one thread's accesses."""
    out = os.path.join(_HERE, "liboracle_san.so") if sanitize else _LIB
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        flags = (["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                  "-fno-sanitize-recover=undefined", "-Wno-unknown-pragmas"]
                 if sanitize else ["-O2", "-fopenmp"])
        subprocess.check_call(["gcc"] + flags + [
            "-fPIC", "-shared", "-std=c11", "-Wall", "-Wextra", "-Wno-unused-parameter",
            _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, out)
    return out


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    path = os.environ.get("ORACLE_LIBRARY")      # another build, e.g. the sanitized one
    if not path:
        path = _LIB
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i64, i32, u64, f64 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint64, ctypes.c_double
    lib.orc_philox4x64_10.argtypes = [P, P, P]
    lib.orc_set_threads.argtypes = [i32]
    lib.orc_max_threads.restype = i32
    lib.orc_start_value.argtypes = [u64, u64, i32, i32]
    lib.orc_start_value.restype = f64
    lib.orc_start_vectors.argtypes = [i64, i32, u64, u64, P, P]
    lib.orc_relax_vector.argtypes = [i64, P, P, P, i32, f64, P, P]
    lib.orc_rescale_vector.argtypes = [i64, P, P, P, P, P]
    lib.orc_algebraic_distance.argtypes = [i64, P, P, P, P, P, i64, i32, i32, f64, u64, u64, P, P, P, P, P]
    lib.orc_strength.argtypes = [i64, P, f64, P]
    lib.orc_normalize_dist.argtypes = [i64, P, P, P, P, P, i32, f64, P]
    lib.orc_budget.argtypes = [i64, f64]
    lib.orc_budget.restype = i64
    lib.orc_sparsify.argtypes = [i64, P, P, P, P, i64, P, i32, f64, P]
    lib.orc_sparsify.restype = i64
    lib.orc_fit_exponent.argtypes = [i64, P, P, P, P, i64, P, i32, f64, P, P]
    lib.orc_fit_exponent.restype = f64
    lib.orc_grad_weights.argtypes = [i64, P, P, P, P, P, i64, i32, i32, f64, u64, u64, P, P, P]
    lib.orc_bin_vertex_key.argtypes = [u64, u64, i32]
    lib.orc_bin_vertex_key.restype = ctypes.c_uint32
    lib.orc_bin_priority.argtypes = [ctypes.c_uint32, i32]
    lib.orc_bin_priority.restype = ctypes.c_uint32
    lib.orc_bin_layout.argtypes = [i64, P, P, P, P, P]
    lib.orc_binned_choices.argtypes = [i64, P, P, P, P, P, u64, u64, f64, P]
    lib.orc_ingest.argtypes = [i64, i64, P, P, P, P, i32, P, P, P, P, P, P]
    lib.orc_subgraph.argtypes = [i64, P, P, P, P, i64, P, P, P, P, P, P]
    lib.orc_ml_seeds.argtypes = [i64, P, P, P, P, P, f64, f64, P]
    lib.orc_ml_aggregates.argtypes = [i64, P, P, P, P, P, f64, P, P]
    lib.orc_ml_aggregates.restype = i64
    lib.orc_ml_sparsify.argtypes = [i64, P, P, P, P, P, i64, i32, i32, f64, u64, u64, i32, i64, P, i32, i32, i32,
                                    f64, f64, f64, u64, P, P]
    lib.orc_ml_level_span.argtypes = [i32, i32, i32, f64, P]
    lib.orc_ml_sparsify.restype = i64
    lib.orc_subgraph.restype = i64
    lib.orc_triangles.argtypes = [i64, P, P, P]
    lib.orc_clustering.argtypes = [i64, P, P, P]
    lib.orc_clustering.restype = f64
    lib.orc_components.argtypes = [i64, P, P, P]
    lib.orc_components.restype = i64
    lib.orc_spearman.argtypes = [i64, P, P]
    lib.orc_spearman.restype = f64
    lib.orc_ingest.restype = i64
    lib.orc_exact_sum_f32.argtypes = [P, i64]
    lib.orc_exact_sum_f32.restype = ctypes.c_float
    lib.orc_sparsify_binned.argtypes = [i64, P, P, P, P, i64, P, u64, u64, f64, P]
    lib.orc_sparsify_binned.restype = i64
    lib.orc_fit_exponent_binned.argtypes = [i64, P, P, P, P, i64, P, u64, u64, f64, P, P]
    lib.orc_fit_exponent_binned.restype = f64
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on (timing only: the
    results do not depend on the count)."""
    os.environ["OMP_NUM_THREADS"] = str(n)
    _load().orc_set_threads(int(n))


def max_threads() -> int:
    """Threads the oracle's next OpenMP loop will use."""
    return int(_load().orc_max_threads())


def philox4x64_10(counter, key) -> np.ndarray:
    lib = _load()
    ctr = np.asarray(counter, dtype=np.uint64).reshape(4).copy()
    k = np.asarray(key, dtype=np.uint64).reshape(2).copy()
    out = np.zeros(4, dtype=np.uint64)
    lib.orc_philox4x64_10(_p(ctr), _p(k), _p(out))
    return out


def start_vectors(n: int, R: int, seed: int, graph_id: int = 0, orig_id=None) -> np.ndarray:
    lib = _load()
    oid = _c(orig_id, np.int32)
    x0 = np.zeros((n, R), dtype=np.float64)
    lib.orc_start_vectors(n, R, seed, graph_id, _p(oid), _p(x0))
    return x0


def relax_vector(g, x0: np.ndarray, k: int, omega: float = 0.5, trace: bool = False):
    """k JOR sweeps of one vector; returns x^(k) (or x^(0..k) if trace)."""
    lib = _load()
    x = np.array(x0, dtype=np.float64, copy=True)
    tr = np.zeros((k + 1, g.n), dtype=np.float64) if trace else None
    lib.orc_relax_vector(g.n, _p(g.row_ptr), _p(g.col), _p(_c(g.w, np.float32)), k, omega,
                         _p(x), _p(tr))
    return tr if trace else x


def rescale_vector(g, x: np.ndarray):
    lib = _load()
    x = np.ascontiguousarray(x, dtype=np.float64)
    xh = np.zeros(g.n, dtype=np.float64)
    lo = ctypes.c_double()
    hi = ctypes.c_double()
    lib.orc_rescale_vector(g.n, _p(g.row_ptr), _p(x), _p(xh), ctypes.byref(lo), ctypes.byref(hi))
    return xh, lo.value, hi.value


def algebraic_distance(g, R: int, k: int, omega: float = 0.5, seed: int = 0,
                       graph_id: int = 0, x0: Optional[np.ndarray] = None,
                       want_vectors: bool = False):
    """Algorithm 1.  Returns rho[m] (and x^(k), xhat, minmax[2R] if asked)."""
    lib = _load()
    rho = np.zeros(g.m, dtype=np.float64)
    xk = np.zeros((g.n, R), dtype=np.float64) if want_vectors else None
    xh = np.zeros((g.n, R), dtype=np.float64) if want_vectors else None
    mm = np.zeros(2 * R, dtype=np.float64) if want_vectors else None
    x0c = _c(x0, np.float64)
    lib.orc_algebraic_distance(g.n, _p(g.row_ptr), _p(g.col), _p(_c(g.w, np.float32)),
                               _p(g.eid), _p(g.orig_id), g.m, R, k, omega, seed, graph_id,
                               _p(x0c), _p(rho), _p(xk), _p(xh), _p(mm))
    if want_vectors:
        return rho, xk, xh, mm
    return rho


def strength(rho: np.ndarray, eps: float = 1e-12) -> np.ndarray:
    lib = _load()
    r = np.ascontiguousarray(rho, dtype=np.float64)
    out = np.zeros_like(r)
    lib.orc_strength(r.size, _p(r), eps, _p(out))
    return out


def normalize_dist(g, rho: np.ndarray, by_strength: bool = True, eps: float = 0.0) -> np.ndarray:
    """Algorithm 1's optional normalization, as a distance: out_e =
    sqrt(rho_e^2 + eps) * sqrt(f_i f_j) with f the weighted degree (or the
    degree), so that the normalized delta is 1 / out_e."""
    lib = _load()
    r = np.ascontiguousarray(rho, dtype=np.float64)
    out = np.zeros(g.m, dtype=np.float64)
    lib.orc_normalize_dist(g.n, _p(g.row_ptr), _p(g.col), _p(_c(g.w, np.float32)), _p(g.eid), _p(r),
                           1 if by_strength else 0, float(eps), _p(out))
    return out


def budget(d: int, e: float) -> int:
    return int(_load().orc_budget(int(d), float(e)))


def sparsify(g, rho: np.ndarray, orient: int, e: float):
    """Algorithm 3.  Returns (keep[m] uint8, n_kept)."""
    lib = _load()
    r = np.ascontiguousarray(rho, dtype=np.float64)
    keep = np.zeros(g.m, dtype=np.uint8)
    kept = lib.orc_sparsify(g.n, _p(g.row_ptr), _p(g.col), _p(g.eid), _p(g.orig_id), g.m,
                            _p(r), orient, e, _p(keep))
    return keep, int(kept)


def fit_exponent(g, rho: np.ndarray, orient: int, target: float):
    """Binary-search fitting of e.  Returns (e, keep[m], n_kept)."""
    lib = _load()
    r = np.ascontiguousarray(rho, dtype=np.float64)
    keep = np.zeros(g.m, dtype=np.uint8)
    kept = ctypes.c_int64()
    e = lib.orc_fit_exponent(g.n, _p(g.row_ptr), _p(g.col), _p(g.eid), _p(g.orig_id), g.m,
                             _p(r), orient, target, _p(keep), ctypes.byref(kept))
    return float(e), keep, int(kept.value)


def grad_weights(g, c: np.ndarray, R: int, k: int, omega: float = 0.5, seed: int = 0,
                 graph_id: int = 0, x0: Optional[np.ndarray] = None) -> np.ndarray:
    """d/dw_e of L = sum_e c_e rho_e (reverse mode, FP64)."""
    lib = _load()
    cc = np.ascontiguousarray(c, dtype=np.float64)
    out = np.zeros(g.m, dtype=np.float64)
    lib.orc_grad_weights(g.n, _p(g.row_ptr), _p(g.col), _p(_c(g.w, np.float32)), _p(g.eid),
                         _p(g.orig_id), g.m, R, k, omega, seed, graph_id, _p(_c(x0, np.float64)),
                         _p(cc), _p(out))
    return out


def bin_vertex_key(seed: int, vertex_key: int, graph_id: int = 0) -> int:
    """Vertex i's 32-bit key for its random neighbour order (SparsifyB)."""
    return int(_load().orc_bin_vertex_key(seed, graph_id, int(vertex_key)))


def bin_priority(vertex_key_bits: int, neighbour_key: int) -> int:
    """Priority of a neighbour in a vertex's random order (SparsifyB)."""
    return int(_load().orc_bin_priority(int(vertex_key_bits) & 0xffffffff, int(neighbour_key)))


def bin_layout(g, rho: np.ndarray):
    """Algorithm 4's binning step: (bin[2m] per CSR entry, nbins[n])."""
    lib = _load()
    r = np.ascontiguousarray(rho, dtype=np.float64)
    b = np.zeros(len(g.col), dtype=np.int32)
    nb = np.zeros(g.n, dtype=np.int64)
    lib.orc_bin_layout(g.n, _p(g.row_ptr), _p(g.eid), _p(r), _p(b), _p(nb))
    return b, nb


def binned_choices(g, rho: np.ndarray, e: float, seed: int, graph_id: int = 0) -> np.ndarray:
    """Algorithm 4's per-vertex choices: chosen[2m] per CSR entry (1 when the
    entry's row vertex selects that edge)."""
    lib = _load()
    r = np.ascontiguousarray(rho, dtype=np.float64)
    ch = np.zeros(len(g.col), dtype=np.uint8)
    lib.orc_binned_choices(g.n, _p(g.row_ptr), _p(g.col), _p(g.eid), _p(g.orig_id), _p(r), seed, graph_id,
                           e, _p(ch))
    return ch


def sparsify_binned(g, rho: np.ndarray, e: float, seed: int, graph_id: int = 0):
    """Algorithm 4 (SparsifyB) at exponent e.  Returns (keep[m] uint8, n_kept)."""
    lib = _load()
    r = np.ascontiguousarray(rho, dtype=np.float64)
    keep = np.zeros(g.m, dtype=np.uint8)
    kept = lib.orc_sparsify_binned(g.n, _p(g.row_ptr), _p(g.col), _p(g.eid), _p(g.orig_id), g.m,
                                   _p(r), seed, graph_id, e, _p(keep))
    return keep, int(kept)


def fit_exponent_binned(g, rho: np.ndarray, target: float, seed: int, graph_id: int = 0):
    """Binary-search fitting of e for SparsifyB.  Returns (e, keep[m], n_kept)."""
    lib = _load()
    r = np.ascontiguousarray(rho, dtype=np.float64)
    keep = np.zeros(g.m, dtype=np.uint8)
    kept = ctypes.c_int64()
    e = lib.orc_fit_exponent_binned(g.n, _p(g.row_ptr), _p(g.col), _p(g.eid), _p(g.orig_id), g.m,
                                    _p(r), seed, graph_id, target, _p(keep), ctypes.byref(kept))
    return float(e), keep, int(kept.value)


def ingest(n: int, u, v, w=None, orig_id=None, order: int = 0):
    """An edge list into the symmetric CSR of the graph model (self-loops
    dropped, repeated pairs merged with summed weights; order 1 stores the
    vertices by decreasing degree, order 2 in reverse Cuthill-McKee order).  Returns (row_ptr, col, w_entries or
    None, eid, orig_id, m, n_dropped); raises ValueError for an endpoint out
    of range."""
    lib = _load()
    uu = np.ascontiguousarray(u, dtype=np.int32)
    vv = np.ascontiguousarray(v, dtype=np.int32)
    ww = None if w is None else np.ascontiguousarray(w, dtype=np.float32)
    oi = _c(orig_id, np.int32)
    m_in = uu.size
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    col = np.zeros(max(1, 2 * m_in), dtype=np.int32)
    eid = np.zeros(max(1, 2 * m_in), dtype=np.int32)
    w_out = np.zeros(max(1, 2 * m_in), dtype=np.float32) if ww is not None else None
    orig = np.zeros(max(1, n), dtype=np.int32)
    dropped = ctypes.c_int64()
    m = lib.orc_ingest(n, m_in, _p(uu), _p(vv), _p(ww), _p(oi), order, _p(row_ptr), _p(col), _p(w_out),
                       _p(eid), _p(orig), ctypes.byref(dropped))
    if m == -1:
        raise ValueError("vertex id out of range")
    if m < 0:
        raise ValueError("a weight is not finite and positive")
    nnz = 2 * m
    return (row_ptr, col[:nnz].copy(), None if w_out is None else w_out[:nnz].copy(), eid[:nnz].copy(),
            orig[:n].copy(), int(m), int(dropped.value))


def exact_sum_f32(x) -> np.float32:
    """The exact sum of positive finite float32 values, rounded once to
    float32 (the merged weight of repeated pairs)."""
    lib = _load()
    xx = np.ascontiguousarray(x, dtype=np.float32)
    return np.float32(lib.orc_exact_sum_f32(_p(xx), xx.size))


def subgraph(g, keep):
    """G_s = (V, {e : keep[e]}) as CSR arrays: (row_ptr, col, w or None,
    eid renumbered over the kept edges, original edge id per entry, m_s)."""
    lib = _load()
    k = np.ascontiguousarray(keep, dtype=np.uint8)
    nnz = len(g.col)
    rp = np.zeros(g.n + 1, dtype=np.int64)
    col = np.zeros(max(1, nnz), dtype=np.int32)
    w = np.zeros(max(1, nnz), dtype=np.float32) if g.w is not None else None
    eid = np.zeros(max(1, nnz), dtype=np.int32)
    oe = np.zeros(max(1, nnz), dtype=np.int32)
    ms = lib.orc_subgraph(g.n, _p(g.row_ptr), _p(g.col), _p(_c(g.w, np.float32)), _p(g.eid), g.m, _p(k), _p(rp),
                          _p(col), _p(w), _p(eid), _p(oe))
    q = int(rp[-1])
    return rp, col[:q].copy(), None if w is None else w[:q].copy(), eid[:q].copy(), oe[:q].copy(), int(ms)


def properties(n: int, row_ptr, col):
    """Triangles lambda_i, clustering c_i and C_G (Eq. cc), component
    labels (smallest id of each component) and their number."""
    lib = _load()
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cl = np.ascontiguousarray(col, dtype=np.int32)
    lam = np.zeros(max(1, n), dtype=np.int64)
    c = np.zeros(max(1, n), dtype=np.float64)
    comp = np.zeros(max(1, n), dtype=np.int32)
    lib.orc_triangles(n, _p(rp), _p(cl), _p(lam))
    cg = lib.orc_clustering(n, _p(rp), _p(lam), _p(c))
    nc = lib.orc_components(n, _p(rp), _p(cl), _p(comp))
    return {"lambda": lam[:n], "c": c[:n], "C_G": float(cg), "comp": comp[:n], "n_components": int(nc)}


def spearman(x, y) -> float:
    """Spearman rank correlation by the Preliminaries' formula (ties share
    the mean of their ranks)."""
    lib = _load()
    xx = np.ascontiguousarray(x, dtype=np.float64)
    yy = np.ascontiguousarray(y, dtype=np.float64)
    return float(lib.orc_spearman(xx.size, _p(xx), _p(yy)))


def ml_seeds(g, rho, eps: float = 1e-12, theta: float = 0.5) -> np.ndarray:
    """Coarsening seeds of Algorithm 6 (uint8 [n])."""
    lib = _load()
    r = np.ascontiguousarray(rho, dtype=np.float64)
    out = np.zeros(max(1, g.n), dtype=np.uint8)
    lib.orc_ml_seeds(g.n, _p(g.row_ptr), _p(g.col), _p(g.eid), _p(g.orig_id), _p(r), eps, theta, _p(out))
    return out[:g.n]


def ml_aggregates(g, rho, is_seed, eps: float = 1e-12):
    """Aggregate of every vertex under the restriction P (Eq. P), and their number."""
    lib = _load()
    r = np.ascontiguousarray(rho, dtype=np.float64)
    s = np.ascontiguousarray(is_seed, dtype=np.uint8)
    agg = np.zeros(max(1, g.n), dtype=np.int32)
    nc = lib.orc_ml_aggregates(g.n, _p(g.row_ptr), _p(g.col), _p(g.eid), _p(g.orig_id), _p(r), eps, _p(s), _p(agg))
    return agg[:g.n], int(nc)


def ml_level_span(n_levels: int, span: int, segment: int, value: float) -> np.ndarray:
    """The per-level ratio vector of the level-span rule (Section 6,
    implementation paragraph), coarsest level first: segment 0, 1, 2 =
    coarsest, middle, finest third of the levels; -1 = no sparsification."""
    lib = _load()
    out = np.zeros(max(1, n_levels), dtype=np.float64)
    lib.orc_ml_level_span(n_levels, span, segment, value, _p(out))
    return out[:n_levels]


def ml_sparsify(g, R: int, k: int, e_levels=None, omega: float = 0.5, seed: int = 0, graph_id: int = 0,
                levels: int = 8, n_min: int = 1000, eps: float = 1e-12, theta: float = 0.5, bin_seed: int = 0,
                fit: bool = False, span: int = 0, segment: int = 0, span_value: float = 0.3):
    """Algorithm 6 (MLSparsify).  e_levels: per-level ratios, coarsest level
    first (a shorter list repeats its last value; negative = no
    sparsification at that level); entries are exponents, or retention
    targets with `fit`.  span > 0 replaces e_levels by the level-span vector
    of the levels reached.  Returns (keep[m], n_kept, depth)."""
    if e_levels is None and span <= 0:
        raise ValueError("ml_sparsify needs e_levels, or span > 0 for the level-span rule")
    lib = _load()
    ev = np.atleast_1d(np.ascontiguousarray(e_levels if e_levels is not None else [0.0], dtype=np.float64))
    if ev.size < levels:
        ev = np.concatenate([ev, np.full(levels - ev.size, ev[-1])])
    keep = np.zeros(max(1, g.m), dtype=np.uint8)
    depth = ctypes.c_int32(0)
    kept = lib.orc_ml_sparsify(g.n, _p(g.row_ptr), _p(g.col), _p(_c(g.w, np.float32)), _p(g.eid), _p(g.orig_id),
                               g.m, R, k, omega, seed, graph_id, levels, n_min, _p(ev), int(fit), span, segment,
                               span_value, eps, theta, bin_seed, _p(keep), ctypes.byref(depth))
    return keep[:g.m], int(kept), int(depth.value)
