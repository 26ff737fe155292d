"""Run in a subprocess by test_sanitizers_cpu.py: drives every entry of the
oracle's C library on small graphs (including empty and edgeless ones) and
prints one JSON line of result digests.  The parent runs it once against
the ordinary oracle build and once against the AddressSanitizer +
UndefinedBehaviorSanitizer build (ORACLE_LIBRARY, with the sanitizer runtime
preloaded) and compares the two lines: a sanitizer report aborts the second
run, and the digests show that the -O1 sanitized build computes the same
values."""
import hashlib
import json
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
from paper_1601_05527_amd import graphs as G  # noqa: E402


def _h(*arrs) -> str:
    d = hashlib.sha256()
    for a in arrs:
        a = np.ascontiguousarray(a)
        d.update(str(a.dtype).encode())
        d.update(a.tobytes())
    return d.hexdigest()[:16]


def main():
    out = {}
    cases = {
        "gnm": G.gnm(300, 1500, 3),
        "cl": G.chung_lu(500, 3000, seed=4),
        "grid": G.grid_long_range(12, 6, seed=5),
        "edgeless": G.from_edges(7, np.zeros(0, int), np.zeros(0, int)),
        "pair": G.from_edges(4, np.array([0, 2]), np.array([1, 3])),
    }
    for name, g in cases.items():
        rho, xk, xh, mm = oracle.algebraic_distance(g, 4, 10, 0.5, seed=1, want_vectors=True)
        out[name + ".rho"] = _h(rho, xk, xh, mm)
        out[name + ".x0"] = _h(oracle.start_vectors(g.n, 3, 2))
        if g.n:
            x0 = oracle.start_vectors(g.n, 1, 2)[:, 0]
            tr = oracle.relax_vector(g, x0, 5, trace=True)
            out[name + ".trace"] = _h(tr, *oracle.rescale_vector(g, tr[-1])[:1])
        out[name + ".strength"] = _h(oracle.strength(rho), oracle.normalize_dist(g, rho),
                                     oracle.normalize_dist(g, rho, by_strength=False, eps=1e-9))
        for orient in (0, 1):
            out[f"{name}.keep{orient}"] = _h(*oracle.sparsify(g, rho, orient, 0.5)[:1])
            if g.m:
                e, keep, _ = oracle.fit_exponent(g, rho, orient, 0.3)
                out[f"{name}.fit{orient}"] = _h(np.float64(e), keep)
        out[name + ".bins"] = _h(*oracle.bin_layout(g, rho), oracle.binned_choices(g, rho, 0.5, 7),
                                 oracle.sparsify_binned(g, rho, 0.5, 7)[0])
        if g.m:
            e, keep, _ = oracle.fit_exponent_binned(g, rho, 0.3, 7)
            out[name + ".fitb"] = _h(np.float64(e), keep)
            c = np.random.default_rng(0).standard_normal(g.m)
            out[name + ".grad"] = _h(oracle.grad_weights(g, c, 3, 6, seed=1))
        keep, _ = oracle.sparsify(g, rho, 0, 0.5)
        sub = oracle.subgraph(g, keep)
        props = oracle.properties(g.n, g.row_ptr, g.col)
        out[name + ".props"] = _h(props["lambda"], props["c"], props["comp"], np.float64(props["C_G"]),
                                  *sub[:2], sub[3], sub[4])
        seeds = oracle.ml_seeds(g, rho)
        out[name + ".ml"] = _h(seeds, oracle.ml_aggregates(g, rho, seeds)[0])
        if g.m:
            keep, kept, depth = oracle.ml_sparsify(g, 4, 8, [0.5], seed=1, levels=4, n_min=20)
            out[name + ".mls"] = _h(keep, np.int64(kept), np.int64(depth))
    rng = np.random.default_rng(9)
    u = rng.integers(0, 40, 200)
    v = rng.integers(0, 40, 200)
    w = rng.uniform(0.5, 2.0, 200).astype(np.float32)
    for order in (0, 1):
        r = oracle.ingest(40, u, v, w, order=order)
        out[f"ingest{order}"] = _h(r[0], r[1], r[2], r[3], r[4], np.int64(r[5]), np.int64(r[6]))
    out["ingest_empty"] = _h(*[a for a in oracle.ingest(5, [], [])[:2]])
    out["sum_f32"] = _h(oracle.exact_sum_f32(w))
    out["spearman"] = _h(np.float64(oracle.spearman(rng.random(50), rng.random(50))))
    out["span"] = _h(oracle.ml_level_span(9, 3, 2, 0.3))
    out["philox"] = _h(oracle.philox4x64_10([1, 2, 3, 4], [5, 6]))
    out["budget"] = [oracle.budget(d, 0.5) for d in (0, 1, 2, 7, 100)]
    print(json.dumps({"library": oracle._load()._name, "digests": out}, sort_keys=True))


if __name__ == "__main__":
    main()
