"""Helpers shared by the GPU parity tests (comparison statistics and the
near-cut rule for sparsified edge sets)."""
import sys

import numpy as np


def announce(name: str) -> None:
    """Name the case before any GPU work, so a failure is attributable."""
    print(f"[case] {name}", flush=True)
    sys.stdout.flush()


def rel_stats(got, want, floor=0.0):
    got = np.asarray(got, dtype=np.float64)
    want = np.asarray(want, dtype=np.float64)
    den = np.maximum(np.abs(want), floor)
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.where(den > 0, np.abs(got - want) / den, np.abs(got - want))
    if rel.size == 0:
        return {"max": 0.0, "p999": 0.0}
    return {"max": float(rel.max()), "p999": float(np.quantile(rel, 0.999)), "rel": rel}


def near_cut_mismatches(g, rho_ref, keep_got, keep_ref, orient, e, tol):
    """Edges whose kept/dropped state differs, minus those explained by
    rounding: an edge within `tol` (relative) of a deciding endpoint's cut in
    the reference distances (the c_i-th key of row i in rank order, or the
    (c_i+1)-th).  Returns the list of unexplained edge ids."""
    import math
    bad = []
    diff = np.nonzero(np.asarray(keep_got) != np.asarray(keep_ref))[0]
    cuts = {}

    def row_cut(i):
        if i not in cuts:
            ps = slice(int(g.row_ptr[i]), int(g.row_ptr[i + 1]))
            vals = np.sort(np.asarray(rho_ref, dtype=np.float64)[g.eid[ps]])
            if orient == 1:
                vals = vals[::-1]
            d = len(vals)
            c = min(d, max(1, int(math.floor(d ** e))))
            cuts[i] = [float(vals[c - 1])] + ([float(vals[c])] if c < d else [])
        return cuts[i]

    for q in diff:
        r = float(rho_ref[q])
        explained = any(abs(r - kc) <= tol * max(abs(kc), 1e-30)
                        for i in (int(g.edge_u[q]), int(g.edge_v[q])) for kc in row_cut(i))
        if not explained:
            bad.append(int(q))
    return bad


def fp32_tolerance(g, x0, xk, minmax, rho_ref, k, tol=1e-5):
    """Per-edge absolute bound on |rho_got - rho_ref| for distances
    computed from vectors stored in FP32: max(tol * rho_e, 2 k eps M_e),
    eps = 2^-24, where M_e = || max(|x_u - mu|, |x_v - mu|) / (hi - lo) ||
    over the R vectors (x = x^(k) in FP64, mu = the s-weighted mean of
    x^(0) per vector, which the relaxation conserves and which the library
    subtracts before its sweeps; hi - lo the rescale span).  Each sweep
    rounds the stored values to eps relative to |x - mu| and the sweep is
    non-expansive, so after k sweeps x_u - x_v carries an absolute error of
    order k eps |x - mu|.  Returns (bound, M_e / rho_e)."""
    deg = np.diff(g.row_ptr)
    rows = np.repeat(np.arange(g.n), deg)
    w = np.ones(len(g.col)) if g.w is None else g.w.astype(np.float64)
    s = np.bincount(rows, weights=w, minlength=g.n)
    mu = (s[:, None] * x0).sum(axis=0) / s.sum()
    R = xk.shape[1]
    span = np.asarray(minmax[R:]) - np.asarray(minmax[:R])
    span = np.where(span > 0, span, np.inf)
    a = np.abs(xk[g.edge_u] - mu) / span
    b = np.abs(xk[g.edge_v] - mu) / span
    M = np.linalg.norm(np.maximum(a, b), axis=1)
    bound = np.maximum(tol * rho_ref, 2.0 * k * 2.0 ** -24 * M)
    with np.errstate(divide="ignore", invalid="ignore"):
        kappa = np.where(rho_ref > 0, M / rho_ref, np.inf)
    return bound, kappa


def check_fp32(g, x0, xk, minmax, rho_got, rho_ref, k, tol=1e-5):
    """(worst ratio of the error to the per-edge bound, stats); passes when
    the ratio is <= 1."""
    bound, kappa = fp32_tolerance(g, x0, xk, minmax, rho_ref, k, tol)
    err = np.abs(np.asarray(rho_got, dtype=np.float64) - rho_ref)
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(bound > 0, err / bound, np.where(err > 0, np.inf, 0.0))
        rel = np.where(rho_ref > 0, err / rho_ref, 0.0)
    if ratio.size == 0:
        return 0.0, {}
    worst = int(np.argmax(ratio))
    return float(ratio.max()), {"max_rel": float(rel.max()), "n_over_tol": int((err > tol * rho_ref).sum()),
                                "kappa_at_worst": float(kappa[worst])}
