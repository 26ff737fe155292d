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
    the reference distances.  Returns the list of unexplained edge ids."""
    import math
    bad = []
    diff = np.nonzero(keep_got != keep_ref)[0]
    for q in diff:
        explained = False
        for i in (int(g.edge_u[q]), int(g.edge_v[q])):
            ps = range(g.row_ptr[i], g.row_ptr[i + 1])
            vals = sorted(float(rho_ref[g.eid[p]]) for p in ps)
            if orient == 1:
                vals = vals[::-1]
            d = len(vals)
            c = min(d, max(1, int(math.floor(d ** e))))
            cut = [vals[c - 1]] + ([vals[c]] if c < d else [])
            r = float(rho_ref[q])
            if any(abs(r - kc) <= tol * max(abs(kc), 1e-30) for kc in cut):
                explained = True
                break
        if not explained:
            bad.append(int(q))
    return bad
