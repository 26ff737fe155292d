"""Seeded synthetic workloads, shared by the benchmark and the parity tests
so that both run the same inputs in the same launch configuration.

Each workload is a dict of sizes and method parameters plus a builder.
None of the method's arithmetic lives here: these are input recipes only
(graph generators from ``graphs``, sizes drawn from numpy generators).

  Every workload relaxes with each connected component centred by its own
  weighted mean; FP32 storage keeps its last FP64_TAIL sweeps in FP64.

  CHUNG_LU   one power-law graph, n = 2^20, 16,000,000 edges, degree exponent
             2.1, lognormal(0, 1) weights; R = 16, k = 20, FP32; LOCAL and
             GLOBAL selection fitted to 30% retention; the selection with
             binning (Algorithm 4) fitted to the same retention; the
             multilevel cycle (Algorithm 6) with at most 9 levels, n_min
             1000, level-span 3 on the finest third, 30% per level.
  BATCH      512 Chung-Lu graphs, n log-uniform in [1e3, 2e5], average degree
             2m/n uniform in [8, 32], lognormal weights; R = 8, k = 20, FP32,
             LOCAL selection at e = 0.5, one captured launch sequence.
  RMAT       R-MAT (a, b, c, d) = (.57, .19, .19, .05), n = 2^24, 2^28
             edges, uniform(0.5, 2) weights; R = 16, k = 30; BF16 storage of
             the test vectors with FP32 arithmetic, the last 12 sweeps stored
             wider (11 in FP32, the last in FP64), beside the FP32 path.
  GRID       512 x 512 4-neighbour grid plus 0.5% extra random long-range
             edges, lognormal weights; R = 8, k = 20, FP32; gradient of
             sum_e c_e rho_e with c_e ~ N(0, 1), checkpoints every 5 sweeps.
  GNM        G(n, m) with n = 2,000, m = 10,000, unit weights, seed 0;
             R = 10, k = 20, FP64; LOCAL selection at e = 0.5.
"""
from __future__ import annotations

import numpy as np

from . import graphs

OMEGA = 0.5
FP64_TAIL = 3        # final sweeps of FP32 storage kept in FP64

CHUNG_LU = dict(n=1 << 20, m=16_000_000, gamma=2.1, seed=2024, R=16, k=20, seed_vec=1, target=0.3,
                bin_seed=17, ml_levels=9, ml_n_min=1000, ml_span=3)
BATCH = dict(G=512, n_lo=1e3, n_hi=2e5, deg_lo=8.0, deg_hi=32.0, seed=3, R=8, k=20, seed_vec=7,
             graph_id=0, e=0.5)
RMAT = dict(scale=24, m=1 << 28, seed=11, R=16, k=30, seed_vec=5, fp32_tail=12, fp64_tail=1, target=0.3)
GRID = dict(side=512, long_frac=0.005, seed=13, R=8, k=20, seed_vec=1, ckpt_every=5)
GNM = dict(n=2000, m=10_000, seed=0, R=10, k=20, seed_vec=0, e=0.5)


def chung_lu_graph(layout: str = "degree"):
    """(graph as drawn, graph as stored on the device).  The stored graph is
    the same graph with vertices relabelled by decreasing degree; results
    are keyed by original ids and do not depend on the relabelling."""
    c = CHUNG_LU
    g = graphs.chung_lu(c["n"], c["m"], gamma=c["gamma"], seed=c["seed"])
    if layout == "degree":
        return g, graphs.relabel(g, graphs.degree_descending_order(g))
    return g, g


def batch_sizes(G: int = BATCH["G"], seed: int = BATCH["seed"]):
    """Vertex and edge counts of the batch: n log-uniform in [n_lo, n_hi],
    average degree 2m/n uniform in [deg_lo, deg_hi]."""
    b = BATCH
    rng = np.random.default_rng(seed)
    ns = np.round(np.exp(rng.uniform(np.log(b["n_lo"]), np.log(b["n_hi"]), G))).astype(np.int64)
    deg = rng.uniform(b["deg_lo"], b["deg_hi"], G)
    ms = np.round(ns * deg / 2).astype(np.int64)
    return ns, ms


def batch_graphs(device="cuda", G: int = BATCH["G"], seed: int = BATCH["seed"]):
    """The batch's graphs as device dicts (graphs.chung_lu_device), each
    stored by decreasing degree."""
    ns, ms = batch_sizes(G, seed)
    return [graphs.chung_lu_device(int(n), int(m), seed=seed * 1_000_003 + q, device=device)
            for q, (n, m) in enumerate(zip(ns, ms))]


def rmat_graph(device="cuda", scale: int = RMAT["scale"], m: int = RMAT["m"]):
    """The R-MAT graph as a device dict, stored by decreasing degree."""
    return graphs.rmat_device(scale, m, seed=RMAT["seed"], weights="uniform", device=device)


def grid_graph(side: int = GRID["side"]):
    """The grid with long-range edges (host graph, natural row-major order)."""
    n_long = int(round(GRID["long_frac"] * 2 * side * (side - 1)))
    return graphs.grid_long_range(side, n_long, seed=GRID["seed"])


def gnm_graph():
    return graphs.gnm(GNM["n"], GNM["m"], GNM["seed"])
