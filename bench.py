#!/usr/bin/env python
"""Benchmark of the algebraic-distance sparsification hot path on one MI355X.

Default workload (one step): a Chung-Lu power-law graph, n = 2^20 vertices,
exactly 16,000,000 undirected edges, degree exponent 2.1, lognormal(0, 1)
weights (seeded, synthetic; it stands in for the paper's real networks), with
  start vectors (Philox, each connected component centred by its own
  weighted mean) -> 20 JOR sweeps of R = 16 vectors (omega = 1/2, FP32
  storage and arithmetic, the last 2 sweeps stored and computed in FP64) ->
  rescale -> per-edge L2 algebraic distance (FP32) ->
  LOCAL and GLOBAL selection, each with e fitted to 30% retention.
The graph is resident in HBM before timing starts.  Vertices are stored in
decreasing-degree order and the graph's connected components are grouped
once (set-up work of the graph, timed apart; results are keyed by the
original ids and do not depend on either).

Prints one JSON line.  `value` is JOR edge-vector updates per second over
the whole step, nnz * R * k / t_step.  The line also carries compact
records of the other workloads (`workloads`: the 512-graph batch, R-MAT in
BF16 and FP32 storage with their accuracy, the adjoint on the grid), unless
--no-extras is given.

Other forms, one JSON line each (--workload): `batch` (512 Chung-Lu graphs
in one captured launch sequence), `bf16` (R-MAT n = 2^24, 2^28 edges, BF16
storage, against the FP32 path and the FP64 path), `adjoint` (512 x 512
grid with long-range edges, forward and weight gradient), `fp64` (G(n, m)
with n = 2,000, m = 10,000 in FP64), `multilevel` (the multilevel cycle of
Algorithm 6 on the default graph; value in input edges per second).  The
inputs are those of paper_1601_05527_amd.workloads.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "JOR edge-vector updates/s (nnz*R*k/s) + % HBM roofline; end-to-end sparsify ms"


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def sweep_bytes(n: int, nnz: int, r: int, bx_in: int, weighted: bool, bx_out: "int | None" = None) -> int:
    """Algorithmic bytes of one JOR sweep: the CSR structure once (int32
    column + FP32 weight per stored entry, int64 row pointer and FP32 1/s
    per row) plus one read of the n x R block in and one write out."""
    bx_out = bx_in if bx_out is None else bx_out
    return nnz * (4 + (4 if weighted else 0)) + (n + 1) * 8 + 4 * n + n * r * (bx_in + bx_out)


def dist_bytes(n: int, nnz: int, m: int, r: int, bx: int) -> int:
    """Algorithmic bytes of the distance pass: row pointers and columns
    once, the edge ids of the upper entries (one per edge), the vector
    block once, one FP32 distance per edge."""
    return (n + 1) * 8 + nnz * 4 + m * 4 + n * r * bx + 4 * m


def relax_sweep_bytes(n: int, nnz: int, r: int, k: int, weighted: bool, store_bytes: int, tail32: int,
                      tail64: int) -> list:
    """Algorithmic bytes of each of the k sweeps: x^(0) in FP32 (FP64 for
    FP64 storage), sweeps 1..k-tail32 stored in `store_bytes` (BF16 2, FP32
    4), then FP32 up to k-tail64, then FP64."""
    def b(t):            # bytes per element of x^(t)
        if t == 0:
            return 8 if store_bytes == 8 else 4
        if t > k - tail64:
            return 8
        if t > k - tail32:
            return 4
        return store_bytes
    return [sweep_bytes(n, nnz, r, b(t - 1), weighted, b(t)) for t in range(1, k + 1)]


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def sweep_traffic() -> "float | None":
    """Memory-side traffic per k_sweep launch from the committed counter
    summary (profiles/k_sweep_traffic.json: the step's sweeps' read requests
    by size, TCC_EA0_RDREQ_128B and _64B, plus WRITE_SIZE, checked on a copy
    of known size), or None when the sweep kernel's source has changed since
    those counters were taken."""
    import hashlib
    try:
        info = json.load(open(os.path.join(ROOT, "profiles", "k_sweep_traffic.json")))
        src = open(os.path.join(ROOT, "paper_1601_05527_amd", "csrc", "ad_relax.hip")).read()
        i = src.index("template <int U, int VEC, typename Tin, typename A>\n__device__ __forceinline__ void gather_rows")
        j = src.index("// Launch plan of the sweep")
    except (OSError, ValueError):
        return None
    if hashlib.sha256(src[i:j].encode()).hexdigest()[:16] != info.get("kernel_source_sha256_16"):
        return None
    return float(info["traffic_bytes_per_launch"])


def oracle_threads() -> int:
    """Threads the oracle's OpenMP loops use (OpenMP's own count once the
    oracle is loaded; before that the environment's or the affinity mask's)."""
    if "oracle" in sys.modules:
        return sys.modules["oracle"].max_threads()
    threads = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS")
    return int(omp) if omp and omp.isdigit() else threads


class Timer:
    """HIP events on the current stream (the stream every library call is
    given) around a region, averaged over `reps` repetitions."""

    def __init__(self, torch):
        self.torch = torch
        self.ev0 = torch.cuda.Event(enable_timing=True)
        self.ev1 = torch.cuda.Event(enable_timing=True)

    def run(self, fn, reps: int) -> float:
        self.torch.cuda.synchronize()
        self.ev0.record()
        for _ in range(reps):
            fn()
        self.ev1.record()
        self.torch.cuda.synchronize()
        return self.ev0.elapsed_time(self.ev1) / reps


def gather_probe_ms(torch, timer, x, col, row_bytes, reps=10):
    """ms of one launch of the pure row-gather probe (libad_probe.so) over
    `col`, rows of `row_bytes` bytes of `x`; None if the probe is not built."""
    import ctypes
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_1601_05527_amd", "libad_probe.so")
    if not os.path.exists(path):
        log("gather probe not built; no gather ceiling reported")
        return None
    lib = ctypes.CDLL(path)
    i64 = ctypes.c_int64
    lib.ad_probe_threads.restype = i64
    lib.ad_probe_threads.argtypes = [ctypes.c_int]
    lib.ad_probe_gather.restype = ctypes.c_int
    lib.ad_probe_gather.argtypes = [ctypes.c_void_p, i64, ctypes.c_int, ctypes.c_void_p, i64, ctypes.c_void_p,
                                    ctypes.c_int, ctypes.c_void_p]
    assert x.is_contiguous() and x.shape[1] * x.element_size() == row_bytes
    blocks = 2048
    sums = torch.empty((lib.ad_probe_threads(blocks), 4), dtype=torch.float32, device=x.device)

    def run():
        rc = lib.ad_probe_gather(x.data_ptr(), x.shape[0], row_bytes, col.data_ptr(), col.numel(),
                                 sums.data_ptr(), blocks, torch.cuda.current_stream().cuda_stream)
        if rc != 0:
            raise RuntimeError(f"ad_probe_gather returned {rc}")

    run()
    return timer.run(run, reps)


def vendor_spmm_ms(torch, timer, dg, x, reps=5):
    """{ms, what} of y = W x with torch's sparse CSR product (the vendor
    sparse library on this device) over the same CSR and vector block, or
    {error} when that path is unavailable."""
    try:
        w = dg.w if dg.w is not None else torch.ones(dg.col.numel(), dtype=torch.float32, device=x.device)
        a = torch.sparse_csr_tensor(dg.row_ptr, dg.col.to(torch.int64), w, size=(dg.n, dg.n))
        y = a @ x
        torch.cuda.synchronize()
        ms = timer.run(lambda: a @ x, reps)
        del a, y
        return {"ms": ms, "what": "torch sparse CSR x dense (W x only, no JOR blend), same CSR and FP32 block"}
    except Exception as ex:   # reported, not fatal: the comparison is context
        return {"error": f"{type(ex).__name__}: {ex}"[:200]}


def traced(api, timer, fn, reps):
    """(ms per call, per-kernel {name: (launches, total ms)}) with the
    library's own per-launch event tracing switched on.  One untimed traced
    call first fills the library's event pool, so the timed calls create no
    events."""
    api.lib.ad_trace_reset()
    api.lib.ad_trace_enable(1)
    fn()
    api.lib.ad_trace_reset()
    ms = timer.run(fn, reps)
    api.lib.ad_trace_enable(0)
    kern = api.trace_summary()
    api.lib.ad_trace_reset()
    return ms, kern


LIMITER = ("memory-side line-request rate: random 64-128 B row gathers, each a 128 B line request "
           "when it misses the XCD's 4 MB L2; random line requests are served at about 55 G/s whether "
           "the lines sit in the Infinity Cache or in HBM, and the FP32 sweep issues about 20.7M per launch "
           "(about 56 G/s) -- see profiles/k_sweep_chung_lu_n2e20_memory_counters.md")


def roofline(kern: dict, bytes_per_launch: float, traffic=None) -> dict:
    launches, total = kern.get("k_sweep", (0, 0.0))
    avg = total / max(1, launches)
    achieved = bytes_per_launch / (avg * 1e-3) / 1e9 if avg > 0 else 0.0
    return {"kernel": "k_sweep", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "bytes_per_launch": bytes_per_launch,
            "avg_launch_ms": avg, "limiter": LIMITER,
            "traffic_source": ("profiles/k_sweep_traffic.json (rocprofv3: read requests x their size from "
                               "TCC_EA0_RDREQ_128B/_64B, plus WRITE_SIZE, per launch, averaged over a step's "
                               "sweeps; a 1 GiB copy checks both; null when the kernel changed since)")}


def base_result(args, value, step_ms, dtype, data, config, roof, cpu, **extra) -> dict:
    out = {
        "metric": METRIC, "value": value, "unit": "edge-vector updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": step_ms, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": dtype, "data": data, "config": config,
        "roofline": roof, "cpu_baseline": cpu,
    }
    out.update(extra)
    return out


def err_stats(got, want, tol):
    """Relative error of every element of got against want (torch tensors
    on the GPU; an exact zero in want needs an exact zero in got): max,
    median, p99, p99.9 (quantiles over a fixed sample of 2^23 when larger)
    and the count beyond tol."""
    import torch
    want = want.double()
    diff = (got.double() - want).abs()
    rel = torch.where(want != 0, diff / want.abs(), torch.where(diff > 0, torch.full_like(diff, float("inf")),
                                                                 torch.zeros_like(diff)))
    beyond = int((rel > tol).sum())
    rel = rel.float()
    qs = torch.tensor([0.5, 0.99, 0.999], device=rel.device)
    n = rel.numel()
    pick = rel if n <= (1 << 23) else rel[torch.randint(0, n, (1 << 23,), device=rel.device,
                                                       generator=torch.Generator(rel.device).manual_seed(0))]
    q = torch.quantile(pick, qs).tolist()
    return {"max": float(rel.max()), "median": q[0], "p99": q[1], "p999": q[2], "tol": tol, "beyond_tol": beyond,
            "n": n}


# ------------------------------------------------------------ Chung-Lu ---

def run_chung_lu(args, api, torch, dev):
    from paper_1601_05527_amd import workloads as W
    c = W.CHUNG_LU
    R, K, OMEGA, TARGET, SEED_VEC = c["R"], c["k"], W.OMEGA, c["target"], c["seed_vec"]
    t0 = time.perf_counter()
    g_orig, g_run = W.chung_lu_graph(args.layout)
    t_setup = time.perf_counter() - t0
    log(f"graph generated and laid out in {t_setup:.1f}s: n={g_run.n} m={g_run.m} d_max={g_run.d_max}")
    dg = api.DeviceGraph.from_host(g_run, dev, keep_host=False)
    n, m, nnz = dg.n, dg.m, 2 * dg.m
    torch.cuda.synchronize()
    TAIL64 = W.FP64_TAIL
    t0 = time.perf_counter()
    comp = dg.components()            # grouped once per graph, like the layout
    torch.cuda.synchronize()
    t_comp = time.perf_counter() - t0
    log(f"{comp.n_comp} connected components grouped in {t_comp * 1e3:.1f} ms")

    # buffers reused by every step
    ws_r = api._workspace(api.relax_workspace_bytes(
        dg, api.relax_opts(R, K, OMEGA, SEED_VEC, rows_per_wave=args.rows_per_wave,
                           hub_degree=args.hub_degree, fp64_tail=TAIL64, comp=comp)), dev)
    ws_s = api._workspace(api.sparsify_fit_both_workspace_bytes(dg), dev)
    ws_d = api._workspace(api.edge_dist_workspace_bytes(dg), dev)
    out = api.RelaxResult(x=torch.empty((n, R), dtype=torch.float64, device=dev),
                          minmax=torch.empty(2 * R, dtype=torch.float64, device=dev),
                          shift=torch.empty((max(1, comp.n_comp), R), dtype=torch.float64, device=dev), ckpt=None,
                          store="f32")
    rho = torch.empty(m, dtype=torch.float32, device=dev)
    keep_l = torch.empty(m, dtype=torch.uint8, device=dev)
    keep_g = torch.empty(m, dtype=torch.uint8, device=dev)
    nk = torch.empty(2, dtype=torch.int64, device=dev)
    fit = {}

    def relax_dist():
        api.relax(dg, R, K, OMEGA, SEED_VEC, ws=ws_r, out=out, rows_per_wave=args.rows_per_wave,
                  hub_degree=args.hub_degree, fp64_tail=TAIL64)
        api.distances(dg, out, out=rho, ws=ws_d)

    def step():
        relax_dist()
        # LOCAL and GLOBAL fits from one ranking pass
        _, _, _, (e_l, e_g) = api.sparsify_fit_both(dg, rho, TARGET, ws=ws_s, keep_local=keep_l,
                                                    keep_global=keep_g, n_kept=nk)
        fit["e_local"], fit["e_global"] = e_l, e_g

    if args.calib_copy_mib > 0:
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {nb} bytes done")
        del src, dst

    timer = Timer(torch)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    step_ms, kern = traced(api, timer, step, args.steps)
    rd_ms = timer.run(relax_dist, args.steps)     # relax + distance alone, the bandwidth path
    # the step without the e-fit: both selections at the fitted exponents
    bud_l = torch.from_numpy(api.budget_table(dg.d_max, fit["e_local"])).to(dev)
    bud_g = torch.from_numpy(api.budget_table(dg.d_max, fit["e_global"])).to(dev)
    keep_fl, keep_fg = torch.empty_like(keep_l), torch.empty_like(keep_g)
    nk_f = torch.empty(2, dtype=torch.int64, device=dev)

    def step_fixed():
        relax_dist()
        api.sparsify(dg, rho, 0, budget=bud_l, ws=ws_s, keep=keep_fl, n_kept=nk_f[0:1])
        api.sparsify(dg, rho, 1, budget=bud_g, ws=ws_s, keep=keep_fg, n_kept=nk_f[1:2])

    step_fixed()
    fixed_ms = timer.run(step_fixed, args.steps)
    fixed_same = bool(torch.equal(keep_fl, keep_l) and torch.equal(keep_fg, keep_g) and torch.equal(nk_f, nk))
    del bud_l, bud_g, keep_fl, keep_fg

    kept_l, kept_g = (int(v) for v in nk.tolist())
    weighted = dg.w is not None
    per_sweep = relax_sweep_bytes(n, nnz, R, K, weighted, 4, K, TAIL64)
    sb = sum(per_sweep) / K           # the k sweeps share one trace scope: bytes of an average sweep
    db = dist_bytes(n, nnz, m, R, 8)
    roof = roofline(kern, sb, sweep_traffic())
    rd_gbs = (sum(per_sweep) + db) / (rd_ms * 1e-3) / 1e9
    # context: the same relaxation with every sweep stored in FP32 (no FP64 tail)
    out32 = api.RelaxResult(x=torch.empty((n, R), dtype=torch.float32, device=dev), minmax=out.minmax.clone(),
                            shift=out.shift.clone(), ckpt=None, store="f32")
    ws_r32 = api._workspace(api.relax_workspace_bytes(dg, api.relax_opts(R, K, OMEGA, SEED_VEC, comp=comp)), dev)
    rho32 = torch.empty_like(rho)

    def relax_dist32():
        api.relax(dg, R, K, OMEGA, SEED_VEC, ws=ws_r32, out=out32)
        api.distances(dg, out32, out=rho32, ws=ws_d)

    relax_dist32()
    rd32_ms = timer.run(relax_dist32, args.steps)
    x32 = out32.x
    del ws_r32, rho32

    # context: a device-to-device copy of 1 GiB (reads and writes 2 GiB), the streaming ceiling
    src = torch.ones(1 << 30, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    copy_ms = timer.run(lambda: dst.copy_(src), 5)
    copy_gbs = 2 * (1 << 30) / (copy_ms * 1e-3) / 1e9
    del src, dst

    # selection with binning (Algorithm 4) fitted to the same retention, on the step's distances
    ws_b = api._workspace(api.sparsify_binned_workspace_bytes(dg), dev)
    keep_b = torch.empty(m, dtype=torch.uint8, device=dev)
    nk_b = torch.empty(1, dtype=torch.int64, device=dev)
    binned = {}

    def binned_fit():
        _, _, e_b = api.sparsify_binned(dg, rho, c["bin_seed"], target=TARGET, ws=ws_b, keep=keep_b, n_kept=nk_b)
        binned["e"] = e_b

    binned_fit()
    b_ms, b_kern = traced(api, timer, binned_fit, max(1, min(args.steps, 5)))
    kept_b = int(nk_b.item())
    binned.update(ms=b_ms, kept=kept_b, ratio=kept_b / m,
                  breakdown_ms={k_: v[1] / max(1, min(args.steps, 5)) for k_, v in sorted(b_kern.items())},
                  what=(f"Algorithm 4 (bins by Scott's rule per vertex, round-robin over the bins in a "
                        f"seeded random order) with e fitted to {int(TARGET * 100)}% retention, on the "
                        "step's own distances; synchronises for the fit"))
    del ws_b

    # Algorithm 1's normalised distance (weighted-degree form) on the step's
    # distances, then the LOCAL fit on it
    rho_n = torch.empty_like(rho)
    norm_ms = timer.run(lambda: api.normalize_dist(dg, rho, by_strength=True, out=rho_n), 5)
    keep_nl, keep_ng = torch.empty_like(keep_l), torch.empty_like(keep_g)
    _, _, _, (e_nl, e_ng) = api.sparsify_fit_both(dg, rho_n, TARGET, ws=ws_s, keep_local=keep_nl,
                                                  keep_global=keep_ng, n_kept=torch.empty_like(nk))
    normalized = {"ms": norm_ms, "e_local_fit": e_nl, "e_global_fit": e_ng,
                  "what": ("per-vertex weighted degrees (a wave per row, FP64) and rho_e * sqrt(s_i s_j) for every "
                           "edge (eps 0); the fits: LOCAL and GLOBAL to the same retention on the normalised "
                           "distances")}
    del rho_n, keep_nl, keep_ng

    # the property comparisons of Section 6 for the step's LOCAL selection
    props = {}

    def compare():
        props.update(api.compare_properties(dg, keep_l))

    compare()
    p_ms = timer.run(compare, 2)
    props.update(ms=p_ms, what=("subgraph of the LOCAL selection, triangles / clustering / components of "
                                "both graphs, Spearman of degrees and of clustering (synchronising calls)"))

    # on-device ingest of the graph as drawn (16M pairs, random labels) into the
    # degree-ordered CSR the step runs on
    gu = torch.from_numpy(g_orig.edge_u).to(dev)
    gv = torch.from_numpy(g_orig.edge_v).to(dev)
    gw = torch.from_numpy(g_orig.edge_w).to(dev)
    di = api.ingest(n, gu, gv, gw, by_degree=True, entry_ids=False)
    same = bool(torch.equal(di.row_ptr, dg.row_ptr) and torch.equal(di.col, dg.col) and
                torch.equal(di.w, dg.w) and torch.equal(di.eid, dg.eid) and torch.equal(di.orig_id, dg.orig_id))
    del di
    ing_ms = timer.run(lambda: api.ingest(n, gu, gv, gw, by_degree=True, entry_ids=False), 3)
    ingest = {"ms": ing_ms, "pairs_per_s": g_orig.m / (ing_ms * 1e-3), "equals_step_layout": same,
              "what": (f"ad_ingest of the {g_orig.m} drawn pairs (random labels, lognormal weights) into the "
                       "symmetric CSR stored by decreasing degree, outputs allocated per call; "
                       f"(host generation and layout of the graph: {t_setup:.1f} s); rcm_ms: the same pairs "
                       "into reverse Cuthill-McKee order; rcm_gather_probe_ms: the gather probe over that "
                       "layout's column array (the degree order's: gather_ceiling.probe_ms)")}
    # the same pairs in reverse Cuthill-McKee order, and the sweep's gather floor in that layout
    dr = api.ingest(n, gu, gv, gw, order="rcm", entry_ids=False)
    ingest["rcm_ms"] = timer.run(lambda: api.ingest(n, gu, gv, gw, order="rcm", entry_ids=False), 2)
    ingest["rcm_gather_probe_ms"] = gather_probe_ms(torch, timer, x32, dr.col, R * 4)
    del dr, gu, gv, gw

    # context: the sweep's neighbour-row gathers alone, with nothing else asked of the
    # memory system (the irregular path's practical ceiling), and the vendor SpMM
    sweep_ms = roof["avg_launch_ms"]
    probe_ms = gather_probe_ms(torch, timer, x32, dg.col, R * 4)
    gather = None
    if probe_ms:
        gather = {"probe_ms": probe_ms, "rows_per_s": nnz / (probe_ms * 1e-3),
                  "sweep_rows_per_s": nnz / (sweep_ms * 1e-3) if sweep_ms else None,
                  "sweep_frac_of_probe": probe_ms / sweep_ms if sweep_ms else None,
                  "what": (f"one launch gathering all {nnz} neighbour rows ({R * 4} B each) in CSR "
                           "order with the graph's own column array, summing them; no weights, no "
                           "output rows, no arithmetic beyond the sum")}
    spmm = vendor_spmm_ms(torch, timer, dg, x32)
    del x32, out32

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cores = oracle_threads()
        log(f"CPU baseline: oracle, R={R}, {args.cpu_sweeps} sweeps, {cores} threads")
        t0 = time.perf_counter()
        oracle.algebraic_distance(g_run, R, args.cpu_sweeps, OMEGA, seed=SEED_VEC)
        t_cpu = time.perf_counter() - t0
        cpu = {"value": nnz * R * args.cpu_sweeps / t_cpu, "unit": "edge-vector updates/s",
               "cores": cores, "kind": "oracle", "cpu_model": cpu_model(),
               "sample": (f"FP64 oracle (Algorithm 1 in the paper's order) on the same graph, all "
                          f"{R} vectors, {args.cpu_sweeps} of the {K} sweeps, then rescale and "
                          f"distances; {t_cpu:.2f}s wall on {cores} threads (about {t_cpu * cores:.0f} "
                          "core-seconds); selection not included")}
        if args.cpu_sweeps_1t > 0:
            oracle.set_threads(1)
            log(f"CPU baseline: oracle, R={R}, {args.cpu_sweeps_1t} sweeps, 1 thread")
            t0 = time.perf_counter()
            oracle.algebraic_distance(g_run, R, args.cpu_sweeps_1t, OMEGA, seed=SEED_VEC)
            t_1 = time.perf_counter() - t0
            oracle.set_threads(cores)
            cpu["single_thread"] = {
                "value": nnz * R * args.cpu_sweeps_1t / t_1, "unit": "edge-vector updates/s", "cores": 1,
                "sample": (f"the same oracle call with {args.cpu_sweeps_1t} sweeps on one thread, "
                           f"{t_1:.2f}s wall including start vectors, rescale and distances")}

    config = {
        "workload": (f"Chung-Lu power-law graph n=2^20, m={c['m']}, gamma={c['gamma']}, "
                     f"lognormal(0,1) weights; R={R}, k={K}, omega={OMEGA}, FP32; LOCAL and "
                     f"GLOBAL selection each fitted to {int(TARGET * 100)}% retention"),
        "precision": (f"FP32 storage and arithmetic for sweeps 1..{K - TAIL64}, sweeps {K - TAIL64 + 1}..{K} "
                      f"stored and computed in FP64, FP32 distances; each connected component centred by its "
                      f"own weighted mean"),
        "n": n, "m": m, "nnz": nnz, "d_max": dg.d_max, "R": R, "k": K, "fp64_tail": TAIL64,
        "components": comp.n_comp, "layout": args.layout, "parallelism": "single GPU",
    }
    return base_result(
        args, nnz * R * K / (step_ms * 1e-3), step_ms, "f32", "synthetic (seeded Chung-Lu graph; no dataset)",
        config, roof, cpu,
        breakdown_ms_per_step={k_: v[1] / args.steps for k_, v in sorted(kern.items())},
        relax_dist_ms=rd_ms, relax_dist_hbm_frac=rd_gbs / HBM_PEAK_GBS,
        step_fixed_e={"ms": fixed_ms, "equals_fitted_masks": fixed_same,
                      "what": "relax + distances + LOCAL and GLOBAL selection at the fitted exponents "
                              "(ad_sparsify twice, budget tables already on the device): the step without the e-fit"},
        relax_dist_fp32_only_ms=rd32_ms,
        copy_ceiling_GBs=copy_gbs,
        gather_ceiling=gather,
        vendor_spmm=spmm,
        binned_selection=binned,
        normalized_distance=normalized,
        ingest=ingest,
        properties=props,
        traffic_over_algorithmic=(roof["traffic"] / sb) if roof["traffic"] else None,
        sweep_updates_per_s=nnz * R / (roof["avg_launch_ms"] * 1e-3) if roof["avg_launch_ms"] else None,
        fit={"e_local": fit["e_local"], "e_global": fit["e_global"], "kept_local": kept_l,
             "kept_global": kept_g, "ratio_local": kept_l / m, "ratio_global": kept_g / m},
        setup_s={"generate_and_layout": t_setup, "components": t_comp})


# ----------------------------------------------------------- multilevel ---

def run_multilevel(args, api, torch, dev):
    """Algorithm 6 alone on the Chung-Lu graph: at most 9 levels, n_min
    1000, level-span 3 on the finest third, each sparsified level keeping
    30% of its edges."""
    from paper_1601_05527_amd import graphs
    from paper_1601_05527_amd import workloads as W
    c = W.CHUNG_LU
    R, K, TARGET = c["R"], c["k"], c["target"]
    _, g_run = W.chung_lu_graph("degree")
    dg = api.DeviceGraph.from_host(g_run, dev, keep_host=False)
    m = dg.m
    kw = dict(levels=c["ml_levels"], n_min=c["ml_n_min"], bin_seed=c["bin_seed"], fit=True, span=c["ml_span"],
              segment=2, span_value=TARGET)
    keep = torch.empty(m, dtype=torch.uint8, device=dev)
    res = {}

    def cycle():
        _, kept, depth = api.ml_sparsify(dg, R, K, omega=W.OMEGA, seed=c["seed_vec"], store="f32", keep=keep, **kw)
        res.update(kept=kept, depth=depth)

    timer = Timer(torch)
    for _ in range(args.warmup):
        cycle()
    torch.cuda.synchronize()
    ms, kern = traced(api, timer, cycle, args.steps)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        ns, ms_ = 1 << 18, 4_000_000
        g0 = graphs.chung_lu(ns, ms_, gamma=c["gamma"], seed=c["seed"])
        gs = graphs.relabel(g0, graphs.degree_descending_order(g0))
        t0 = time.perf_counter()
        oracle.ml_sparsify(gs, R, K, None, omega=W.OMEGA, seed=c["seed_vec"], **kw)
        t_cpu = time.perf_counter() - t0
        cpu = {"value": gs.m / t_cpu, "unit": "input edges/s", "cores": oracle_threads(), "kind": "oracle",
               "sample": (f"FP64 oracle multilevel cycle, same parameters, on a Chung-Lu graph of the same kind "
                          f"with n=2^18 and {gs.m} edges; {t_cpu:.2f}s wall")}
    config = {
        "workload": (f"Algorithm 6 on the Chung-Lu graph n=2^20, m={c['m']}, gamma={c['gamma']}, lognormal "
                     f"weights; R={R}, k={K}, FP32 relaxation at every level; at most {c['ml_levels']} levels, "
                     f"n_min={c['ml_n_min']}, level-span {c['ml_span']} on the finest third, each sparsified "
                     f"level keeping {int(TARGET * 100)}% of its edges"),
        "n": dg.n, "m": m, "R": R, "k": K, "parallelism": "single GPU",
    }
    return base_result(args, m / (ms * 1e-3), ms, "f32", "synthetic (seeded Chung-Lu graph; no dataset)", config,
                       None, cpu, metric="multilevel sparsification throughput", unit="input edges/s",
                       kept=res["kept"], depth=res["depth"], ratio=res["kept"] / m,
                       breakdown_ms_per_step={k_: v[1] / args.steps for k_, v in sorted(kern.items())})


# --------------------------------------------------------------- batch ---

def run_batch(args, api, torch, dev):
    from paper_1601_05527_amd import graphs
    from paper_1601_05527_amd import workloads as W
    b_ = W.BATCH
    R, K = b_["R"], b_["k"]
    t0 = time.perf_counter()
    ds = W.batch_graphs(dev)
    dgs = [api.DeviceGraph.from_tensors(d) for d in ds]
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    n = sum(d.n for d in dgs)
    m = sum(d.m for d in dgs)
    nnz = 2 * m
    log(f"{len(dgs)} graphs generated in {t_gen:.1f}s: n={n} m={m}")
    t0 = time.perf_counter()
    b = api.Batch(dgs, R, K, W.OMEGA, seed=b_["seed_vec"], graph_id=b_["graph_id"], orient=api.AD_LOCAL,
                  e=b_["e"], autotune=True, fp64_tail=W.FP64_TAIL)
    torch.cuda.synchronize()
    t_create = time.perf_counter() - t0
    log(f"batch created (pack, autotune, capture) in {t_create:.1f}s; rows_per_wave={b.rows_per_wave}")
    timer = Timer(torch)
    for _ in range(args.warmup):
        b.run()
    step_ms = timer.run(b.run, args.steps)
    # the same launch sequence uncaptured, traced per kernel
    unc_ms, kern = traced(api, timer, lambda: b.run(captured=False), args.steps)
    weighted = True
    roof = roofline(kern, sum(relax_sweep_bytes(n, nnz, R, K, weighted, 4, K, W.FP64_TAIL)) / K)
    kept = int(b.fetch()[2].sum().item())
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cores = oracle_threads()
        budget_s = args.cpu_seconds
        done_nnz, t_cpu, q = 0, 0.0, 0
        while q < len(ds) and t_cpu < budget_s:
            g = graphs.device_to_host(ds[q])
            t0 = time.perf_counter()
            oracle.algebraic_distance(g, R, K, W.OMEGA, seed=b_["seed_vec"], graph_id=b_["graph_id"] + q)
            t_cpu += time.perf_counter() - t0
            done_nnz += 2 * g.m
            q += 1
        cpu = {"value": done_nnz * R * K / t_cpu, "unit": "edge-vector updates/s", "cores": cores,
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": (f"FP64 oracle on the first {q} of the {len(ds)} graphs ({done_nnz // 2} edges), "
                          f"R={R}, all {K} sweeps, rescale and distances; {t_cpu:.2f}s; selection not included")}
    config = {
        "workload": (f"batch of {len(dgs)} Chung-Lu graphs (gamma 2.1, lognormal weights), n log-uniform in "
                     f"[1e3, 2e5], average degree uniform in [8, 32]; R={R}, k={K}, FP32 (last "
                     f"{W.FP64_TAIL} sweeps FP64, components centred apart); LOCAL selection "
                     f"at e={b_['e']}; one captured launch sequence, rows_per_wave autotuned"),
        "graphs": len(dgs), "n": n, "m": m, "nnz": nnz, "R": R, "k": K,
        "rows_per_wave": b.rows_per_wave, "parallelism": "single GPU",
    }
    b.close()
    return base_result(args, nnz * R * K / (step_ms * 1e-3), step_ms, "f32",
                       "synthetic (seeded Chung-Lu graphs; no dataset)", config, roof, cpu,
                       uncaptured_ms_per_step=unc_ms,
                       breakdown_ms_per_step={k_: v[1] / args.steps for k_, v in sorted(kern.items())},
                       kept=kept, setup_s={"generate": t_gen, "create": t_create})


# ---------------------------------------------------------------- BF16 ---

def run_bf16(args, api, torch, dev):
    """R-MAT n = 2^24, 2^28 edges: BF16 storage (the step timed in the line)
    beside the FP32 path, both against the library's FP64 path."""
    from paper_1601_05527_amd import graphs
    from paper_1601_05527_amd import workloads as W
    c = W.RMAT
    R, K, TAIL, TAIL64, TARGET = c["R"], c["k"], c["fp32_tail"], c["fp64_tail"], c["target"]
    t0 = time.perf_counter()
    d = W.rmat_graph(dev)
    dg = api.DeviceGraph.from_tensors(d)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    n, m, nnz = dg.n, dg.m, 2 * dg.m
    log(f"R-MAT generated in {t_gen:.1f}s: n={n} m={m} d_max={dg.d_max}")
    t0 = time.perf_counter()
    comp = dg.components()
    torch.cuda.synchronize()
    t_comp = time.perf_counter() - t0
    log(f"{comp.n_comp} components grouped in {t_comp:.2f}s")
    ws_d = api._workspace(api.edge_dist_workspace_bytes(dg), dev)
    ws_s = api._workspace(api.sparsify_fit_both_workspace_bytes(dg), dev)
    keep_l = torch.empty(m, dtype=torch.uint8, device=dev)
    keep_g = torch.empty(m, dtype=torch.uint8, device=dev)
    nk = torch.empty(2, dtype=torch.int64, device=dev)
    fits = {}
    tails = {"bf16": (TAIL, TAIL64), "f32": (K, W.FP64_TAIL), "f64": (K, 0)}

    def make(store):
        t32, t64 = tails[store]
        opts = api.relax_opts(R, K, W.OMEGA, c["seed_vec"], store=store, fp32_tail=t32, fp64_tail=t64, comp=comp)
        ws = api._workspace(api.relax_workspace_bytes(dg, opts), dev)
        out = api.RelaxResult(x=torch.empty((n, R), dtype=torch.float64, device=dev),
                              minmax=torch.empty(2 * R, dtype=torch.float64, device=dev),
                              shift=torch.empty((max(1, comp.n_comp), R), dtype=torch.float64, device=dev),
                              ckpt=None, store=store)
        rho_s = torch.empty(m, dtype=torch.float64 if store == "f64" else torch.float32, device=dev)

        def relax_dist():
            api.relax(dg, R, K, W.OMEGA, c["seed_vec"], store=store, fp32_tail=t32, fp64_tail=t64, ws=ws, out=out)
            api.distances(dg, out, out=rho_s, ws=ws_d)

        def step():
            relax_dist()
            _, _, _, (e_l, e_g) = api.sparsify_fit_both(dg, rho_s, TARGET, ws=ws_s, keep_local=keep_l,
                                                        keep_global=keep_g, n_kept=nk)
            fits[(store, "local")], fits[(store, "global")] = e_l, e_g
        return step, relax_dist, rho_s, ws, out

    timer = Timer(torch)
    results = {}
    for store in ("bf16", "f32"):
        step, relax_dist, rho_s, ws, out = make(store)
        for _ in range(args.warmup):
            step()
        ms, kern = traced(api, timer, step, args.steps)
        rd_ms = timer.run(relax_dist, args.steps)
        relax_dist()
        results[store] = {"ms": ms, "relax_dist_ms": rd_ms, "kern": kern, "rho": rho_s}
        del ws, out
        log(f"{store}: {ms:.2f} ms per step, relax+dist {rd_ms:.2f} ms")
    # reference: the library's FP64 path (FP64 storage and arithmetic; its parity with the oracle is tested)
    _, relax_dist64, rho64, ws64, out64 = make("f64")
    relax_dist64()
    torch.cuda.synchronize()
    acc = {"reference": "the library's FP64 path on the GPU (FP64 storage and arithmetic)",
           "bf16": err_stats(results["bf16"]["rho"], rho64, 2e-2),
           "f32": err_stats(results["f32"]["rho"], rho64, 1e-5)}
    del rho64, ws64, out64
    weighted = True
    per = relax_sweep_bytes(n, nnz, R, K, weighted, 2, TAIL, TAIL64)
    roof = roofline(results["bf16"]["kern"], sum(per) / K)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        g = graphs.device_to_host(d)
        x0 = oracle.start_vectors(g.n, 1, c["seed_vec"], 0, g.orig_id)[:, 0].copy()
        sweeps = args.cpu_sweeps
        t0 = time.perf_counter()
        oracle.relax_vector(g, x0, sweeps, W.OMEGA)
        t_cpu = time.perf_counter() - t0
        cpu = {"value": nnz * sweeps / t_cpu, "unit": "edge-vector updates/s", "cores": oracle_threads(),
               "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"FP64 oracle, 1 of the {R} vectors, {sweeps} of the {K} sweeps on the same graph; "
                         f"{t_cpu:.2f}s"}
        del g
    ms = results["bf16"]["ms"]
    config = {
        "workload": (f"R-MAT (a,b,c,d)=(.57,.19,.19,.05) n=2^{c['scale']}, m={m}, uniform(0.5,2) weights; "
                     f"R={R}, k={K}, test vectors stored in BF16 (last {TAIL} sweeps wider: {TAIL - TAIL64} FP32, "
                     f"{TAIL64} FP64), FP32 arithmetic; components centred apart and re-centred before every "
                     f"BF16 sweep; LOCAL and GLOBAL selection each fitted to {int(TARGET * 100)}% retention"),
        "n": n, "m": m, "nnz": nnz, "d_max": dg.d_max, "R": R, "k": K, "fp32_tail": TAIL, "fp64_tail": TAIL64,
        "components": comp.n_comp, "parallelism": "single GPU",
    }
    return base_result(
        args, nnz * R * K / (ms * 1e-3), ms, "bf16 storage, f32 arithmetic",
        "synthetic (seeded R-MAT graph; no dataset)", config, roof, cpu,
        fp32_path={"ms_per_step": results["f32"]["ms"], "relax_dist_ms": results["f32"]["relax_dist_ms"],
                   "value": nnz * R * K / (results["f32"]["ms"] * 1e-3), "fp64_tail": W.FP64_TAIL,
                   "breakdown_ms_per_step": {k_: v[1] / args.steps
                                             for k_, v in sorted(results["f32"]["kern"].items())}},
        relax_dist_ms=results["bf16"]["relax_dist_ms"],
        breakdown_ms_per_step={k_: v[1] / args.steps for k_, v in sorted(results["bf16"]["kern"].items())},
        accuracy=acc, fit={f"{s}_{o}": v for (s, o), v in fits.items()},
        setup_s={"generate": t_gen, "components": t_comp})


# ------------------------------------------------------------- adjoint ---

def run_adjoint(args, api, torch, dev):
    import numpy as np
    from paper_1601_05527_amd import workloads as W
    c = W.GRID
    R, K, CK = c["R"], c["k"], c["ckpt_every"]
    g = W.grid_graph()
    dg = api.DeviceGraph.from_host(g, dev)
    n, m, nnz = dg.n, dg.m, 2 * dg.m
    cvec = torch.from_numpy(np.random.default_rng(c["seed"]).normal(size=m).astype(np.float32)).to(dev)
    comp = dg.components()
    opts = api.relax_opts(R, K, W.OMEGA, c["seed_vec"], ckpt_every=CK, comp=comp)
    ws_r = api._workspace(api.relax_workspace_bytes(dg, opts), dev)
    ws_d = api._workspace(api.edge_dist_workspace_bytes(dg), dev)
    nck = int(api.lib.ad_relax_num_checkpoints(api.ctypes.byref(opts)))
    out = api.RelaxResult(x=torch.empty((n, R), dtype=torch.float32, device=dev),
                          minmax=torch.empty(2 * R, dtype=torch.float64, device=dev),
                          shift=torch.empty((max(1, comp.n_comp), R), dtype=torch.float64, device=dev),
                          ckpt=torch.empty((nck, n, R), dtype=torch.float32, device=dev), store="f32")
    rho = torch.empty(m, dtype=torch.float32, device=dev)
    gw = torch.empty(m, dtype=torch.float32, device=dev)
    opts_b = api.relax_opts(R, K, W.OMEGA, c["seed_vec"], ckpt_every=CK, comp=comp)
    ws_b = api._workspace(int(api.lib.ad_relax_backward_workspace_size(api.ctypes.byref(dg.abi()),
                                                                       api.ctypes.byref(opts_b))), dev)

    def forward():
        api.relax(dg, R, K, W.OMEGA, c["seed_vec"], ckpt_every=CK, ws=ws_r, out=out)
        api.edge_dist(dg, out.x, out.minmax, out=rho, ws=ws_d)

    def backward():
        api.relax_backward(dg, out, R, K, cvec, W.OMEGA, c["seed_vec"], ckpt_every=CK, ws=ws_b, out=gw)

    def step():
        forward()
        backward()

    timer = Timer(torch)
    for _ in range(args.warmup):
        step()
    f_ms = timer.run(forward, args.steps)
    b_ms = timer.run(backward, args.steps)
    step_ms, kern = traced(api, timer, step, args.steps)
    roof = roofline(kern, sweep_bytes(n, nnz, R, 4, True))
    # the gradient against the FP64 oracle's reverse mode (test infrastructure, outside the timed region)
    import oracle
    t0 = time.perf_counter()
    want = oracle.grad_weights(g, cvec.cpu().numpy().astype(np.float64), R, K, W.OMEGA, seed=c["seed_vec"])
    t_cpu = time.perf_counter() - t0
    got = gw.cpu().numpy().astype(np.float64)
    per = np.abs(got - want) / (np.abs(want) + 1e-3 * np.abs(want).max())
    grad_err = {"rel_l2": float(np.linalg.norm(got - want) / np.linalg.norm(want)), "max_per_edge": float(per.max()),
                "p999_per_edge": float(np.quantile(per, 0.999)),
                "per_edge_measure": "|g - g_oracle| / (|g_oracle| + 1e-3 max |g_oracle|)"}
    cpu = None
    if not args.no_cpu_baseline:
        cpu = {"value": nnz * R * K / t_cpu, "unit": "edge-vector updates/s (forward + gradient)",
               "cores": oracle_threads(), "kind": "oracle", "cpu_model": cpu_model(),
               "sample": f"FP64 oracle reverse-mode gradient on the same graph, R={R}, k={K}; {t_cpu:.2f}s"}
    config = {
        "workload": (f"{c['side']}x{c['side']} grid plus {g.m - 2 * c['side'] * (c['side'] - 1)} random long-range "
                     f"edges, lognormal weights; R={R}, k={K}, FP32; gradient of sum_e c_e rho_e with respect to "
                     f"every edge weight, checkpoints every {CK} sweeps; value counts the forward sweeps only"),
        "n": n, "m": m, "nnz": nnz, "R": R, "k": K, "ckpt_every": CK, "parallelism": "single GPU",
    }
    return base_result(args, nnz * R * K / (step_ms * 1e-3), step_ms, "f32",
                       "synthetic (seeded grid with long-range edges; no dataset)", config, roof, cpu,
                       forward_ms=f_ms, backward_ms=b_ms, backward_over_forward=b_ms / f_ms, gradient_error=grad_err,
                       breakdown_ms_per_step={k_: v[1] / args.steps for k_, v in sorted(kern.items())})


# ---------------------------------------------------------------- FP64 ---

def run_fp64(args, api, torch, dev):
    import numpy as np
    from paper_1601_05527_amd import workloads as W
    c = W.GNM
    R, K, E = c["R"], c["k"], c["e"]
    g = W.gnm_graph()
    dg = api.DeviceGraph.from_host(g, dev)
    n, m, nnz = dg.n, dg.m, 2 * dg.m
    res = {}

    def step():
        r = api.relax(dg, R, K, W.OMEGA, c["seed_vec"], store="f64")
        rho = api.edge_dist(dg, r.x, r.minmax)
        keep, nk = api.sparsify(dg, rho, api.AD_LOCAL, E)
        res["rho"], res["keep"] = rho, keep

    timer = Timer(torch)
    for _ in range(args.warmup):
        step()
    step_ms, kern = traced(api, timer, step, args.steps)
    roof = roofline(kern, sweep_bytes(n, nnz, R, 8, False))
    import oracle
    t0 = time.perf_counter()
    rho_o = oracle.algebraic_distance(g, R, K, W.OMEGA, seed=c["seed_vec"])
    keep_o, _ = oracle.sparsify(g, rho_o, 0, E)
    t_cpu = time.perf_counter() - t0
    rho_g = res["rho"].cpu().numpy()
    cpu = None if args.no_cpu_baseline else {
        "value": nnz * R * K / t_cpu, "unit": "edge-vector updates/s", "cores": oracle_threads(), "kind": "oracle",
        "sample": f"the whole workload: FP64 oracle distances and LOCAL selection; {t_cpu * 1e3:.1f} ms"}
    config = {"workload": f"G(n,m) n={n}, m={m}, unit weights, seed 0; R={R}, k={K}, FP64; LOCAL selection e={E}",
              "n": n, "m": m, "nnz": nnz, "R": R, "k": K, "parallelism": "single GPU"}
    return base_result(args, nnz * R * K / (step_ms * 1e-3), step_ms, "f64", "synthetic (seeded G(n,m); no dataset)",
                       config, roof, cpu,
                       oracle_max_rel_err=float(np.max(np.abs(rho_g - rho_o) / rho_o)),
                       kept_equal_oracle=bool(np.array_equal(res["keep"].cpu().numpy(), keep_o)),
                       breakdown_ms_per_step={k_: v[1] / args.steps for k_, v in sorted(kern.items())})


def extras(args, api, torch, dev) -> dict:
    """Compact records of the batch, R-MAT and adjoint workloads for the
    default line (fewer steps, no CPU baselines; each workload's own line
    holds the full record)."""
    import copy
    import gc
    sub = copy.copy(args)
    sub.steps, sub.warmup, sub.no_cpu_baseline = args.extra_steps, 1, True
    out = {}
    keep = ("value", "unit", "ms_per_step", "dtype", "roofline")
    for name, fn in (("batch", run_batch), ("rmat", run_bf16), ("adjoint", run_adjoint)):
        t0 = time.perf_counter()
        r = fn(sub, api, torch, dev)
        rec = {k_: r[k_] for k_ in keep}
        rec["roofline"] = {k_: r["roofline"][k_] for k_ in ("achieved", "frac", "avg_launch_ms")}
        rec["workload"] = r["config"]["workload"]
        rec["steps"] = sub.steps
        for k_ in ("uncaptured_ms_per_step", "kept", "fp32_path", "accuracy", "forward_ms", "backward_ms",
                   "backward_over_forward", "gradient_error", "relax_dist_ms", "breakdown_ms_per_step"):
            if k_ in r:
                rec[k_] = r[k_]
        rec["wall_s"] = time.perf_counter() - t0
        out[name] = rec
        log(f"{name}: {rec['ms_per_step']:.2f} ms per step ({rec['wall_s']:.0f} s with set-up)")
        del r
        gc.collect()
        torch.cuda.empty_cache()
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["chung-lu", "batch", "bf16", "adjoint", "fp64", "multilevel"],
                    default="chung-lu")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=6, help="sweeps in the oracle's bounded CPU sample")
    ap.add_argument("--cpu-sweeps-1t", type=int, default=2,
                    help="sweeps in the oracle's one-thread sample of the Chung-Lu workload (0: none)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="batch workload: oracle time budget for its graph sample")
    ap.add_argument("--layout", choices=["degree", "given"], default="degree")
    ap.add_argument("--rows-per-wave", type=int, default=0)
    ap.add_argument("--hub-degree", type=int, default=0)
    ap.add_argument("--no-extras", action="store_true",
                    help="default workload: leave out the compact batch / R-MAT / adjoint records")
    ap.add_argument("--extra-steps", type=int, default=3, help="timed steps of each compact record")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="before timing, copy a buffer of this many MiB device to device "
                         "(a kernel of known traffic for calibrating memory counters)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: every workload "
              "here runs on a single MI355X", file=sys.stderr)
        return 2

    import torch

    from paper_1601_05527_amd import api

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    run = {"chung-lu": run_chung_lu, "batch": run_batch, "bf16": run_bf16, "adjoint": run_adjoint,
           "fp64": run_fp64, "multilevel": run_multilevel}[args.workload]
    result = run(args, api, torch, dev)
    if args.workload == "chung-lu" and not args.no_extras:
        import gc
        gc.collect()
        torch.cuda.empty_cache()
        result["workloads"] = extras(args, api, torch, dev)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
