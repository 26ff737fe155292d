"""Python binding of libad (the C ABI in ``include/ad.h``).

Argument marshalling only: every step of the computation runs in the HIP
library.  Tensors live on the current HIP device; calls are enqueued on
``torch.cuda.current_stream()``.  Importing this module loads ``libad.so``
and raises if it has not been built -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import graphs as _graphs

_HERE = os.path.dirname(os.path.abspath(__file__))
# AD_LIBRARY names another build of the library (the host-sanitized one of
# build_lib.build_sanitized()); by default the in-tree libad.so.
LIB_PATH = os.environ.get("AD_LIBRARY") or os.path.join(_HERE, "libad.so")

AD_F64, AD_F32, AD_BF16 = 0, 1, 2
AD_LOCAL, AD_GLOBAL = 0, 1
_DTYPES = {"f64": AD_F64, "f32": AD_F32, "bf16": AD_BF16}
_STATUS = {0: "AD_OK", 1: "AD_ERR_INVALID_ARG", 2: "AD_ERR_UNSUPPORTED", 3: "AD_ERR_WORKSPACE",
           4: "AD_ERR_GRAPH", 5: "AD_ERR_HIP", 6: "AD_ERR_INTERNAL"}


class ADGraph(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("m", ctypes.c_int64), ("row_ptr", ctypes.c_void_p),
                ("col", ctypes.c_void_p), ("w", ctypes.c_void_p), ("eid", ctypes.c_void_p),
                ("orig_id", ctypes.c_void_p), ("d_max", ctypes.c_int32),
                ("col_orig", ctypes.c_void_p)]


class ADComponents(ctypes.Structure):
    _fields_ = [("n_comp", ctypes.c_int64), ("n_chunks", ctypes.c_int64), ("comp_of", ctypes.c_void_p),
                ("members", ctypes.c_void_p), ("comp_start", ctypes.c_void_p), ("chunk_start", ctypes.c_void_p)]


class ADRelaxOpts(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int32), ("k", ctypes.c_int32), ("omega", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("graph_id", ctypes.c_uint64), ("store", ctypes.c_int),
                ("fp32_tail", ctypes.c_int32), ("ckpt_every", ctypes.c_int32),
                ("rows_per_wave", ctypes.c_int32), ("hub_degree", ctypes.c_int32),
                ("fp64_tail", ctypes.c_int32), ("comp", ctypes.POINTER(ADComponents))]


class ADBatchOpts(ctypes.Structure):
    _fields_ = [("orient", ctypes.c_int), ("e", ctypes.c_double), ("autotune", ctypes.c_int32)]


class ADMLOpts(ctypes.Structure):
    _fields_ = [("R", ctypes.c_int32), ("k", ctypes.c_int32), ("omega", ctypes.c_double),
                ("seed", ctypes.c_uint64), ("graph_id", ctypes.c_uint64), ("store", ctypes.c_int),
                ("levels", ctypes.c_int32), ("n_min", ctypes.c_int64), ("e_host", ctypes.c_void_p),
                ("eps", ctypes.c_double), ("theta", ctypes.c_double), ("bin_seed", ctypes.c_uint64),
                ("fit", ctypes.c_int32), ("span", ctypes.c_int32), ("segment", ctypes.c_int32),
                ("span_value", ctypes.c_double), ("fp64_tail", ctypes.c_int32)]


class ADError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def _load_lib():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1601_05527_amd.build_lib")
    lib = ctypes.CDLL(LIB_PATH)
    P, S = ctypes.c_void_p, ctypes.c_size_t
    G = ctypes.POINTER(ADGraph)
    O = ctypes.POINTER(ADRelaxOpts)
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    st = ctypes.c_int
    sig = {
        "ad_relax_workspace_size": (S, [G, O]),
        "ad_relax_num_checkpoints": (i32, [O]),
        "ad_relax": (st, [G, O, P, P, P, P, P, P, S, P]),
        "ad_edge_dist_workspace_size": (S, [G]),
        "ad_edge_dist": (st, [G, i32, ctypes.c_int, P, P, ctypes.c_int, P, P, S, P]),
        "ad_edge_dist_noalloc_max_bytes": (S, []),
        "ad_edge_dist_noalloc": (st, [G, i32, ctypes.c_int, P, P, ctypes.c_int, P, P]),
        "ad_components_workspace_size": (S, [G]),
        "ad_compare_properties_workspace_size": (S, [G]),
        "ad_compare_properties": (st, [G, P, P, P, S, P]),
        "ad_components_build": (st, [G, P, P, P, P, ctypes.POINTER(i64), ctypes.POINTER(i64), P, S, P]),
        "ad_budget_table": (st, [i32, f64, P]),
        "ad_sparsify_workspace_size": (S, [G]),
        "ad_sparsify": (st, [G, ctypes.c_int, P, ctypes.c_int, P, P, P, P, S, P]),
        "ad_sparsify_fit": (st, [G, ctypes.c_int, P, ctypes.c_int, f64, P, P, P, P, S, P]),
        "ad_sparsify_fit_both_workspace_size": (S, [G]),
        "ad_normalize_dist_workspace_size": (S, [G]),
        "ad_normalize_dist": (st, [G, ctypes.c_int, P, ctypes.c_int32, f64, P, P, S, P]),
        "ad_subgraph_workspace_size": (S, [G]),
        "ad_subgraph": (st, [G, P, P, P, P, P, P, ctypes.POINTER(i64), P, S, P]),
        "ad_graph_properties_workspace_size": (S, [G]),
        "ad_graph_properties": (st, [G, P, P, P, P, P, S, P]),
        "ad_spearman_workspace_size": (S, [i64]),
        "ad_spearman": (st, [i64, P, P, ctypes.POINTER(f64), P, S, P]),
        "ad_ingest_workspace_size": (S, [i64, i64]),
        "ad_ingest": (st, [i64, i64, P, P, P, P, i32, P, P, P, P, P, ctypes.POINTER(i64), ctypes.POINTER(i32),
                           ctypes.POINTER(i64), P, S, P]),
        "ad_sparsify_binned_workspace_size": (S, [G]),
        "ad_sparsify_binned": (st, [G, ctypes.c_int, P, ctypes.c_uint64, ctypes.c_uint64, f64, f64, P, P,
                                    ctypes.POINTER(ctypes.c_double), P, S, P]),
        "ad_ml_aggregate_workspace_size": (S, [G]),
        "ad_ml_aggregate": (st, [G, ctypes.c_int, P, f64, f64, P, P, ctypes.POINTER(i64), P, S, P]),
        "ad_ml_level_span": (st, [i32, i32, i32, f64, P]),
        "ad_ml_sparsify": (st, [G, ctypes.POINTER(ADMLOpts), P, ctypes.POINTER(i64), ctypes.POINTER(i32), P]),
        "ad_sparsify_fit_both": (st, [G, ctypes.c_int, P, f64, P, P, P, P, P, S, P]),
        "ad_edge_dist_select_workspace_size": (S, [G]),
        "ad_edge_dist_sparsify": (st, [G, i32, ctypes.c_int, P, P, P, ctypes.c_int, P, P, P, P, S, P]),
        "ad_edge_dist_fit_both": (st, [G, i32, ctypes.c_int, P, P, P, f64, P, P, P, P, P, S, P]),
        "ad_relax_backward_workspace_size": (S, [G, O]),
        "ad_relax_backward": (st, [G, O, P, P, P, P, P, P, P, S, P]),
        "ad_edge_to_entries": (st, [G, P, P, P]),
        "ad_graph_col_orig": (st, [G, P, P]),
        "ad_batch_create": (st, [i32, G, O, ctypes.POINTER(ADBatchOpts), ctypes.POINTER(P), P]),
        "ad_batch_run": (st, [P, P]),
        "ad_batch_run_uncaptured": (st, [P, P]),
        "ad_batch_info": (st, [P, P, P, P]),
        "ad_batch_results": (st, [P, P, P, P, P]),
        "ad_batch_copy_results": (st, [P, P, P, P, P, P]),
        "ad_batch_destroy": (None, [P]),
        "ad_validate_workspace_size": (S, [G]),
        "ad_validate_graph": (st, [G, P, S, P]),
        "ad_trace_enable": (None, [i32]),
        "ad_trace_reset": (None, []),
        "ad_trace_summary": (st, [ctypes.c_char_p, S]),
        "ad_status_string": (ctypes.c_char_p, [st]),
        "ad_last_error": (ctypes.c_char_p, []),
        "ad_abi_version": (i32, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load_lib()


def _check(status: int) -> None:
    if status != 0:
        raise ADError(status, lib.ad_last_error().decode())


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _workspace(nbytes: int, device) -> torch.Tensor:
    # torch's caching allocator returns 256-byte-aligned blocks; check anyway.
    ws = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
    if ws.data_ptr() % 256:
        raise ADError(3, "workspace allocation is not 256-byte aligned")
    return ws


def trace_summary() -> dict:
    """{kernel name: (launches, total ms)} recorded while ad_trace_enable(1)."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(lib.ad_trace_summary(buf, len(buf)))
    out = {}
    for line in buf.value.decode().splitlines():
        name, cnt, ms = line.split()
        out[name] = (int(cnt), float(ms))
    return out


# ---------------------------------------------------------------- graphs ---

@dataclass
class DeviceGraph:
    """A symmetric CSR resident on the device, plus the ABI struct."""

    n: int
    m: int
    d_max: int
    row_ptr: torch.Tensor
    col: torch.Tensor
    w: Optional[torch.Tensor]
    eid: torch.Tensor
    orig_id: Optional[torch.Tensor]
    host: Optional[_graphs.Graph] = None
    col_orig: Optional[torch.Tensor] = None
    comp: Optional["Components"] = None

    @classmethod
    def from_host(cls, g: _graphs.Graph, device="cuda", keep_host: bool = True,
                  entry_ids: bool = True) -> "DeviceGraph":
        """Copy the CSR to the device; with entry_ids also build the
        per-entry neighbour ids (ad_graph_col_orig) used by ranking."""
        dev = torch.device(device)

        def t(a, dt):
            return torch.from_numpy(np.ascontiguousarray(a, dtype=dt)).to(dev)

        dg = cls(n=g.n, m=g.m, d_max=g.d_max,
                 row_ptr=t(g.row_ptr, np.int64), col=t(g.col, np.int32),
                 w=None if g.w is None else t(g.w, np.float32),
                 eid=t(g.eid, np.int32), orig_id=t(g.orig_id, np.int32),
                 host=g if keep_host else None)
        if entry_ids and g.m > 0:
            dg.col_orig = torch.empty(2 * g.m, dtype=torch.int32, device=dev)
            gs = dg.abi()
            _check(lib.ad_graph_col_orig(ctypes.byref(gs), _ptr(dg.col_orig), _stream()))
        return dg

    @classmethod
    def from_tensors(cls, d: dict, entry_ids: bool = True) -> "DeviceGraph":
        """Wrap a device graph dict (graphs.chung_lu_device / rmat_device)."""
        dg = cls(n=d["n"], m=d["m"], d_max=d["d_max"], row_ptr=d["row_ptr"].contiguous(),
                 col=d["col"].contiguous(), w=None if d["w"] is None else d["w"].contiguous(),
                 eid=d["eid"].contiguous(), orig_id=d["orig_id"].contiguous(), host=None)
        if entry_ids and dg.m > 0:
            dg.col_orig = torch.empty(2 * dg.m, dtype=torch.int32, device=dg.row_ptr.device)
            gs = dg.abi()
            _check(lib.ad_graph_col_orig(ctypes.byref(gs), _ptr(dg.col_orig), _stream()))
        return dg

    @property
    def device(self):
        return self.row_ptr.device

    def abi(self) -> ADGraph:
        return ADGraph(self.n, self.m, self.row_ptr.data_ptr(),
                       self.col.data_ptr() if self.col.numel() else None,
                       None if self.w is None else self.w.data_ptr(),
                       self.eid.data_ptr() if self.eid.numel() else None,
                       None if self.orig_id is None else self.orig_id.data_ptr(),
                       self.d_max,
                       None if self.col_orig is None else self.col_orig.data_ptr())

    def with_weights(self, w_entries: Optional[torch.Tensor]) -> "DeviceGraph":
        # positive weights keep the components, so the grouping carries over
        return DeviceGraph(self.n, self.m, self.d_max, self.row_ptr, self.col, w_entries,
                           self.eid, self.orig_id, self.host, self.col_orig, self.comp)

    def components(self) -> "Components":
        """The graph's connected components grouped for the per-component
        centring of ``ad_relax`` (``ad_components_build``), built on first use
        and kept with the graph.  Synchronises the current stream."""
        if self.comp is None:
            self.comp = components(self)
        return self.comp


@dataclass
class Components:
    """Device arrays of ``ad_components`` plus the ABI struct."""

    n_comp: int
    n_chunks: int
    comp_of: torch.Tensor        # int32 [n], -1 for isolated vertices
    members: torch.Tensor        # int32 [n]
    comp_start: torch.Tensor     # int64 [n + 1]
    chunk_start: torch.Tensor    # int64 [n + 1]

    def abi(self) -> ADComponents:
        return ADComponents(self.n_comp, self.n_chunks, self.comp_of.data_ptr(), self.members.data_ptr(),
                            self.comp_start.data_ptr(), self.chunk_start.data_ptr())


def components(dg: DeviceGraph) -> Components:
    """``ad_components_build``: connected components of the graph, grouped.
    Synchronises the current stream."""
    dev = dg.device
    g = dg.abi()
    n1 = max(1, dg.n)
    out = Components(0, 0, torch.empty(n1, dtype=torch.int32, device=dev),
                     torch.empty(n1, dtype=torch.int32, device=dev),
                     torch.empty(n1 + 1, dtype=torch.int64, device=dev),
                     torch.empty(n1 + 1, dtype=torch.int64, device=dev))
    ws = _workspace(lib.ad_components_workspace_size(ctypes.byref(g)), dev)
    nc, nch = ctypes.c_int64(0), ctypes.c_int64(0)
    _check(lib.ad_components_build(ctypes.byref(g), _ptr(out.comp_of), _ptr(out.members), _ptr(out.comp_start),
                                   _ptr(out.chunk_start), ctypes.byref(nc), ctypes.byref(nch), _ptr(ws), ws.numel(),
                                   _stream()))
    out.n_comp, out.n_chunks = nc.value, nch.value
    return out


def validate_graph(dg: DeviceGraph) -> None:
    """Structural check of the CSR on the device (synchronises)."""
    g = dg.abi()
    ws = _workspace(lib.ad_validate_workspace_size(ctypes.byref(g)), dg.device)
    _check(lib.ad_validate_graph(ctypes.byref(g), _ptr(ws), ws.numel(), _stream()))


# ----------------------------------------------------------------- relax ---

@dataclass
class RelaxResult:
    x: torch.Tensor          # [n, R] x^(k) minus the shift of each vertex's component
    minmax: torch.Tensor     # [2R] float64, of x^(k) itself
    shift: torch.Tensor      # [n_comp, R] (per component) or [R] float64
    ckpt: Optional[torch.Tensor]
    store: str
    comp: Optional[Components] = None
    opts: Optional[ADRelaxOpts] = None

    def x_true(self) -> torch.Tensor:
        """x^(k) itself in float64: the stored values plus their shifts."""
        x = self.x.to(torch.float64)
        if self.comp is None:
            return x + self.shift.reshape(1, -1)
        c = self.comp.comp_of[:x.shape[0]].to(torch.int64)
        sh = self.shift.reshape(-1, x.shape[1])[c.clamp(min=0)]
        return x + torch.where((c >= 0)[:, None], sh, torch.zeros_like(sh))

    @property
    def rho_dtype(self) -> torch.dtype:
        """Distances are FP64 for FP64 storage, else FP32."""
        return torch.float64 if self.store == "f64" else torch.float32


def relax_opts(R: int, k: int, omega: float = 0.5, seed: int = 0, graph_id: int = 0,
               store: str = "f32", fp32_tail: int = 2, ckpt_every: int = 0,
               rows_per_wave: int = 0, hub_degree: int = 0, fp64_tail: int = 0,
               comp: Optional[Components] = None) -> ADRelaxOpts:
    o = ADRelaxOpts(R, k, omega, seed, graph_id, _DTYPES[store], fp32_tail, ckpt_every,
                    rows_per_wave, hub_degree, fp64_tail, None)
    if comp is not None:
        o._comp_abi = comp.abi()             # kept alive with the options
        o.comp = ctypes.pointer(o._comp_abi)
    return o


def relax_workspace_bytes(dg: DeviceGraph, opts: ADRelaxOpts) -> int:
    g = dg.abi()
    return int(lib.ad_relax_workspace_size(ctypes.byref(g), ctypes.byref(opts)))


def relax(dg: DeviceGraph, R: int, k: int, omega: float = 0.5, seed: int = 0, graph_id: int = 0,
          store: str = "f32", x0: Optional[torch.Tensor] = None, fp32_tail: int = 2,
          ckpt_every: int = 0, rows_per_wave: int = 0, hub_degree: int = 0,
          ws: Optional[torch.Tensor] = None, out: Optional[RelaxResult] = None,
          fp64_tail: int = 0, per_component: bool = True) -> RelaxResult:
    """Start vectors + k JOR sweeps + rescale statistics (``ad_relax``).
    With ``per_component`` each connected component is centred by its own
    weighted mean (the graph's components are built once and cached); the
    last ``fp64_tail`` sweeps of FP32 / BF16 storage are stored in FP64, and
    x is then float64."""
    comp = dg.components() if per_component else None
    opts = relax_opts(R, k, omega, seed, graph_id, store, fp32_tail, ckpt_every, rows_per_wave,
                      hub_degree, fp64_tail, comp)
    g = dg.abi()
    dev = dg.device
    sdt = torch.float64 if store == "f64" else torch.float32
    xdt = torch.float64 if (store == "f64" or fp64_tail > 0) else torch.float32
    nsh = max(1, comp.n_comp) if comp is not None else 1
    if out is None:
        nck = int(lib.ad_relax_num_checkpoints(ctypes.byref(opts)))
        out = RelaxResult(
            x=torch.empty((dg.n, R), dtype=xdt, device=dev),
            minmax=torch.empty(2 * R, dtype=torch.float64, device=dev),
            shift=torch.empty((nsh, R) if comp is not None else (R,), dtype=torch.float64, device=dev),
            ckpt=torch.empty((nck, dg.n, R), dtype=sdt, device=dev) if nck else None,
            store=store)
    out.comp, out.opts = comp, opts
    if x0 is not None:
        if x0.dtype != sdt or tuple(x0.shape) != (dg.n, R) or not x0.is_contiguous():
            raise ValueError("x0 must be a contiguous [n, R] tensor of the storage dtype")
    if ws is None:
        ws = _workspace(lib.ad_relax_workspace_size(ctypes.byref(g), ctypes.byref(opts)), dev)
    _check(lib.ad_relax(ctypes.byref(g), ctypes.byref(opts), _ptr(x0), _ptr(out.x), _ptr(out.minmax),
                        _ptr(out.shift), _ptr(out.ckpt), _ptr(ws), ws.numel(), _stream()))
    return out


# -------------------------------------------------------------- distance ---

def edge_dist_workspace_bytes(dg: DeviceGraph) -> int:
    g = dg.abi()
    return int(lib.ad_edge_dist_workspace_size(ctypes.byref(g)))


def edge_dist(dg: DeviceGraph, x: torch.Tensor, minmax: torch.Tensor,
              out: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
              rho_dtype: Optional[torch.dtype] = None) -> torch.Tensor:
    """rho[m] = L2 distance of the rescaled vectors (``ad_edge_dist``);
    rho_dtype defaults to out's dtype, else x's."""
    R = x.shape[1]
    dt = AD_F64 if x.dtype == torch.float64 else AD_F32
    if rho_dtype is None:
        rho_dtype = out.dtype if out is not None else x.dtype
    if out is None:
        out = torch.empty(dg.m, dtype=rho_dtype, device=x.device)
    rt = AD_F64 if out.dtype == torch.float64 else AD_F32
    g = dg.abi()
    if ws is None:
        ws = _workspace(lib.ad_edge_dist_workspace_size(ctypes.byref(g)), x.device)
    _check(lib.ad_edge_dist(ctypes.byref(g), R, dt, _ptr(x), _ptr(minmax), rt, _ptr(out), _ptr(ws), ws.numel(),
                            _stream()))
    return out


def distances(dg: DeviceGraph, res: RelaxResult, out: Optional[torch.Tensor] = None,
              ws: Optional[torch.Tensor] = None) -> torch.Tensor:
    """``edge_dist`` of a relaxation: FP64 rho for FP64 storage, else FP32."""
    return edge_dist(dg, res.x, res.minmax, out=out, ws=ws, rho_dtype=res.rho_dtype)


def normalize_dist(dg: DeviceGraph, rho: torch.Tensor, by_strength: bool = True, eps: float = 0.0,
                   out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Algorithm 1's optional normalization as a distance (``ad_normalize_dist``):
    out_e = sqrt(rho_e^2 + eps) * sqrt(f_i f_j), f the weighted degree (or the
    degree); the normalized delta is 1 / out_e."""
    if out is None:
        out = torch.empty_like(rho)
    g = dg.abi()
    ws = _workspace(lib.ad_normalize_dist_workspace_size(ctypes.byref(g)), rho.device)
    dt = AD_F64 if rho.dtype == torch.float64 else AD_F32
    _check(lib.ad_normalize_dist(ctypes.byref(g), dt, _ptr(rho), 1 if by_strength else 0, float(eps), _ptr(out),
                                 _ptr(ws), ws.numel(), _stream()))
    return out


# ------------------------------------------------------------- selection ---

def budget_table(d_max: int, e: float) -> np.ndarray:
    out = np.zeros(d_max + 1, dtype=np.int32)
    _check(lib.ad_budget_table(d_max, float(e), out.ctypes.data_as(ctypes.c_void_p)))
    return out


def sparsify_workspace_bytes(dg: DeviceGraph) -> int:
    g = dg.abi()
    return int(lib.ad_sparsify_workspace_size(ctypes.byref(g)))


def sparsify(dg: DeviceGraph, rho: torch.Tensor, orient: int, e: Optional[float] = None,
             budget: Optional[torch.Tensor] = None, ws: Optional[torch.Tensor] = None,
             keep: Optional[torch.Tensor] = None, n_kept: Optional[torch.Tensor] = None):
    """Algorithm 3 at a fixed exponent (``ad_sparsify``); returns (keep, n_kept)."""
    dev = rho.device
    if budget is None:
        budget = torch.from_numpy(budget_table(dg.d_max, e)).to(dev)
    g = dg.abi()
    if ws is None:
        ws = _workspace(lib.ad_sparsify_workspace_size(ctypes.byref(g)), dev)
    if keep is None:
        keep = torch.empty(dg.m, dtype=torch.uint8, device=dev)
    if n_kept is None:
        n_kept = torch.empty(1, dtype=torch.int64, device=dev)
    dt = AD_F64 if rho.dtype == torch.float64 else AD_F32
    _check(lib.ad_sparsify(ctypes.byref(g), dt, _ptr(rho), orient, _ptr(budget), _ptr(keep), _ptr(n_kept),
                           _ptr(ws), ws.numel(), _stream()))
    return keep, n_kept


def sparsify_fit(dg: DeviceGraph, rho: torch.Tensor, orient: int, target: float,
                 ws: Optional[torch.Tensor] = None, keep: Optional[torch.Tensor] = None,
                 n_kept: Optional[torch.Tensor] = None):
    """Algorithm 3 with e fitted to a retention target (``ad_sparsify_fit``);
    returns (keep, n_kept, e).  Synchronises the current stream."""
    dev = rho.device
    g = dg.abi()
    if ws is None:
        ws = _workspace(lib.ad_sparsify_workspace_size(ctypes.byref(g)), dev)
    if keep is None:
        keep = torch.empty(dg.m, dtype=torch.uint8, device=dev)
    if n_kept is None:
        n_kept = torch.empty(1, dtype=torch.int64, device=dev)
    e_used = ctypes.c_double(-1.0)
    dt = AD_F64 if rho.dtype == torch.float64 else AD_F32
    _check(lib.ad_sparsify_fit(ctypes.byref(g), dt, _ptr(rho), orient, float(target), _ptr(keep),
                               _ptr(n_kept), ctypes.byref(e_used), _ptr(ws), ws.numel(), _stream()))
    return keep, n_kept, e_used.value


def sparsify_fit_both_workspace_bytes(dg: DeviceGraph) -> int:
    g = dg.abi()
    return int(lib.ad_sparsify_fit_both_workspace_size(ctypes.byref(g)))


def sparsify_fit_both(dg: DeviceGraph, rho: torch.Tensor, target: float,
                      ws: Optional[torch.Tensor] = None, keep_local: Optional[torch.Tensor] = None,
                      keep_global: Optional[torch.Tensor] = None, n_kept: Optional[torch.Tensor] = None):
    """LOCAL and GLOBAL fits from one ranking pass (``ad_sparsify_fit_both``);
    returns (keep_local, keep_global, n_kept[2], (e_local, e_global)).
    Synchronises the current stream."""
    dev = rho.device
    g = dg.abi()
    if ws is None:
        ws = _workspace(lib.ad_sparsify_fit_both_workspace_size(ctypes.byref(g)), dev)
    if keep_local is None:
        keep_local = torch.empty(dg.m, dtype=torch.uint8, device=dev)
    if keep_global is None:
        keep_global = torch.empty(dg.m, dtype=torch.uint8, device=dev)
    if n_kept is None:
        n_kept = torch.empty(2, dtype=torch.int64, device=dev)
    e_used = (ctypes.c_double * 2)(-1.0, -1.0)
    dt = AD_F64 if rho.dtype == torch.float64 else AD_F32
    _check(lib.ad_sparsify_fit_both(ctypes.byref(g), dt, _ptr(rho), float(target), _ptr(keep_local),
                                    _ptr(keep_global), _ptr(n_kept), e_used, _ptr(ws), ws.numel(), _stream()))
    return keep_local, keep_global, n_kept, (e_used[0], e_used[1])


# ------------------------------------------- distance and selection, fused --

def edge_dist_select_workspace_bytes(dg: DeviceGraph) -> int:
    g = dg.abi()
    return int(lib.ad_edge_dist_select_workspace_size(ctypes.byref(g)))


def _fused_prep(dg, x, rho, ws):
    if rho is None:
        rho = torch.empty(dg.m, dtype=torch.float32, device=x.device)
    if rho.dtype != torch.float32:
        raise ValueError("the fused calls write FP32 distances")
    g = dg.abi()
    if ws is None:
        ws = _workspace(lib.ad_edge_dist_select_workspace_size(ctypes.byref(g)), x.device)
    dt = AD_F64 if x.dtype == torch.float64 else AD_F32
    return g, rho, ws, dt


def edge_dist_sparsify(dg: DeviceGraph, res: RelaxResult, orient: int, e: Optional[float] = None,
                       budget: Optional[torch.Tensor] = None, rho: Optional[torch.Tensor] = None,
                       ws: Optional[torch.Tensor] = None, keep: Optional[torch.Tensor] = None,
                       n_kept: Optional[torch.Tensor] = None):
    """Distances and Algorithm 3 at a fixed exponent in one call
    (``ad_edge_dist_sparsify``); returns (rho, keep, n_kept)."""
    x = res.x
    dev = x.device
    g, rho, ws, dt = _fused_prep(dg, x, rho, ws)
    if budget is None:
        budget = torch.from_numpy(budget_table(dg.d_max, e)).to(dev)
    if keep is None:
        keep = torch.empty(dg.m, dtype=torch.uint8, device=dev)
    if n_kept is None:
        n_kept = torch.empty(1, dtype=torch.int64, device=dev)
    _check(lib.ad_edge_dist_sparsify(ctypes.byref(g), x.shape[1], dt, _ptr(x), _ptr(res.minmax), _ptr(rho), orient,
                                     _ptr(budget), _ptr(keep), _ptr(n_kept), _ptr(ws), ws.numel(), _stream()))
    return rho, keep, n_kept


def edge_dist_fit_both(dg: DeviceGraph, res: RelaxResult, target: float, rho: Optional[torch.Tensor] = None,
                       ws: Optional[torch.Tensor] = None, keep_local: Optional[torch.Tensor] = None,
                       keep_global: Optional[torch.Tensor] = None, n_kept: Optional[torch.Tensor] = None):
    """Distances and both fitted orders in one call (``ad_edge_dist_fit_both``);
    returns (rho, keep_local, keep_global, n_kept[2], (e_local, e_global)).
    Synchronises the current stream."""
    x = res.x
    dev = x.device
    g, rho, ws, dt = _fused_prep(dg, x, rho, ws)
    if keep_local is None:
        keep_local = torch.empty(dg.m, dtype=torch.uint8, device=dev)
    if keep_global is None:
        keep_global = torch.empty(dg.m, dtype=torch.uint8, device=dev)
    if n_kept is None:
        n_kept = torch.empty(2, dtype=torch.int64, device=dev)
    e_used = (ctypes.c_double * 2)(-1.0, -1.0)
    _check(lib.ad_edge_dist_fit_both(ctypes.byref(g), x.shape[1], dt, _ptr(x), _ptr(res.minmax), _ptr(rho),
                                     float(target), _ptr(keep_local), _ptr(keep_global), _ptr(n_kept), e_used,
                                     _ptr(ws), ws.numel(), _stream()))
    return rho, keep_local, keep_global, n_kept, (e_used[0], e_used[1])


# --------------------------------------------------------------- adjoint ---

def relax_backward(dg: DeviceGraph, res: RelaxResult, R: int, k: int, grad_rho: torch.Tensor,
                   omega: float = 0.5, seed: int = 0, graph_id: int = 0, ckpt_every: int = 5,
                   ws: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """dL/dw_e given dL/drho_e (``ad_relax_backward``)."""
    opts = relax_opts(R, k, omega, seed, graph_id, "f32", 2, ckpt_every, comp=res.comp)
    g = dg.abi()
    if ws is None:
        ws = _workspace(lib.ad_relax_backward_workspace_size(ctypes.byref(g), ctypes.byref(opts)), dg.device)
    if out is None:
        out = torch.empty(dg.m, dtype=torch.float32, device=dg.device)
    _check(lib.ad_relax_backward(ctypes.byref(g), ctypes.byref(opts), _ptr(res.ckpt), _ptr(res.x),
                                 _ptr(res.minmax), _ptr(res.shift), _ptr(grad_rho), _ptr(out), _ptr(ws),
                                 ws.numel(), _stream()))
    return out


def edge_to_entries(dg: DeviceGraph, w_edge: torch.Tensor) -> torch.Tensor:
    """CSR-order weights w_entries[p] = w_edge[eid[p]] (``ad_edge_to_entries``)."""
    out = torch.empty(2 * dg.m, dtype=torch.float32, device=w_edge.device)
    g = dg.abi()
    _check(lib.ad_edge_to_entries(ctypes.byref(g), _ptr(w_edge.contiguous()), _ptr(out), _stream()))
    return out


class AlgDist(torch.autograd.Function):
    """rho = AlgDist.apply(w_edge, dg, R, k, omega, seed, ckpt_every).

    Forward: ad_relax (FP32, checkpoints every ``ckpt_every`` sweeps) and
    ad_edge_dist with the edge weights ``w_edge`` [m].  Backward:
    ad_relax_backward gives dL/dw_e from dL/drho_e."""

    @staticmethod
    def forward(ctx, w_edge, dg, R, k, omega=0.5, seed=0, ckpt_every=5):
        w_edge = w_edge.detach().contiguous().float()
        dgw = dg.with_weights(edge_to_entries(dg, w_edge))
        res = relax(dgw, R, k, omega, seed, store="f32", ckpt_every=ckpt_every)
        rho = distances(dgw, res)
        ctx.dgw, ctx.res = dgw, res
        ctx.args = (R, k, omega, seed, ckpt_every)
        return rho

    @staticmethod
    def backward(ctx, grad_rho):
        R, k, omega, seed, ckpt_every = ctx.args
        gw = relax_backward(ctx.dgw, ctx.res, R, k, grad_rho.contiguous().float(), omega, seed,
                            ckpt_every=ckpt_every)
        return gw, None, None, None, None, None, None


# --------------------------------------------------------------- batches ---

class Batch:
    """Many graphs relaxed, measured and sparsified (fixed e) as one captured
    launch sequence (``ad_batch_*``).  Graph q uses start-vector key word
    graph_id + q; results equal running each graph alone, bit for bit."""

    def __init__(self, graphs, R: int, k: int, omega: float = 0.5, seed: int = 0, graph_id: int = 0,
                 orient: int = AD_LOCAL, e: float = 0.5, autotune: bool = True,
                 rows_per_wave: int = 0, hub_degree: int = 0, fp64_tail: int = 0):
        self.graphs = list(graphs)        # keep the inputs alive while packing
        self.G = len(self.graphs)
        self.R = R
        arr = (ADGraph * self.G)(*[dg.abi() for dg in self.graphs])
        opts = relax_opts(R, k, omega, seed, graph_id, "f32", 2, 0, rows_per_wave, hub_degree, fp64_tail)
        bo = ADBatchOpts(orient, float(e), 1 if autotune else 0)
        h = ctypes.c_void_p()
        _check(lib.ad_batch_create(self.G, arr, ctypes.byref(opts), ctypes.byref(bo), ctypes.byref(h), _stream()))
        self._h = h
        ro = np.zeros(self.G + 1, dtype=np.int64)
        eo = np.zeros(self.G + 1, dtype=np.int64)
        rpw = ctypes.c_int32()
        _check(lib.ad_batch_info(h, ro.ctypes.data_as(ctypes.c_void_p), eo.ctypes.data_as(ctypes.c_void_p),
                                 ctypes.byref(rpw)))
        self.row_off, self.edge_off, self.rows_per_wave = ro, eo, rpw.value
        dev = self.graphs[0].device
        self.rho = torch.empty(int(eo[-1]), dtype=torch.float32, device=dev)
        self.keep = torch.empty(int(eo[-1]), dtype=torch.uint8, device=dev)
        self.n_kept = torch.empty(self.G, dtype=torch.int64, device=dev)
        self.minmax = torch.empty((self.G, 2 * R), dtype=torch.float64, device=dev)

    def run(self, captured: bool = True) -> None:
        fn = lib.ad_batch_run if captured else lib.ad_batch_run_uncaptured
        _check(fn(self._h, _stream()))

    def fetch(self):
        """Copy the last run's outputs into this object's tensors; returns
        (rho, keep, n_kept, minmax) for the packed edge ranges edge_off."""
        _check(lib.ad_batch_copy_results(self._h, _ptr(self.rho), _ptr(self.keep), _ptr(self.n_kept),
                                         _ptr(self.minmax), _stream()))
        return self.rho, self.keep, self.n_kept, self.minmax

    def close(self) -> None:
        if self._h:
            lib.ad_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------ whole path ---

def sparsify_graph(dg: DeviceGraph, R: int, k: int, orient: int, e: Optional[float] = None,
                   target: Optional[float] = None, omega: float = 0.5, seed: int = 0,
                   store: str = "f32", fp64_tail: int = 2):
    """Algorithm 1 then Algorithm 3 on one graph (components centred apart,
    the last ``fp64_tail`` sweeps of FP32 storage in FP64).  Returns a dict
    with rho, keep, n_kept and the exponent used."""
    res = relax(dg, R, k, omega, seed, store=store, fp64_tail=0 if store == "f64" else fp64_tail)
    rho = distances(dg, res)
    if target is not None:
        keep, n_kept, e_used = sparsify_fit(dg, rho, orient, target)
    else:
        keep, n_kept = sparsify(dg, rho, orient, e)
        e_used = e
    return {"rho": rho, "keep": keep, "n_kept": n_kept, "e": e_used, "relax": res}


def sparsify_binned_workspace_bytes(dg: DeviceGraph) -> int:
    g = dg.abi()
    return int(lib.ad_sparsify_binned_workspace_size(ctypes.byref(g)))


def sparsify_binned(dg: DeviceGraph, rho: torch.Tensor, seed: int, e: float = 0.5, target: float = 0.0,
                    graph_id: int = 0, ws: Optional[torch.Tensor] = None, keep: Optional[torch.Tensor] = None,
                    n_kept: Optional[torch.Tensor] = None):
    """Algorithm 4, selection with binning (``ad_sparsify_binned``): at the
    fixed exponent e, or with e fitted to `target` when target > 0.  Returns
    (keep, n_kept, e_used).  Synchronises the current stream."""
    dev = rho.device
    g = dg.abi()
    if ws is None:
        ws = _workspace(lib.ad_sparsify_binned_workspace_size(ctypes.byref(g)), dev)
    if keep is None:
        keep = torch.empty(dg.m, dtype=torch.uint8, device=dev)
    if n_kept is None:
        n_kept = torch.empty(1, dtype=torch.int64, device=dev)
    e_used = ctypes.c_double(-1.0)
    dt = AD_F64 if rho.dtype == torch.float64 else AD_F32
    _check(lib.ad_sparsify_binned(ctypes.byref(g), dt, _ptr(rho), int(seed) & (2 ** 64 - 1),
                                  int(graph_id) & (2 ** 64 - 1), float(e), float(target), _ptr(keep),
                                  _ptr(n_kept), ctypes.byref(e_used), _ptr(ws), ws.numel(), _stream()))
    return keep, n_kept, e_used.value


# ---------------------------------------------------------------- ingest ---

_ORDERS = {"listed": 0, "degree": 1, "rcm": 2}


def ingest(n: int, u: torch.Tensor, v: torch.Tensor, w: Optional[torch.Tensor] = None,
           orig_id: Optional[torch.Tensor] = None, by_degree: bool = True,
           entry_ids: bool = True, order: Optional[str] = None) -> DeviceGraph:
    """An undirected edge list on the device into a ``DeviceGraph``
    (``ad_ingest``): self-loops dropped, repeated pairs merged (weights
    summed), vertices stored by decreasing degree unless ``by_degree`` is
    False; ``order`` ("listed", "degree" or "rcm", reverse Cuthill-McKee)
    overrides ``by_degree``.  Synchronises the current stream."""
    code = _ORDERS[order] if order is not None else (1 if by_degree else 0)
    dev = u.device
    m_in = int(u.numel())
    u = u.to(torch.int32).contiguous()
    v = v.to(torch.int32).contiguous()
    if w is not None:
        w = w.to(torch.float32).contiguous()
    row_ptr = torch.empty(n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(max(1, 2 * m_in), dtype=torch.int32, device=dev)
    eid = torch.empty(max(1, 2 * m_in), dtype=torch.int32, device=dev)
    w_out = torch.empty(max(1, 2 * m_in), dtype=torch.float32, device=dev) if w is not None else None
    orig = torch.empty(max(1, n), dtype=torch.int32, device=dev)
    ws = _workspace(lib.ad_ingest_workspace_size(n, m_in), dev)
    m = ctypes.c_int64(0)
    d_max = ctypes.c_int32(0)
    dropped = ctypes.c_int64(0)
    _check(lib.ad_ingest(n, m_in, _ptr(u), _ptr(v), _ptr(w), _ptr(orig_id), code, _ptr(row_ptr),
                         _ptr(col), _ptr(w_out), _ptr(eid), _ptr(orig), ctypes.byref(m), ctypes.byref(d_max),
                         ctypes.byref(dropped), _ptr(ws), ws.numel(), _stream()))
    nnz = 2 * m.value
    dg = DeviceGraph(n=n, m=m.value, d_max=d_max.value, row_ptr=row_ptr, col=col[:nnz], w=None if w is None else
                     w_out[:nnz], eid=eid[:nnz], orig_id=orig[:n])
    dg.n_dropped = dropped.value      # type: ignore[attr-defined]
    if entry_ids and dg.m > 0:
        dg.col_orig = torch.empty(2 * dg.m, dtype=torch.int32, device=dev)
        gs = dg.abi()
        _check(lib.ad_graph_col_orig(ctypes.byref(gs), _ptr(dg.col_orig), _stream()))
    return dg


# ------------------------------------------------------------ properties ---

def subgraph(dg: DeviceGraph, keep: torch.Tensor, entry_ids: bool = True) -> DeviceGraph:
    """The sparsified graph (V, {e : keep[e]}) as a ``DeviceGraph``
    (``ad_subgraph``); ``orig_edge`` maps each entry to the original edge id.
    Synchronises the current stream."""
    dev = keep.device
    g = dg.abi()
    nnz = max(1, 2 * dg.m)
    row_ptr = torch.empty(dg.n + 1, dtype=torch.int64, device=dev)
    col = torch.empty(nnz, dtype=torch.int32, device=dev)
    eid = torch.empty(nnz, dtype=torch.int32, device=dev)
    oe = torch.empty(nnz, dtype=torch.int32, device=dev)
    w = torch.empty(nnz, dtype=torch.float32, device=dev) if dg.w is not None else None
    ws = _workspace(lib.ad_subgraph_workspace_size(ctypes.byref(g)), dev)
    ms = ctypes.c_int64(0)
    _check(lib.ad_subgraph(ctypes.byref(g), _ptr(keep.to(torch.uint8).contiguous()), _ptr(row_ptr), _ptr(col),
                           _ptr(w), _ptr(eid), _ptr(oe), ctypes.byref(ms), _ptr(ws), ws.numel(), _stream()))
    q = 2 * ms.value
    deg_max = int((row_ptr[1:] - row_ptr[:-1]).max().item()) if dg.n > 0 else 0
    sg = DeviceGraph(n=dg.n, m=ms.value, d_max=deg_max, row_ptr=row_ptr, col=col[:q],
                     w=None if w is None else w[:q], eid=eid[:q], orig_id=dg.orig_id)
    sg.orig_edge = oe[:q]      # type: ignore[attr-defined]
    if entry_ids and sg.m > 0:
        sg.col_orig = torch.empty(q, dtype=torch.int32, device=dev)
        gs = sg.abi()
        _check(lib.ad_graph_col_orig(ctypes.byref(gs), _ptr(sg.col_orig), _stream()))
    return sg


def graph_properties(dg: DeviceGraph) -> dict:
    """Triangles, clustering (per vertex and C_G of Eq. cc) and components
    (``ad_graph_properties``).  Synchronises the current stream."""
    dev = dg.device
    g = dg.abi()
    n = max(1, dg.n)
    lam = torch.empty(n, dtype=torch.int64, device=dev)
    c = torch.empty(n, dtype=torch.float64, device=dev)
    comp = torch.empty(n, dtype=torch.int32, device=dev)
    summary = (ctypes.c_double * 2)()
    ws = _workspace(lib.ad_graph_properties_workspace_size(ctypes.byref(g)), dev)
    _check(lib.ad_graph_properties(ctypes.byref(g), _ptr(lam), _ptr(c), _ptr(comp), summary, _ptr(ws), ws.numel(),
                                   _stream()))
    return {"lambda": lam[:dg.n], "c": c[:dg.n], "comp": comp[:dg.n], "C_G": summary[0],
            "n_components": int(summary[1])}


def spearman(x: torch.Tensor, y: torch.Tensor) -> float:
    """Spearman rank correlation by the Preliminaries' formula (``ad_spearman``)."""
    x = x.to(torch.float64).contiguous()
    y = y.to(torch.float64).contiguous()
    n = x.numel()
    ws = _workspace(lib.ad_spearman_workspace_size(n), x.device)
    rho = ctypes.c_double(0.0)
    _check(lib.ad_spearman(n, _ptr(x), _ptr(y), ctypes.byref(rho), _ptr(ws), ws.numel(), _stream()))
    return rho.value


def compare_properties(dg: DeviceGraph, keep: torch.Tensor) -> dict:
    """The comparisons of Section 6 that need no external package
    (``ad_compare_properties``): the sparsified graph's C_G and component
    count against the original's (and their ratio), and Spearman
    correlations of the degree and clustering distributions.  Synchronises
    the current stream."""
    g = dg.abi()
    ws = _workspace(lib.ad_compare_properties_workspace_size(ctypes.byref(g)), dg.device)
    out = (ctypes.c_double * 8)()
    _check(lib.ad_compare_properties(ctypes.byref(g), _ptr(keep.to(torch.uint8).contiguous()),
                                     ctypes.cast(out, ctypes.c_void_p), _ptr(ws), ws.numel(), _stream()))
    return {"m": dg.m, "m_kept": int(out[0]), "C_G": out[1], "C_G_sparse": out[2],
            "components": int(out[3]), "components_sparse": int(out[4]), "comp_ratio": out[5],
            "degree_spearman": out[6], "clustering_spearman": out[7]}


# ------------------------------------------------------------ multilevel ---

def ml_aggregate(dg: DeviceGraph, rho: torch.Tensor, eps: float = 1e-12, theta: float = 0.5):
    """One coarsening step of Algorithm 6 (``ad_ml_aggregate``): returns
    (agg int32 [n], is_seed uint8 [n], n_coarse).  Synchronises the current
    stream."""
    dev = rho.device
    g = dg.abi()
    ws = _workspace(lib.ad_ml_aggregate_workspace_size(ctypes.byref(g)), dev)
    agg = torch.empty(max(1, dg.n), dtype=torch.int32, device=dev)
    is_seed = torch.empty(max(1, dg.n), dtype=torch.uint8, device=dev)
    nc = ctypes.c_int64(0)
    dt = AD_F64 if rho.dtype == torch.float64 else AD_F32
    _check(lib.ad_ml_aggregate(ctypes.byref(g), dt, _ptr(rho.contiguous()), float(eps), float(theta), _ptr(agg),
                               _ptr(is_seed), ctypes.byref(nc), _ptr(ws), ws.numel(), _stream()))
    return agg[:dg.n], is_seed[:dg.n], nc.value


def ml_level_span(n_levels: int, span: int, segment: int, value: float) -> np.ndarray:
    """The level-span ratio vector (``ad_ml_level_span``), coarsest level first."""
    out = (ctypes.c_double * max(1, n_levels))()
    _check(lib.ad_ml_level_span(n_levels, span, segment, float(value), ctypes.cast(out, ctypes.c_void_p)))
    return np.array(out[:n_levels], dtype=np.float64)


def ml_sparsify(dg: DeviceGraph, R: int, k: int, e_levels=None, omega: float = 0.5, seed: int = 0,
                graph_id: int = 0, levels: int = 8, n_min: int = 1000, store: str = "f32", eps: float = 1e-12,
                theta: float = 0.5, bin_seed: int = 0, fit: bool = False, span: int = 0, segment: int = 0,
                span_value: float = 0.3, keep: Optional[torch.Tensor] = None, fp64_tail: int = 2):
    """Algorithm 6, MLSparsify (``ad_ml_sparsify``).  ``e_levels``: the
    per-level ratio vector, coarsest level first, one entry per level (a
    negative entry skips SparsifyB at that level); exponents, or retention
    targets with ``fit``.  ``span > 0`` uses the level-span vector of the
    levels reached instead.  FP32 relaxations store their last ``fp64_tail``
    sweeps in FP64.  Returns (keep uint8 [m], n_kept, depth).  Synchronises
    the current stream."""
    if span > 0:
        ev = [0.0] * max(levels, 1)
    else:
        if e_levels is None:
            raise ValueError("ml_sparsify needs e_levels, or span > 0 for the level-span rule")
        ev = [float(x) for x in np.atleast_1d(np.asarray(e_levels, dtype=np.float64))]
        if len(ev) != levels:
            raise ValueError(f"e_levels has {len(ev)} entries for {levels} levels")
    e_arr = (ctypes.c_double * len(ev))(*ev)
    o = ADMLOpts(R=R, k=k, omega=omega, seed=int(seed) & (2 ** 64 - 1), graph_id=int(graph_id) & (2 ** 64 - 1),
                 store=_DTYPES[store], levels=levels, n_min=n_min,
                 e_host=ctypes.cast(e_arr, ctypes.c_void_p).value, eps=eps, theta=theta,
                 bin_seed=int(bin_seed) & (2 ** 64 - 1), fit=int(fit), span=span, segment=segment,
                 span_value=span_value, fp64_tail=fp64_tail if store == "f32" else 0)
    g = dg.abi()
    if keep is None:
        keep = torch.empty(max(1, dg.m), dtype=torch.uint8, device=dg.row_ptr.device)
    kept = ctypes.c_int64(0)
    depth = ctypes.c_int32(0)
    _check(lib.ad_ml_sparsify(ctypes.byref(g), ctypes.byref(o), _ptr(keep), ctypes.byref(kept), ctypes.byref(depth),
                              _stream()))
    return keep[:dg.m], kept.value, depth.value
