"""MI355X colour-coding tree counter: thin Python binding over libcc.so (include/cc.h).

The binding only marshals arguments: device memory comes from PyTorch tensors, streams are
PyTorch's current HIP stream, and every step of the counting path runs in the library's HIP
kernels. There is no CPU fallback: if libcc.so is missing or a tensor is not on the GPU, the
calls raise.

Verbs (Section 2 "Subgraph-counting problem" and Algorithm 1 of the paper):
  Plan(edges)           load tree template (partition into active/passive sub-templates)
  Graph(row_ptr, col)   load CSR graph (validated, work lists built)
  colour(graph, k, ..)  random colourings
  count(plan, graph, colours)   colourful embedding counts X per colouring
  estimate(plan, X)     mean(X) * k^k / k! / |Aut(T)|
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass
from functools import lru_cache

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libcc.so")

CC_PLAN_CENTRE_SMALLEST = 1
CC_PLAN_NO_SHARING = 2
CC_GRAPH_TRUST = 1
CC_MAX_PACKED = 4096  # largest B of one packed count

_STATUS = {0: "CC_OK", -1: "CC_EINVAL", -2: "CC_ERANGE", -3: "CC_ENOMEM", -4: "CC_ENOSPC",
           -5: "CC_EDEVICE", -6: "CC_EINTERNAL"}


class CCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class _PlanInfo(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("root", ctypes.c_int32), ("n_splits", ctypes.c_int32),
                ("aut", ctypes.c_double), ("units_per_edge", ctypes.c_int64),
                ("table3_memory", ctypes.c_int64), ("table3_compute", ctypes.c_int64),
                ("gather_doubles_per_edge", ctypes.c_int64), ("combine_fma_per_vertex", ctypes.c_int64),
                ("peak_live_columns", ctypes.c_int64), ("device_bytes", ctypes.c_size_t)]


class _SplitMaps(ctypes.Structure):
    _fields_ = [("act", ctypes.c_int32), ("pas", ctypes.c_int32), ("out", ctypes.c_int32),
                ("split_off", ctypes.c_int64), ("fold_off", ctypes.c_int64), ("mask_off", ctypes.c_int64),
                ("full_off", ctypes.c_int64), ("emap_off", ctypes.c_int64),
                ("proj_src_off", ctypes.c_int64), ("proj_fold_off", ctypes.c_int64), ("Wn", ctypes.c_int32)]


class _TableDesc(ctypes.Structure):
    _fields_ = [("size", ctypes.c_int32), ("width", ctypes.c_int32), ("stride", ctypes.c_int64),
                ("offset", ctypes.c_int64)]


class _BudgetInfo(ctypes.Structure):
    _fields_ = [("workspace_bytes", ctypes.c_size_t), ("host_bytes", ctypes.c_size_t),
                ("parked_tables", ctypes.c_int32), ("proj_classes", ctypes.c_int32),
                ("arena_columns", ctypes.c_int64),
                ("unbounded_columns", ctypes.c_int64)]


class _GraphInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz", ctypes.c_int64), ("max_degree", ctypes.c_int64),
                ("n_light", ctypes.c_int64), ("n_hubs", ctypes.c_int64), ("n_chunks", ctypes.c_int64),
                ("hub_threshold", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("cols_per_lane", ctypes.c_int32), ("proj_classes", ctypes.c_int32),
                ("packed_tile", ctypes.c_int32)]


class _Instance(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("graph", ctypes.c_void_p), ("colours_dev", ctypes.c_void_p),
                ("X_dev", ctypes.c_void_p), ("vertex_dev", ctypes.c_void_p)]


CC_BATCH_LEVELS = 1


def CC_BATCH_SHARE(d: int) -> int:
    return (d & 0xFF) << 8


class _Tuning(ctypes.Structure):
    _fields_ = [("hub_threshold", ctypes.c_int32), ("chunk", ctypes.c_int32),
                ("cols_per_lane", ctypes.c_int32), ("proj_classes", ctypes.c_int32),
                ("packed_tile", ctypes.c_int32)]


EXPORTS = ["cc_last_error", "cc_plan_create", "cc_plan_info_get", "cc_plan_split_get",
           "cc_plan_bind_device", "cc_plan_destroy", "cc_entry_order", "cc_plan_split_maps",
           "cc_plan_constants_get", "cc_graph_workspace_bytes", "cc_graph_prepare",
           "cc_graph_info_get", "cc_graph_release", "cc_color", "cc_count_workspace_bytes", "cc_count",
           "cc_count_inspect", "cc_plan_table_get", "cc_count_projection", "cc_count_noalloc",
           "cc_count_budget_plan", "cc_count_budget",
           "cc_count_packed_workspace_bytes", "cc_count_packed", "cc_stream_check", "cc_iterations",
           "cc_multi_create", "cc_multi_info_get", "cc_multi_step_get", "cc_multi_destroy",
           "cc_count_packed_multi_workspace_bytes",
           "cc_count_packed_multi", "cc_count_packed_multi_persistent_workspace_bytes",
           "cc_count_packed_multi_persistent",
           "cc_estimate", "cc_estimate_median_of_means", "cc_profile_enable", "cc_profile_read",
           "cc_batch_create", "cc_batch_workspace_bytes", "cc_batch_run", "cc_batch_check", "cc_batch_destroy"]


@lru_cache(maxsize=1)
def lib() -> ctypes.CDLL:
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build() or "
                           "python paper_1804_09764_amd/_build.py")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    I32, I64, U32, U64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "cc_last_error": (ctypes.c_char_p, []),
        "cc_plan_create": (ctypes.c_int, [I32, P, I32, U32, ctypes.POINTER(P)]),
        "cc_plan_info_get": (ctypes.c_int, [P, ctypes.POINTER(_PlanInfo)]),
        "cc_plan_split_get": (ctypes.c_int, [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32),
                                             ctypes.POINTER(I32)]),
        "cc_plan_bind_device": (ctypes.c_int, [P, P, ctypes.c_size_t, P]),
        "cc_plan_destroy": (None, [P]),
        "cc_entry_order": (ctypes.c_int, [I32, I32, P, I64]),
        "cc_plan_split_maps": (ctypes.c_int, [P, I32, ctypes.POINTER(_SplitMaps)]),
        "cc_plan_constants_get": (ctypes.c_int, [P, P, ctypes.c_size_t]),
        "cc_graph_workspace_bytes": (ctypes.c_int, [I64, I64, P, ctypes.POINTER(ctypes.c_size_t)]),
        "cc_graph_prepare": (ctypes.c_int, [I64, I64, P, P, P, ctypes.c_size_t, P, U32, P,
                                            ctypes.POINTER(P)]),
        "cc_graph_info_get": (ctypes.c_int, [P, ctypes.POINTER(_GraphInfo)]),
        "cc_graph_release": (None, [P]),
        "cc_color": (ctypes.c_int, [P, I32, U64, U64, I32, P, P]),
        "cc_count_workspace_bytes": (ctypes.c_int, [P, P, ctypes.POINTER(ctypes.c_size_t)]),
        "cc_count": (ctypes.c_int, [P, P, P, I32, P, ctypes.c_size_t, P, P, P]),
        "cc_count_inspect": (ctypes.c_int, [P, P, P, I32, P, ctypes.c_size_t, P, P]),
        "cc_plan_table_get": (ctypes.c_int, [P, P, I32, ctypes.POINTER(_TableDesc)]),
        "cc_count_projection": (ctypes.c_int, [P, P, P, I32]),
        "cc_count_noalloc": (ctypes.c_int, [P, P, P, I32, P, P, P]),
        "cc_count_budget_plan": (ctypes.c_int, [P, P, ctypes.c_size_t, ctypes.POINTER(_BudgetInfo)]),
        "cc_count_budget": (ctypes.c_int, [P, P, P, I32, ctypes.c_size_t, P, ctypes.c_size_t, P, ctypes.c_size_t,
                                           P, P, P]),
        "cc_count_packed_workspace_bytes": (ctypes.c_int, [P, P, I32, ctypes.POINTER(ctypes.c_size_t)]),
        "cc_count_packed": (ctypes.c_int, [P, P, P, I32, P, ctypes.c_size_t, P, P, P]),
        "cc_stream_check": (ctypes.c_int, [P]),
        "cc_multi_create": (ctypes.c_int, [I32, P, ctypes.POINTER(P)]),
        "cc_multi_info_get": (ctypes.c_int, [P, ctypes.POINTER(I32), ctypes.POINTER(I64), ctypes.POINTER(I32)]),
        "cc_multi_step_get": (ctypes.c_int, [P, I32, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
        "cc_multi_destroy": (None, [P]),
        "cc_count_packed_multi_workspace_bytes": (ctypes.c_int, [P, P, I32, ctypes.POINTER(ctypes.c_size_t)]),
        "cc_count_packed_multi": (ctypes.c_int, [P, P, P, I32, P, ctypes.c_size_t, P, P]),
        "cc_count_packed_multi_persistent_workspace_bytes": (ctypes.c_int, [P, P, I32,
                                                                            ctypes.POINTER(ctypes.c_size_t)]),
        "cc_count_packed_multi_persistent": (ctypes.c_int, [P, P, P, I32, P, ctypes.c_size_t, P, P]),
        "cc_iterations": (ctypes.c_int, [I32, ctypes.c_double, ctypes.c_double, ctypes.POINTER(I64),
                                         ctypes.POINTER(I32)]),
        "cc_estimate": (ctypes.c_int, [P, P, I32, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double)]),
        "cc_estimate_median_of_means": (ctypes.c_int, [P, P, I32, I32, ctypes.POINTER(ctypes.c_double)]),
        "cc_profile_enable": (ctypes.c_int, [P, I32]),
        "cc_batch_create": (ctypes.c_int, [I32, P, U32, ctypes.POINTER(P)]),
        "cc_batch_workspace_bytes": (ctypes.c_int, [P, ctypes.POINTER(ctypes.c_size_t)]),
        "cc_batch_run": (ctypes.c_int, [P, P, ctypes.c_size_t, P]),
        "cc_batch_check": (ctypes.c_int, [P, P]),
        "cc_batch_destroy": (None, [P]),
        "cc_profile_read": (ctypes.c_int, [P, I32, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


def _check(rc: int):
    if rc != 0:
        raise CCError(rc, lib().cc_last_error().decode())


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _dev_ptr(t, dtype=None, name="tensor"):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


@dataclass
class PlanInfo:
    k: int
    root: int
    n_splits: int
    aut: float
    units_per_edge: int
    table3_memory: int
    table3_compute: int
    gather_doubles_per_edge: int
    combine_fma_per_vertex: int
    peak_live_columns: int
    device_bytes: int


class Plan:
    """A tree template and its partition (host); `bind()` uploads its constant tables to the GPU."""

    def __init__(self, edges, root: int = -1, flags: int = 0, bind: bool = True, device=None):
        e = np.ascontiguousarray(np.asarray(edges, dtype=np.int32).reshape(-1, 2))
        self.edges = e
        self.k = e.shape[0] + 1
        h = ctypes.c_void_p()
        _check(lib().cc_plan_create(self.k, e.ctypes.data if e.size else None, root, flags,
                                    ctypes.byref(h)))
        self._h = h
        self._dev = None
        inf = _PlanInfo()
        _check(lib().cc_plan_info_get(self._h, ctypes.byref(inf)))
        self.info = PlanInfo(*(getattr(inf, f[0]) for f in _PlanInfo._fields_))
        self.splits = []
        for i in range(self.info.n_splits):
            s, a, p = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            _check(lib().cc_plan_split_get(self._h, i, ctypes.byref(s), ctypes.byref(a), ctypes.byref(p)))
            self.splits.append((s.value, a.value, p.value))
        if bind:
            self.bind(device)

    def bind(self, device=None, stream=None):
        import torch
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        nbytes = max(int(self.info.device_bytes), 256)
        self._dev = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        _check(lib().cc_plan_bind_device(self._h, ctypes.c_void_p(self._dev.data_ptr()), nbytes, _stream(stream)))
        return self

    @property
    def handle(self):
        return self._h

    def split_maps(self, i: int) -> dict:
        """Table ids and map offsets of split i in the plan's constants (cc_plan_split_maps)."""
        m = _SplitMaps()
        _check(lib().cc_plan_split_maps(self._h, i, ctypes.byref(m)))
        return {f[0]: getattr(m, f[0]) for f in _SplitMaps._fields_}

    def constants(self) -> np.ndarray:
        """Host copy of the plan's device constants (uint8; cc_plan_constants_get)."""
        out = np.zeros(max(self.info.device_bytes, 1), dtype=np.uint8)
        _check(lib().cc_plan_constants_get(self._h, out.ctypes.data, out.nbytes))
        return out[:self.info.device_bytes]

    def profile(self, enable: bool = True):
        """Record per-split kernel times of later counts with this plan (HIP events)."""
        _check(lib().cc_profile_enable(self._h, 1 if enable else 0))

    def profile_read(self):
        """(gather_ms[n_splits], finish_ms[n_splits], colourings[n_splits]) recorded so far."""
        n = self.info.n_splits
        g = np.zeros(n, dtype=np.float64)
        f = np.zeros(n, dtype=np.float64)
        c = np.zeros(n, dtype=np.int64)
        _check(lib().cc_profile_read(self._h, n, g.ctypes.data if n else None, f.ctypes.data if n else None,
                                     c.ctypes.data if n else None))
        return g, f, c

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().cc_plan_destroy(h)
            except Exception:
                pass
            self._h = None


class Graph:
    """A CSR graph resident on the GPU (int64 row_ptr, int32 col) with its prepared work lists."""

    def __init__(self, row_ptr, col, hub_threshold: int = 0, chunk: int = 0, trust: bool = False,
                 cols_per_lane: int = 0, proj_classes: int = 0, packed_tile: int = 0, stream=None):
        import torch
        self.row_ptr = row_ptr
        self.col = col
        n = row_ptr.numel() - 1
        nnz = col.numel()
        self.n, self.nnz = n, nnz
        tun = _Tuning(hub_threshold, chunk, cols_per_lane, proj_classes, packed_tile)
        nb = ctypes.c_size_t()
        _check(lib().cc_graph_workspace_bytes(n, nnz, ctypes.byref(tun), ctypes.byref(nb)))
        self._ws = torch.empty(max(nb.value, 256), dtype=torch.uint8, device=row_ptr.device)
        h = ctypes.c_void_p()
        _check(lib().cc_graph_prepare(n, nnz, _dev_ptr(row_ptr, torch.int64, "row_ptr"),
                                      _dev_ptr(col, torch.int32, "col") if nnz else None,
                                      ctypes.c_void_p(self._ws.data_ptr()), self._ws.numel(),
                                      ctypes.byref(tun), CC_GRAPH_TRUST if trust else 0, _stream(stream),
                                      ctypes.byref(h)))
        self._h = h
        gi = _GraphInfo()
        _check(lib().cc_graph_info_get(self._h, ctypes.byref(gi)))
        self.info = {f[0]: getattr(gi, f[0]) for f in _GraphInfo._fields_}

    @classmethod
    def from_numpy(cls, row_ptr, col, device="cuda", **kw):
        import torch
        rp = torch.from_numpy(np.ascontiguousarray(row_ptr, dtype=np.int64)).to(device)
        cl = torch.from_numpy(np.ascontiguousarray(col, dtype=np.int32)).to(device)
        return cls(rp, cl, **kw)

    @property
    def handle(self):
        return self._h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().cc_graph_release(h)
            except Exception:
                pass
            self._h = None


def colour(graph: Graph, k: int, seed: int, first_iter: int = 0, B: int = 1, out=None, stream=None):
    """B counter-based random colourings, uint8 tensor [B, n] on the graph's device."""
    import torch
    if out is None:
        out = torch.empty((B, graph.n), dtype=torch.uint8, device=graph.row_ptr.device)
    _check(lib().cc_color(graph.handle, k, seed, first_iter, B, _dev_ptr(out, torch.uint8, "colours"),
                          _stream(stream)))
    return out


class Workspace:
    """Caller-owned count workspace (reused across calls with the same plan/graph shapes)."""

    def __init__(self):
        self.buf = None

    def get(self, nbytes: int, device):
        import torch
        if self.buf is None or self.buf.numel() < nbytes or self.buf.device != device:
            self.buf = None
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        return self.buf


def count_workspace_bytes(plan: Plan, graph: Graph) -> int:
    nb = ctypes.c_size_t()
    _check(lib().cc_count_workspace_bytes(plan.handle, graph.handle, ctypes.byref(nb)))
    return nb.value


def count(plan: Plan, graph: Graph, colours, per_vertex: bool = False, workspace: Workspace | None = None,
          out=None, vertex_out=None, stream=None):
    """X[b] for each colouring row of `colours` ([B, n] uint8 on the GPU); float64 tensors."""
    import torch
    if colours.dim() == 1:
        colours = colours.view(1, -1)
    B = colours.shape[0]
    if colours.shape[1] != graph.n:
        raise ValueError("colours must be [B, n]")
    dev = graph.row_ptr.device
    ws = (workspace or Workspace()).get(count_workspace_bytes(plan, graph), dev)
    X = out if out is not None else torch.empty(B, dtype=torch.float64, device=dev)
    V = None
    if per_vertex:
        V = vertex_out if vertex_out is not None else torch.empty((B, graph.n), dtype=torch.float64, device=dev)
    _check(lib().cc_count(plan.handle, graph.handle, _dev_ptr(colours, torch.uint8, "colours"), B,
                          ctypes.c_void_p(ws.data_ptr()), ws.numel(), _dev_ptr(X, torch.float64, "X"),
                          _dev_ptr(V, torch.float64, "vertex_out"), _stream(stream)))
    return (X, V) if per_vertex else X


CC_NOALLOC_SCRATCH_BYTES = 128 << 20  # the fixed workspace of cc_count_noalloc, per GPU


def count_noalloc(plan: Plan, graph: Graph, colours, out, vertex_out=None, stream=None):
    """cc_count_noalloc: X[b] for each colouring row of `colours` into the caller's `out` (float64,
    B) and optionally `vertex_out` (float64, [B, n]), with the library's fixed workspace: no device
    memory is allocated by this call."""
    import torch
    if colours.dim() == 1:
        colours = colours.view(1, -1)
    B = colours.shape[0]
    if colours.shape[1] != graph.n:
        raise ValueError("colours must be [B, n]")
    if out.numel() < B:
        raise ValueError("out must hold B doubles")
    if vertex_out is not None and vertex_out.numel() < B * graph.n:
        raise ValueError("vertex_out must hold B * n doubles")
    _check(lib().cc_count_noalloc(plan.handle, graph.handle, _dev_ptr(colours, torch.uint8, "colours"), B,
                                  _dev_ptr(out, torch.float64, "out"), _dev_ptr(vertex_out, torch.float64, "vertex_out"),
                                  _stream(stream)))
    return out


def count_budget_plan(plan: Plan, graph: Graph, budget: int) -> dict:
    """cc_count_budget_plan: the device workspace, host bytes, parked tables and arena widths of a
    count within `budget` bytes of device workspace (CCError CC_ENOSPC if it cannot fit)."""
    info = _BudgetInfo()
    rc = lib().cc_count_budget_plan(plan.handle, graph.handle, int(budget), ctypes.byref(info))
    out = {f[0]: getattr(info, f[0]) for f in _BudgetInfo._fields_}
    _check(rc)
    return out


def count_budget(plan: Plan, graph: Graph, colours, budget: int, per_vertex: bool = False,
                 workspace: Workspace | None = None, host=None, out=None, vertex_out=None, stream=None):
    """X[b] for each colouring row of `colours` within `budget` bytes of device workspace
    (cc_count_budget): tables idle across the peak wait in `host` (a pinned uint8 CPU tensor that
    must stay alive until the stream has passed the count; when None, one is allocated here and the
    call waits for the stream before returning)."""
    import torch
    if colours.dim() == 1:
        colours = colours.view(1, -1)
    B = colours.shape[0]
    if colours.shape[1] != graph.n:
        raise ValueError("colours must be [B, n]")
    info = count_budget_plan(plan, graph, budget)
    dev = graph.row_ptr.device
    ws = (workspace or Workspace()).get(info["workspace_bytes"], dev)
    own_host = host is None
    if own_host:
        try:
            host = torch.empty(max(info["host_bytes"], 1), dtype=torch.uint8, pin_memory=True)
        except Exception:  # the host refuses to lock that much: pageable, copies staged
            host = torch.empty(max(info["host_bytes"], 1), dtype=torch.uint8)
    if host.is_cuda or host.numel() < info["host_bytes"]:
        raise ValueError("host must be a CPU tensor of at least host_bytes bytes")
    X = out if out is not None else torch.empty(B, dtype=torch.float64, device=dev)
    V = None
    if per_vertex:
        V = vertex_out if vertex_out is not None else torch.empty((B, graph.n), dtype=torch.float64, device=dev)
    _check(lib().cc_count_budget(plan.handle, graph.handle, _dev_ptr(colours, torch.uint8, "colours"), B, int(budget),
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(host.data_ptr()),
                                 host.numel(), _dev_ptr(X, torch.float64, "X"),
                                 _dev_ptr(V, torch.float64, "vertex_out"), _stream(stream)))
    if own_host:
        (stream if stream is not None else torch.cuda.current_stream()).synchronize()
    return (X, V) if per_vertex else X


def count_inspect(plan: Plan, graph: Graph, colours, last: int, workspace: Workspace | None = None,
                  vertex_out=None, stream=None):
    """Run the splits 0..last of one colouring (`colours`: n uint8 on the GPU) and stop
    (cc_count_inspect). Returns the workspace tensor (uint8) that holds the tables, and the
    per-vertex root counts (float64, n) when split `last` is the root split, else None."""
    import torch
    colours = colours.reshape(-1)
    if colours.numel() != graph.n:
        raise ValueError("colours must have n entries")
    dev = graph.row_ptr.device
    ws = (workspace or Workspace()).get(count_workspace_bytes(plan, graph), dev)
    V = None
    if plan.split_maps(last)["out"] == -2:
        V = vertex_out if vertex_out is not None else torch.empty(graph.n, dtype=torch.float64, device=dev)
    _check(lib().cc_count_inspect(plan.handle, graph.handle, _dev_ptr(colours, torch.uint8, "colours"), last,
                                  ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                                  _dev_ptr(V, torch.float64, "vertex_out"), _stream(stream)))
    return ws, V


def count_projection(plan: Plan, graph: Graph) -> list[int]:
    """Colour classes per projected pass of each split in cc_count (0: unprojected)."""
    n = plan.info.n_splits
    out = (ctypes.c_int32 * max(n, 1))()
    _check(lib().cc_count_projection(plan.handle, graph.handle, out, max(n, 1)))
    return [int(x) for x in out[:n]]


def table_desc(plan: Plan, graph: Graph, table: int) -> dict:
    """Where table `table` lives in a count workspace (cc_plan_table_get): size, width, stride
    (doubles between rows), offset (bytes)."""
    d = _TableDesc()
    _check(lib().cc_plan_table_get(plan.handle, graph.handle, table, ctypes.byref(d)))
    return {f[0]: getattr(d, f[0]) for f in _TableDesc._fields_}


def table_rows(ws, desc: dict, vertices):
    """Rows of the given vertices of a table in a count workspace, as a float64 GPU tensor
    [len(vertices), width] (a gather over the caller's workspace tensor; no kernel of the library)."""
    import torch
    nbytes = ws.numel() - desc["offset"]
    flat = ws[desc["offset"]:desc["offset"] + nbytes // 8 * 8].view(torch.float64)
    idx = torch.as_tensor(vertices, dtype=torch.int64, device=ws.device)
    base = (idx * desc["stride"]).unsqueeze(1) + torch.arange(desc["width"], device=ws.device).unsqueeze(0)
    return flat[base]


def count_packed_workspace_bytes(plan: Plan, graph: Graph, B: int) -> int:
    nb = ctypes.c_size_t()
    _check(lib().cc_count_packed_workspace_bytes(plan.handle, graph.handle, B, ctypes.byref(nb)))
    return nb.value


def count_packed(plan: Plan, graph: Graph, colours, per_vertex: bool = False, workspace: Workspace | None = None,
                 out=None, vertex_out=None, stream=None):
    """X[b] for the B colourings of `colours` ([B, n] uint8 on the GPU) counted together, one row of
    the tables holding all B colourings (cc_count_packed). The per-vertex counts, if asked, are
    [n, B]."""
    import torch
    if colours.dim() == 1:
        colours = colours.view(1, -1)
    B = colours.shape[0]
    if colours.shape[1] != graph.n:
        raise ValueError("colours must be [B, n]")
    dev = graph.row_ptr.device
    ws = (workspace or Workspace()).get(count_packed_workspace_bytes(plan, graph, B), dev)
    X = out if out is not None else torch.empty(B, dtype=torch.float64, device=dev)
    V = None
    if per_vertex:
        V = vertex_out if vertex_out is not None else torch.empty((graph.n, B), dtype=torch.float64, device=dev)
    _check(lib().cc_count_packed(plan.handle, graph.handle, _dev_ptr(colours, torch.uint8, "colours"), B,
                                 ctypes.c_void_p(ws.data_ptr()), ws.numel(), _dev_ptr(X, torch.float64, "X"),
                                 _dev_ptr(V, torch.float64, "vertex_out"), _stream(stream)))
    return (X, V) if per_vertex else X


def stream_check(stream=None):
    """Synchronise `stream` (default: the current one) and raise CCError on a device error."""
    _check(lib().cc_stream_check(_stream(stream)))


class Multi:
    """Several templates of one size counted together over the same colourings, sharing the
    tables of equal rooted sub-templates (cc_multi_*)."""

    def __init__(self, plans):
        self.plans = list(plans)
        arr = (ctypes.c_void_p * len(self.plans))(*[p.handle.value for p in self.plans])
        h = ctypes.c_void_p()
        _check(lib().cc_multi_create(len(self.plans), arr, ctypes.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    @property
    def info(self) -> dict:
        st, ns, nt = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
        _check(lib().cc_multi_info_get(self._h, ctypes.byref(st), ctypes.byref(ns), ctypes.byref(nt)))
        return {"steps": st.value, "splits": ns.value, "tables": nt.value}

    @property
    def steps(self) -> list[tuple[int, int]]:
        """(plan index, split index) of every split that runs, in execution order."""
        out = []
        for i in range(self.info["steps"]):
            p, j = ctypes.c_int32(), ctypes.c_int32()
            _check(lib().cc_multi_step_get(self._h, i, ctypes.byref(p), ctypes.byref(j)))
            out.append((p.value, j.value))
        return out

    def workspace_bytes(self, graph: "Graph", B: int, persistent: bool = False) -> int:
        nb = ctypes.c_size_t()
        fn = (lib().cc_count_packed_multi_persistent_workspace_bytes if persistent
              else lib().cc_count_packed_multi_workspace_bytes)
        _check(fn(self._h, graph.handle, B, ctypes.byref(nb)))
        return nb.value

    def count(self, graph: "Graph", colours, workspace: Workspace | None = None, out=None, stream=None,
              persistent: bool = False):
        """X[p, b] for every template p and colouring b of `colours` ([B, n] uint8 on the GPU):
        one launch per split (cc_count_packed_multi) or one persistent launch for all of them
        (cc_count_packed_multi_persistent, persistent=True)."""
        import torch
        if colours.dim() == 1:
            colours = colours.view(1, -1)
        B = colours.shape[0]
        if colours.shape[1] != graph.n:
            raise ValueError("colours must be [B, n]")
        dev = graph.row_ptr.device
        ws = (workspace or Workspace()).get(self.workspace_bytes(graph, B, persistent), dev)
        X = out if out is not None else torch.empty((len(self.plans), B), dtype=torch.float64, device=dev)
        fn = lib().cc_count_packed_multi_persistent if persistent else lib().cc_count_packed_multi
        _check(fn(self._h, graph.handle, _dev_ptr(colours, torch.uint8, "colours"), B,
                  ctypes.c_void_p(ws.data_ptr()), ws.numel(), _dev_ptr(X, torch.float64, "X"), _stream(stream)))
        return X

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().cc_multi_destroy(h)
            except Exception:
                pass
            self._h = None


def entry_order(k: int, m: int) -> np.ndarray:
    """Storage order of a table row of m-sets over the k-1 colours other than the anchor's:
    element pos is the colex rank of the set stored at position pos (cc_entry_order)."""
    n = math.comb(k - 1, m) if 0 <= m <= k - 1 else 0
    out = np.zeros(max(n, 1), dtype=np.int32)
    _check(lib().cc_entry_order(k, m, out.ctypes.data, n))
    return out[:n]


def estimate(plan: Plan, X) -> tuple[float, float]:
    """mean(X) * k^k / k! / |Aut(T)| and its standard error (host)."""
    x = np.ascontiguousarray(np.asarray(X, dtype=np.float64).reshape(-1))
    est, se = ctypes.c_double(), ctypes.c_double()
    _check(lib().cc_estimate(plan.handle, x.ctypes.data, len(x), ctypes.byref(est), ctypes.byref(se)))
    return est.value, se.value


def iterations(k: int, epsilon: float, delta: float) -> tuple[int, int]:
    """(colourings per group, groups) for an (epsilon, delta)-approximation (cc_iterations)."""
    s, t = ctypes.c_int64(), ctypes.c_int32()
    _check(lib().cc_iterations(k, epsilon, delta, ctypes.byref(s), ctypes.byref(t)))
    return s.value, t.value


def estimate_median_of_means(plan: Plan, X, groups: int) -> float:
    x = np.ascontiguousarray(np.asarray(X, dtype=np.float64).reshape(-1))
    est = ctypes.c_double()
    _check(lib().cc_estimate_median_of_means(plan.handle, x.ctypes.data, len(x), groups, ctypes.byref(est)))
    return est.value


class Batch:
    """Many (plan, graph, colouring) instances counted in one persistent launch (cc_batch_*).

    `instances` is a list of (plan, graph, colours, X_out, vertex_out) with colours a uint8 GPU
    tensor of n entries, X_out a float64 GPU tensor view of one element and vertex_out either
    None or a float64 GPU tensor of n entries. Every instance gets exactly the result that
    count() would give it alone.
    """

    def __init__(self, instances, levels: bool = False, share: int = 1):
        import torch
        self._keep = list(instances)
        arr = (_Instance * max(len(instances), 1))()
        for i, (plan, graph, col, X, V) in enumerate(instances):
            if col.numel() != graph.n:
                raise ValueError("colours must have n entries")
            arr[i].plan = plan.handle.value
            arr[i].graph = graph.handle.value
            arr[i].colours_dev = _dev_ptr(col, torch.uint8, "colours").value if graph.n else None
            arr[i].X_dev = _dev_ptr(X, torch.float64, "X").value
            arr[i].vertex_dev = _dev_ptr(V, torch.float64, "vertex_out").value if V is not None else None
        flags = (CC_BATCH_LEVELS if levels else 0) | CC_BATCH_SHARE(share)
        h = ctypes.c_void_p()
        _check(lib().cc_batch_create(len(instances), arr, flags, ctypes.byref(h)))
        self._h = h
        nb = ctypes.c_size_t()
        _check(lib().cc_batch_workspace_bytes(self._h, ctypes.byref(nb)))
        self.workspace_bytes = nb.value
        self._dev = instances[0][1].row_ptr.device if instances else None

    def run(self, workspace=None, stream=None):
        """Queue the batch; `workspace` is a Workspace, a uint8 GPU tensor of at least
        workspace_bytes, or None (allocated here)."""
        import torch
        if isinstance(workspace, torch.Tensor):
            if workspace.numel() < self.workspace_bytes or workspace.dtype != torch.uint8:
                raise ValueError("workspace tensor too small")
            ws = workspace
        else:
            ws = (workspace or Workspace()).get(self.workspace_bytes, self._dev)
        self._ws = ws
        _check(lib().cc_batch_run(self._h, ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream(stream)))

    def check(self, stream=None):
        _check(lib().cc_batch_check(self._h, _stream(stream)))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().cc_batch_destroy(h)
            except Exception:
                pass
            self._h = None


def count_batched(plans, graph: Graph, colours, levels: bool = False, workspace: Workspace | None = None,
                  stream=None):
    """X[t, b] for every plan t and colouring row b of `colours` ([B, n] uint8) in one batch."""
    import torch
    if colours.dim() == 1:
        colours = colours.view(1, -1)
    B = colours.shape[0]
    X = torch.empty((len(plans), B), dtype=torch.float64, device=graph.row_ptr.device)
    inst = [(p, graph, colours[b], X[t, b:b + 1], None) for t, p in enumerate(plans) for b in range(B)]
    batch = Batch(inst, levels=levels)
    batch.run(workspace, stream)
    return X, batch
