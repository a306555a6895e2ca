"""Python binding of libfrnn (include/frnn.h): argument marshalling only.

Every step of the graph build runs in the HIP library; this module allocates
device memory through PyTorch, passes raw pointers and the current HIP stream,
and maps status codes to exceptions.  It never computes edges itself: if the
library is missing, importing or calling it raises.
"""

from __future__ import annotations

import ctypes
import dataclasses
import os
import threading

import numpy as np

import torch  # loaded first so libfrnn binds to the HIP runtime PyTorch already uses

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfrnn.so")

FRNN_OK, FRNN_ERR_ARG, FRNN_ERR_NONFINITE, FRNN_ERR_CAPACITY = 0, 1, 2, 3
FRNN_ERR_WORKSPACE, FRNN_ERR_UNSUPPORTED, FRNN_ERR_HIP = 4, 5, 6
MAX_D = 64
MAX_K = 4096
NOALLOC_SCRATCH_MIB = 64
FLAG_TIMING = 1
FLAG_EVENTS_RESIDENT = 2
STAGES = ("bounds", "keys", "cells", "scatter", "search", "totals", "place")


class FrnnError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"frnn status {status}: {message}")
        self.status = status


class FrnnConfig(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("axes", ctypes.c_int32), ("cell_div", ctypes.c_int32),
                ("grid_mult", ctypes.c_int32), ("flags", ctypes.c_int32)]


class FrnnStats(ctypes.Structure):
    _fields_ = [("n_edges", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("n_cells", ctypes.c_int64), ("axes", ctypes.c_int32), ("grid", ctypes.c_int32 * 4),
                ("dims", ctypes.c_int32 * 4), ("cell", ctypes.c_float * 4),
                ("capped_queries", ctypes.c_int32), ("overflow_queries", ctypes.c_int32),
                ("stage_ms", ctypes.c_float * len(STAGES)), ("survivors", ctypes.c_int64)]

    def as_dict(self) -> dict:
        a = self.axes
        return {"n_edges": self.n_edges, "candidates": self.candidates, "n_cells": self.n_cells,
                "axes": a, "grid": list(self.grid)[:a], "dims": list(self.dims)[:a], "cell": list(self.cell)[:a],
                "capped_queries": self.capped_queries, "overflow_queries": self.overflow_queries,
                "stage_ms": dict(zip(STAGES, self.stage_ms)), "survivors": self.survivors}


@dataclasses.dataclass(frozen=True)
class Config:
    """Speed-only tunables; every choice yields the same edges."""

    dims: tuple[int, ...] | None = None         # 3 or 4 binned coordinates (default: the last ones)
    axes: int = 0                               # binned count when dims is None (0: automatic)
    cell_div: int = 1                           # cell edge = r (1 + 2^-10) / cell_div
    grid_mult: int = 0                          # search workgroups per resident slot (0: automatic)
    timing: bool = False                        # per-stage HIP event timing in the stats
    events_resident: bool = False               # batch event table already in the workspace

    def to_c(self) -> FrnnConfig:
        c = FrnnConfig()
        c.axes = int(self.axes)
        if self.dims is not None:
            if len(self.dims) not in (3, 4):
                raise ValueError("dims must name 3 or 4 coordinates")
            for p, v in enumerate(self.dims):
                c.dims[p] = int(v)
            c.axes = len(self.dims)
        c.cell_div = int(self.cell_div)
        c.grid_mult = int(self.grid_mult)
        c.flags = (FLAG_TIMING if self.timing else 0) | (FLAG_EVENTS_RESIDENT if self.events_resident else 0)
        return c


_lock = threading.Lock()
_lib = None


def _declare(lib: ctypes.CDLL) -> ctypes.CDLL:
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.frnn_workspace_bytes.restype = ctypes.c_size_t
    lib.frnn_workspace_bytes.argtypes = [i64, i32]
    lib.frnn_build.restype = ctypes.c_int
    lib.frnn_build.argtypes = [vp, i64, i32, ctypes.c_float, i32, vp, ctypes.c_size_t, vp, vp, i64,
                               ctypes.POINTER(i64), ctypes.POINTER(FrnnConfig),
                               ctypes.POINTER(FrnnStats), vp]
    lib.frnn_build_noalloc.restype = ctypes.c_int
    lib.frnn_build_noalloc.argtypes = [vp, i64, i32, ctypes.c_float, i32, vp, vp, i64, ctypes.POINTER(i64),
                                       ctypes.POINTER(FrnnConfig), ctypes.POINTER(FrnnStats), vp]
    lib.frnn_batch_workspace_bytes.restype = ctypes.c_size_t
    lib.frnn_batch_workspace_bytes.argtypes = [ctypes.POINTER(i64), i32, i32]
    lib.frnn_build_batch.restype = ctypes.c_int
    lib.frnn_build_batch.argtypes = [vp, ctypes.POINTER(i64), i32, i32, ctypes.c_float, i32, vp, ctypes.c_size_t,
                                     vp, vp, i64, ctypes.POINTER(i64), ctypes.POINTER(FrnnConfig),
                                     ctypes.POINTER(FrnnStats), vp]
    lib.frnn_build_batch_async.restype = ctypes.c_int
    lib.frnn_build_batch_async.argtypes = [vp, ctypes.POINTER(i64), i32, i32, ctypes.c_float, i32, vp,
                                           ctypes.c_size_t, vp, vp, i64, vp, ctypes.POINTER(FrnnConfig), vp]
    lib.frnn_build_events_async.restype = ctypes.c_int
    lib.frnn_build_events_async.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(i64), i32, i32,
                                            ctypes.c_float, i32, vp, ctypes.c_size_t, vp, vp, i64, vp,
                                            ctypes.POINTER(FrnnConfig), vp]
    lib.frnn_components_workspace_bytes.restype = ctypes.c_size_t
    lib.frnn_components_workspace_bytes.argtypes = [i64]
    for name, last in (("frnn_components", ctypes.POINTER(ctypes.c_int64)), ("frnn_components_async", vp)):
        fn = getattr(lib, name)
        fn.restype = ctypes.c_int
        fn.argtypes = [vp, vp, i64, i64, vp, ctypes.c_float, vp, ctypes.c_size_t, vp, last, vp]
    lib.frnn_status_string.restype = ctypes.c_char_p
    lib.frnn_status_string.argtypes = [ctypes.c_int]
    return lib


def lib() -> ctypes.CDLL:
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise ImportError(f"{LIB_PATH} is missing: build it with "
                                  "`python -m paper_2202_06929_amd.build_lib`")
            _lib = _declare(ctypes.CDLL(LIB_PATH))
    return _lib


def status_string(status: int) -> str:
    return lib().frnn_status_string(status).decode()


def workspace_bytes(n: int, d: int) -> int:
    return int(lib().frnn_workspace_bytes(n, d))


def _stream_handle(device: torch.device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _check_points(points: torch.Tensor) -> None:
    if not isinstance(points, torch.Tensor) or points.device.type != "cuda":
        raise TypeError("points must be a GPU tensor")
    if points.dtype != torch.float32 or points.dim() != 2 or not points.is_contiguous():
        raise TypeError("points must be a contiguous float32 tensor [n, d]")


def build_into(points: torch.Tensor, r: float, K: int, workspace: torch.Tensor,
               src: torch.Tensor, dst: torch.Tensor, config: Config | None = None,
               stats: FrnnStats | None = None) -> tuple[int, int]:
    """One call of frnn_build on caller-provided buffers.  Returns (status, E)."""
    n, d = points.shape
    E = ctypes.c_int64(0)
    cfg = config.to_c() if config is not None else None
    st = lib().frnn_build(
        ctypes.c_void_p(points.data_ptr()), n, d, ctypes.c_float(r), K,
        ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
        ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), src.numel(),
        ctypes.byref(E), ctypes.byref(cfg) if cfg is not None else None,
        ctypes.byref(stats) if stats is not None else None,
        ctypes.c_void_p(_stream_handle(points.device)))
    return st, int(E.value)


def build(points: torch.Tensor, r: float, K: int, config: Config | None = None,
          capacity: int | None = None, return_stats: bool = False):
    """Edges of the FRNN graph: int64 [2, E] on the points' device, (i asc, j asc).

    Row 0 holds the query i, row 1 the neighbour j.  With return_stats=True,
    returns (edges, stats dict).  The returned tensor may be a view with a row
    stride larger than E.
    """
    _check_points(points)
    n, d = points.shape
    if n == 0:
        empty = torch.empty((2, 0), dtype=torch.int64, device=points.device)
        return (empty, FrnnStats().as_dict()) if return_stats else empty
    cap = max(1, int(capacity)) if capacity is not None else max(1024, 16 * n)
    stats = FrnnStats()
    for attempt in range(2):
        wsb = workspace_bytes(n, d)
        if wsb == 0:
            raise FrnnError(FRNN_ERR_ARG, "invalid sizes")
        ws = torch.empty(wsb, dtype=torch.uint8, device=points.device)
        out = torch.empty((2, cap), dtype=torch.int64, device=points.device)
        st, E = build_into(points, r, K, ws, out[0], out[1], config, stats)
        if st == FRNN_OK:
            edges = out[:, :E]
            return (edges, stats.as_dict()) if return_stats else edges
        if st == FRNN_ERR_CAPACITY and attempt == 0:
            cap = E
            continue
        raise FrnnError(st, status_string(st))
    raise FrnnError(FRNN_ERR_CAPACITY, "capacity retry failed")


def build_noalloc_into(points: torch.Tensor, r: float, K: int, src: torch.Tensor, dst: torch.Tensor,
                       config: Config | None = None, stats: FrnnStats | None = None) -> tuple[int, int]:
    """One call of frnn_build_noalloc (no workspace: the library's fixed device
    array) on caller-provided outputs.  Returns (status, E)."""
    _check_points(points)
    n, d = points.shape
    E = ctypes.c_int64(0)
    cfg = config.to_c() if config is not None else None
    st = lib().frnn_build_noalloc(
        ctypes.c_void_p(points.data_ptr()), n, d, ctypes.c_float(r), K,
        ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), src.numel(),
        ctypes.byref(E), ctypes.byref(cfg) if cfg is not None else None,
        ctypes.byref(stats) if stats is not None else None,
        ctypes.c_void_p(_stream_handle(points.device)))
    return st, int(E.value)


def _offsets_array(offsets) -> np.ndarray:
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if off.ndim != 1 or off.size < 2:
        raise ValueError("offsets must be int64 [n_events + 1]")
    return off


def batch_workspace_bytes(offsets, d: int) -> int:
    off = _offsets_array(offsets)
    return int(lib().frnn_batch_workspace_bytes(off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                                off.size - 1, d))


def build_batch_into(points: torch.Tensor, offsets, r: float, K: int, workspace: torch.Tensor,
                     src: torch.Tensor, dst: torch.Tensor, config: Config | None = None,
                     stats: FrnnStats | None = None) -> tuple[int, np.ndarray]:
    """One call of frnn_build_batch on caller buffers.  Returns (status, edge_offsets)."""
    off = _offsets_array(offsets)
    n_events = off.size - 1
    eo = np.zeros(n_events + 1, dtype=np.int64)
    cfg = config.to_c() if config is not None else None
    st = lib().frnn_build_batch(
        ctypes.c_void_p(points.data_ptr()), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n_events,
        points.shape[1], ctypes.c_float(r), K, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
        ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), src.numel(),
        eo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(cfg) if cfg is not None else None,
        ctypes.byref(stats) if stats is not None else None, ctypes.c_void_p(_stream_handle(points.device)))
    return st, eo


def build_batch(points: torch.Tensor, offsets, r: float, K: int, config: Config | None = None,
                capacity: int | None = None, return_stats: bool = False):
    """Edges of several events searched independently in one pass.

    points holds the events' rows back to back; offsets (int64 [n_events + 1]) marks
    where each event starts.  Returns (edges int64 [2, E], edge_offsets numpy int64
    [n_events + 1]): event e's edges are edges[:, edge_offsets[e]:edge_offsets[e+1]],
    with indices local to the event and sorted by (i, j).
    """
    _check_points(points)
    off = _offsets_array(offsets)
    d = points.shape[1]
    rows = int(off[-1] - off[0])
    cap = max(1, int(capacity)) if capacity is not None else max(1024, 16 * rows)
    stats = FrnnStats()
    for attempt in range(2):
        wsb = batch_workspace_bytes(off, d)
        if wsb == 0:
            raise FrnnError(FRNN_ERR_ARG, "invalid sizes")
        ws = torch.empty(wsb, dtype=torch.uint8, device=points.device)
        out = torch.empty((2, cap), dtype=torch.int64, device=points.device)
        st, eo = build_batch_into(points, off, r, K, ws, out[0], out[1], config, stats)
        if st == FRNN_OK:
            edges = out[:, :int(eo[-1])]
            return (edges, eo, stats.as_dict()) if return_stats else (edges, eo)
        if st == FRNN_ERR_CAPACITY and attempt == 0:
            cap = int(eo[-1])
            continue
        raise FrnnError(st, status_string(st))
    raise FrnnError(FRNN_ERR_CAPACITY, "capacity retry failed")


def build_batch_async(points: torch.Tensor, offsets, r: float, K: int, workspace: torch.Tensor,
                      src: torch.Tensor, dst: torch.Tensor, edge_offsets: torch.Tensor,
                      config: Config | None = None) -> int:
    """Enqueues frnn_build_batch_async on the current stream and returns its status.

    edge_offsets: device int64 [n_events + 2]; after the stream reaches this point it
    holds the per-event edge ranges, the total, then a status word (0, 2 or 3).
    """
    off = _offsets_array(offsets)
    n_events = off.size - 1
    if edge_offsets.numel() < n_events + 2 or edge_offsets.dtype != torch.int64:
        raise ValueError("edge_offsets must be a device int64 tensor of n_events + 2 entries")
    cfg = config.to_c() if config is not None else None
    return lib().frnn_build_batch_async(
        ctypes.c_void_p(points.data_ptr()), off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n_events,
        points.shape[1], ctypes.c_float(r), K, ctypes.c_void_p(workspace.data_ptr()), workspace.numel(),
        ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), src.numel(),
        ctypes.c_void_p(edge_offsets.data_ptr()), ctypes.byref(cfg) if cfg is not None else None,
        ctypes.c_void_p(_stream_handle(points.device)))


class AsyncBatch:
    """Repeated frnn_build_batch_async calls on the same points, offsets, radius, cap,
    workspace, outputs and config, each with its own edge_offsets buffer: the fixed
    arguments are marshalled once, on the stream current at construction.  The
    tensors must stay alive and in place while the object is used.
    """

    def __init__(self, points: torch.Tensor, offsets, r: float, K: int, workspace: torch.Tensor,
                 src: torch.Tensor, dst: torch.Tensor, config: Config | None = None):
        self._off = _offsets_array(offsets)  # kept alive: the call reads it
        self._n_events = self._off.size - 1
        self._cfg = config.to_c() if config is not None else None
        self._fn = lib().frnn_build_batch_async
        self._head = (ctypes.c_void_p(points.data_ptr()), self._off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                      self._n_events, points.shape[1], ctypes.c_float(r), K, ctypes.c_void_p(workspace.data_ptr()),
                      workspace.numel(), ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
                      src.numel())
        self._tail = (ctypes.byref(self._cfg) if self._cfg is not None else None,
                      ctypes.c_void_p(_stream_handle(points.device)))

    def __call__(self, edge_offsets: torch.Tensor) -> int:
        """Enqueues one build; edge_offsets as for build_batch_async.  Returns its status."""
        if edge_offsets.numel() < self._n_events + 2 or edge_offsets.dtype != torch.int64:
            raise ValueError("edge_offsets must be a device int64 tensor of n_events + 2 entries")
        return self._fn(*self._head, ctypes.c_void_p(edge_offsets.data_ptr()), *self._tail)


def build_events_async(event_points: list[torch.Tensor], r: float, K: int, workspace: torch.Tensor,
                       src: torch.Tensor, dst: torch.Tensor, edge_offsets: torch.Tensor,
                       config: Config | None = None) -> int:
    """Enqueues frnn_build_events_async for events held in separate device tensors.

    The workspace size is batch_workspace_bytes of the events' cumulative sizes;
    edge_offsets (device int64 [n_events + 2]) receives the ranges and the status.
    """
    if not event_points:
        raise ValueError("no events")
    d = event_points[0].shape[1]
    for p in event_points:
        if p.dtype != torch.float32 or p.dim() != 2 or p.shape[1] != d or not p.is_contiguous():
            raise TypeError("every event must be a contiguous float32 tensor [n, d]")
    n_events = len(event_points)
    ptrs = (ctypes.c_void_p * n_events)(*[p.data_ptr() if p.shape[0] else 0 for p in event_points])
    sizes = np.array([p.shape[0] for p in event_points], dtype=np.int64)
    cfg = config.to_c() if config is not None else None
    return lib().frnn_build_events_async(
        ptrs, sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), n_events, d, ctypes.c_float(r), K,
        ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), ctypes.c_void_p(src.data_ptr()),
        ctypes.c_void_p(dst.data_ptr()), src.numel(), ctypes.c_void_p(edge_offsets.data_ptr()),
        ctypes.byref(cfg) if cfg is not None else None, ctypes.c_void_p(_stream_handle(event_points[0].device)))


def components_workspace_bytes(n_vertices: int) -> int:
    return int(lib().frnn_components_workspace_bytes(n_vertices))


def _edge_arrays(src: torch.Tensor, dst: torch.Tensor, scores: torch.Tensor | None):
    for t in (src, dst):
        if t.dtype != torch.int64 or t.dim() != 1 or not t.is_contiguous() or not t.is_cuda:
            raise TypeError("src and dst must be contiguous 1-D int64 device tensors")
    if src.numel() != dst.numel():
        raise ValueError("src and dst differ in length")
    if scores is not None and (scores.dtype != torch.float32 or scores.numel() != src.numel()
                               or not scores.is_contiguous() or not scores.is_cuda):
        raise TypeError("scores must be a contiguous float32 device tensor with one entry per edge")


def components(src: torch.Tensor, dst: torch.Tensor, n_vertices: int, scores: torch.Tensor | None = None,
               threshold: float = 0.0) -> tuple[torch.Tensor, int]:
    """Track labels: (labels int64 [n_vertices], number of components).

    Weakly connected components of the kept edges (all edges, or those with
    scores > threshold), each vertex labeled with the smallest vertex id of its
    component (frnn_components)."""
    _edge_arrays(src, dst, scores)
    dev = src.device
    labels = torch.empty(max(n_vertices, 0), dtype=torch.int64, device=dev)
    ws = torch.empty(max(components_workspace_bytes(n_vertices), 256), dtype=torch.uint8, device=dev)
    nc = ctypes.c_int64(0)
    st = lib().frnn_components(
        ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), src.numel(), n_vertices,
        ctypes.c_void_p(scores.data_ptr()) if scores is not None else None, ctypes.c_float(threshold),
        ctypes.c_void_p(ws.data_ptr()), ws.numel(), ctypes.c_void_p(labels.data_ptr()), ctypes.byref(nc),
        ctypes.c_void_p(_stream_handle(dev)))
    if st != FRNN_OK:
        raise FrnnError(st, status_string(st))
    return labels, int(nc.value)


def components_async(src: torch.Tensor, dst: torch.Tensor, n_vertices: int, workspace: torch.Tensor,
                     labels: torch.Tensor, result: torch.Tensor, scores: torch.Tensor | None = None,
                     threshold: float = 0.0) -> int:
    """Enqueues frnn_components_async on the current stream; result (device int64 [2])
    receives the number of components and a status word."""
    _edge_arrays(src, dst, scores)
    return lib().frnn_components_async(
        ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), src.numel(), n_vertices,
        ctypes.c_void_p(scores.data_ptr()) if scores is not None else None, ctypes.c_float(threshold),
        ctypes.c_void_p(workspace.data_ptr()), workspace.numel(), ctypes.c_void_p(labels.data_ptr()),
        ctypes.c_void_p(result.data_ptr()), ctypes.c_void_p(_stream_handle(src.device)))
