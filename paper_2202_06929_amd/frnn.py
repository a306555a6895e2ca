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

import torch  # loaded first so libfrnn binds to the HIP runtime PyTorch already uses

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libfrnn.so")

FRNN_OK, FRNN_ERR_ARG, FRNN_ERR_NONFINITE, FRNN_ERR_CAPACITY = 0, 1, 2, 3
FRNN_ERR_WORKSPACE, FRNN_ERR_UNSUPPORTED, FRNN_ERR_HIP = 4, 5, 6
MAX_D = 64
MAX_K = 4096
FLAG_TIMING = 1
STAGES = ("bounds", "keys", "cells", "scatter", "search", "long", "offsets", "place")


class FrnnError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"frnn status {status}: {message}")
        self.status = status


class FrnnConfig(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 3), ("cell_div", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("flags", ctypes.c_int32)]


class FrnnStats(ctypes.Structure):
    _fields_ = [("n_edges", ctypes.c_int64), ("candidates", ctypes.c_int64),
                ("n_cells", ctypes.c_int64), ("grid", ctypes.c_int32 * 3),
                ("dims", ctypes.c_int32 * 3), ("cell", ctypes.c_float * 3),
                ("capped_queries", ctypes.c_int32), ("overflow_queries", ctypes.c_int32),
                ("stage_ms", ctypes.c_float * 8)]

    def as_dict(self) -> dict:
        return {"n_edges": self.n_edges, "candidates": self.candidates, "n_cells": self.n_cells,
                "grid": list(self.grid), "dims": list(self.dims), "cell": list(self.cell),
                "capped_queries": self.capped_queries, "overflow_queries": self.overflow_queries,
                "stage_ms": dict(zip(STAGES, self.stage_ms))}


@dataclasses.dataclass(frozen=True)
class Config:
    """Speed-only tunables; every choice yields the same edges."""

    dims: tuple[int, int, int] | None = None  # binned coordinates (default: the last three)
    cell_div: int = 1                           # cell edge = r (1 + 2^-10) / cell_div
    tile: int = 0
    timing: bool = False                        # per-stage HIP event timing in the stats

    def to_c(self) -> FrnnConfig:
        c = FrnnConfig()
        if self.dims is not None:
            for p in range(3):
                c.dims[p] = int(self.dims[p])
        c.cell_div = int(self.cell_div)
        c.tile = int(self.tile)
        c.flags = FLAG_TIMING if self.timing else 0
        return c


_lock = threading.Lock()
_lib = None


def _declare(lib: ctypes.CDLL) -> ctypes.CDLL:
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.frnn_workspace_bytes.restype = ctypes.c_size_t
    lib.frnn_workspace_bytes.argtypes = [i64, i32, i64]
    lib.frnn_build.restype = ctypes.c_int
    lib.frnn_build.argtypes = [vp, i64, i32, ctypes.c_float, i32, vp, ctypes.c_size_t, vp, vp, i64,
                               ctypes.POINTER(i64), ctypes.POINTER(FrnnConfig),
                               ctypes.POINTER(FrnnStats), vp]
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


def workspace_bytes(n: int, d: int, edge_capacity: int) -> int:
    return int(lib().frnn_workspace_bytes(n, d, edge_capacity))


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
        wsb = workspace_bytes(n, d, cap)
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
