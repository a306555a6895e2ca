"""Python access to the CPU oracle of track labeling (components_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use it; the product path never imports it.  It shares no code with the
HIP library.  The labeling rule is stated in the C file's header: kept edges
(score above the threshold, or all edges without scores), weakly connected
components, each vertex labeled with the smallest vertex id of its component.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "components_oracle.c")
LIB = os.path.join(HERE, "_build", "libcomponents.so")
CFLAGS = ["-O2", "-std=c11", "-fPIC", "-shared"]

_lock = threading.Lock()
_lib = None


class OracleError(RuntimeError):
    def __init__(self, status: int):
        super().__init__(f"components oracle status {status}")
        self.status = status


def build(src: str = SRC, out: str = LIB, extra_flags: list[str] | None = None) -> str:
    """Compile the oracle into a shared library (always recompiles)."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cmd = ["gcc", *CFLAGS, *(extra_flags or []), src, "-o", out + ".tmp"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(out + ".tmp", out)
    return out


def _declare(lib: ctypes.CDLL) -> ctypes.CDLL:
    i64p = ctypes.POINTER(ctypes.c_int64)
    lib.oracle_components.restype = ctypes.c_int
    lib.oracle_components.argtypes = [i64p, i64p, ctypes.c_int64, ctypes.c_int64,
                                      ctypes.POINTER(ctypes.c_float), ctypes.c_float, i64p]
    return lib


def load(path: str | None = None) -> ctypes.CDLL:
    """Load a compiled oracle (building the default one if it is absent or stale)."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build()
            _lib = _declare(ctypes.CDLL(LIB))
    return _lib


def labels(src, dst, n: int, scores=None, threshold: float = 0.0,
           lib: ctypes.CDLL | None = None) -> np.ndarray:
    """Component label (smallest member id) of every vertex 0..n-1, int64 [n]."""
    lib = lib or load()
    s = np.ascontiguousarray(src, dtype=np.int64)
    d = np.ascontiguousarray(dst, dtype=np.int64)
    if s.shape != d.shape or s.ndim != 1:
        raise ValueError("src and dst must be 1-D arrays of the same length")
    sc = None
    if scores is not None:
        sc = np.ascontiguousarray(scores, dtype=np.float32)
        if sc.shape != s.shape:
            raise ValueError("scores must have one entry per edge")
    out = np.empty(max(n, 0), dtype=np.int64)
    i64p = ctypes.POINTER(ctypes.c_int64)
    st = lib.oracle_components(
        s.ctypes.data_as(i64p), d.ctypes.data_as(i64p), s.size, n,
        sc.ctypes.data_as(ctypes.POINTER(ctypes.c_float)) if sc is not None else None,
        ctypes.c_float(threshold), out.ctypes.data_as(i64p))
    if st != 0:
        raise OracleError(st)
    return out
