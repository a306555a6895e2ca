"""Python access to the CPU oracle of the FRNN graph (frnn_oracle.c).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use it; the product path never imports it.  It shares no code with the
HIP library and imports nothing from the package except, in callers, the seeded
event generator.

The arithmetic lives in frnn_oracle.c (see its header for the definition it
follows).  This file only compiles it with a plain C compiler and marshals numpy
arrays in and out.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "frnn_oracle.c")
BUILD_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(BUILD_DIR, "liboracle.so")

# -ffp-contract=off keeps every product and sum separately rounded; -fno-fast-math
# keeps IEEE semantics (no flush of subnormals, no reassociation).
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]

OK, ERR_ARG, ERR_NONFINITE, ERR_CAPACITY = 0, 1, 2, 3

_lock = threading.Lock()
_lib = None


class OracleError(RuntimeError):
    def __init__(self, status: int):
        names = {ERR_ARG: "bad argument", ERR_NONFINITE: "non-finite coordinate",
                 ERR_CAPACITY: "capacity"}
        super().__init__(f"oracle status {status}: {names.get(status, 'unknown')}")
        self.status = status


def build(src: str = SRC, out: str = LIB, extra_flags: list[str] | None = None) -> str:
    """Compile the oracle into a shared library (always recompiles)."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cmd = ["gcc", *CFLAGS, *(extra_flags or []), src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    os.replace(out + ".tmp", out)
    return out


def _declare(lib: ctypes.CDLL) -> ctypes.CDLL:
    f32p = ctypes.POINTER(ctypes.c_float)
    i64p = ctypes.POINTER(ctypes.c_int64)
    for name in ("oracle_frnn_brute", "oracle_frnn_grid"):
        fn = getattr(lib, name)
        fn.restype = ctypes.c_int
        fn.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_int32,
                       i64p, i64p, ctypes.c_int64, i64p]
    lib.oracle_frnn_degrees.restype = ctypes.c_int
    lib.oracle_frnn_degrees.argtypes = [f32p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float, i64p]
    lib.oracle_pair_dist.restype = None
    lib.oracle_pair_dist.argtypes = [f32p, ctypes.c_int32, i64p, i64p, ctypes.c_int64, f32p]
    return lib


def load(path: str | None = None) -> ctypes.CDLL:
    """Load a compiled oracle (building the default one if it is absent)."""
    global _lib
    if path is not None:
        return _declare(ctypes.CDLL(path))
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
                build()
            _lib = _declare(ctypes.CDLL(LIB))
    return _lib


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _as_points(points) -> np.ndarray:
    X = np.ascontiguousarray(np.asarray(points, dtype=np.float32))
    if X.ndim != 2:
        raise ValueError("points must be [n, d]")
    return X


def _run(fn_name: str, points, r: float, K: int, lib: ctypes.CDLL | None) -> np.ndarray:
    lib = lib or load()
    X = _as_points(points)
    n, d = X.shape
    fn = getattr(lib, fn_name)
    cap = max(1024, 16 * n)
    for _ in range(2):
        src = np.zeros(cap, dtype=np.int64)
        dst = np.zeros(cap, dtype=np.int64)
        E = np.zeros(1, dtype=np.int64)
        st = fn(_ptr(X, ctypes.c_float), n, d, ctypes.c_float(r), K,
                _ptr(src, ctypes.c_int64), _ptr(dst, ctypes.c_int64), cap, _ptr(E, ctypes.c_int64))
        if st == OK:
            e = int(E[0])
            return np.stack([src[:e], dst[:e]])
        if st != ERR_CAPACITY:
            raise OracleError(st)
        cap = int(E[0])
    raise OracleError(ERR_CAPACITY)


def frnn_grid(points, r: float, K: int, lib: ctypes.CDLL | None = None) -> np.ndarray:
    """Edges of the FRNN graph by the grid route: int64 [2, E], (i asc, j asc)."""
    return _run("oracle_frnn_grid", points, r, K, lib)


def frnn_brute(points, r: float, K: int, lib: ctypes.CDLL | None = None) -> np.ndarray:
    """Edges of the FRNN graph by testing every ordered pair (O(n^2))."""
    return _run("oracle_frnn_brute", points, r, K, lib)


def degrees(points, r: float, lib: ctypes.CDLL | None = None) -> np.ndarray:
    """|N(i)| before the cap, for every i (O(n^2))."""
    lib = lib or load()
    X = _as_points(points)
    n, d = X.shape
    deg = np.zeros(max(n, 1), dtype=np.int64)
    st = lib.oracle_frnn_degrees(_ptr(X, ctypes.c_float), n, d, ctypes.c_float(r),
                                 _ptr(deg, ctypes.c_int64))
    if st != OK:
        raise OracleError(st)
    return deg[:n]


def pair_dist(points, i: np.ndarray, j: np.ndarray, lib: ctypes.CDLL | None = None) -> np.ndarray:
    """D(i, j) of the definition for each listed pair (float32)."""
    lib = lib or load()
    X = _as_points(points)
    i = np.ascontiguousarray(i, dtype=np.int64)
    j = np.ascontiguousarray(j, dtype=np.int64)
    out = np.zeros(max(i.size, 1), dtype=np.float32)
    lib.oracle_pair_dist(_ptr(X, ctypes.c_float), X.shape[1], _ptr(i, ctypes.c_int64),
                         _ptr(j, ctypes.c_int64), i.size, _ptr(out, ctypes.c_float))
    return out[: i.size]
