"""Autotuner of the grid search: picks the cell size, the binned coordinates (three
or four, and which) and the search grid (workgroups per resident slot) for a
workload by timing each candidate on a sample batch.

Every candidate must return byte-identical edges (they are speed-only choices of
the same exact search); the tuner checks that on the device and refuses to pick
otherwise.  Choices are cached in a JSON file keyed by (GPU architecture, d, size
bucket, r, K), so a workload is tuned once per machine.
"""

from __future__ import annotations

import dataclasses
import json
import math
import os
import time

import numpy as np
import torch

from . import frnn

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "frnn_mi355x_tune.json")


def candidates(d: int) -> list[frnn.Config]:
    """Four binned coordinates (when d >= 5: the last four, and for d >= 8 a spread
    of four), then three binned coordinates crossed with cell divisions 1-3: the last
    three (leading terms of the distance sum unbinned, so the early exit bites), the
    first three, and a spread of coordinates.  The search grid is then tuned for the
    best of these (grid_candidates)."""
    out = []
    if d >= 5:
        out.append(frnn.Config(axes=4))
    if d >= 8:
        out.append(frnn.Config(dims=(d // 2 - 1, d // 2, d // 2 + 1, d - 1)))
    dim_sets = [None, (0, 1, 2)]
    if d >= 6:
        dim_sets.append((d // 2, d // 2 + 1, d - 1))
    for dims in dim_sets:
        for div in (1, 2, 3):
            out.append(frnn.Config(dims=dims, axes=3 if dims is None else 0, cell_div=div))
    return out


def grid_candidates(best: frnn.Config) -> list[frnn.Config]:
    return [dataclasses.replace(best, grid_mult=m) for m in (1, 2, 4)]


def describe(cfg: frnn.Config) -> str:
    return f"dims={cfg.dims} axes={cfg.axes} div={cfg.cell_div} grid={cfg.grid_mult}"


def size_bucket(rows: int) -> int:
    return int(round(math.log2(max(rows, 1)) * 2))


def cache_key(arch: str, d: int, rows: int, r: float, K: int) -> str:
    return f"{arch}|d={d}|b={size_bucket(rows)}|r={r:.6g}|K={K}"


def _sync() -> None:
    torch.cuda.synchronize()


def _arch() -> str:
    props = torch.cuda.get_device_properties(0)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def tune(points: torch.Tensor, offsets, r: float, K: int, repeats: int = 5,
         cache_path: str | None = DEFAULT_CACHE, cands: list[frnn.Config] | None = None,
         log=None) -> tuple[frnn.Config, dict]:
    """Times every candidate on the batch (points, offsets); returns the fastest config
    and a report {config: median seconds}.  Raises if candidates disagree."""
    off = np.asarray(offsets, dtype=np.int64)
    rows = int(off[-1] - off[0])
    d = points.shape[1]
    key = cache_key(_arch(), d, rows, r, K)
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
        if key in cache:
            c = cache[key]
            return frnn.Config(dims=tuple(c["dims"]) if c["dims"] else None, axes=c.get("axes", 0),
                               cell_div=c["cell_div"], grid_mult=c.get("grid_mult", 0)), c
    first = cands or candidates(d)
    _, eo0 = frnn.build_batch(points, off, r, K, config=first[0])
    cap = int(eo0[-1]) + 1024
    ws_bytes = max(frnn.batch_workspace_bytes(off, d), 1)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=points.device)
    out = torch.empty((2, cap), dtype=torch.int64, device=points.device)
    ref = {}
    timings = {}

    def run(cfgs):
        for cfg in cfgs:
            st, eo = frnn.build_batch_into(points, off, r, K, ws, out[0], out[1], cfg)
            if st != frnn.FRNN_OK:
                raise frnn.FrnnError(st, frnn.status_string(st))
            E = int(eo[-1])
            if not ref:
                ref["edges"] = out[:, :E].clone()
                ref["eo"] = eo.copy()
            elif not (np.array_equal(eo, ref["eo"]) and torch.equal(out[:, :E], ref["edges"])):
                raise AssertionError(f"config {cfg} changed the edges: the search is not exact")
            ts = []
            for _ in range(repeats):
                _sync()
                t0 = time.perf_counter()
                frnn.build_batch_into(points, off, r, K, ws, out[0], out[1], cfg)
                ts.append(time.perf_counter() - t0)
            timings[cfg] = float(np.median(ts))
            if log:
                log(f"tune {cfg}: {timings[cfg] * 1e3:.3f} ms")

    run(first)
    if not cands:
        run(grid_candidates(min(timings, key=timings.get)))
    best = min(timings, key=timings.get)
    report = {"dims": list(best.dims) if best.dims else None, "axes": best.axes, "cell_div": best.cell_div,
              "grid_mult": best.grid_mult, "seconds": timings[best], "key": key,
              "all": {describe(c): t for c, t in timings.items()}}
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        cache = {}
        if os.path.exists(cache_path):
            with open(cache_path) as f:
                cache = json.load(f)
        cache[key] = report
        with open(cache_path + ".tmp", "w") as f:
            json.dump(cache, f, indent=1)
        os.replace(cache_path + ".tmp", cache_path)
    return best, report
