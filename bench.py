"""Benchmark of the FRNN graph build on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload single|high|tiny]

A step is one pass of the whole path over one synthetic event already resident in
HBM: bounds, keys, cell scan, scatter, neighbour search and edge placement (long
lists included).  The timed steps run back to back on one stream through the
asynchronous entry point; synchronous calls (each returning the edge count to the
host) give the per-event latency percentiles.  The default workload is
the single event of 120,000 points in 8-D (r = 0.1, K = 256).

Prints one JSON line with throughput (events/s), edges/s, per-event latency
percentiles, the roofline of the dominant kernel (the neighbour search) from
HIP-event timings taken inside this run, and the CPU oracle timed on this host.
"""

from __future__ import annotations

import argparse
import dataclasses
import gc
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks: HBM3E 8 TB/s; FP32 vector 157.3 TFLOP/s (256 CUs x
# 2.4 GHz x 256 FLOP per CU and cycle, which counts a fused multiply-add as two
# operations and packed FP32 as two lanes).  The distance test may use neither
# (every product and sum is rounded on its own), so its own issue ceiling is one
# FP32 operation per lane and cycle: 256 CUs x 64 lanes x 2.4 GHz = 39.3 T/s,
# reported beside the published figure, never in its place.
HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
PLAIN_LANE_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
PATH_HBM_TARGET = 0.5
METRIC = "events/s and edges/s at 120k hits; p50/p99 per-event latency; HBM GB/s vs peak"
LATENCY_SAMPLES = 200


def log(msg: str) -> None:
    print(msg, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", choices=["single", "high", "tiny", "knn"], default="single")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cell-div", type=int, default=None)
    ap.add_argument("--axes", type=int, default=0, choices=[0, 3, 4], help="binned coordinates (0: automatic)")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--no-labeling", action="store_true")
    ap.add_argument("--copy-probe", action="store_true", help="run the counter calibration copy and exit")
    ap.add_argument("--summarize", nargs="+", metavar="DIR",
                    help="print a markdown summary of rocprofv3 output folders (TRACE FETCH WRITE CFETCH CWRITE "
                         "[SQ]) and exit")
    ap.add_argument("--commands", nargs="+", default=None, help="the profiling commands, for the summary")
    ap.add_argument("--lds", nargs=2, default=None, metavar=("DIR", "COMMAND"),
                    help="rocprofv3 folder and command of an LdsBankConflict / MeanOccupancyPerCU pass")
    ap.add_argument("--bench-line", default=None,
                    help="stdout of the profiled bench run (its JSON line gives n, d and E for the summary)")
    ap.add_argument("--batch-only", type=int, default=0, metavar="CALLS",
                    help="build the 64-event batch CALLS times with the default binned coordinates and "
                         "default grid (a run to profile) and exit")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("TITLE", "TRACE", "COMMAND"),
                    help="print a markdown table of kernel durations from one rocprofv3 kernel-trace folder and exit")
    return ap.parse_args()


def search_bytes(n: int, dpad: int, n_cells: int, E: int) -> int:
    """Algorithmic HBM bytes of one search launch: each sorted row read once, the
    sorted rows' (original row, cell) words, cell starts, kept counts and the
    unsorted neighbour lists (4 bytes per edge)."""
    return n * dpad * 4 + 8 * n + 4 * (n_cells + 1) + 4 * n + 4 * E


def cells_max(n: int) -> int:
    """Cells reserved (cleared and scanned) for an event of n points."""
    return min(max(2 * n, 1 << 15), 1 << 24)


def kernel_bytes(kernel: str, n: int, d: int, E: int, axes: int = 4) -> int | None:
    """Algorithmic HBM bytes of one launch of each kernel of the path on one event
    (inputs read once, outputs written once): what the counted traffic of the
    profile is compared with."""
    dpad = next(p for p in (4, 8, 12, 16, 24, 32, 48, 64) if d <= p)
    cells = cells_max(n)
    tiles = (n + 255) // 256
    table = {
        # points read; histogram cleared
        "k_bounds": 4 * n * d + 4 * cells,
        # binned coordinates read; packed cell and rank written; one counter updated per point
        "k_keys": 4 * axes * n + 8 * n + 8 * min(n, cells),
        # histogram read, cell starts written (the search's wave starts, 4 bytes a
        # wave, are under 2% of this and not counted)
        "k_scan_cells": 4 * cells + 4 * (cells + 1),
        # packed cell, rank, cell start and row read; padded row, (row, cell) pair and inverse written
        "k_scatter": 12 * n + 4 * n * d + 4 * n * dpad + 12 * n,
        "k_search": search_bytes(n, dpad, cells, E),
        # kept counts read, tile totals written
        "k_kept_sums": 4 * n + 8 * tiles,
        # kept counts and list entries read, int64 edges written
        "k_place": 4 * n + 4 * E + 16 * E,
        # labeling of the event's graph (n vertices, E edges): parents initialised;
        # edges read and one parent per source updated; edges read again with the
        # parents of their ends; parents read and int64 labels written
        "k_cc_init": 4 * n,
        "k_cc_minhook": 16 * E + 8 * n,
        "k_cc_hook": 16 * E + 8 * n,
        "k_cc_label": 4 * n + 8 * n,
    }
    for k, v in table.items():
        if kernel == k or kernel.startswith(k + "<"):
            return v
    return None


def path_bytes(n: int, d: int, E: int) -> int:
    """Algorithmic HBM bytes of the whole path per event: points read for bounds,
    keys and scatter, sorted rows written and read by the search (5 n d 4), about
    40 bytes of per-point indices, and 16 bytes per int64 edge."""
    return 5 * n * d * 4 + 40 * n + 16 * E


def host_threads() -> int:
    """Host threads this process may use (its CPU affinity), at most 16: the GPU
    box's share of host cores for one GPU."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(spec, X, single_s: float = 6.0, multi_s: float = 1.5) -> dict:
    """The CPU oracle (plain C grid route, unchanged) on the same event.

    Two legs: one host thread, repeated for about single_s seconds (at least 3
    runs); then every usable host thread (host_threads()) each building the event
    over and over for about multi_s seconds of wall time, events being independent.
    `value` is the all-threads rate with `cores` the threads used; the one-thread
    rate is reported beside it."""
    import threading

    from oracle import oracle
    oracle.load()
    runs = []
    t0 = time.perf_counter()
    while len(runs) < 3 or time.perf_counter() - t0 < single_s:
        t = time.perf_counter()
        oracle.frnn_grid(X, spec.r, spec.K)
        runs.append(time.perf_counter() - t)
    one = len(runs) / sum(runs)

    threads = host_threads()
    counts = [0] * threads
    stop = time.perf_counter() + multi_s

    def work(k):
        while time.perf_counter() < stop or counts[k] == 0:
            oracle.frnn_grid(X, spec.r, spec.K)  # the C call runs outside the interpreter lock
            counts[k] += 1

    pool = [threading.Thread(target=work, args=(k,)) for k in range(threads)]
    t = time.perf_counter()
    for th in pool:
        th.start()
    for th in pool:
        th.join()
    wall = time.perf_counter() - t
    many = sum(counts) / wall
    return {"value": many, "unit": "events/s", "cores": threads, "kind": "oracle",
            "sample": f"the same event (n={spec.n}, d={spec.d}) built by the oracle's grid route: {sum(counts)} "
                      f"builds on {threads} host threads in {wall:.1f} s of wall time (one event per thread at a "
                      f"time); and {len(runs)} builds on one thread, {sum(runs):.1f} s (median "
                      f"{statistics.median(runs):.3f} s)",
            "single_core": {"value": one, "unit": "events/s", "cores": 1},
            "host_cpu": host_cpu(), "host_cpus_visible": os.cpu_count()}


def kernel_source_digest() -> str:
    """First 16 hex digits of the SHA-256 of the kernel sources; a stored traffic
    figure is used only while it matches."""
    import hashlib
    h = hashlib.sha256()
    for f in ("frnn_kernels.hip", "frnn_internal.h"):
        with open(os.path.join(ROOT, "paper_2202_06929_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "single_event_120k.md")


def stored_traffic(kernel: str) -> int | None:
    """HBM bytes per launch of `kernel` from the committed counter summary, or None
    when the summary is missing or was taken from other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            text = f.read()
    except OSError:
        return None
    digest = None
    value = None
    for line in text.splitlines():
        if line.startswith("kernel sources sha256/16:"):
            digest = line.split(":", 1)[1].strip()
        if line.startswith(f"traffic {kernel} bytes per launch:"):
            value = int(line.split(":", 1)[1].strip())
    return value if digest == kernel_source_digest() else None


def stored_duration_us(kernel: str) -> float | None:
    """Average duration of `kernel` in the committed kernel-trace summary (rocprofv3),
    or None when it is missing or was taken from other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            text = f.read()
    except OSError:
        return None
    digest = None
    value = None
    for line in text.splitlines():
        if line.startswith("kernel sources sha256/16:"):
            digest = line.split(":", 1)[1].strip()
        cells = [c.strip() for c in line.strip().strip("|").split("|")]
        if value is None and len(cells) == 5 and cells[0] == kernel:
            try:
                value = float(cells[2])
            except ValueError:
                pass
    return value if digest == kernel_source_digest() else None


def stored_valu(kernel: str) -> float | None:
    """VALU issue utilisation of `kernel` from the committed counter summary, or
    None when it is missing or was taken from other kernel sources."""
    try:
        with open(TRAFFIC_FILE) as f:
            text = f.read()
    except OSError:
        return None
    digest = None
    value = None
    for line in text.splitlines():
        if line.startswith("kernel sources sha256/16:"):
            digest = line.split(":", 1)[1].strip()
        if line.startswith(f"valu {kernel} issue utilisation:"):
            value = float(line.split(":", 1)[1].strip())
    return value if digest == kernel_source_digest() else None


def identity() -> dict:
    """GPU, ROCm and host of this run."""
    import torch
    props = torch.cuda.get_device_properties(0)
    rocm = None
    for f in ("/opt/rocm/.info/version", "/opt/rocm/.info/version-dev"):
        try:
            with open(f) as fh:
                rocm = fh.read().strip()
                break
        except OSError:
            pass
    return {"gpu": props.name, "arch": getattr(props, "gcnArchName", "?"), "cus": props.multi_processor_count,
            "hbm_gib": round(props.total_memory / 2 ** 30, 1), "rocm": rocm, "hip_runtime": torch.version.hip,
            "torch": torch.__version__, "host_cpu": host_cpu(), "host_cpus_visible": os.cpu_count()}


def copy_bandwidth(gib: float = 1.0, reps: int = 10) -> dict:
    """Device-to-device copy of `gib` GiB: read + write bytes over the best HIP-event time."""
    import torch
    n = int(gib * 2 ** 30) // 4
    a = torch.ones(n, device="cuda:0")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    best = float("inf")
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        b.copy_(a)
        e.record()
        e.synchronize()
        best = min(best, s.elapsed_time(e) * 1e-3)
    gbs = 2 * n * 4 / best / 1e9
    del a, b
    torch.cuda.empty_cache()
    return {"gbs": gbs, "frac_of_peak": gbs / HBM_PEAK_GBS, "bytes_per_copy": 2 * n * 4,
            "how": f"torch copy of {gib:g} GiB on the device, best of {reps} HIP-event timings"}


def copy_probe() -> None:
    """A plain device copy of 256 MiB, five times: the calibration run for the HBM
    byte counters (FETCH_SIZE / WRITE_SIZE per dispatch against known bytes)."""
    import torch
    n = 64 * 1024 * 1024
    a = torch.rand(n, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_per_dispatch": n * 4, "dispatches": 5}), flush=True)


def batch_only(calls: int) -> None:
    """The benchmark's 64-event batch built `calls` times with one fixed config."""
    import numpy as np
    import torch

    from paper_2202_06929_amd import events, frnn
    sizes = events.batched_sizes()
    evs = [events.generate(events.batched_spec(n, 100 + k))[0] for k, n in enumerate(sizes)]
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pts = torch.from_numpy(np.concatenate(evs)).to("cuda:0")
    cfg = frnn.Config()
    for k in range(calls):
        edges, eo = frnn.build_batch(pts, offsets, 0.1, 256, cfg)
    torch.cuda.synchronize()
    print(json.dumps({"batch_calls": calls, "rows": int(offsets[-1]), "edges": int(eo[-1])}), flush=True)


def summarize_trace(title: str, trace_dir: str, command: str) -> str:
    """Markdown table of the library's kernel durations in one kernel-trace folder."""
    import csv
    import glob
    hits = glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True)
    if not hits:
        raise FileNotFoundError(f"kernel_stats.csv under {trace_dir}")

    def short(k):
        return k.replace("(anonymous namespace)::", "").replace("frnn::", "").replace("void ", "").split("(")[0]

    out = [f"# rocprofv3 summary: {title}", "", f"kernel sources sha256/16: {kernel_source_digest()}", "",
           f"command: `{command}`", "", "| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
    for r in csv.DictReader(open(hits[0])):
        if short(r["Name"]).startswith("k_"):
            out.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                       f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} |")
    return "\n".join(out + [""])


# MI355X issue model: 256 CUs x 4 SIMDs; a wave64 VALU instruction occupies a
# SIMD for 4 cycles, at most one per SIMD at a time.
SIMDS = 1024
VALU_CYCLES = 4


def summarize(trace_dir: str, fetch_dir: str, write_dir: str, cfetch_dir: str, cwrite_dir: str,
              commands: list[str], sq_dir: str | None = None, bench_line: str | None = None,
              lds_dir: str | None = None, lds_command: str | None = None) -> str:
    """Markdown summary of rocprofv3 outputs: kernel durations, HBM bytes per
    dispatch scaled by the copy calibration (beside each kernel's algorithmic
    bytes, from the event's n, d and E in the profiled run's own JSON line when
    given) and, given a folder of SQ/GRBM counters, VALU issue utilisation per
    kernel."""
    import csv
    import glob

    def one(d, name):
        hits = glob.glob(os.path.join(d, "**", name), recursive=True)
        if not hits:
            raise FileNotFoundError(f"{name} under {d}")
        return hits[0]

    def short(k):
        return k.replace("(anonymous namespace)::", "").replace("frnn::", "").replace("void ", "").split("(")[0]

    rows = [r for r in csv.DictReader(open(one(trace_dir, "*kernel_stats.csv"))) if short(r["Name"]).startswith("k_")]
    out = ["# rocprofv3 summary: single event, 120,000 points, 8-D float32, r=0.1, K=256", "",
           f"kernel sources sha256/16: {kernel_source_digest()}", "", "## Kernel durations", "",
           f"command: `{commands[0]}`", "", "| kernel | calls | avg us | min us | max us |", "|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| {short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                   f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} |")

    def counters(d, counter):
        acc = {}
        for r in csv.DictReader(open(one(d, "*counter_collection.csv"))):
            if r["Counter_Name"] == counter:
                acc.setdefault(short(r["Kernel_Name"]), []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in acc.items()}

    fetch, write = counters(fetch_dir, "FETCH_SIZE"), counters(write_dir, "WRITE_SIZE")
    cf, cw = counters(cfetch_dir, "FETCH_SIZE"), counters(cwrite_dir, "WRITE_SIZE")
    copy_kib = 256 * 1024
    ck = next(k for k in cf if "copy" in k.lower())
    f_scale, w_scale = copy_kib / cf[ck], copy_kib / cw[ck]
    out += ["", "## HBM bytes per dispatch", "", f"commands: `{commands[1]}`; `{commands[2]}`",
            f"calibration: `{commands[3]}`; `{commands[4]}`", "",
            f"copy kernel `{ck}` of 256 MiB reads FETCH_SIZE {cf[ck]:.0f} KiB and WRITE_SIZE {cw[ck]:.0f} KiB "
            f"per dispatch: scale factors fetch x{f_scale:.3f}, write x{w_scale:.3f}", "",
            "| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | scaled bytes | algorithmic bytes | counted / algorithmic |",
            "|---|---|---|---|---|---|"]
    ev = None
    if bench_line:
        with open(bench_line) as f:
            for line in f:
                if line.startswith("{"):
                    ev = json.loads(line)
    ours = [k for k in fetch if k.startswith("k_")]
    for k in ours:
        b = int(round((fetch[k] * f_scale + write.get(k, 0.0) * w_scale) * 1024))
        alg = None
        if ev is not None:
            alg = kernel_bytes(k, ev["config"]["n"], ev["config"]["d"], ev["edges"], ev["config"]["axes"])
        a_txt = f"{alg}" if alg else "—"
        r_txt = f"{b / alg:.2f}" if alg else "—"
        out.append(f"| {k} | {fetch[k]:.1f} | {write.get(k, 0.0):.1f} | {b} | {a_txt} | {r_txt} |")
    if ev is not None:
        out += ["", f"algorithmic bytes for n = {ev['config']['n']}, d = {ev['config']['d']}, "
                    f"E = {ev['edges']}, {ev['config']['axes']} binned coordinates (the profiled run's own line)"]
    lines = []
    for k in ours:
        b = int(round((fetch[k] * f_scale + write.get(k, 0.0) * w_scale) * 1024))
        lines.append(f"traffic {k} bytes per launch: {b}")
    if sq_dir is not None:
        dur = {short(r["Name"]): float(r["AverageNs"]) * 1e-9 for r in rows}
        sq = {c: counters(sq_dir, c) for c in ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS",
                                             "SQ_INSTS_SMEM")}
        cmd = commands[5] if len(commands) > 5 else "?"
        out += ["## VALU issue utilisation", "", f"command: `{cmd}`", "",
                f"utilisation = SQ_INSTS_VALU x {VALU_CYCLES} cycles / (average duration x 2.4 GHz x {SIMDS} SIMDs): "
                "the share of the SIMDs' cycles that issued VALU work", "",
                "| kernel | waves | VALU instr | SALU instr | LDS instr | SMEM instr | VALU util |",
                "|---|---|---|---|---|---|---|"]
        vlines = []
        for k in ours:
            if k not in sq["SQ_INSTS_VALU"] or k not in dur:
                continue
            t = dur[k]
            util = sq["SQ_INSTS_VALU"][k] * VALU_CYCLES / (t * 2.4e9 * SIMDS)
            out.append(f"| {k} | {sq['SQ_WAVES'].get(k, 0):.0f} | {sq['SQ_INSTS_VALU'][k]:.0f} | "
                       f"{sq['SQ_INSTS_SALU'].get(k, 0):.0f} | {sq['SQ_INSTS_LDS'].get(k, 0):.0f} | "
                       f"{sq['SQ_INSTS_SMEM'].get(k, 0):.0f} | {util:.3f} |")
            vlines.append(f"valu {k} issue utilisation: {util:.4f}")
        out += [""] + vlines + [""]
    if lds_dir is not None:
        conf, occ = counters(lds_dir, "LdsBankConflict"), counters(lds_dir, "MeanOccupancyPerCU")
        out += ["## LDS bank conflicts and occupancy", "", f"command: `{lds_command or '?'}`", "",
                "LdsBankConflict: bank-conflict cycles per LDS access cycle (SQ_LDS_BANK_CONFLICT over "
                "SQ_LDS_IDX_ACTIVE less the conflicts); MeanOccupancyPerCU: resident waves per CU averaged over "
                "the kernel's time", "", "| kernel | LDS bank conflicts per access | mean waves per CU |", "|---|---|---|"]
        for k in ours:
            if k in conf or k in occ:
                c = f"{conf[k]:.3f}" if k in conf else "—"
                o = f"{occ[k]:.1f}" if k in occ else "—"
                out.append(f"| {k} | {c} | {o} |")
        out.append("")
    out += [""] + lines + [""]
    return "\n".join(out)


def batched_bench(steps: int, warmup: int, log) -> dict:
    """64 events of 20k-150k hits in one launch sequence, captured in a HIP graph.

    Compares the plain loop (one frnn_build per event) with one batched call and
    with replays of the captured batch; every batched event's edges are checked
    byte-for-byte against the same event built alone.
    """
    import numpy as np
    import torch

    from paper_2202_06929_amd import events, frnn, tune

    sizes = events.batched_sizes()
    evs = [events.generate(events.batched_spec(n, 100 + k))[0] for k, n in enumerate(sizes)]
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    dev = torch.device("cuda:0")
    pts = torch.from_numpy(np.concatenate(evs)).to(dev)
    r, K, d = 0.1, 256, 8
    cfg, treport = tune.tune(pts, offsets, r, K, log=log)
    log(f"batched: tuned config {cfg} ({treport.get('seconds', 0) * 1e3:.2f} ms per batch)")

    # Plain loop: one call (and one synchronisation) per event.
    views = [pts[int(offsets[k]):int(offsets[k + 1])] for k in range(len(sizes))]
    caps = [16 * n for n in sizes]
    wss = [torch.empty(frnn.workspace_bytes(n, d), dtype=torch.uint8, device=dev) for n in sizes]
    outs = [torch.empty((2, c), dtype=torch.int64, device=dev) for c in caps]
    alone = []
    for k in range(len(sizes)):
        st, E = frnn.build_into(views[k], r, K, wss[k], outs[k][0], outs[k][1], cfg)
        assert st == frnn.FRNN_OK
        alone.append(outs[k][:, :E].cpu())
    def plain_pass():
        for k in range(len(sizes)):
            frnn.build_into(views[k], r, K, wss[k], outs[k][0], outs[k][1], cfg)
    for _ in range(max(1, warmup // 4)):
        plain_pass()
    torch.cuda.synchronize()
    t = time.perf_counter()
    reps = max(2, steps // 20)
    for _ in range(reps):
        plain_pass()
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t) / reps

    # One batched call, then a captured graph of the same batch replayed.
    total_e = sum(a.shape[1] for a in alone)
    cap = total_e + 4096
    ws = torch.empty(frnn.batch_workspace_bytes(offsets, d), dtype=torch.uint8, device=dev)
    out = torch.empty((2, cap), dtype=torch.int64, device=dev)
    st, eo = frnn.build_batch_into(pts, offsets, r, K, ws, out[0], out[1], cfg)
    assert st == frnn.FRNN_OK and eo[-1] == total_e
    for k in range(len(sizes)):
        got = out[:, int(eo[k]):int(eo[k + 1])].cpu()
        assert torch.equal(got, alone[k]), f"event {k}: batched edges differ from the event alone"
    t = time.perf_counter()
    for _ in range(reps):
        frnn.build_batch_into(pts, offsets, r, K, ws, out[0], out[1], cfg)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t) / reps

    eo_dev = torch.zeros(len(sizes) + 2, dtype=torch.int64, device=dev)
    rcfg = dataclasses.replace(cfg, events_resident=True)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        st = frnn.build_batch_async(pts, offsets, r, K, ws, out[0], out[1], eo_dev, rcfg)
        assert st == frnn.FRNN_OK
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        st = frnn.build_batch_async(pts, offsets, r, K, ws, out[0], out[1], eo_dev, rcfg)
    assert st == frnn.FRNN_OK
    for _ in range(3):
        out.fill_(-1)
        graph.replay()
        torch.cuda.synchronize()
        e_host = eo_dev.cpu().numpy()
        assert e_host[-1] == 0 and np.array_equal(e_host[:-1], eo), "graph replay: wrong edge ranges"
        for k in (0, len(sizes) // 2, len(sizes) - 1):
            assert torch.equal(out[:, int(eo[k]):int(eo[k + 1])].cpu(), alone[k]), "graph replay: edges differ"
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record()
    for _ in range(reps):
        graph.replay()
    end.record()
    torch.cuda.synchronize()
    t_graph = start.elapsed_time(end) * 1e-3 / reps
    n_ev = len(sizes)
    return {"workload": f"batched: {n_ev} events, hits uniform in [20000, 150000] (total {int(offsets[-1])}), "
                        "8-D float32, r=0.1, K=256",
            "config": {"dims": list(cfg.dims) if cfg.dims else None, "axes": cfg.axes, "cell_div": cfg.cell_div,
                       "grid_mult": cfg.grid_mult},
            "events_per_s_plain_loop": n_ev / t_plain, "events_per_s_batched_call": n_ev / t_batch,
            "events_per_s_graph": n_ev / t_graph, "ms_per_batch_graph": t_graph * 1e3,
            "edges_per_s_graph": total_e / t_graph, "edges": total_e,
            "speedup_graph_vs_plain": t_plain / t_graph, "parity": "every event identical to the event alone",
            "tune": treport.get("all")}


SERVED_LOADS = (0.5, 0.8, 1.0, 1.2, 2.0)


def served_bench(log, n_arrivals: int = 1000, n_distinct: int = 250, loads=SERVED_LOADS) -> dict:
    """Poisson arrivals of events with log-uniform hit counts in [10k, 300k].

    n_distinct events are drawn once (sizes log-uniform in [10k, 300k]) and request
    k carries event k mod n_distinct.  The plain loop's capacity (events/s of one
    synchronous call per event, back to back) is measured first; then, for every
    offered load in `loads` (a multiple of that capacity), the same trace of
    n_arrivals Poisson arrivals runs through the plain loop and through the
    continuous-batching server, and every served result is compared byte for byte
    with the plain loop's result for the same request.
    """
    import numpy as np
    import torch

    from paper_2202_06929_amd import events, frnn, serve

    r, K, d = 0.1, 256, 8
    base = events.served_trace(n_arrivals, rate_hz=1.0)
    pts = [events.generate(events.batched_spec(n, 10_000 + k))[0] for k, (_, n) in enumerate(base[:n_distinct])]
    dev = torch.device("cuda:0")
    dev_pts = [torch.from_numpy(x).to(dev) for x in pts]
    ev_of = [k % n_distinct for k in range(n_arrivals)]

    def build(req):
        return frnn.build(req.points, r, K)

    # Plain-loop capacity on these events (warm, back to back).
    for k in range(10):
        build(serve.Request(rid=k, arrival=0.0, points=dev_pts[k]))
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k in range(n_arrivals):
        build(serve.Request(rid=k, arrival=0.0, points=dev_pts[ev_of[k]]))
    torch.cuda.synchronize()
    capacity = n_arrivals / (time.perf_counter() - t)

    def idle(until):
        while time.perf_counter() < until:
            pass

    ex = serve.GpuExecutor(r, K, d, n_streams=3)
    warm = [serve.Request(rid=k, arrival=0.0, points=dev_pts[k]) for k in range(40)]
    serve.Server(ex, hbm_budget=64 << 30, max_batch=64, idle=idle).run(warm)
    rows = []
    for load in loads:
        rate = load * capacity
        arrivals = [a / rate for a, _ in base]  # the unit-rate trace scaled to the offered rate

        def trace():
            return [serve.Request(rid=k, arrival=arrivals[k], points=dev_pts[ev_of[k]]) for k in range(n_arrivals)]

        plain_trace = trace()
        plain = serve.plain_loop(plain_trace, build, idle=idle)
        served_trace = trace()
        served = serve.Server(ex, hbm_budget=64 << 30, max_batch=64, idle=idle).run(served_trace)
        same = all(q.status == serve.OK and torch.equal(q.edges, p.edges) for q, p in zip(served_trace, plain_trace))
        if not same:
            raise RuntimeError(f"served results differ from the plain loop's at load {load}")
        log(f"served x{load}: plain p50 {plain.p50_ms:.2f} p99 {plain.p99_ms:.2f} ms, {plain.events_per_s:.0f}/s; "
            f"server p50 {served.p50_ms:.2f} p99 {served.p99_ms:.2f} ms, {served.events_per_s:.0f}/s, "
            f"mean batch {served.mean_batch:.1f}")
        rows.append({"load": load, "offered_events_per_s": rate, "plain": plain.as_dict(), "server": served.as_dict(),
                     "server_vs_plain_events_per_s": served.events_per_s / plain.events_per_s,
                     "server_vs_plain_p99": served.p99_ms / plain.p99_ms})
    return {"workload": f"served: {n_arrivals} Poisson arrivals per load, each carrying one of {n_distinct} events "
                        "with hits log-uniform in [10000, 300000] (8-D float32, r=0.1, K=256), HBM budget 64 GB, "
                        "3 streams, batches of at most 64",
            "plain_capacity_events_per_s": capacity, "loads": rows,
            "parity": "every served result identical to the plain loop's result for the same request"}


def labeling_bench(spec, X, pts, steps: int, warmup: int, log, cpu: bool) -> dict:
    """Track labeling (weakly connected components) of the event's FRNN graph.

    Steps run back to back through frnn_components_async, each result slot checked
    afterwards; one launch of each kernel is timed with HIP events on the stream.
    The labels are compared with the CPU oracle's on the oracle's own edge list.
    """
    import numpy as np
    import torch

    from paper_2202_06929_amd import frnn

    dev = pts.device
    edges = frnn.build(pts, spec.r, spec.K)
    src, dst = edges[0].contiguous(), edges[1].contiguous()
    n, E = spec.n, int(src.numel())
    ws = torch.empty(frnn.components_workspace_bytes(n), dtype=torch.uint8, device=dev)
    lab = torch.empty(n, dtype=torch.int64, device=dev)
    res = torch.full((warmup + steps, 2), -1, dtype=torch.int64, device=dev)
    for w in range(warmup):
        frnn.components_async(src, dst, n, ws, lab, res[w])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        frnn.components_async(src, dst, n, ws, lab, res[warmup + k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    r = res.cpu().numpy()
    if not ((r[:, 1] == 0).all() and (r[:, 0] == r[0, 0]).all()):
        raise RuntimeError("a labeling step failed")
    got = lab.cpu().numpy()
    from oracle import components as cc_oracle
    from oracle import oracle
    g = oracle.frnn_grid(X, spec.r, spec.K)
    want = cc_oracle.labels(g[0], g[1], n)
    if not np.array_equal(got, want):
        raise RuntimeError("labels differ from the oracle")
    # Algorithmic bytes: both endpoint arrays read once (16 E), the parent array
    # written, read back and the int64 labels written (4 n + 4 n + 8 n).
    alg = 16 * E + 16 * n
    per = wall / steps
    out = {"workload": f"labels of the single event's FRNN graph: {n} vertices, {E} edges",
           "events_per_s": steps / wall, "ms_per_event": per * 1e3, "components": int(r[0, 0]),
           "hbm_gbs_algorithmic": alg / per / 1e9, "hbm_frac": alg / per / 1e9 / HBM_PEAK_GBS,
           "alg_bytes": alg, "parity": "labels identical to the oracle's"}
    if cpu:
        runs = []
        t = time.perf_counter()
        while len(runs) < 3 or time.perf_counter() - t < 3.0:
            a = time.perf_counter()
            cc_oracle.labels(g[0], g[1], n)
            runs.append(time.perf_counter() - a)
        out["cpu_oracle_events_per_s"] = len(runs) / sum(runs)
    log(f"labeling: {out['ms_per_event']:.3f} ms per event, {out['components']} components")
    return out


def main():
    args = parse()
    if args.batch_only:
        batch_only(args.batch_only)
        return
    if args.summarize_trace:
        title, trace, command = args.summarize_trace
        print(summarize_trace(title, trace, command))
        return
    if args.summarize:
        if len(args.summarize) not in (5, 6):
            raise SystemExit("--summarize takes TRACE FETCH WRITE CFETCH CWRITE [SQ]")
        cmds = args.commands or ["?"] * len(args.summarize)
        print(summarize(*args.summarize[:5], commands=cmds,
                        sq_dir=args.summarize[5] if len(args.summarize) == 6 else None,
                        bench_line=args.bench_line, lds_dir=args.lds[0] if args.lds else None,
                        lds_command=args.lds[1] if args.lds else None))
        return
    if args.copy_probe:
        copy_probe()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(events are independent, so more GPUs would each run this same path)", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2202_06929_amd import events, frnn

    spec = {"single": events.SINGLE, "high": events.HIGH, "tiny": events.TINY, "knn": events.KNN}[args.workload]
    X, _ = events.generate(spec)
    dev = torch.device("cuda:0")
    pts = torch.from_numpy(X).to(dev)
    n, d = X.shape
    cfg = frnn.Config(cell_div=args.cell_div or 1, axes=args.axes)
    cap = 16 * n
    offs = np.array([0, n], dtype=np.int64)
    ws = torch.empty(max(frnn.workspace_bytes(n, d), frnn.batch_workspace_bytes(offs, d)),
                     dtype=torch.uint8, device=dev)
    out = torch.empty((2, cap), dtype=torch.int64, device=dev)

    def step(config=cfg, stats=None):
        st, E = frnn.build_into(pts, spec.r, spec.K, ws, out[0], out[1], config, stats)
        if st != frnn.FRNN_OK:
            raise frnn.FrnnError(st, frnn.status_string(st))
        return E

    E = step()
    # Throughput: K steps back to back through the asynchronous entry point (edge
    # range and status land in device memory, one slot per step, so no step waits
    # for the host; the call's fixed arguments are marshalled once); every step's
    # status and edge count are checked afterwards.
    eo = torch.full((args.warmup + args.steps, 3), -1, dtype=torch.int64, device=dev)
    slots = [eo[k] for k in range(args.warmup + args.steps)]
    src, dst = out[0], out[1]
    # Python's cyclic garbage collector is off while steps are enqueued and timed
    # (as timeit does): a collection in the middle of the loop stalled the host for
    # over a millisecond, which left the GPU idle and showed in short timed regions.
    gc.collect()
    gc.disable()
    call = frnn.AsyncBatch(pts, offs, spec.r, spec.K, ws, src, dst, cfg)
    for w in range(args.warmup):
        call(slots[w])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        call(slots[args.warmup + k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    events_per_s = args.steps / wall
    eo_h = eo.cpu().numpy()
    if not ((eo_h[:, 2] == 0).all() and (eo_h[:, 1] == E).all() and (eo_h[:, 0] == 0).all()):
        raise RuntimeError(f"a pipelined step failed: statuses {set(eo_h[:, 2].tolist())}, counts {set(eo_h[:, 1].tolist())}")

    # Latency: synchronous calls, each waiting for its edge count on the host
    # (at least LATENCY_SAMPLES of them, so that p99 is not the maximum).
    lat = []
    n_lat = max(LATENCY_SAMPLES, args.steps)
    t1 = time.perf_counter()
    for _ in range(n_lat):
        a = time.perf_counter()
        step()
        lat.append(time.perf_counter() - a)
    sync_events_per_s = n_lat / (time.perf_counter() - t1)

    # Same steps again with HIP events around every stage (on the stream the
    # kernels run on) for the per-kernel durations of the roofline.
    tcfg = dataclasses.replace(cfg, timing=True)
    stage_sum = {k: 0.0 for k in frnn.STAGES}
    stats = frnn.FrnnStats()
    for _ in range(args.steps):
        step(tcfg, stats)
        for k, v in stats.as_dict()["stage_ms"].items():
            stage_sum[k] += v
    stage_ms = {k: v / args.steps for k, v in stage_sum.items()}
    gc.enable()
    st = stats.as_dict()
    # Pairs the paper's three-coordinate grid examines for the same edges (one call
    # with three binned coordinates, same cell edge): the work this search replaces.
    st3 = frnn.FrnnStats()
    E3 = step(dataclasses.replace(cfg, axes=3, dims=None), st3)
    if E3 != E:
        raise RuntimeError(f"three binned coordinates gave {E3} edges, four gave {E}")
    pairs3 = st3.as_dict()["candidates"]

    dpad = next(p for p in (4, 8, 12, 16, 24, 32, 48, 64) if d <= p)
    t_search = stage_ms["search"] * 1e-3
    sb = search_bytes(n, dpad, st["n_cells"], E)
    # Algorithmic work of the search: 3d + 1 FP32 operations (d differences, d
    # squares, d sums, one comparison) per examined pair, no early exit counted.
    ops = st["candidates"] * (3 * d + 1)
    # Executed work: every examined pair gets its leading terms (two for rows of up to
    # 8 floats, four for 12-float rows, three for wider ones) and a comparison; pairs
    # below r2 after them get the remaining terms of the padded row and a comparison.
    lead = 2 if dpad <= 8 else (4 if dpad == 12 else 3)
    executed = st["candidates"] * (3 * lead + 1) + st["survivors"] * (3 * (dpad - lead) + 1)
    kname = f"k_search<{dpad}, {'true' if spec.K < 16 else 'false'}>"
    # The same kernel's average under rocprofv3 (committed summary of the default
    # run, same sources): HIP events around a kernel also count its dispatch.
    prof_us = stored_duration_us(kname) if args.workload == "single" else None
    roofline = {"bound": "alu", "achieved": ops / t_search / 1e12, "peak": FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": ops / t_search / 1e12 / FP32_PEAK_TFLOPS,
                "traffic": stored_traffic(kname) if args.workload == "single" else None, "kernel": kname, "kernel_us": t_search * 1e6,
                "work": f"{st['candidates']} examined pairs x (3d+1) FP32 ops = {ops}",
                "timing": "HIP events on the call's stream around the search kernel, averaged over a second "
                          "pass of the same steps",
                "plain_lane_peak": PLAIN_LANE_PEAK_TOPS,
                "frac_of_plain_lane_peak": ops / t_search / 1e12 / PLAIN_LANE_PEAK_TOPS,
                "executed_ops": executed, "survivors": st["survivors"],
                "executed_frac": executed / t_search / 1e12 / FP32_PEAK_TFLOPS,
                "kernel_us_profile": prof_us,
                "frac_profile": ops / (prof_us * 1e-6) / 1e12 / FP32_PEAK_TFLOPS if prof_us else None,
                "three_coordinate_grid_pairs": pairs3,
                "three_coordinate_grid_frac": pairs3 * (3 * d + 1) / t_search / 1e12 / FP32_PEAK_TFLOPS,
                "valu_issue_util": stored_valu(kname) if args.workload == "single" else None}
    roofline_hbm = {"bound": "hbm", "achieved": sb / t_search / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": sb / t_search / 1e9 / HBM_PEAK_GBS, "bytes": sb}
    t_step = wall / args.steps
    pb = path_bytes(n, d, E)
    lat_ms = sorted(x * 1e3 for x in lat)
    result = {
        "metric": METRIC if args.workload == "single" else f"events/s ({args.workload} event)",
        "value": events_per_s, "unit": "events/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_step * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload} event: {n} points, {d}-D float32, r={spec.r}, K={spec.K}",
                   "n": n, "d": d, "r": spec.r, "K": spec.K, "seed": spec.seed,
                   "cell_div": cfg.cell_div, "axes": st["axes"], "dims": st["dims"], "grid": st["grid"]},
        "edges": E, "edges_per_s": E * events_per_s,
        "timing": "value: steps pipelined on one stream through frnn_build_batch_async (no host round trip per "
                  "step); p50/p99 and sync_events_per_s: synchronous frnn_build calls, each returning its edge "
                  "count to the host",
        "sync_events_per_s": sync_events_per_s,
        "p50_ms": lat_ms[len(lat_ms) // 2], "p99_ms": lat_ms[min(len(lat_ms) - 1, int(0.99 * len(lat_ms)))],
        "latency_samples": n_lat,
        "path_hbm_gbs": pb / t_step / 1e9, "path_hbm_frac": pb / t_step / 1e9 / HBM_PEAK_GBS,
        "path_hbm_target_frac": PATH_HBM_TARGET, "path_bytes": pb,
        "stage_us": {k: v * 1e3 for k, v in stage_ms.items()},
        "candidates": st["candidates"],
        "roofline": roofline, "roofline_hbm": roofline_hbm,
    }
    result["identity"] = identity()
    result["copy_bandwidth"] = copy_bandwidth()
    result["path_hbm_frac_of_copy"] = result["path_hbm_gbs"] / result["copy_bandwidth"]["gbs"]
    if args.workload == "single" and not args.no_labeling:
        result["labeling"] = labeling_bench(spec, X, pts, args.steps, args.warmup, log, not args.no_cpu_baseline)
    if not args.no_batched:
        result["batched"] = batched_bench(args.steps, args.warmup, log)
    if not args.no_served:
        result["served"] = served_bench(log)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(spec, X)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
