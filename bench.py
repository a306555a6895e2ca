"""Benchmark of the FRNN graph build on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload single|high|tiny]

A step is one whole frnn_build call over one synthetic event already resident in
HBM: bounds, keys, cell scan, scatter, neighbour search, long lists, offsets and
edge placement, plus the read-back of the edge count.  The default workload is
the single event of 120,000 points in 8-D (r = 0.1, K = 256).

Prints one JSON line with throughput (events/s), edges/s, per-event latency
percentiles, the roofline of the dominant kernel (the neighbour search) from
HIP-event timings taken inside this run, and the CPU oracle timed on this host.
"""

from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks.  Plain FP32 VALU lane-ops: 256 CUs x 64 lanes x 2.4 GHz
# = 39.3 T/s (the 157.3 TFLOP/s vector figure counts fused multiply-add as two
# and packed FP32 as two lanes; this path may use neither).
HBM_PEAK_GBS = 8000.0
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", choices=["single", "high", "tiny"], default="single")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cell-div", type=int, default=None)
    return ap.parse_args()


def search_bytes(n: int, dpad: int, n_cells: int, E: int) -> int:
    """Algorithmic HBM bytes of one search launch: each sorted row read once,
    row ids, cell starts, kept counts and list positions, the unsorted edge store."""
    return n * dpad * 4 + 4 * n + 4 * (n_cells + 1) + 4 * n + 8 * n + 4 * E


def path_bytes(n: int, d: int, E: int) -> int:
    """Algorithmic HBM bytes of the whole path per event: points read for bounds,
    keys and scatter, sorted rows written and read by the search (5 n d 4), about
    40 bytes of per-point indices, and 16 bytes per int64 edge."""
    return 5 * n * d * 4 + 40 * n + 16 * E


def cpu_baseline(spec, X) -> dict:
    from oracle import oracle
    oracle.load()
    runs = []
    for _ in range(3):
        t = time.perf_counter()
        oracle.frnn_grid(X, spec.r, spec.K)
        runs.append(time.perf_counter() - t)
    med = statistics.median(runs)
    return {"value": 1.0 / med, "unit": "events/s", "cores": 1, "kind": "oracle",
            "sample": f"one full event (n={spec.n}, d={spec.d}), grid route, single thread, "
                      f"median of 3 runs ({med:.2f} s each)"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(events are independent, so more GPUs would each run this same path)", file=sys.stderr)
        sys.exit(2)
    import torch

    from paper_2202_06929_amd import events, frnn

    spec = {"single": events.SINGLE, "high": events.HIGH, "tiny": events.TINY}[args.workload]
    X, _ = events.generate(spec)
    dev = torch.device("cuda:0")
    pts = torch.from_numpy(X).to(dev)
    n, d = X.shape
    cfg = frnn.Config(cell_div=args.cell_div) if args.cell_div else frnn.Config()
    cap = 16 * n
    ws = torch.empty(frnn.workspace_bytes(n, d, cap), dtype=torch.uint8, device=dev)
    out = torch.empty((2, cap), dtype=torch.int64, device=dev)

    def step(config=cfg, stats=None):
        st, E = frnn.build_into(pts, spec.r, spec.K, ws, out[0], out[1], config, stats)
        if st != frnn.FRNN_OK:
            raise frnn.FrnnError(st, frnn.status_string(st))
        return E

    for _ in range(args.warmup):
        E = step()
    torch.cuda.synchronize()
    lat = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        a = time.perf_counter()
        E = step()
        lat.append(time.perf_counter() - a)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    events_per_s = args.steps / wall

    # Same steps again with HIP events around every stage (on the stream the
    # kernels run on) for the per-kernel durations of the roofline.
    tcfg = frnn.Config(dims=cfg.dims, cell_div=cfg.cell_div, timing=True)
    stage_sum = {k: 0.0 for k in frnn.STAGES}
    stats = frnn.FrnnStats()
    for _ in range(args.steps):
        step(tcfg, stats)
        for k, v in stats.as_dict()["stage_ms"].items():
            stage_sum[k] += v
    stage_ms = {k: v / args.steps for k, v in stage_sum.items()}
    st = stats.as_dict()

    dpad = next(p for p in (4, 8, 12, 16, 24, 32, 48, 64) if d <= p)
    t_search = stage_ms["search"] * 1e-3
    sb = search_bytes(n, dpad, st["n_cells"], E)
    ops = st["candidates"] * (3 * d + 1)
    roofline = {"bound": "alu", "achieved": ops / t_search / 1e12, "peak": VALU_PEAK_TOPS,
                "unit": "TFLOP/s", "frac": ops / t_search / 1e12 / VALU_PEAK_TOPS, "traffic": None,
                "kernel": "k_search", "kernel_us": t_search * 1e6,
                "work": f"{st['candidates']} candidate pairs x (3d+1) FP32 ops"}
    roofline_hbm = {"bound": "hbm", "achieved": sb / t_search / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": sb / t_search / 1e9 / HBM_PEAK_GBS, "bytes": sb}
    t_step = wall / args.steps
    pb = path_bytes(n, d, E)
    lat_ms = sorted(x * 1e3 for x in lat)
    result = {
        "metric": "events/s at 120k hits" if args.workload == "single" else f"events/s ({args.workload} event)",
        "value": events_per_s, "unit": "events/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": t_step * 1e3, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{args.workload} event: {n} points, {d}-D float32, r={spec.r}, K={spec.K}",
                   "n": n, "d": d, "r": spec.r, "K": spec.K, "seed": spec.seed,
                   "cell_div": cfg.cell_div, "dims": st["dims"], "grid": st["grid"]},
        "edges": E, "edges_per_s": E * events_per_s,
        "p50_ms": lat_ms[len(lat_ms) // 2], "p99_ms": lat_ms[min(len(lat_ms) - 1, int(0.99 * len(lat_ms)))],
        "path_hbm_gbs": pb / t_step / 1e9, "path_hbm_frac": pb / t_step / 1e9 / HBM_PEAK_GBS,
        "stage_us": {k: v * 1e3 for k, v in stage_ms.items()},
        "candidates": st["candidates"],
        "roofline": roofline, "roofline_hbm": roofline_hbm,
    }
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(spec, X)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
