"""Parity of the HIP path with the CPU oracle: identical bytes, edge for edge.

The edge list is unique (definition in include/frnn.h), so the bar is exact
equality of the int64 [2, E] arrays.  Every case runs through the C interface
via the ctypes binding.
"""

import functools
import os
import sys

import numpy as np
import pytest
import torch

from oracle import invariants, oracle
from paper_2202_06929_amd import events, frnn

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_edges(X, r, K, **kw):
    pts = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(DEV)
    e = frnn.build(pts, r, K, **kw)
    torch.cuda.synchronize()
    return e.cpu().numpy()


@functools.lru_cache(maxsize=None)
def event_and_oracle(name):
    spec = {"tiny": events.TINY, "single": events.SINGLE, "high": events.HIGH}[name]
    X, _ = events.generate(spec)
    return spec, X, oracle.frnn_grid(X, spec.r, spec.K)


def assert_same(got, want):
    assert got.dtype == np.int64 and want.dtype == np.int64
    assert got.shape == want.shape, (got.shape, want.shape)
    if not np.array_equal(got, want):
        bad = np.flatnonzero((got != want).any(0))[:5]
        raise AssertionError(f"first differing edges at {bad.tolist()}: got {got[:, bad].T.tolist()} "
                             f"want {want[:, bad].T.tolist()}")


@pytest.mark.parametrize("name", ["tiny", "single", "high"])
def test_workload_events_match_oracle(name):
    spec, X, want = event_and_oracle(name)
    log(f"parity {name}: n={spec.n} d={spec.d} r={spec.r} K={spec.K}")
    got, st = frnn.build(torch.from_numpy(X).to(DEV), spec.r, spec.K, return_stats=True)
    torch.cuda.synchronize()
    assert_same(got.cpu().numpy(), want)
    assert st["n_edges"] == want.shape[1]
    assert st["capped_queries"] == 0


@pytest.mark.parametrize("case", events.stress_cases(), ids=lambda c: c.name)
def test_stress_cases_match_oracle(case):
    log(f"stress {case.name}: n={len(case.points)} r={case.r} K={case.K}")
    want = oracle.frnn_grid(case.points, case.r, case.K)
    got = gpu_edges(case.points, case.r, case.K)
    assert_same(got, want)


@pytest.mark.parametrize("d", [3, 4, 5, 7, 8, 9, 12, 13, 16, 17, 24, 31, 48, 64])
def test_every_dimension_bucket(d):
    spec = events.EventSpec(n=3000, d=d, n_clusters=250, size_lo=5, size_hi=15, sigma=0.02,
                            noise_frac=0.1, r=0.1 * max(1.0, (d / 8) ** 0.5), K=16, seed=100 + d)
    X, _ = events.generate(spec)
    log(f"dimension d={d}")
    assert_same(gpu_edges(X, spec.r, spec.K), oracle.frnn_grid(X, spec.r, spec.K))


@pytest.mark.parametrize("cfg", [
    frnn.Config(), frnn.Config(axes=3), frnn.Config(dims=(0, 1, 2)), frnn.Config(dims=(2, 0, 5)),
    frnn.Config(dims=(0, 1, 2, 3)), frnn.Config(dims=(6, 0, 3, 5)),
    frnn.Config(cell_div=2), frnn.Config(cell_div=3), frnn.Config(dims=(0, 1, 2), cell_div=2),
    frnn.Config(grid_mult=1), frnn.Config(grid_mult=8), frnn.Config(axes=3, grid_mult=8),
], ids=["default", "three_axes", "lead_dims", "mixed_dims", "lead_dims4", "mixed_dims4", "div2", "div3",
        "lead_div2", "grid1", "grid8", "three_axes_grid8"])
@pytest.mark.parametrize("name", ["tiny", "single"])
def test_every_config_gives_the_same_edges(cfg, name):
    spec, X, want = event_and_oracle(name)
    log(f"config {cfg} on {name}")
    assert_same(gpu_edges(X, spec.r, spec.K, config=cfg), want)


@pytest.mark.parametrize("d", [4, 5])
def test_four_axes_on_few_coordinates(d):
    """Four binned coordinates when d is 4 (every coordinate binned, so the
    leading terms of the sum are binned too) and 5."""
    spec = events.EventSpec(n=4000, d=d, n_clusters=300, size_lo=5, size_hi=15, sigma=0.02,
                            noise_frac=0.1, r=0.1, K=32, seed=60 + d)
    X, _ = events.generate(spec)
    log(f"four axes, d={d}")
    want = oracle.frnn_grid(X, spec.r, spec.K)
    got, st = frnn.build(torch.from_numpy(X).to(DEV), spec.r, spec.K, config=frnn.Config(axes=4),
                         return_stats=True)
    torch.cuda.synchronize()
    assert st["axes"] == 4 and st["dims"] == list(range(d - 4, d))
    assert_same(got.cpu().numpy(), want)


def test_repeated_runs_are_identical():
    spec, X, want = event_and_oracle("single")
    pts = torch.from_numpy(X).to(DEV)
    first = frnn.build(pts, spec.r, spec.K).cpu().numpy()
    for _ in range(9):
        assert np.array_equal(frnn.build(pts, spec.r, spec.K).cpu().numpy(), first)
    assert_same(first, want)


def test_capacity_error_reports_the_needed_count_and_retry_succeeds():
    spec, X, want = event_and_oracle("tiny")
    pts = torch.from_numpy(X).to(DEV)
    n, d = X.shape
    cap = 100
    ws = torch.empty(frnn.workspace_bytes(n, d), dtype=torch.uint8, device=DEV)
    out = torch.empty((2, cap), dtype=torch.int64, device=DEV)
    st, E = frnn.build_into(pts, spec.r, spec.K, ws, out[0], out[1])
    assert st == frnn.FRNN_ERR_CAPACITY and E == want.shape[1]
    got = frnn.build(pts, spec.r, spec.K, capacity=100)  # retries once with the exact count
    assert_same(got.cpu().numpy(), want)
    exact = frnn.build(pts, spec.r, spec.K, capacity=E)
    assert exact.is_contiguous()
    assert_same(exact.cpu().numpy(), want)


def test_non_finite_input_is_rejected():
    X, _ = events.generate(events.TINY)
    for bad in (np.nan, np.inf, -np.inf):
        Y = X.copy()
        Y[777, 5] = bad
        with pytest.raises(frnn.FrnnError) as e:
            gpu_edges(Y, 0.1, 64)
        assert e.value.status == frnn.FRNN_ERR_NONFINITE
    # a good call right after an error still works
    assert_same(gpu_edges(X, 0.1, 64), event_and_oracle("tiny")[2])


def test_dyadic_exact_points():
    X, _ = events.dyadic_event(5000, 8, 9)
    assert_same(gpu_edges(X, 0.2, 64), oracle.frnn_grid(X, 0.2, 64))


def test_ragged_sizes_and_small_events():
    rng = np.random.Generator(np.random.PCG64(5))
    for n in (1, 2, 3, 63, 64, 65, 255, 256, 257, 4095, 4096, 4097, 9001):
        X = rng.uniform(-0.3, 0.3, size=(n, 6)).astype(np.float32)
        log(f"ragged n={n}")
        assert_same(gpu_edges(X, 0.15, 20), oracle.frnn_grid(X, 0.15, 20))


def test_invariants_on_the_high_occupancy_event():
    """Every property of the definition on the 300k 12-D event's GPU edges: no
    self-loops, D < r2 for every edge (recomputed by the oracle's distance), at most
    K per query, canonical order, kept count min(|N(i)|, K) and symmetry.  |N(i)|
    comes from the oracle's grid route with a cap that cannot bind."""
    spec, X, want = event_and_oracle("high")
    got = gpu_edges(X, spec.r, spec.K)
    uncapped = np.bincount(oracle.frnn_grid(X, spec.r, 4096)[0], minlength=spec.n)
    invariants.check(X, spec.r, spec.K, got, uncapped_degrees=uncapped)


# ------------------------------------------------------------------ batches

def _batch_case(seed=21):
    """Events of uneven sizes (including empty and single-point ones) back to back."""
    evs = [events.generate(events.TINY)[0]]
    for k, n in enumerate((5000, 0, 1, 777, 12000, 2, 3001)):
        spec = events.batched_spec(n, seed + k) if n >= 24 else None
        if spec is None:
            X = np.random.Generator(np.random.PCG64(seed + k)).uniform(-0.05, 0.05, size=(n, 8)).astype(np.float32)
        else:
            X, _ = events.generate(spec)
        evs.append(X)
    evs.append(next(c for c in events.stress_cases() if c.name == "S1_clump_cap").points)
    return evs


def test_batch_matches_each_event_alone():
    evs = _batch_case()
    offsets = np.concatenate([[0], np.cumsum([len(x) for x in evs])]).astype(np.int64)
    pts = torch.from_numpy(np.concatenate(evs)).to(DEV)
    log(f"batch of {len(evs)} events, {offsets[-1]} rows")
    edges, eo = frnn.build_batch(pts, offsets, 0.1, 64)
    edges = edges.cpu().numpy()
    assert eo[0] == 0 and np.all(np.diff(eo) >= 0)
    for e, X in enumerate(evs):
        got = edges[:, eo[e]:eo[e + 1]]
        assert_same(np.ascontiguousarray(got), oracle.frnn_grid(X, 0.1, 64))
        if len(X):
            alone = gpu_edges(X, 0.1, 64)
            assert_same(np.ascontiguousarray(got), alone)


def test_batch_capacity_and_nonfinite():
    evs = _batch_case()
    offsets = np.concatenate([[0], np.cumsum([len(x) for x in evs])]).astype(np.int64)
    pts = torch.from_numpy(np.concatenate(evs)).to(DEV)
    edges, eo = frnn.build_batch(pts, offsets, 0.1, 64, capacity=10)  # retries with the total needed
    want_total = sum(oracle.frnn_grid(X, 0.1, 64).shape[1] for X in evs)
    assert eo[-1] == want_total
    bad = np.concatenate(evs)
    bad[offsets[3] + 100 if offsets[4] - offsets[3] > 100 else offsets[1] + 5, 2] = np.nan
    with pytest.raises(frnn.FrnnError) as e:
        frnn.build_batch(torch.from_numpy(bad).to(DEV), offsets, 0.1, 64)
    assert e.value.status == frnn.FRNN_ERR_NONFINITE


def test_captured_batch_graph_replays_match_eager():
    evs = _batch_case()
    offsets = np.concatenate([[0], np.cumsum([len(x) for x in evs])]).astype(np.int64)
    pts = torch.from_numpy(np.concatenate(evs)).to(DEV)
    edges, eo = frnn.build_batch(pts, offsets, 0.1, 64)
    eager = edges.cpu().numpy()
    cap = int(eo[-1]) + 100
    ws = torch.empty(frnn.batch_workspace_bytes(offsets, 8), dtype=torch.uint8, device=DEV)
    out = torch.empty((2, cap), dtype=torch.int64, device=DEV)
    eo_dev = torch.zeros(len(evs) + 2, dtype=torch.int64, device=DEV)
    assert frnn.build_batch_async(pts, offsets, 0.1, 64, ws, out[0], out[1], eo_dev) == frnn.FRNN_OK
    torch.cuda.synchronize()
    cfg = frnn.Config(events_resident=True)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        assert frnn.build_batch_async(pts, offsets, 0.1, 64, ws, out[0], out[1], eo_dev, cfg) == frnn.FRNN_OK
    for rep in range(4):
        out.fill_(-7)
        eo_dev.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        e_host = eo_dev.cpu().numpy()
        assert e_host[-1] == 0, f"replay {rep}: status {e_host[-1]}"
        assert np.array_equal(e_host[:-1], eo), f"replay {rep}: edge ranges differ"
        assert_same(np.ascontiguousarray(out[:, :int(eo[-1])].cpu().numpy()), eager)


def test_events_entry_point_matches_oracle():
    """frnn_build_events_async with each event in its own allocation (no gather)."""
    evs = _batch_case()
    tensors = [torch.from_numpy(np.ascontiguousarray(X)).to(DEV) for X in evs]
    offsets = np.concatenate([[0], np.cumsum([len(x) for x in evs])]).astype(np.int64)
    want = [oracle.frnn_grid(X, 0.1, 64) for X in evs]
    cap = sum(w.shape[1] for w in want) + 64
    ws = torch.empty(frnn.batch_workspace_bytes(offsets, 8), dtype=torch.uint8, device=DEV)
    out = torch.full((2, cap), -7, dtype=torch.int64, device=DEV)
    eo = torch.full((len(evs) + 2,), -1, dtype=torch.int64, device=DEV)
    log(f"events entry point: {len(evs)} events")
    assert frnn.build_events_async(tensors, 0.1, 64, ws, out[0], out[1], eo) == frnn.FRNN_OK
    torch.cuda.synchronize()
    eo = eo.cpu().numpy()
    assert eo[-1] == 0
    got = out.cpu().numpy()
    for e in range(len(evs)):
        assert_same(np.ascontiguousarray(got[:, eo[e]:eo[e + 1]]), want[e])


def test_served_requests_match_oracle():
    """The continuous-batching server on the GPU: every request's edges equal the oracle's."""
    from paper_2202_06929_amd import serve

    spec = events.batched_spec(1, 0)
    reqs = []
    host = []
    for k, (t, n) in enumerate(events.served_trace(24, 20000.0, lo=200, hi=15000, seed=5)):
        X, _ = events.generate(events.batched_spec(n, 1000 + k))
        host.append(X)
        reqs.append(serve.Request(rid=k, arrival=t, points=torch.from_numpy(X).to(DEV)))
    ex = serve.GpuExecutor(spec.r, spec.K, host[0].shape[1], n_streams=3)
    stats = serve.Server(ex, hbm_budget=8 << 30, max_batch=8).run(reqs)
    log(f"served: {stats}")
    assert stats.completed == len(reqs)
    for req, X in zip(reqs, host):
        assert_same(np.ascontiguousarray(req.edges.cpu().numpy()), oracle.frnn_grid(X, spec.r, spec.K))


@pytest.mark.parametrize("K", [1, 2, 3, 8, 15, 16])
def test_small_caps_keep_the_nearest(K):
    """Caps below the list size: the search picks the K nearest by (D, j) itself."""
    spec = events.TINY
    X, _ = events.generate(spec)
    log(f"small cap K={K} on the tiny event")
    assert_same(gpu_edges(X, spec.r, K), oracle.frnn_grid(X, spec.r, K))


@pytest.mark.parametrize("d", [3, 8, 12, 16])
@pytest.mark.parametrize("K", [1, 4, 15])
def test_small_caps_on_dense_cells(d, K):
    """Caps below the list size where cells hold many queries: several query tiles
    per cell with a partial last one, at each row width of the capped search."""
    X = events.dense_cells(d)
    log(f"small cap K={K} on dense cells d={d}")
    want = oracle.frnn_grid(X, 0.1, K)
    assert_same(gpu_edges(X, 0.1, K), want)
    assert_same(gpu_edges(X, 0.1, K, config=frnn.Config(dims=(0, 1, 2))), want)
    if d >= 4:
        assert_same(gpu_edges(X, 0.1, K, config=frnn.Config(dims=(0, 1, 2, 3))), want)


def test_nearest_eight_on_the_single_event():
    """The kNN-then-radius workload: K = 8 binds for about half the queries."""
    spec = events.KNN
    X, _ = events.generate(spec)
    log(f"knn workload n={spec.n} K={spec.K}")
    pts = torch.from_numpy(X).to(DEV)
    stats = frnn.FrnnStats()
    cap = 16 * spec.n
    ws = torch.empty(frnn.workspace_bytes(spec.n, spec.d), dtype=torch.uint8, device=DEV)
    out = torch.empty((2, cap), dtype=torch.int64, device=DEV)
    st, E = frnn.build_into(pts, spec.r, spec.K, ws, out[0], out[1], None, stats)
    assert st == frnn.FRNN_OK
    want = oracle.frnn_grid(X, spec.r, spec.K)
    assert_same(out[:, :E].cpu().numpy(), want)
    assert stats.capped_queries == int((np.bincount(oracle.frnn_grid(X, spec.r, 4096)[0], minlength=spec.n)
                                        > spec.K).sum())


def test_large_batch_uses_grouped_offsets():
    """More than 4096 placement tiles (over a million rows): output offsets come from
    the two-level totals; every event equals the event built alone."""
    sizes = [120_000] * 9
    evs = [events.generate(events.batched_spec(n, 500 + k))[0] for k, n in enumerate(sizes)]
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    assert (offsets[-1] + 255) // 256 > 4096
    pts = torch.from_numpy(np.concatenate(evs)).to(DEV)
    log(f"large batch: {offsets[-1]} rows")
    edges, eo = frnn.build_batch(pts, offsets, 0.1, 256)
    edges = edges.cpu().numpy()
    for e, X in enumerate(evs):
        got = np.ascontiguousarray(edges[:, eo[e]:eo[e + 1]])
        assert_same(got, gpu_edges(X, 0.1, 256))
        if e in (0, 8):
            assert_same(got, oracle.frnn_grid(X, 0.1, 256))


def _oracle_many(events_, r, K):
    """The oracle's edges of several events, computed on parallel host threads
    (the C oracle runs outside the interpreter lock)."""
    from concurrent.futures import ThreadPoolExecutor
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(workers) as pool:
        return list(pool.map(lambda X: oracle.frnn_grid(X, r, K), events_))


@functools.lru_cache(maxsize=None)
def benchmark_batch():
    """The benchmark's 64 events (20k-150k hits each) and the oracle's edges of each."""
    sizes = events.batched_sizes()
    evs = [events.generate(events.batched_spec(n, 100 + k))[0] for k, n in enumerate(sizes)]
    return sizes, evs, _oracle_many(evs, 0.1, 256)


@pytest.mark.parametrize("cfg", [frnn.Config(), frnn.Config(grid_mult=4), frnn.Config(dims=(4, 5, 7))],
                         ids=["default", "grid4", "three_axes_457"])
def test_benchmark_batch_of_64_events(cfg):
    """The benchmark's batch (64 events of 20k-150k hits): every event equals the
    oracle's edges of that event, with four binned coordinates and with three."""
    sizes, evs, want = benchmark_batch()
    offsets = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    pts = torch.from_numpy(np.concatenate(evs)).to(DEV)
    log(f"benchmark batch: {offsets[-1]} rows, {cfg}")
    edges, eo = frnn.build_batch(pts, offsets, 0.1, 256, cfg)
    edges = edges.cpu().numpy()
    assert eo[-1] == sum(w.shape[1] for w in want)
    for e in range(len(evs)):
        assert_same(np.ascontiguousarray(edges[:, eo[e]:eo[e + 1]]), want[e])


def test_served_stream_of_full_size_events_matches_oracle():
    """The served workload at its own scale: Poisson arrivals of events with hit
    counts log-uniform in [10k, 300k] (one of 300k added), 8-D, r = 0.1, K = 256,
    through the continuous-batching server on three streams; every request's edges
    equal the oracle's."""
    from paper_2202_06929_amd import serve

    trace = events.served_trace(15, 20000.0, seed=17)
    trace.append((trace[4][0], 300_000))  # arrives together with request 4
    host = [events.generate(events.batched_spec(n, 2000 + k))[0] for k, (_, n) in enumerate(trace)]
    log(f"served full-size stream: sizes {[len(X) for X in host]}")
    assert max(len(X) for X in host) >= 250_000 and min(len(X) for X in host) < 30_000
    reqs = [serve.Request(rid=k, arrival=t, points=torch.from_numpy(X).to(DEV))
            for k, ((t, _), X) in enumerate(zip(trace, host))]
    ex = serve.GpuExecutor(0.1, 256, 8, n_streams=3)
    stats = serve.Server(ex, hbm_budget=64 << 30, max_batch=8).run(reqs)
    log(f"served: {stats}")
    assert stats.completed == len(reqs)
    got = [np.ascontiguousarray(req.edges.cpu().numpy()) for req in reqs]
    for g, w in zip(got, _oracle_many(host, 0.1, 256)):
        assert_same(g, w)


def test_prepared_async_batch_matches_the_plain_call():
    evs = _batch_case()
    offsets = np.concatenate([[0], np.cumsum([len(x) for x in evs])]).astype(np.int64)
    pts = torch.from_numpy(np.concatenate(evs)).to(DEV)
    log(f"prepared async batch: {len(evs)} events, {offsets[-1]} rows")
    want, eo_want = frnn.build_batch(pts, offsets, 0.1, 64)
    cap = want.shape[1] + 64
    ws = torch.empty(frnn.batch_workspace_bytes(offsets, 8), dtype=torch.uint8, device=DEV)
    out = torch.full((2, cap), -7, dtype=torch.int64, device=DEV)
    slots = torch.full((3, len(evs) + 2), -1, dtype=torch.int64, device=DEV)
    call = frnn.AsyncBatch(pts, offsets, 0.1, 64, ws, out[0], out[1])
    for k in range(3):
        assert call(slots[k]) == frnn.FRNN_OK
    torch.cuda.synchronize()
    got = slots.cpu().numpy()
    for k in range(3):
        assert np.array_equal(got[k, :-1], eo_want) and got[k, -1] == 0
    assert torch.equal(out[:, :want.shape[1]], want)
    with pytest.raises(ValueError):
        call(torch.zeros(1, dtype=torch.int64, device=DEV))
