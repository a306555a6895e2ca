"""Parity of the HIP track labeling (frnn_components) with the CPU oracle.

Labels are unique (each vertex gets the smallest vertex id of its weakly connected
component), so the bar is exact equality of the int64 label arrays.  Every case
goes through the C interface via the ctypes binding.
"""

import sys

import numpy as np
import pytest
import torch

from oracle import components as cc_oracle
from oracle import oracle
from paper_2202_06929_amd import events, frnn

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_labels(src, dst, n, scores=None, threshold=0.0):
    s = torch.from_numpy(np.ascontiguousarray(src, dtype=np.int64)).to(DEV)
    d = torch.from_numpy(np.ascontiguousarray(dst, dtype=np.int64)).to(DEV)
    sc = None if scores is None else torch.from_numpy(np.ascontiguousarray(scores, dtype=np.float32)).to(DEV)
    lab, nc = frnn.components(s, d, n, sc, threshold)
    torch.cuda.synchronize()
    return lab.cpu().numpy(), nc


def random_graph(seed, n, e):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(0, n, size=e).astype(np.int64), rng.integers(0, n, size=e).astype(np.int64)


@pytest.mark.parametrize("seed,n,e", [(1, 1, 0), (2, 1, 3), (3, 10, 5), (4, 1000, 700), (5, 5000, 5000),
                                      (6, 20000, 60000), (7, 100_000, 50_000), (8, 300, 0)])
def test_random_graphs_match_oracle(seed, n, e):
    src, dst = random_graph(seed, n, e)
    log(f"components random n={n} e={e} seed={seed}")
    got, nc = gpu_labels(src, dst, n)
    want = cc_oracle.labels(src, dst, n)
    assert np.array_equal(got, want)
    assert nc == len(np.unique(want))


def test_long_chain_and_star():
    # A path given in a shuffled order (deep trees) and a star (one hub).
    n = 50_000
    rng = np.random.Generator(np.random.PCG64(21))
    perm = rng.permutation(n)
    src, dst = perm[:-1].astype(np.int64), perm[1:].astype(np.int64)
    order = rng.permutation(n - 1)
    log("components chain")
    got, nc = gpu_labels(src[order], dst[order], n)
    assert nc == 1 and (got == 0).all()
    hub = np.full(n - 1, n - 1, dtype=np.int64)
    got, nc = gpu_labels(hub, np.arange(n - 1, dtype=np.int64), n)
    assert nc == 1 and (got == 0).all()


def test_scores_and_strict_threshold():
    src, dst = random_graph(31, 4000, 8000)
    rng = np.random.Generator(np.random.PCG64(32))
    scores = rng.uniform(0, 1, size=src.size).astype(np.float32)
    scores[::5] = np.float32(0.7)  # exactly at the threshold: dropped
    log("components scores")
    got, nc = gpu_labels(src, dst, 4000, scores, 0.7)
    want = cc_oracle.labels(src, dst, 4000, scores, 0.7)
    assert np.array_equal(got, want) and nc == len(np.unique(want))


@pytest.mark.parametrize("name", ["tiny", "single"])
def test_labels_of_the_frnn_graph(name):
    spec = {"tiny": events.TINY, "single": events.SINGLE}[name]
    X, _ = events.generate(spec)
    pts = torch.from_numpy(X).to(DEV)
    log(f"components of the {name} event graph")
    edges = frnn.build(pts, spec.r, spec.K)
    lab, nc = frnn.components(edges[0].contiguous(), edges[1].contiguous(), spec.n)
    torch.cuda.synchronize()
    g = oracle.frnn_grid(X, spec.r, spec.K)
    want = cc_oracle.labels(g[0], g[1], spec.n)
    assert np.array_equal(lab.cpu().numpy(), want)
    assert nc == len(np.unique(want))


def test_repeated_runs_are_identical():
    src, dst = random_graph(41, 30_000, 40_000)
    first, _ = gpu_labels(src, dst, 30_000)
    for _ in range(5):
        again, _ = gpu_labels(src, dst, 30_000)
        assert np.array_equal(again, first)


def test_endpoint_out_of_range_is_reported():
    src = np.array([0, 1, 7], dtype=np.int64)
    dst = np.array([1, 2, 3], dtype=np.int64)
    with pytest.raises(frnn.FrnnError) as e:
        gpu_labels(src, dst, 5)
    assert e.value.status == frnn.FRNN_ERR_ARG


def test_async_and_captured_graph_replays_match():
    src, dst = random_graph(51, 8000, 12000)
    want = cc_oracle.labels(src, dst, 8000)
    s = torch.from_numpy(src).to(DEV)
    d = torch.from_numpy(dst).to(DEV)
    ws = torch.empty(frnn.components_workspace_bytes(8000), dtype=torch.uint8, device=DEV)
    lab = torch.empty(8000, dtype=torch.int64, device=DEV)
    res = torch.zeros(2, dtype=torch.int64, device=DEV)
    assert frnn.components_async(s, d, 8000, ws, lab, res) == frnn.FRNN_OK
    torch.cuda.synchronize()
    assert np.array_equal(lab.cpu().numpy(), want) and res[1].item() == 0
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        assert frnn.components_async(s, d, 8000, ws, lab, res) == frnn.FRNN_OK
    for rep in range(4):
        lab.fill_(-1)
        res.fill_(-1)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert res[1].item() == 0, f"replay {rep}"
        assert res[0].item() == len(np.unique(want))
        assert np.array_equal(lab.cpu().numpy(), want), f"replay {rep}"


def test_no_vertices():
    # No labeling pass runs; the count and the status still reach the caller.
    empty = torch.zeros(0, dtype=torch.int64, device=DEV)
    lab, nc = frnn.components(empty, empty, 0)
    torch.cuda.synchronize()
    assert lab.numel() == 0 and nc == 0
    one = torch.zeros(1, dtype=torch.int64, device=DEV)
    with pytest.raises(frnn.FrnnError) as e:
        frnn.components(one, one, 0)
    assert e.value.status == frnn.FRNN_ERR_ARG
