"""The autotuner without a GPU: a stub build stands in for the HIP library, so the
tuner's own logic (timing every candidate, refusing a candidate whose edges
differ, the JSON cache keyed by architecture, dimension, size bucket, r and K) is
checked on the CPU."""

import json
import time

import numpy as np
import pytest
import torch

from paper_2202_06929_amd import frnn, tune

EDGES = 40


class StubLibrary:
    """frnn's batch entry points on CPU tensors: every config returns the same edges
    unless it is listed in `wrong`; each config takes `cost(cfg)` seconds."""

    def __init__(self, cost, wrong=()):
        self.cost = cost
        self.wrong = set(wrong)
        self.calls = 0

    def edges(self, cfg):
        e = torch.arange(2 * EDGES, dtype=torch.int64).reshape(2, EDGES)
        if (cfg.dims, cfg.cell_div, cfg.grid_mult) in self.wrong:
            e = e.clone()
            e[1, 7] += 1
        return e

    def build_batch_into(self, points, off, r, K, ws, src, dst, cfg=None, stats=None):
        self.calls += 1
        time.sleep(self.cost(cfg))
        e = self.edges(cfg)
        src[:EDGES] = e[0]
        dst[:EDGES] = e[1]
        return frnn.FRNN_OK, np.array([0, EDGES // 2, EDGES], dtype=np.int64)

    def build_batch(self, points, off, r, K, config=None):
        return self.edges(config), np.array([0, EDGES // 2, EDGES], dtype=np.int64)


@pytest.fixture
def stub(monkeypatch):
    def install(cost, wrong=()):
        lib = StubLibrary(cost, wrong)
        monkeypatch.setattr(frnn, "build_batch_into", lib.build_batch_into)
        monkeypatch.setattr(frnn, "build_batch", lib.build_batch)
        monkeypatch.setattr(frnn, "batch_workspace_bytes", lambda off, d: 4096)
        monkeypatch.setattr(tune, "_arch", lambda: "stub")
        monkeypatch.setattr(tune, "_sync", lambda: None)
        return lib
    return install


def points(rows=1000, d=8):
    return torch.zeros((rows, d), dtype=torch.float32)


def cost_fast_lead_dims(cfg):
    # (0, 1, 2) with cell_div 2 is five times faster than everything else.
    return 0.0005 if (cfg.dims, cfg.cell_div) == ((0, 1, 2), 2) else 0.0025


def test_picks_the_fastest_config_then_tunes_its_grid(stub, tmp_path):
    lib = stub(cost_fast_lead_dims)
    cache = str(tmp_path / "tune.json")
    best, report = tune.tune(points(), [0, 600, 1000], 0.1, 256, repeats=2, cache_path=cache)
    assert (best.dims, best.cell_div) == ((0, 1, 2), 2)
    n_first = len(tune.candidates(8))
    assert len(report["all"]) == n_first + len(tune.grid_candidates(best))
    assert report["key"] == tune.cache_key("stub", 8, 1000, 0.1, 256)
    stored = json.load(open(cache))[report["key"]]
    assert stored["dims"] == [0, 1, 2] and stored["cell_div"] == 2 and stored["axes"] == 0


def test_cache_hit_skips_timing_and_other_sizes_miss(stub, tmp_path):
    lib = stub(cost_fast_lead_dims)
    cache = str(tmp_path / "tune.json")
    first, _ = tune.tune(points(), [0, 1000], 0.1, 256, repeats=1, cache_path=cache)
    calls = lib.calls
    again, rep = tune.tune(points(), [0, 1000], 0.1, 256, repeats=1, cache_path=cache)
    assert lib.calls == calls, "a cached workload must not be timed again"
    assert (again.dims, again.cell_div, again.grid_mult) == (first.dims, first.cell_div, first.grid_mult)
    # A size in another bucket, another K or another r is a miss.
    for off, r, K in (([0, 4000], 0.1, 256), ([0, 1000], 0.1, 64), ([0, 1000], 0.2, 256)):
        before = lib.calls
        tune.tune(points(off[-1]), off, r, K, repeats=1, cache_path=cache)
        assert lib.calls > before
    assert len(json.load(open(cache))) == 4


def test_a_candidate_that_changes_the_edges_is_refused(stub, tmp_path):
    stub(lambda cfg: 0.0, wrong={((0, 1, 2), 3, 0)})
    cache = str(tmp_path / "tune.json")
    with pytest.raises(AssertionError, match="changed the edges"):
        tune.tune(points(), [0, 1000], 0.1, 256, repeats=1, cache_path=cache)
    import os
    assert not os.path.exists(cache), "nothing may be cached after a refusal"
