"""Lists longer than the search keeps: collected again by the placement pass.

Tight clumps give every query of a clump exactly (clump size - 1) neighbours, so
the lists around the 16-slot boundary (15, 16, 17), lists several placement
windows long, caps that equal the count or cut it, and the largest cap all run
through the long-list path, alone and in a batch, against the CPU oracle.
"""

import sys

import numpy as np
import pytest
import torch

from oracle import oracle
from paper_2202_06929_amd import events, frnn

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
SIZES = [16, 17, 18, 33, 64, 200, 600]


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def assert_same(got, want):
    assert got.shape == want.shape, (got.shape, want.shape)
    if not np.array_equal(got, want):
        bad = np.flatnonzero((got != want).any(0))[:5]
        raise AssertionError(f"first differing edges at {bad.tolist()}: got {got[:, bad].T.tolist()} "
                             f"want {want[:, bad].T.tolist()}")


@pytest.mark.parametrize("d", [3, 8, 12])
@pytest.mark.parametrize("K", [4096, 200, 33, 32, 17, 16, 8, 1])
def test_long_lists_around_the_list_size_and_the_cap(d, K):
    X = events.tight_clumps(SIZES, d, 0.1, seed=5 + d, noise=300)
    log(f"long lists: n={len(X)} d={d} K={K}")
    want = oracle.frnn_grid(X, 0.1, K)
    got, st = frnn.build(torch.from_numpy(X).to(DEV), 0.1, K, return_stats=True)
    torch.cuda.synchronize()
    assert_same(got.cpu().numpy(), want)
    # A list is long when it has more than 16 entries (with K >= 16 a list of at
    # most 16 is also within the cap).
    assert st["overflow_queries"] == sum(m for m in SIZES if m - 1 > 16)
    assert st["capped_queries"] == sum(m for m in SIZES if m - 1 > K)


def test_largest_cap_on_a_clump_larger_than_it():
    X = events.tight_clumps([4200], 8, 0.1, seed=41, noise=100)
    K = frnn.MAX_K
    log(f"largest cap: n={len(X)} K={K}")
    want = oracle.frnn_grid(X, 0.1, K)
    got = frnn.build(torch.from_numpy(X).to(DEV), 0.1, K)
    torch.cuda.synchronize()
    assert want.shape[1] == 4200 * K
    assert_same(got.cpu().numpy(), want)


def test_long_lists_in_a_batch():
    evs = [events.tight_clumps(SIZES[: k + 2], 8, 0.1, seed=60 + k, noise=50 * k) for k in range(5)]
    evs.insert(2, np.zeros((0, 8), dtype=np.float32))
    offsets = np.concatenate([[0], np.cumsum([len(x) for x in evs])]).astype(np.int64)
    log(f"long lists in a batch of {len(evs)} events, {offsets[-1]} rows")
    for K in (4096, 40):
        edges, eo = frnn.build_batch(torch.from_numpy(np.concatenate(evs)).to(DEV), offsets, 0.1, K)
        edges = edges.cpu().numpy()
        for e, X in enumerate(evs):
            assert_same(np.ascontiguousarray(edges[:, eo[e]:eo[e + 1]]), oracle.frnn_grid(X, 0.1, K))
