"""Properties every FRNN edge list must have, whatever produced it.

TEST INFRASTRUCTURE ONLY.  These follow from the graph's definition (paper,
Sections 2 and 3.4: edges join points closer than a fixed radius) and from the
cap rule (at most K neighbours per query, nearest first, index breaking ties):

  * every edge joins two different points (no self-loops);
  * every edge (i, j) has D(i, j) < fl32(r * r);
  * no query keeps more than K neighbours;
  * the list is in canonical order: i ascending, then j ascending, no repeats;
  * (i, j) in E and |N(j)| <= K  implies  (j, i) in E  (symmetry wherever the cap
    does not bind; the whole graph is symmetric when no query is capped);
  * the real-number distance agrees with the float32 test away from the radius:
    pairs with squared distance below r^2 (1 - tol) are edges of uncapped queries,
    pairs above r^2 (1 + tol) never are.
"""

from __future__ import annotations

import numpy as np

from . import oracle


def edge_keys(edges: np.ndarray, n: int) -> np.ndarray:
    return edges[0].astype(np.int64) * max(n, 1) + edges[1].astype(np.int64)


def check(points: np.ndarray, r: float, K: int, edges: np.ndarray,
          uncapped_degrees: np.ndarray | None = None) -> None:
    """Raises AssertionError naming the first property that fails."""
    X = np.ascontiguousarray(points, dtype=np.float32)
    n = X.shape[0]
    edges = np.asarray(edges)
    assert edges.ndim == 2 and edges.shape[0] == 2, "edges must be [2, E]"
    assert edges.dtype == np.int64, "edges must be int64"
    i, j = edges[0], edges[1]
    if edges.shape[1] == 0:
        if uncapped_degrees is not None:
            assert int(np.sum(np.minimum(uncapped_degrees, K))) == 0, "edges missing"
        return
    assert i.min() >= 0 and j.min() >= 0 and i.max() < n and j.max() < n, "index out of range"
    assert np.all(i != j), "self-loop"
    keys = edge_keys(edges, n)
    assert np.all(np.diff(keys) > 0), "not in canonical (i, j) order or repeated edge"
    deg = np.bincount(i, minlength=n)
    assert deg.max() <= K, "more than K neighbours kept"
    D = oracle.pair_dist(X, i, j)
    r2 = np.float32(r) * np.float32(r)
    assert np.all(D < r2), "edge with D >= r^2"
    if uncapped_degrees is not None:
        assert np.array_equal(deg, np.minimum(uncapped_degrees, K)), "kept count != min(|N(i)|, K)"
        uncapped_j = uncapped_degrees[j] <= K
        rev = edge_keys(np.stack([j[uncapped_j], i[uncapped_j]]), n)
        assert np.all(np.isin(rev, keys)), "missing reverse edge of an uncapped query"


def check_against_reals(points: np.ndarray, r: float, K: int, edges: np.ndarray,
                        rel_tol: float = 1e-5) -> None:
    """Compares with float64 squared distances, away from the radius (row blocks of n)."""
    X = np.asarray(points, dtype=np.float64)
    n = X.shape[0]
    i, j = edges[0], edges[1]
    deg = np.bincount(i, minlength=n) if edges.shape[1] else np.zeros(n, np.int64)
    r2 = float(r) * float(r)
    bs = 256
    for a in range(0, n, bs):
        b = min(n, a + bs)
        d2 = ((X[a:b, None, :] - X[None, :, :]) ** 2).sum(-1)
        d2[np.arange(b - a), np.arange(a, b)] = np.inf  # no self pairs
        mask = np.zeros_like(d2, dtype=bool)
        sel = (i >= a) & (i < b)
        mask[i[sel] - a, j[sel]] = True
        outside = d2 > r2 * (1 + rel_tol)
        assert not np.any(mask & outside), "an edge lies well outside the radius"
        inside = d2 < r2 * (1 - rel_tol)
        rows = (inside.sum(1) < K) & (deg[a:b] < K)
        miss = inside[rows] & ~mask[rows]
        assert not np.any(miss), "a pair well inside the radius is not an edge"
