"""Seeded synthetic events shaped like the latent embeddings the graph builder consumes.

The paper's metric-learning stage (Section 2) places the spacepoints of one track
close together in a Euclidean latent space and spacepoints of different tracks far
apart.  Its measured workloads are TrackML events, which are not available here, so
every event is synthetic: clusters stand for tracks (a handful to twenty hits each),
a uniform background stands for hits that belong to no reconstructable track.

This module only draws random numbers.  It holds none of the graph builder's
arithmetic, so it can serve both the GPU path and the CPU oracle with the same
bytes.

Recipe (one event):
  1. cluster centres ~ U[-1, 1]^d (float64);
  2. cluster sizes ~ integers in [lo, hi];
  3. sizes adjusted by +-1, cyclically over clusters 0, 1, 2, ... and only within
     [lo, hi], until they add up to the clustered quota n - round(noise_frac * n);
  4. clustered points = centre + N(0, sigma^2) per dimension;
  5. noise points ~ U[-1, 1]^d;
  6. concatenate, round to float32 (round to nearest even), shuffle with one
     permutation of n.
The returned labels are the cluster index (or -1 for noise), for diagnostics only.
"""

from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class EventSpec:
    """Shape of one synthetic event."""

    n: int
    d: int
    n_clusters: int
    size_lo: int
    size_hi: int
    sigma: float
    noise_frac: float
    r: float
    K: int
    seed: int

    def with_seed(self, seed: int) -> "EventSpec":
        return dataclasses.replace(self, seed=seed)


# The workloads used throughout the tests and the benchmark.
TINY = EventSpec(n=2_000, d=8, n_clusters=150, size_lo=8, size_hi=15, sigma=0.02,
                 noise_frac=0.10, r=0.1, K=64, seed=1)
SINGLE = EventSpec(n=120_000, d=8, n_clusters=10_000, size_lo=5, size_hi=18, sigma=0.02,
                   noise_frac=0.15, r=0.1, K=256, seed=2)
HIGH = EventSpec(n=300_000, d=12, n_clusters=22_000, size_lo=6, size_hi=20, sigma=0.03,
                 noise_frac=0.20, r=0.12, K=512, seed=3)
# Nearest K, then the radius cut (the k-nearest-neighbour semantics of Section
# 3.1): the single event's points with K = 8, which binds for about half the
# queries (clusters of up to 18 points).
KNN = dataclasses.replace(SINGLE, K=8)


def batched_spec(n: int, seed: int) -> EventSpec:
    """An event of the batched / served streams: the single-event shape scaled to n.

    The cluster count keeps the single-event ratio of one cluster per 12 hits.
    """
    return EventSpec(n=n, d=8, n_clusters=max(1, round(n / 12)), size_lo=5, size_hi=18,
                     sigma=0.02, noise_frac=0.15, r=0.1, K=256, seed=seed)


def batched_sizes(n_events: int = 64, lo: int = 20_000, hi: int = 150_000,
                  seed: int = 99) -> list[int]:
    """Hit counts of a batch: uniform integers in [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return [int(v) for v in rng.integers(lo, hi + 1, size=n_events)]


def served_trace(n_events: int, rate_hz: float, lo: int = 10_000, hi: int = 300_000,
                 seed: int = 7) -> list[tuple[float, int]]:
    """Poisson arrivals at a fixed rate with log-uniform hit counts in [lo, hi].

    Returns (arrival time in seconds from t=0, hit count) per event.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    gaps = rng.exponential(1.0 / rate_hz, size=n_events)
    t = np.cumsum(gaps) - gaps[0]
    sizes = np.exp(rng.uniform(math.log(lo), math.log(hi), size=n_events))
    return [(float(a), int(round(s))) for a, s in zip(t, sizes)]


def _cluster_sizes(rng: np.random.Generator, count: int, lo: int, hi: int, quota: int) -> np.ndarray:
    if count * lo > quota or count * hi < quota:
        raise ValueError(f"{count} clusters of {lo}..{hi} points cannot hold {quota} points")
    sizes = rng.integers(lo, hi + 1, size=count).astype(np.int64)
    diff = int(quota - sizes.sum())
    step = 1 if diff > 0 else -1
    c = 0
    while diff != 0:
        nxt = sizes[c] + step
        if lo <= nxt <= hi:
            sizes[c] = nxt
            diff -= step
        c = (c + 1) % count
    return sizes


def generate(spec: EventSpec) -> tuple[np.ndarray, np.ndarray]:
    """Draw one event.  Returns (points float32 [n, d] C-contiguous, labels int64 [n])."""
    n, d = spec.n, spec.d
    if n < 0 or d < 1:
        raise ValueError("need n >= 0 and d >= 1")
    rng = np.random.Generator(np.random.PCG64(spec.seed))
    n_noise = int(round(spec.noise_frac * n))
    quota = n - n_noise
    if quota > 0 and spec.n_clusters > 0:
        centres = rng.uniform(-1.0, 1.0, size=(spec.n_clusters, d))
        sizes = _cluster_sizes(rng, spec.n_clusters, spec.size_lo, spec.size_hi, quota)
        clustered = np.repeat(centres, sizes, axis=0)
        clustered = clustered + rng.normal(0.0, spec.sigma, size=clustered.shape)
        labels_c = np.repeat(np.arange(spec.n_clusters, dtype=np.int64), sizes)
    else:
        n_noise = n
        clustered = np.zeros((0, d))
        labels_c = np.zeros(0, dtype=np.int64)
    noise = rng.uniform(-1.0, 1.0, size=(n_noise, d))
    pts = np.concatenate([clustered, noise], axis=0).astype(np.float32)
    labels = np.concatenate([labels_c, np.full(n_noise, -1, dtype=np.int64)])
    perm = rng.permutation(n)
    return np.ascontiguousarray(pts[perm]), labels[perm]


def cluster_sizes_of(labels: np.ndarray) -> np.ndarray:
    """Sizes of the clusters present in an event's labels (noise excluded)."""
    lab = labels[labels >= 0]
    if lab.size == 0:
        return np.zeros(0, dtype=np.int64)
    return np.bincount(lab)


@dataclasses.dataclass(frozen=True)
class StressCase:
    """A hand-shaped input that drives a corner of the method (the cap, ties, one cell, ...)."""

    name: str
    points: np.ndarray
    r: float
    K: int


def _clump(rng: np.random.Generator, count: int, d: int, sigma: float) -> np.ndarray:
    return rng.uniform(-0.5, 0.5, size=(1, d)) + rng.normal(0.0, sigma, size=(count, d))


def stress_cases(seed: int = 11) -> list[StressCase]:
    """Inputs beyond the clustered workloads: each stresses one corner case.

    S1  a tight clump of 300 points with K = 64: the cap binds for every clump point;
    S2  50 copies of one point with K = 8: distance ties broken by index;
    S3  pairs exactly at / just inside the radius (strict comparison);
    S4  r = 10 with K = 64 and K = 400: every pair within radius, nearest-K and complete graph;
    S5  n = 0, 1, 2 and 100 identical points;
    S6  5,000 points whose coordinates 0-2 and d-3..d-1 are all equal: one grid cell;
    S7  coordinates spread over +-1e4 with r = 0.1: grid sizes hit their caps;
    S8  coordinates near 1e-20 so squared distances are subnormal.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    out: list[StressCase] = []
    d = 8

    s1 = np.concatenate([_clump(rng, 300, d, 0.001), rng.uniform(-1, 1, size=(700, d))])
    out.append(StressCase("S1_clump_cap", s1[rng.permutation(len(s1))].astype(np.float32), 0.1, 64))

    base = rng.uniform(-1, 1, size=(1, d))
    s2 = np.concatenate([np.repeat(base, 50, axis=0), base + rng.normal(0, 0.01, size=(30, d)),
                         rng.uniform(-1, 1, size=(200, d))])
    out.append(StressCase("S2_duplicates_ties", s2[rng.permutation(len(s2))].astype(np.float32), 0.1, 8))

    # Point 1 sits exactly r = 0.5 from point 0 (D == r2, excluded); point 2 sits at
    # 0.5 - 2^-25, just inside.
    s3 = np.zeros((3, 3), dtype=np.float32)
    s3[1, 0] = 0.5
    s3[2, 0] = np.float32(0.5 - 2.0 ** -25)
    out.append(StressCase("S3_boundary", s3, 0.5, 8))

    s4 = rng.uniform(-1, 1, size=(300, d)).astype(np.float32)
    out.append(StressCase("S4_knn_r10_K64", s4, 10.0, 64))
    out.append(StressCase("S4_complete_r10_K400", s4, 10.0, 400))

    out.append(StressCase("S5_empty", np.zeros((0, d), np.float32), 0.1, 8))
    out.append(StressCase("S5_single", rng.uniform(-1, 1, size=(1, d)).astype(np.float32), 0.1, 8))
    out.append(StressCase("S5_pair", np.array([[0.0] * d, [0.05] + [0.0] * (d - 1)], np.float32), 0.1, 8))
    out.append(StressCase("S5_identical", np.repeat(rng.uniform(-1, 1, size=(1, d)), 100, axis=0)
                          .astype(np.float32), 0.1, 200))

    s6 = np.zeros((5000, d))
    s6[:, 3:5] = rng.uniform(-1, 1, size=(5000, 2))
    s6[:, :3] = 0.25
    s6[:, d - 3:] = -0.25
    out.append(StressCase("S6_one_cell", s6.astype(np.float32), 0.1, 64))

    s7 = np.concatenate([rng.uniform(-1e4, 1e4, size=(2500, d)), _clump(rng, 500, d, 0.02)])
    out.append(StressCase("S7_wide_extent", s7[rng.permutation(len(s7))].astype(np.float32), 0.1, 32))

    s8 = (rng.normal(0, 1e-20, size=(400, d))).astype(np.float32)
    out.append(StressCase("S8_subnormal", s8, 2e-20, 16))
    return out


def dense_cells(d: int, seed: int = 23) -> np.ndarray:
    """2,600 float32 points in d dimensions for radius 0.1, with crowded cells.

    A clump of 300 points (sigma 0.01) and 200 points sharing their binned
    coordinates 0-2 and d-3..d-1 (one cell) give cells of hundreds of queries, so
    the search runs many query tiles per cell, ending in a partial one; three
    clumps of 300 with sigma 0.1 f / sqrt(d), f = 1.0, 1.2, 1.5, give hundreds of
    queries with 5 to 16 neighbours at every d; 1,200 uniform points in [-1, 1]^d
    surround them.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    slab = rng.uniform(-1, 1, size=(200, d))
    slab[:, :3] = 0.3
    slab[:, d - 3:] = -0.3
    parts = [_clump(rng, 300, d, 0.01), slab]
    parts += [_clump(rng, 300, d, 0.1 * f / np.sqrt(d)) for f in (1.0, 1.2, 1.5)]
    parts.append(rng.uniform(-1, 1, size=(1200, d)))
    X = np.concatenate(parts)
    return X[rng.permutation(len(X))].astype(np.float32)


def tight_clumps(sizes, d: int, r: float, seed: int, noise: int = 0) -> np.ndarray:
    """Clumps whose points all lie within r of one another, far from each other.

    Clump k has sizes[k] points drawn uniformly from a cube of half-edge
    r / (2.5 sqrt(d)) around a centre on a lattice of spacing 4r, so every point
    has exactly sizes[k] - 1 neighbours within r; `noise` uniform points are
    spread far outside the clumps (a cube of edge 10^4 r).  Shuffled float32.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    half = r / (2.5 * np.sqrt(d))
    parts = []
    for k, m in enumerate(sizes):
        centre = np.zeros(d)
        centre[0] = 4.0 * r * k
        parts.append(centre + rng.uniform(-half, half, size=(int(m), d)))
    if noise:
        parts.append(rng.uniform(0.0, 1e4 * r, size=(noise, d)) + np.array([-2e4 * r] + [0.0] * (d - 1)))
    X = np.concatenate(parts) if parts else np.zeros((0, d))
    return X[rng.permutation(len(X))].astype(np.float32)


def dyadic_event(n: int, d: int, seed: int, step_log2: int = 6,
                 n_clusters: int = 40, sigma: float = 0.05) -> tuple[np.ndarray, np.ndarray]:
    """Clustered points snapped to multiples of 2^-step_log2 in [-1, 1].

    Returns (points float32 [n, d], integer coordinates int64 [n, d]) with
    points == ints * 2^-step_log2 exactly.  With step 2^-6 and d <= 16 every
    difference, square and partial sum of squares is a multiple of 2^-12 below
    2^8, so float32 arithmetic on these points is exact.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    scale = 2 ** step_log2
    centres = rng.uniform(-0.8, 0.8, size=(n_clusters, d))
    which = rng.integers(0, n_clusters, size=n)
    raw = centres[which] + rng.normal(0.0, sigma, size=(n, d))
    ints = np.clip(np.rint(raw * scale), -scale, scale).astype(np.int64)
    return (ints.astype(np.float64) / scale).astype(np.float32), ints
