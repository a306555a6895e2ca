"""The seeded generator: determinism and the shape the workloads promise."""

import numpy as np
import pytest

from paper_2202_06929_amd import events


def test_same_seed_same_bytes_and_new_seed_new_bytes():
    a, la = events.generate(events.TINY)
    b, lb = events.generate(events.TINY)
    c, _ = events.generate(events.TINY.with_seed(2))
    assert a.tobytes() == b.tobytes() and np.array_equal(la, lb)
    assert a.tobytes() != c.tobytes()


@pytest.mark.parametrize("spec", [events.TINY, events.SINGLE, events.HIGH], ids=["tiny", "single", "high"])
def test_counts_and_ranges(spec):
    X, labels = events.generate(spec)
    assert X.shape == (spec.n, spec.d) and X.dtype == np.float32 and X.flags.c_contiguous
    n_noise = int(round(spec.noise_frac * spec.n))
    assert int((labels < 0).sum()) == n_noise
    sizes = events.cluster_sizes_of(labels)
    assert len(sizes) == spec.n_clusters
    assert sizes.min() >= spec.size_lo and sizes.max() <= spec.size_hi
    assert sizes.sum() == spec.n - n_noise
    noise = X[labels < 0]
    assert noise.min() >= -1 and noise.max() <= 1
    # cluster spread: per-coordinate std of (point - cluster mean) close to sigma
    lab = labels[labels >= 0]
    means = np.zeros((spec.n_clusters, spec.d))
    np.add.at(means, lab, X[labels >= 0])
    means /= sizes[:, None]
    resid = X[labels >= 0] - means[lab]
    corr = np.sqrt(np.mean(sizes / (sizes - 1.0)))
    assert abs(resid.std() * corr / spec.sigma - 1) < 0.05


def test_batched_and_served_streams():
    sizes = events.batched_sizes()
    assert len(sizes) == 64 and min(sizes) >= 20_000 and max(sizes) <= 150_000
    tr = events.served_trace(500, rate_hz=1000.0)
    t = np.array([a for a, _ in tr])
    n = np.array([s for _, s in tr])
    assert t[0] == 0.0 and np.all(np.diff(t) >= 0)
    assert n.min() >= 10_000 and n.max() <= 300_000
    assert abs(np.mean(np.diff(t)) * 1000.0 - 1) < 0.15
    spec = events.batched_spec(50_000, 123)
    X, labels = events.generate(spec)
    assert X.shape == (50_000, 8)


def test_dyadic_points_are_exact_multiples():
    X, A = events.dyadic_event(300, 8, 3)
    assert np.array_equal(X.astype(np.float64) * 64, A.astype(np.float64))
    assert np.abs(A).max() <= 64
