"""Pins of the track-labeling oracle (weakly connected components, each vertex
labeled with the smallest vertex id of its component).

The oracle is checked against things other than itself: SciPy's connected
components routine, a label-propagation fixed point written out here, hand-built
graphs with known answers, and the structural invariants of a min-id labeling.
Planted mistakes in private copies of the C source must each fail a pin.
"""

import numpy as np
import pytest
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components

from oracle import components, oracle
from paper_2202_06929_amd import events


def scipy_min_labels(src, dst, n, keep=None):
    if keep is not None:
        src, dst = src[keep], dst[keep]
    g = coo_matrix((np.ones(src.size), (src, dst)), shape=(n, n))
    _, comp = connected_components(g, directed=True, connection="weak")
    mins = np.full(comp.max() + 1 if n else 0, n, dtype=np.int64)
    np.minimum.at(mins, comp, np.arange(n))
    return mins[comp]


def propagate(src, dst, n, keep=None):
    """Fixed point of label[u] = label[v] = min(label[u], label[v]) over kept edges."""
    lab = np.arange(n, dtype=np.int64)
    s, d = (src, dst) if keep is None else (src[keep], dst[keep])
    changed = True
    while changed:
        m = np.minimum(lab[s], lab[d])
        new = lab.copy()
        np.minimum.at(new, s, m)
        np.minimum.at(new, d, m)
        changed = not np.array_equal(new, lab)
        lab = new
    return lab


def random_graph(seed, n, e):
    rng = np.random.Generator(np.random.PCG64(seed))
    src = rng.integers(0, n, size=e)
    dst = rng.integers(0, n, size=e)
    return src.astype(np.int64), dst.astype(np.int64)


def check_invariants(src, dst, n, lab, keep=None):
    v = np.arange(n)
    assert (lab <= v).all()
    assert np.array_equal(lab[lab], lab)
    s, d = (src, dst) if keep is None else (src[keep], dst[keep])
    assert np.array_equal(lab[s], lab[d])


@pytest.mark.parametrize("seed,n,e", [(1, 1, 0), (2, 10, 5), (3, 50, 40), (4, 500, 300), (5, 2000, 1500),
                                      (6, 3000, 6000), (7, 100, 0)])
def test_matches_scipy_and_propagation(seed, n, e):
    src, dst = random_graph(seed, n, e)
    got = components.labels(src, dst, n)
    assert np.array_equal(got, scipy_min_labels(src, dst, n))
    assert np.array_equal(got, propagate(src, dst, n))
    check_invariants(src, dst, n, got)


def test_threshold_is_strict_and_scores_select_edges():
    rng = np.random.Generator(np.random.PCG64(11))
    src, dst = random_graph(12, 400, 600)
    scores = rng.uniform(0, 1, size=src.size).astype(np.float32)
    scores[::7] = np.float32(0.5)  # exactly at the threshold: dropped
    keep = scores > np.float32(0.5)
    got = components.labels(src, dst, 400, scores, 0.5)
    assert np.array_equal(got, scipy_min_labels(src, dst, 400, keep))
    assert np.array_equal(got, propagate(src, dst, 400, keep))
    check_invariants(src, dst, 400, got, keep)
    # A single edge at the threshold joins nothing; just above, it joins.
    one = components.labels(np.array([3]), np.array([1]), 5, np.array([0.25], np.float32), 0.25)
    assert one.tolist() == [0, 1, 2, 3, 4]
    one = components.labels(np.array([3]), np.array([1]), 5, np.array([np.nextafter(np.float32(0.25), np.float32(1))],
                                                                       np.float32), 0.25)
    assert one.tolist() == [0, 1, 2, 1, 4]


def test_hand_built_graphs():
    # Direction is ignored; every component is named by its smallest member.
    src = np.array([7, 5, 9, 4])
    dst = np.array([3, 7, 0, 4])  # 3-7-5, 0-9, a self-loop on 4
    assert components.labels(src, dst, 10).tolist() == [0, 1, 2, 3, 4, 3, 6, 3, 8, 0]
    # A chain given back to front, with a duplicated edge.
    n = 6
    src = np.array([5, 4, 3, 2, 1, 1])
    dst = np.array([4, 3, 2, 1, 0, 0])
    assert components.labels(src, dst, n).tolist() == [0] * n
    # No edges: every vertex is alone.
    assert components.labels(np.zeros(0, np.int64), np.zeros(0, np.int64), 4).tolist() == [0, 1, 2, 3]
    assert components.labels(np.zeros(0, np.int64), np.zeros(0, np.int64), 0).tolist() == []


def test_bad_endpoints_are_rejected():
    with pytest.raises(components.OracleError):
        components.labels(np.array([0]), np.array([5]), 5)
    with pytest.raises(components.OracleError):
        components.labels(np.array([-1]), np.array([0]), 5)


def test_frnn_graph_of_the_tiny_event():
    X, truth = events.generate(events.TINY)
    g = oracle.frnn_grid(X, events.TINY.r, events.TINY.K)
    got = components.labels(g[0], g[1], X.shape[0])
    assert np.array_equal(got, scipy_min_labels(g[0], g[1], X.shape[0]))
    check_invariants(g[0], g[1], X.shape[0], got)
    # Clusters are far apart relative to r, so most clusters form one component.
    assert len(np.unique(got)) < X.shape[0]


MUTATIONS = {
    # adjacency stored one way only: components of the directed reachability
    "one_direction": ("        adj[first[b] + fill[b]++] = a;\n", "        adj[first[b] + fill[b]++] = b;\n"),
    # threshold taken as >= instead of >
    "threshold_ge": ("if (scores && !(scores[e] > threshold))", "if (scores && !(scores[e] >= threshold))"),
    # searches started from the largest vertex: components named by their largest member
    "max_label": ("    for (int64_t v = 0; v < n; ++v) {\n        if (label[v] >= 0)",
                  "    for (int64_t v = n - 1; v >= 0; --v) {\n        if (label[v] >= 0)"),
    # neighbours labeled with the current vertex instead of the search's start
    "label_parent": ("                    label[w] = v;", "                    label[w] = u;"),
}


def pins(lib):
    out = {}
    try:
        src, dst = random_graph(3, 50, 40)
        out["scipy"] = np.array_equal(components.labels(src, dst, 50, lib=lib), scipy_min_labels(src, dst, 50))
        rng = np.random.Generator(np.random.PCG64(11))
        s2, d2 = random_graph(12, 400, 600)
        sc = rng.uniform(0, 1, size=s2.size).astype(np.float32)
        sc[::7] = np.float32(0.5)
        keep = sc > np.float32(0.5)
        out["threshold"] = np.array_equal(components.labels(s2, d2, 400, sc, 0.5, lib=lib),
                                          propagate(s2, d2, 400, keep))
        out["hand"] = components.labels(np.array([7, 5, 9, 4]), np.array([3, 7, 0, 4]), 10, lib=lib).tolist() == \
            [0, 1, 2, 3, 4, 3, 6, 3, 8, 0]
    except components.OracleError:
        out["error"] = False
    return out


def test_pins_pass_on_shipped_oracle():
    assert all(pins(components.load()).values())


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(components.SRC).read()
    assert old in src, name
    path = tmp_path / f"mut_{name}.c"
    path.write_text(src.replace(old, new))
    lib = components.load(components.build(str(path), str(tmp_path / f"lib_{name}.so")))
    res = pins(lib)
    assert not all(res.values()), f"mutation {name} passed every pin: {res}"
