"""Pins of the CPU oracle against what the definition and the mathematics fix.

The paper defines the graph as all pairs of points closer than a constant radius
in the embedding space (Section 2) and builds it with a grid-cell search
(Section 3.4).  It prints no worked example, so the oracle is pinned by:
  * the O(n^2) definition (brute force) on tiny and stress inputs, and written
    out in numpy float32 for sampled queries of the full-size benchmark events;
  * exact-arithmetic inputs checked against scipy's k-d tree and against
    integer squared distances (nearest-K reduction, the Section 3.1 reading);
  * float64 distances away from the radius;
  * closed-form cases derived by hand (strict radius, summation order, no fused
    multiply-add, subnormals, duplicate ties, complete graph);
  * the expected edge count of the clustered generator (chi-square closed form).
"""

from fractions import Fraction

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st
from scipy.spatial import cKDTree
from scipy.stats import chi2

from oracle import invariants, oracle
from paper_2202_06929_amd import events


def fl32(x) -> Fraction:
    """Round an exact rational to the nearest float32 (ties to even), normal range only."""
    x = Fraction(x)
    if x == 0:
        return Fraction(0)
    sign = -1 if x < 0 else 1
    x = abs(x)
    e = 0
    while x >= 2:
        x /= 2
        e += 1
    while x < 1:
        x *= 2
        e -= 1
    m = x * 2 ** 23
    q = m.numerator // m.denominator
    rem = m - q
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and q % 2 == 1):
        q += 1
    return sign * Fraction(q, 2 ** 23) * Fraction(2) ** e


def as_set(edges):
    return set(zip(edges[0].tolist(), edges[1].tolist()))


# ---------------------------------------------------------------- brute force

def _sampled_definition(X, r, K, queries):
    """N(i) of the definition for the given queries against every point, written
    out with numpy float32 arithmetic: differences, squares and the sum over the
    coordinates in ascending order, each rounded to float32 (numpy fuses nothing),
    the strict test against fl32(r * r), then the cap by (D, j)."""
    X = np.ascontiguousarray(X, dtype=np.float32)
    r32 = np.float32(r)
    r2 = np.float32(r32 * r32)
    out = {}
    for i in queries:
        t = X - X[i]
        acc = t[:, 0] * t[:, 0]
        for k in range(1, X.shape[1]):
            acc = acc + t[:, k] * t[:, k]
        hit = np.flatnonzero(acc < r2)
        hit = hit[hit != i]
        order = np.lexsort((hit, acc[hit]))  # by D, then j
        out[i] = np.sort(hit[order][:K])
    return out


@pytest.mark.parametrize("spec", [events.SINGLE, events.HIGH], ids=["single_120k", "high_300k_12d"])
def test_grid_matches_the_definition_on_sampled_queries_at_full_size(spec):
    # The benchmark events themselves: 300 queries drawn at random, each against
    # every point of the event.
    X, _ = events.generate(spec)
    g = oracle.frnn_grid(X, spec.r, spec.K)
    rng = np.random.Generator(np.random.PCG64(31))
    queries = rng.choice(len(X), size=300, replace=False)
    want = _sampled_definition(X, spec.r, spec.K, queries)
    starts = np.searchsorted(g[0], np.arange(len(X) + 1))
    n_hits = 0
    for i in queries:
        got = g[1, starts[i]:starts[i + 1]]
        assert np.array_equal(got, want[i]), i
        n_hits += len(got)
    assert n_hits > 300  # the sample holds real neighbour lists


def test_grid_equals_brute_tiny_event():
    X, _ = events.generate(events.TINY)
    g = oracle.frnn_grid(X, events.TINY.r, events.TINY.K)
    b = oracle.frnn_brute(X, events.TINY.r, events.TINY.K)
    assert g.shape[1] > 10_000
    assert np.array_equal(g, b)


@pytest.mark.parametrize("case", events.stress_cases(), ids=lambda c: c.name)
def test_grid_equals_brute_stress(case):
    g = oracle.frnn_grid(case.points, case.r, case.K)
    b = oracle.frnn_brute(case.points, case.r, case.K)
    assert np.array_equal(g, b)
    if case.points.shape[0]:
        invariants.check(case.points, case.r, case.K, g, oracle.degrees(case.points, case.r))


@st.composite
def small_inputs(draw):
    n = draw(st.integers(0, 300))
    d = draw(st.integers(3, 12))
    seed = draw(st.integers(0, 2 ** 31))
    rng = np.random.Generator(np.random.PCG64(seed))
    kind = draw(st.sampled_from(["uniform", "clumps", "dups", "lattice"]))
    if kind == "uniform":
        X = rng.uniform(-1, 1, size=(n, d))
    elif kind == "clumps":
        c = rng.uniform(-1, 1, size=(max(1, n // 20), d))
        X = c[rng.integers(0, len(c), size=n)] + rng.normal(0, 0.05, size=(n, d))
    elif kind == "dups":
        c = rng.uniform(-1, 1, size=(max(1, n // 10), d))
        X = c[rng.integers(0, len(c), size=n)]
    else:
        X = rng.integers(-4, 5, size=(n, d)) * 0.125
    r = draw(st.sampled_from([0.05, 0.1, 0.125, 0.25, 0.3, 0.6, 2.0]))
    K = draw(st.integers(1, 40))
    return X.astype(np.float32), r, K


@settings(max_examples=60, deadline=None, suppress_health_check=[HealthCheck.too_slow])
@given(small_inputs())
def test_grid_equals_brute_random(inp):
    X, r, K = inp
    g = oracle.frnn_grid(X, r, K)
    b = oracle.frnn_brute(X, r, K)
    assert np.array_equal(g, b)
    if X.shape[0]:
        invariants.check(X, r, K, g, oracle.degrees(X, r))


# ------------------------------------------------------ exact-arithmetic inputs

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dyadic_points_match_kdtree(seed):
    # All float32 steps are exact on these points, so D(i,j) is the true squared
    # distance.  r2 = fl32(0.2^2) is not a multiple of 2^-12, so no pair sits on
    # the radius and '<' and '<=' agree: the edge set is the k-d tree's pair set.
    X, _ = events.dyadic_event(1500, 8, seed)
    r, K = 0.2, 10_000
    got = as_set(oracle.frnn_grid(X, r, K))
    r2 = float(np.float32(r) * np.float32(r))
    assert (Fraction(r2) * 4096).denominator != 1
    pairs = cKDTree(X.astype(np.float64)).query_pairs(np.sqrt(r2), output_type="ndarray")
    want = set(map(tuple, pairs.tolist())) | set((j, i) for i, j in pairs.tolist())
    assert len(want) > 1000
    assert got == want


@pytest.mark.parametrize("K", [1, 3, 7, 25, 398])
def test_dyadic_nearest_k_matches_integer_lexsort(K):
    # With r larger than every distance, Out(i) is the K nearest by (D, j): the
    # exact k-nearest-neighbour search of Section 3.1 with index tie-break.  On
    # dyadic points D(i,j) = sum (a_i - a_j)^2 / 4096 exactly (integer arithmetic).
    # K = 398 = n - 2 leaves every query exactly one neighbour over the cap.
    X, A = events.dyadic_event(400, 6, 5, n_clusters=6, sigma=0.03)
    got = oracle.frnn_grid(X, 100.0, K)
    n = len(X)
    Dint = ((A[:, None, :] - A[None, :, :]) ** 2).sum(-1)
    rows, cols = [], []
    for i in range(n):
        j = np.arange(n)
        keep = j != i
        order = np.lexsort((j[keep], Dint[i, keep]))[:K]
        sel = np.sort(j[keep][order])
        rows += [i] * len(sel)
        cols += sel.tolist()
    want = np.array([rows, cols], dtype=np.int64)
    assert np.array_equal(got, want)


def test_float64_band_tiny_event():
    X, _ = events.generate(events.TINY)
    g = oracle.frnn_grid(X, events.TINY.r, events.TINY.K)
    invariants.check_against_reals(X, events.TINY.r, events.TINY.K, g)
    invariants.check(X, events.TINY.r, events.TINY.K, g, oracle.degrees(X, events.TINY.r))


# ------------------------------------------------------------ hand derivations

def test_radius_is_strict():
    # r = 0.5: r2 = 0.25 exactly.  Point 1 is at distance 0.5 from point 0, so
    # D(0,1) = 0.25 = r2 and the pair is not an edge.  Point 2 is at 0.5 - 2^-25:
    # D = 0.25 - 2^-25 + 2^-50, which rounds to 0.25 - 2^-25 < r2 (spacing below
    # 0.25 is 2^-26), so it is.  Points 1 and 2 are 2^-25 apart.
    X = np.zeros((3, 3), np.float32)
    X[1, 0] = 0.5
    X[2, 0] = np.float32(0.5 - 2.0 ** -25)
    assert fl32((Fraction(1, 2) - Fraction(1, 2 ** 25)) ** 2) == Fraction(1, 4) - Fraction(1, 2 ** 25)
    for route in (oracle.frnn_grid, oracle.frnn_brute):
        assert as_set(route(X, 0.5, 8)) == {(0, 2), (1, 2), (2, 0), (2, 1)}


def test_radius_squared_is_rounded_to_float32():
    # r = 0.5 + 2^-24: r^2 = 0.25 + 2^-24 + 2^-48 exactly, which rounds to
    # r2 = 0.25 + 2^-24 (spacing 2^-25 in [0.25, 0.5)).  P1 - P0 = (0.5, 2^-12, 0)
    # gives D = fl(0.25 + 2^-24) = 0.25 + 2^-24 = r2: not an edge.  Comparing with
    # the unrounded r^2 would accept it.
    X = np.zeros((2, 3), np.float32)
    X[1, 0] = 0.5
    X[1, 1] = np.float32(2.0 ** -12)
    r = np.float32(0.5 + 2.0 ** -24)
    assert fl32(Fraction(float(r)) ** 2) == Fraction(1, 4) + Fraction(1, 2 ** 24)
    for route in (oracle.frnn_grid, oracle.frnn_brute):
        assert route(X, float(r), 8).shape == (2, 0)


def test_summation_order_is_ascending():
    # d = 9.  P1 - P0 = (2^-13 x8, 0.75).  Ascending order first adds eight
    # squares 2^-26 exactly (2^-23), then 0.5625: D = 0.5625 + 2^-23, exactly.
    # r = 0.75 + 2^-24 gives r2 = fl(0.5625 + 1.5*2^-24 + 2^-48) = 0.5625 + 2^-23
    # (spacing 2^-24 in [0.5, 1)).  So D == r2: not an edge.  Adding 0.5625 first
    # would absorb every 2^-26 (a quarter spacing) and give D = 0.5625 < r2.
    # P2 - P0 = (2^-13 x4, 0 x4, 0.75): D = 0.5625 + 2^-24 < r2 in either order.
    # P2 - P1 = (0 x4, 2^-13 x4, 0): D = 2^-24 < r2.
    t = np.float32(2.0 ** -13)
    X = np.zeros((3, 9), np.float32)
    X[1, :8] = t
    X[1, 8] = 0.75
    X[2, :4] = t
    X[2, 8] = 0.75
    r = np.float32(0.75 + 2.0 ** -24)
    assert float(r) == 0.75 + 2.0 ** -24
    r2 = fl32(Fraction(float(r)) ** 2)
    assert r2 == Fraction(9, 16) + Fraction(1, 2 ** 23)
    for route in (oracle.frnn_grid, oracle.frnn_brute):
        assert as_set(route(X, float(r), 8)) == {(0, 2), (2, 0), (1, 2), (2, 1)}


def test_products_are_rounded_before_the_sum():
    # d = 3, P1 - P0 = (1, t, 0) with t = 12000050 * 2^-25.  Separately rounded:
    # fl(t^2) then fl(1 + fl(t^2)) = D_sep; a fused multiply-add would give
    # D_fma = fl(1 + t^2), one spacing higher.  r (bits 0x3f87f076) has
    # fl(r^2) = D_fma, so the pair is an edge only without fusion.
    t = Fraction(12000050, 2 ** 25)
    r = np.array([0x3F87F076], np.uint32).view(np.float32)[0]
    r2 = fl32(Fraction(float(r)) ** 2)
    d_sep = fl32(1 + fl32(t * t))
    d_fma = fl32(1 + t * t)
    assert d_sep < r2 == d_fma
    X = np.zeros((2, 3), np.float32)
    X[1, 0] = 1.0
    X[1, 1] = np.float32(float(t))
    assert Fraction(float(X[1, 1])) == t
    for route in (oracle.frnn_grid, oracle.frnn_brute):
        assert as_set(route(X, float(r), 8)) == {(0, 1), (1, 0)}
    np.testing.assert_array_equal(oracle.pair_dist(X, np.array([0]), np.array([1])),
                                  np.array([float(d_sep)], np.float32))


def test_subnormal_distances_are_kept():
    # P1 - P0 = (2^-70, 0, 0): D = 2^-140, a subnormal float32, and r = 2^-69
    # gives r2 = 2^-138 (also subnormal).  D < r2: an edge.  Flushing subnormals
    # to zero would make both 0 and drop the edge.  P2 - P0 = (2^-76, 0, 0):
    # 2^-152 rounds to 0 (below half the smallest subnormal 2^-149), D = 0 < r2.
    X = np.zeros((3, 3), np.float32)
    X[1, 0] = np.float32(2.0 ** -70)
    X[2, 0] = np.float32(2.0 ** -76)
    r = float(np.float32(2.0 ** -69))
    got = as_set(oracle.frnn_brute(X, r, 8))
    assert got == {(0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)}
    assert as_set(oracle.frnn_grid(X, r, 8)) == got
    D = oracle.pair_dist(X, np.array([0, 0]), np.array([1, 2]))
    assert D[0] == np.float32(2.0 ** -140) and D[1] == 0.0


def test_duplicate_ties_take_smallest_indices():
    # S2: 50 copies of one point, K = 8.  For a copy i, every other copy is at
    # D = 0, the smallest possible, so Out(i) is the 8 smallest indices among the
    # other copies (index breaks the tie).
    case = next(c for c in events.stress_cases() if c.name == "S2_duplicates_ties")
    X = case.points
    g = oracle.frnn_grid(X, case.r, case.K)
    groups = {}
    for idx, row in enumerate(map(bytes, X)):
        groups.setdefault(row, []).append(idx)
    dup = max(groups.values(), key=len)
    assert len(dup) == 50
    for i in dup:
        others = [j for j in dup if j != i][:8]
        assert g[1][g[0] == i].tolist() == others


def test_complete_graph_when_radius_covers_everything():
    case = next(c for c in events.stress_cases() if c.name == "S4_complete_r10_K400")
    n = len(case.points)
    g = oracle.frnn_grid(case.points, case.r, case.K)
    assert g.shape[1] == n * (n - 1)
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = ii != jj
    assert np.array_equal(g, np.stack([ii[keep], jj[keep]]))


# ------------------------------------------------------------- closed forms

@pytest.mark.parametrize("spec", [events.TINY, events.SINGLE], ids=["tiny", "single"])
def test_edge_count_matches_cluster_closed_form(spec):
    # Two points of one cluster differ by N(0, 2 sigma^2) per coordinate, so
    # |x_a - x_b|^2 / (2 sigma^2) ~ chi^2_d and a same-cluster ordered pair is an
    # edge with probability F_{chi^2_d}(r^2 / (2 sigma^2)).  Pairs across clusters
    # or with noise are rare at these densities (8-ball of radius 0.1 has volume
    # 4e-8), and K never binds (clusters have at most 20 points).
    X, labels = events.generate(spec)
    g = oracle.frnn_grid(X, spec.r, spec.K)
    sizes = events.cluster_sizes_of(labels).astype(np.float64)
    p = chi2.cdf(spec.r ** 2 / (2 * spec.sigma ** 2), spec.d)
    expected = float(np.sum(sizes * (sizes - 1))) * p
    assert abs(g.shape[1] - expected) / expected < 0.02
    same = labels[g[0]] == labels[g[1]]
    assert same.mean() > 0.995


# --------------------------------------------------------------- arguments

def test_rejects_non_finite_and_bad_arguments():
    X = np.zeros((4, 3), np.float32)
    X[2, 1] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.frnn_grid(X, 0.1, 4)
    assert e.value.status == oracle.ERR_NONFINITE
    X[2, 1] = np.inf
    with pytest.raises(oracle.OracleError):
        oracle.frnn_brute(X, 0.1, 4)
    Y = np.zeros((4, 3), np.float32)
    for r, K in ((0.0, 4), (-1.0, 4), (float("nan"), 4), (float("inf"), 4), (0.1, 0)):
        with pytest.raises(oracle.OracleError) as e:
            oracle.frnn_grid(Y, r, K)
        assert e.value.status == oracle.ERR_ARG


def test_empty_and_single_point():
    for n in (0, 1):
        X = np.zeros((n, 5), np.float32)
        assert oracle.frnn_grid(X, 0.1, 3).shape == (2, 0)
        assert oracle.frnn_brute(X, 0.1, 3).shape == (2, 0)
