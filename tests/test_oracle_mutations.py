"""The oracle's pins catch plausible mistakes.

Each case below plants one mistake in a private copy of the oracle's C source (or
its build flags), builds it on the CPU, and checks that at least one pin of
test_oracle fails against the planted copy.  The shipped oracle is untouched.
"""

import os
from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial import cKDTree

from oracle import invariants, oracle
from paper_2202_06929_amd import events

MUTATIONS = {
    "first_term_dropped": ("for (int k = 0; k < d; ++k) {\n        float t",
                           "for (int k = 1; k < d; ++k) {\n        float t"),
    "last_term_dropped": ("for (int k = 0; k < d; ++k) {\n        float t",
                          "for (int k = 0; k < d - 1; ++k) {\n        float t"),
    "wrong_index": ("float t = xi[k] - xj[k];", "float t = xi[k] - xj[k ? k - 1 : 0];"),
    "wrong_sign": ("float t = xi[k] - xj[k];", "float t = xi[k] + xj[k];"),
    "reversed_order": ("for (int k = 0; k < d; ++k) {\n        float t",
                       "for (int k = d - 1; k >= 0; --k) {\n        float t"),
    "radius_not_strict": ("D < r2", "D <= r2"),
    "radius_in_double": ("const float r2 = r * r;", "const double r2 = (double)r * (double)r;"),
    "missing_cells": ("for (int dz = -1; dz <= 1; ++dz)", "for (int dz = -1; dz <= 0; ++dz)"),
    "cells_too_small": ("const double c = (double)r * (1.0 + 1.0 / 1024.0);",
                        "const double c = (double)r * 0.5;"),
    "cap_off_by_one": ("if (keep > K) {", "if (keep > K + 1) {"),
    "tie_break_reversed": ("return (x->j > y->j) - (x->j < y->j);\n}\n\nstatic int cmp_hit_index",
                           "return (x->j < y->j) - (x->j > y->j);\n}\n\nstatic int cmp_hit_index"),
    "self_loop_in_grid": ("if (j == i) continue;\n                        float D",
                          "float D"),
    "cap_by_index_only": ("qsort(h->v, (size_t)h->len, sizeof(hit_t), cmp_hit_dist_then_index);",
                          "qsort(h->v, (size_t)h->len, sizeof(hit_t), cmp_hit_index);"),
}


# Mistakes planted at every occurrence (both routes) rather than at the first.
EVERYWHERE = {"radius_not_strict", "radius_in_double"}


def _as_set(edges):
    return set(zip(edges[0].tolist(), edges[1].tolist()))


def pins(lib) -> dict:
    """Runs the pins against one build of the oracle; returns {pin: passed}."""
    res = {}

    def run(name, fn):
        try:
            res[name] = bool(fn())
        except Exception:  # a crash or an error status is a failed pin
            res[name] = False

    X, _ = events.generate(events.TINY)

    def brute_vs_grid():
        g = oracle.frnn_grid(X, 0.1, 64, lib=lib)
        return np.array_equal(g, oracle.frnn_brute(X, 0.1, 64, lib=lib)) and g.shape[1] > 10_000

    def invariants_tiny():
        g = oracle.frnn_grid(X, 0.1, 64, lib=lib)
        invariants.check(X, 0.1, 64, g, oracle.degrees(X, 0.1))
        invariants.check_against_reals(X[:600], 0.1, 64, oracle.frnn_grid(X[:600], 0.1, 64, lib=lib))
        return True

    def kdtree():
        Y, _ = events.dyadic_event(1000, 8, 0)
        r2 = float(np.float32(0.2) * np.float32(0.2))
        pairs = cKDTree(Y.astype(np.float64)).query_pairs(np.sqrt(r2), output_type="ndarray")
        want = set(map(tuple, pairs.tolist())) | set((j, i) for i, j in pairs.tolist())
        return _as_set(oracle.frnn_grid(Y, 0.2, 10_000, lib=lib)) == want

    def knn():
        Y, A = events.dyadic_event(200, 6, 5, n_clusters=4, sigma=0.03)
        Dint = ((A[:, None, :] - A[None, :, :]) ** 2).sum(-1)
        ok = True
        for K in (5, 198):  # 198 = n - 2: every query has exactly K + 1 neighbours
            got = oracle.frnn_grid(Y, 100.0, K, lib=lib)
            rows, cols = [], []
            for i in range(len(Y)):
                j = np.arange(len(Y))
                keep = j != i
                sel = np.sort(j[keep][np.lexsort((j[keep], Dint[i, keep]))[:K]])
                rows += [i] * len(sel)
                cols += sel.tolist()
            ok = ok and np.array_equal(got, np.array([rows, cols], dtype=np.int64))
        return ok

    def strict():
        Y = np.zeros((3, 3), np.float32)
        Y[1, 0] = 0.5
        Y[2, 0] = np.float32(0.5 - 2.0 ** -25)
        ok = _as_set(oracle.frnn_grid(Y, 0.5, 8, lib=lib)) == {(0, 2), (1, 2), (2, 0), (2, 1)}
        Z = np.zeros((2, 3), np.float32)
        Z[1, 0] = 0.5
        Z[1, 1] = np.float32(2.0 ** -12)
        r = float(np.float32(0.5 + 2.0 ** -24))
        return ok and oracle.frnn_grid(Z, r, 8, lib=lib).shape[1] == 0

    def order():
        t = np.float32(2.0 ** -13)
        Y = np.zeros((3, 9), np.float32)
        Y[1, :8] = t
        Y[1, 8] = 0.75
        Y[2, :4] = t
        Y[2, 8] = 0.75
        r = float(np.float32(0.75 + 2.0 ** -24))
        return _as_set(oracle.frnn_grid(Y, r, 8, lib=lib)) == {(0, 2), (2, 0), (1, 2), (2, 1)}

    def no_fma():
        Y = np.zeros((2, 3), np.float32)
        Y[1, 0] = 1.0
        Y[1, 1] = np.float32(float(Fraction(12000050, 2 ** 25)))
        r = float(np.array([0x3F87F076], np.uint32).view(np.float32)[0])
        return _as_set(oracle.frnn_brute(Y, r, 8, lib=lib)) == {(0, 1), (1, 0)}

    def ties():
        case = next(c for c in events.stress_cases() if c.name == "S2_duplicates_ties")
        g = oracle.frnn_grid(case.points, case.r, case.K, lib=lib)
        groups = {}
        for idx, row in enumerate(map(bytes, case.points)):
            groups.setdefault(row, []).append(idx)
        dup = max(groups.values(), key=len)
        return all(g[1][g[0] == i].tolist() == [j for j in dup if j != i][:8] for i in dup)

    for name, fn in [("brute_vs_grid", brute_vs_grid), ("invariants", invariants_tiny),
                     ("kdtree", kdtree), ("knn", knn), ("strict", strict), ("order", order),
                     ("no_fma", no_fma), ("ties", ties)]:
        run(name, fn)
    return res


def test_pins_pass_on_shipped_oracle():
    res = pins(oracle.load())
    assert all(res.values()), res


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = open(oracle.SRC).read()
    assert old in src, f"mutation anchor for {name} not found"
    mutated = src.replace(old, new, 1) if name not in EVERYWHERE else src.replace(old, new)
    path = tmp_path / "mut.c"
    path.write_text(mutated)
    lib_path = oracle.build(str(path), str(tmp_path / "libmut.so"))
    res = pins(oracle.load(lib_path))
    assert not all(res.values()), f"no pin caught {name}: {res}"


def test_fused_multiply_add_build_is_caught(tmp_path):
    if os.uname().machine != "x86_64":
        pytest.skip("fma flag is x86-specific")
    lib_path = oracle.build(oracle.SRC, str(tmp_path / "libfma.so"),
                            extra_flags=["-ffp-contract=fast", "-mfma"])
    res = pins(oracle.load(lib_path))
    assert not res["no_fma"], res
