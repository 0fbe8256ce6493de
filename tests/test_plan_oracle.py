"""Pins of the topology oracle (Sec. VII) against the paper: the worked
schedules of Fig. 2, Lemma 2 (geometric progress and its tightness tree),
Lemma 3 (readiness-weighted reduction), Lemma 4 (D_N), "#rakes +
#compressions = N - 1" (Sec. IX-B) and the star row of Table I."""
import json
import math
import os

import numpy as np
import pytest

from oracle import plan as pl
from paper_2608_01332_amd import workloads as w

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_fig2_labels():
    g = json.load(open(os.path.join(GOLD, "fig2_schedules.json")))
    for name, case in g["cases"].items():
        P = pl.make_plan(case["parent"])
        got = {str(v): f"{k}{r}" for v, (k, r, _) in P["removed"].items()}
        assert got == case["labels"], name
        assert P["rounds"] == case["rounds"], name


def _trees():
    rng = np.random.default_rng(4)
    out = [w.tree_chain(50), w.tree_star(40), w.tree_balanced(63), w.tree_comb(41),
           w.tree_caterpillar(30, 3), w.lemma2_tight_tree(16)]
    for _ in range(8):
        par = w.tree_chainprob(int(rng.integers(2, 300)), float(rng.uniform(0.3, 0.99)), rng)
        out.append(w.permute_labels(par, rng)[0])
    return out


@pytest.mark.parametrize("parent", _trees())
def test_progress_and_counts(parent):
    N = len(parent)
    P = pl.make_plan(parent)
    assert len(P["removed"]) == N - 1                      # every non-root node once
    # Lemma 2: each round removes >= ceil(N_r / 3) of the N_r nodes present
    present = N
    for r in range(1, P["rounds"] + 1):
        gone = sum(1 for v in P["removed"].values() if v[1] == r)
        assert 3 * gone >= present
        present -= gone
    assert present == 1
    R = 0
    while 1.5 ** R < N:
        R += 1
    assert P["rounds"] <= R
    assert P["levels"] <= pl.depth_bound(N)               # Lemma 4
    # k - 1 combinations per reduction of k contributions (Lemma 3)
    by = {}
    for v, (k, r, _) in P["removed"].items():
        if k == "R":
            by[(parent_at_removal(P, parent, v), r)] = by.get((parent_at_removal(P, parent, v), r), 0) + 1
    assert len(P["combines"]) == sum(k - 1 for k in by.values())
    assert len(P["absorbs"]) == len(by)


def parent_at_removal(P, parent, v):
    # the node that absorbs v's contribution: the nearest ancestor not compressed before v's rake
    r = P["removed"][v][1]
    a = parent[v]
    while a >= 0 and a in P["removed"] and P["removed"][a][0] == "C" and P["removed"][a][1] < r:
        a = parent[a]
    return a


def test_lemma2_tight():
    for k in (2, 4, 8, 32):
        par = w.lemma2_tight_tree(k)
        P = pl.make_plan(par)
        first = sum(1 for v in P["removed"].values() if v[1] == 1)
        assert len(par) == 3 * k and first == k


def test_table1_star_exact_and_soft_rows():
    g = json.load(open(os.path.join(GOLD, "table1_levels.json")))
    for topo, row in g["rows"].items():
        for N, paper_levels in zip(g["N"], row):
            lv = pl.make_plan(getattr(w, "tree_" + topo)(N))["levels"]
            if topo in g["exact_rows"]:
                assert lv == paper_levels, (topo, N)
            else:
                assert lv <= pl.depth_bound(N)
                assert lv <= 4 * math.log2(N) + 4


def _prefix(a, b):
    (ra, da), (rb, db) = a, b
    return da <= db and (rb >> (db - da)) == ra


@pytest.mark.parametrize("seed", range(20))
def test_sfe_reduction_lemma3(seed):
    """Lemma 3: codewords prefix-free and in sibling order, k-1 combinations, final level
    <= ceil(log2 W) + 1."""
    rng = np.random.default_rng(seed)
    k = int(rng.integers(1, 40))
    levels = [int(v) for v in rng.integers(0, 12, size=k)]
    tree, codes = pl._sfe_tree(levels)
    for i in range(k):
        for j in range(k):
            if i != j:
                assert not _prefix(codes[i], codes[j])
    # lexicographic order of the dyadic intervals is the sibling order
    lo = [r / 2 ** d for r, d in codes]
    assert all(lo[i] < lo[i + 1] for i in range(k - 1))
    leaves, ncomb, out = [], [0], [0]

    def walk(t, depth):
        if isinstance(t, int):
            leaves.append(t)
            out[0] = max(out[0], levels[t] + depth)
            return
        ncomb[0] += 1
        walk(t[0], depth + 1)
        walk(t[1], depth + 1)

    walk(tree, 0)
    assert leaves == list(range(k))
    assert ncomb[0] == k - 1
    W = sum(2 ** l for l in levels)
    assert out[0] <= math.ceil(math.log2(W)) + 1


def test_depth_bound_values():
    # D_N = floor(log2(2N-1) + ceil(log_{3/2} N) log2 36)
    for N in (2, 16, 100, 4096, 65536):
        R = math.ceil(math.log(N) / math.log(1.5) - 1e-12)
        approx = math.floor(math.log2(2 * N - 1) + R * math.log2(36))
        assert abs(pl.depth_bound(N) - approx) <= 1
