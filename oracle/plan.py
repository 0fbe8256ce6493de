"""Topology-only rake-compress schedule of Sec. VII, written out plainly.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Structural rounds (Sec. VII-A): at the start of a round every non-root leaf
is raked; then, in the tree left after those rakes, a maximal set of
pairwise non-adjacent non-root unary nodes is compressed, chosen greedily in
increasing node id (a node is taken unless its parent or its child was
already taken).

Dependency levels (Sec. VII-B, eq. (earliest-level)): initial node and edge
data have producer level 0; every primitive (rake, combine, absorb,
compress) runs at 1 + the largest producer level of its inputs and gives its
output that level.  Rake contributions to one parent in one round are
reduced by the readiness-weighted alphabetic Shannon-Fano-Elias code of
eq. (readiness-code-data): weights w_j = 2^{l_j}, code lengths
ceil(log2(W / w_j)) + 1, the codeword of j the leading bits of the midpoint
F_j + p_j / 2; the binary trie of the codewords with unary vertices
suppressed is the reduction tree (Lemma 3).  All arithmetic is exact
(Python integers).

Readings where the paper is silent:
* sibling order is the order of a parent's outgoing edges, an edge keeping
  its position when a compression replaces it; initially children are in
  increasing id.
* a parent with a single contribution in a round has no combination; its
  absorption reads the rake contribution directly.
"""
from __future__ import annotations


def _sfe_tree(levels):
    """Order-preserving reduction tree for contributions with producer levels
    `levels` (sibling order).  Returns a nested structure: an int (leaf index)
    or a pair (left, right)."""
    k = len(levels)
    w = [1 << l for l in levels]
    W = sum(w)
    codes = []
    S = 0
    for j in range(k):
        d = 0
        while (w[j] << d) < W:      # smallest d with 2^d >= W / w_j
            d += 1
        d += 1                      # d_j^0 = ceil(log2(W / w_j)) + 1
        num = (2 * S + w[j]) << d   # midpoint (2 S_j + w_j) / (2 W), scaled by 2^d
        rj = num // (2 * W)
        codes.append((rj, d))
        S += w[j]

    def bit(j, pos):
        rj, d = codes[j]
        return (rj >> (d - 1 - pos)) & 1

    def build(lo, hi, depth):
        while True:
            if lo == hi:
                return lo
            s = None
            for j in range(lo, hi + 1):
                if bit(j, depth) == 1:
                    s = j
                    break
            if s is None or s == lo:        # all words agree at this bit: unary trie vertex
                depth += 1
                continue
            return (build(lo, s - 1, depth + 1), build(s, hi, depth + 1))

    return build(0, k - 1, 0), codes


def make_plan(parent):
    """Return a dict describing the schedule:
      removed[v] = (kind 'R'|'C', round, level)   for every non-root v
      combines   = list of (parent, round, level, tuple(sorted child ids covered))
      absorbs    = list of (parent, round, level)
      rounds, levels (number of nonempty dependency levels)."""
    parent = [int(p) for p in parent]
    N = len(parent)
    roots = [v for v in range(N) if parent[v] < 0]
    assert len(roots) == 1
    root = roots[0]
    cur_par = list(parent)
    kids = [[] for _ in range(N)]           # current children, in sibling order
    for j in range(N):
        if parent[j] >= 0:
            kids[parent[j]].append(j)
    lvlU = [0] * N                           # producer level of node datum U_v
    lvlE = [0] * N                           # producer level of the edge entering v
    alive = [True] * N
    removed = {}
    combines = []
    absorbs = []
    rnd = 0
    nalive = N
    while nalive > 1:
        rnd += 1
        # ---- rakes
        leaves = [v for v in range(N) if alive[v] and v != root and not kids[v]]
        lvl_of = {}
        for j in leaves:
            lv = 1 + max(lvlU[j], lvlE[j])
            removed[j] = ("R", rnd, lv)
            lvl_of[j] = lv
        by_parent = {}
        for j in leaves:
            by_parent.setdefault(cur_par[j], []).append(j)
        for i, js in by_parent.items():
            js.sort(key=lambda j: kids[i].index(j))
            tree, _ = _sfe_tree([lvl_of[j] for j in js])

            def walk(t):
                if isinstance(t, int):
                    return lvl_of[js[t]], (js[t],)
                la, ca = walk(t[0])
                lb, cb = walk(t[1])
                lv = 1 + max(la, lb)
                combines.append((i, rnd, lv, tuple(sorted(ca + cb))))
                return lv, ca + cb

            agg_level, _ = walk(tree)
            lv = 1 + max(lvlU[i], agg_level)
            absorbs.append((i, rnd, lv))
            lvlU[i] = lv
        for j in leaves:
            alive[j] = False
            kids[cur_par[j]].remove(j)
            nalive -= 1
        # ---- compressions: greedy maximal non-adjacent set of non-root unary nodes
        selected = set()
        for v in range(N):
            if alive[v] and v != root and len(kids[v]) == 1:
                if cur_par[v] in selected or kids[v][0] in selected:
                    continue
                selected.add(v)
        for j in sorted(selected):
            i = cur_par[j]
            k = kids[j][0]
            lv = 1 + max(lvlE[j], lvlU[j], lvlE[k])
            removed[j] = ("C", rnd, lv)
            lvlE[k] = lv
            cur_par[k] = i
            pos = kids[i].index(j)
            kids[i][pos] = k
            alive[j] = False
            nalive -= 1
    all_levels = [r[2] for r in removed.values()] + [c[2] for c in combines] + [a[2] for a in absorbs]
    return {"removed": removed, "combines": combines, "absorbs": absorbs, "rounds": rnd,
            "levels": max(all_levels) if all_levels else 0}


def depth_bound(N: int) -> int:
    """D_N of Lemma 4, eq. (dependency-level-bound), exactly:
    floor(log2(2N-1) + ceil(log_{3/2} N) * log2 36)."""
    import math
    from fractions import Fraction
    if N <= 1:
        return 0
    # R = ceil(log_{3/2} N): smallest R with (3/2)^R >= N
    R = 0
    while Fraction(3, 2) ** R < N:
        R += 1
    # floor(log2((2N-1) * 36^R)) exactly, via integer bit length
    val = (2 * N - 1) * 36 ** R
    return val.bit_length() - 1
