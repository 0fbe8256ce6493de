"""Pins of the oracle's adjoint (gradients through the solve) against finite
differences of the dense KKT solve.

The reference is L(theta) = g . z(theta) with z = (x, u, y) from a dense LAPACK
solve of eq. (kkt) (oracle/dense_kkt.py), which shares nothing with the
Riccati recursion the adjoint uses.  L is linear in (q, r, c), so central
differences there are exact up to rounding and are checked entry by entry;
for the matrix blocks the directional derivative along a random direction is
checked (central differences, step 1e-6, error O(h^2)).  A dropped term, a
wrong sign, a transposed outer product or a parent/child mix-up in any block
changes these directional derivatives by O(1).
"""
import zlib

import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import dense_kkt as dk
from oracle import riccati as orc
from paper_2608_01332_amd import workloads as w

FIELDS = ("Q", "q", "c", "Delta", "R", "S", "r", "A", "B")
EDGE = ("R", "S", "r", "A", "B")


def _loss(parent, d, seed):
    x, u, y = dk.solve_kkt(parent, d)
    root = int(np.nonzero(np.asarray(parent) < 0)[0][0])
    u = u.copy()
    u[root] = 0.0
    return float((seed["x"] * x).sum() + (seed["u"] * u).sum() + (seed["lam"] * y).sum())


def _cases():
    return [("chain", w.tree_chain(6), 2, 1, 1, False), ("star", w.tree_star(7), 3, 2, 0, True),
            ("balanced", w.tree_balanced(9), 2, 2, 1, True), ("random", None, 3, 1, 1, True)]


@pytest.mark.parametrize("name,parent,n,m,delta,cross", _cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_adjoint_matches_finite_differences(name, parent, n, m, delta, cross):
    rng = np.random.default_rng(zlib.crc32(("adj" + name).encode()))
    if parent is None:
        parent, _ = w.permute_labels(w.tree_chainprob(10, 0.6, rng), rng)
    spec = w.DataSpec(n, m, delta_rank=max(1, n // 2) if delta else 0, delta_scale=0.5, cross=cross)
    d = w.lqr_data(parent, spec, rng)
    N = len(parent)
    root = int(np.nonzero(parent < 0)[0][0])
    seed = {"x": rng.standard_normal((N, n)), "u": rng.standard_normal((N, m)), "lam": rng.standard_normal((N, n))}
    seed["u"][root] = 0.0
    sol = orc.tree_riccati(parent, d)
    g = oadj.adjoint(parent, d, sol, seed)
    L0 = _loss(parent, d, seed)
    scale = max(abs(L0), 1.0)
    # right-hand side: exact, entry by entry (non-root slots of r)
    for f in ("q", "r", "c"):
        for idx in np.ndindex(d[f].shape):
            if f == "r" and idx[0] == root:
                continue
            h = 1e-3
            dp = {k: v.copy() for k, v in d.items()}
            dm = {k: v.copy() for k, v in d.items()}
            dp[f][idx] += h
            dm[f][idx] -= h
            fd = (_loss(parent, dp, seed) - _loss(parent, dm, seed)) / (2 * h)
            assert abs(fd - g[f][idx]) <= 1e-9 * scale, (f, idx, fd, g[f][idx])
    # matrix blocks: directional derivatives along random directions
    for f in ("Q", "Delta", "R", "S", "A", "B"):
        for trial in range(2):
            D = rng.standard_normal(d[f].shape)
            if f in EDGE:
                D[root] = 0.0
            h = 1e-6
            dp = {k: v.copy() for k, v in d.items()}
            dm = {k: v.copy() for k, v in d.items()}
            dp[f] = dp[f] + h * D
            dm[f] = dm[f] - h * D
            fd = (_loss(parent, dp, seed) - _loss(parent, dm, seed)) / (2 * h)
            an = float((g[f] * D).sum())
            assert abs(fd - an) <= 1e-6 * max(abs(an), scale), (f, trial, fd, an)
    for f in EDGE:
        assert np.all(g[f][root] == 0.0)


def test_adjoint_of_rhs_is_the_transpose_map():
    """dL/d(q, r, c) for L = g . z is the map (q, r, c) -> z transposed.  The map
    is linear, z = -M^{-1} (q, r, c), and M is symmetric, so
    <solve(a), b> = <a, solve(b)> for any two right-hand sides a, b."""
    rng = np.random.default_rng(99)
    parent = w.tree_chainprob(40, 0.7, rng)
    d = w.lqr_data(parent, w.DataSpec(3, 2, delta_rank=1, cross=True), rng)
    N = len(parent)
    root = int(np.nonzero(parent < 0)[0][0])

    def lin(qrc):
        dd = dict(d)
        dd["q"], dd["r"], dd["c"] = qrc
        o = orc.tree_riccati(parent, dd)
        return o["x"], o["u"], o["lam"]

    def draw():
        q, r, c = rng.standard_normal((N, 3)), rng.standard_normal((N, 2)), rng.standard_normal((N, 3))
        r[root] = 0.0
        return q, r, c

    a, b = draw(), draw()
    za, zb = lin(a), lin(b)
    lhs = sum(float((za[k] * b[k]).sum()) for k in range(3))
    rhs = sum(float((a[k] * zb[k]).sum()) for k in range(3))
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))
