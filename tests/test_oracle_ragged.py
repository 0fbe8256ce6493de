"""Pins of the ragged-dimension oracle (per-node state, per-edge control
dimensions).

The sequential recursion with rectangular blocks is checked against the
dense solve of eq. (kkt) assembled with the same block sizes (unique solution,
Prop. 1) on random small trees with random dimensions, Delta >= 0 and a cross
term; the dense ragged assembly itself is pinned against the uniform dense
KKT solve (oracle/dense_kkt.py, pinned in test_oracle.py) when all dimensions
are equal, and the ragged recursion against the uniform C oracle likewise."""
import numpy as np
import pytest

from oracle import dense_kkt as dk
from oracle import ragged as org
from oracle import riccati as orc
from paper_2608_01332_amd import workloads as w


def _uniform_blocks(d, parent):
    N = len(parent)
    root = int(np.nonzero(parent < 0)[0][0])
    out = {k: [np.array(d[k][v]) for v in range(N)] for k in d}
    # the root's edge blocks are empty
    out["S"][root] = np.zeros((0, 0))
    out["A"][root] = np.zeros((d["A"].shape[1], 0))
    out["B"][root] = np.zeros((d["B"].shape[1], 0))
    out["R"][root] = np.zeros((0, 0))
    out["r"][root] = np.zeros(0)
    return out


@pytest.mark.parametrize("seed", range(12))
def test_ragged_recursion_matches_dense_kkt(seed):
    rng = np.random.default_rng(500 + seed)
    N = int(rng.integers(1, 25))
    par, nn, mm, d = w.ragged_instance(N, 4, 3, rng, p=float(rng.uniform(0.3, 0.9)), delta=seed % 2 == 0,
                                       cross=seed % 3 != 0)
    x, u, y = org.solve_kkt_ragged(par, nn, mm, d)
    o = org.tree_riccati_ragged(par, nn, mm, d)
    for v in range(N):
        assert np.abs(o["x"][v] - x[v]).max(initial=0) < 1e-12
        assert np.abs(o["lam"][v] - y[v]).max(initial=0) < 1e-12
        if par[v] >= 0:
            assert np.abs(o["u"][v] - u[v]).max(initial=0) < 1e-12
            assert o["K"][v].shape == (mm[v], nn[par[v]])
        assert o["P"][v].shape == (nn[v], nn[v])
        assert np.allclose(o["P"][v], o["P"][v].T, atol=1e-12)


@pytest.mark.parametrize("n,m", [(1, 1), (3, 2), (4, 3)])
def test_ragged_with_equal_dims_is_the_uniform_problem(n, m):
    rng = np.random.default_rng(70 + n)
    par = w.tree_chainprob(14, 0.6, rng)
    d = w.lqr_data(par, w.DataSpec(n, m, delta_rank=max(1, n // 2), delta_scale=0.3, cross=True), rng)
    nn = np.full(len(par), n, dtype=np.int32)
    mm = np.full(len(par), m, dtype=np.int32)
    mm[par < 0] = 0
    b = _uniform_blocks(d, par)
    x, u, y = org.solve_kkt_ragged(par, nn, mm, b)
    xu, uu, yu = dk.solve_kkt(par, d)
    ref = orc.tree_riccati(par, d)
    o = org.tree_riccati_ragged(par, nn, mm, b)
    for v in range(len(par)):
        assert np.abs(x[v] - xu[v]).max() < 1e-12 and np.abs(y[v] - yu[v]).max() < 1e-12
        assert np.abs(o["P"][v] - ref["P"][v]).max() < 1e-12
        if par[v] >= 0:
            assert np.abs(u[v] - uu[v]).max() < 1e-12
            assert np.abs(o["K"][v] - ref["K"][v]).max() < 1e-12


def test_pack_and_unpack_are_inverse():
    rng = np.random.default_rng(3)
    par, nn, mm, d = w.ragged_instance(30, 5, 3, rng)
    flat = w.pack_ragged(d)
    for k, blocks in d.items():
        back = w.unpack_ragged(flat[k], [b.shape for b in blocks])
        for a, b in zip(back, blocks):
            assert a.shape == b.shape and np.array_equal(a, b)
