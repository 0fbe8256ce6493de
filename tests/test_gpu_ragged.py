"""GPU solves with per-node state and per-edge control dimensions
(rcr_ragged_plan_create + rcr_ragged_solve) against the ragged FP64 oracle.

Every block of K, P, x, u, lam (packed arrays) within 1e-9 of the oracle
relative to the largest entry of its field; with equal dimensions the ragged
path equals rcr_solve on the same data bit for bit; a one-node tree (empty
edge arrays) works; MIXED32 reaches the KKT residual bar after refinement."""
import numpy as np
import pytest

from oracle import ragged as org
from paper_2608_01332_amd import rcr
from paper_2608_01332_amd import workloads as w

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(flat):
    return {k: torch.from_numpy(np.ascontiguousarray(v, dtype=np.float64)).to("cuda:0") for k, v in flat.items()}


def _shapes(par, nn, mm):
    N = len(par)
    npar = [int(nn[par[v]]) if par[v] >= 0 else 0 for v in range(N)]
    return {"K": [(int(mm[v]), npar[v]) for v in range(N)], "P": [(int(nn[v]), int(nn[v])) for v in range(N)],
            "x": [(int(nn[v]),) for v in range(N)], "u": [(int(mm[v]),) for v in range(N)],
            "lam": [(int(nn[v]),) for v in range(N)]}


def _check(out, ref, par, nn, mm, tol):
    sh = _shapes(par, nn, mm)
    for k in rcr.SOLUTION_FIELDS:
        got = w.unpack_ragged(out[k].cpu().numpy(), sh[k])
        scale = max(max((np.abs(b).max(initial=0) for b in ref[k]), default=0.0), 1e-300)
        err = max((np.abs(g - r).max(initial=0) for g, r in zip(got, ref[k])), default=0.0)
        assert err / scale <= tol, (k, err / scale)


@pytest.mark.parametrize("N,nmax,mmax,nmin", [(300, 4, 2, 1), (2000, 8, 3, 2), (1500, 12, 4, 5), (800, 16, 4, 9),
                                              (1, 6, 3, 6), (2, 3, 2, 1), (600, 5, 5, 1), (32768, 12, 4, 6)])
def test_ragged_matches_oracle(N, nmax, mmax, nmin):
    print(f"[gpu-ragged] N={N} n<={nmax} m<={mmax}", flush=True)
    rng = np.random.default_rng(N * 7 + nmax)
    par, nn, mm, d = w.ragged_instance(N, nmax, mmax, rng, nmin=nmin)
    plan = rcr.Plan.ragged(par, nn, mm)
    assert (plan.n, plan.m) == (int(nn.max()), max(int(mm.max()), 1))
    out = rcr.ragged_solve(plan, _dev(w.pack_ragged(d)), check=True, kkt_residual=True)
    torch.cuda.synchronize()
    assert out["kkt_residual"] <= 1e-8
    _check(out, org.tree_riccati_ragged(par, nn, mm, d), par, nn, mm, 1e-9)


def test_ragged_mixed32():
    print("[gpu-ragged] mixed32", flush=True)
    rng = np.random.default_rng(11)
    par, nn, mm, d = w.ragged_instance(3000, 8, 3, rng, nmin=3)
    plan = rcr.Plan.ragged(par, nn, mm)
    out = rcr.ragged_solve(plan, _dev(w.pack_ragged(d)), precision=rcr.MIXED32, refine_steps=1, check=True,
                           kkt_residual=True)
    torch.cuda.synchronize()
    assert out["kkt_residual"] <= 1e-8
    ref = org.tree_riccati_ragged(par, nn, mm, d)
    sh = _shapes(par, nn, mm)
    for k in ("x", "u", "lam"):
        got = w.unpack_ragged(out[k].cpu().numpy(), sh[k])
        scale = max(np.abs(b).max(initial=0) for b in ref[k])
        assert max(np.abs(g - r).max(initial=0) for g, r in zip(got, ref[k])) / scale <= 1e-7, k


def test_ragged_equal_dims_equals_uniform_solve():
    print("[gpu-ragged] equal dimensions", flush=True)
    rng = np.random.default_rng(5)
    par = w.tree_chainprob(3000, 0.9, rng)
    d = w.lqr_data(par, w.DataSpec(8, 3, delta_rank=4, cross=True), rng)
    root = int(np.nonzero(par < 0)[0][0])
    nn = np.full(len(par), 8, dtype=np.int32)
    mm = np.full(len(par), 3, dtype=np.int32)
    plan_u = rcr.Plan(par, 8, 3)
    ref = rcr.solve(plan_u, rcr.to_device(d), check=True)
    rg = rcr.Plan.ragged(par, nn, mm)
    flat = {}
    for k in rcr.PROBLEM_FIELDS:  # packed: the root's edge blocks are dropped
        a = d[k]
        if k in ("R", "S", "r", "A", "B"):
            a = np.delete(a, root, axis=0)
        flat[k] = a.reshape(-1)
    out = rcr.ragged_solve(rg, _dev(flat), check=True)
    torch.cuda.synchronize()
    keep = torch.ones(len(par), dtype=torch.bool)
    keep[root] = False
    assert torch.equal(out["P"], ref["P"].reshape(-1))
    assert torch.equal(out["x"], ref["x"].reshape(-1)) and torch.equal(out["lam"], ref["lam"].reshape(-1))
    assert torch.equal(out["K"], ref["K"][keep.cuda()].reshape(-1))
    assert torch.equal(out["u"], ref["u"][keep.cuda()].reshape(-1))
