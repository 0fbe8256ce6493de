"""GPU factor/solve split (rcr_factor + rcr_solve_rhs) and the adjoint solve.

Algorithm 1 factors once (Steps 2-3) and solves each right-hand side with the
vector passes of Steps 4-6.  Each right-hand side solved on one factor is
checked against the FP64 oracle run on that right-hand side (<= 1e-9 relative
per result array in FP64; KKT residual <= 1e-8 and x, u, lam <= 1e-7 in MIXED32
after refinement), the split launches no factor-class kernel in the solve, and
its results equal rcr_solve's bit for bit (the same arithmetic in the same
order).  The adjoint (rcr_adjoint) is checked against the oracle's adjoint,
which is pinned by finite differences of the dense KKT solve."""
import sys
import zlib

import numpy as np
import pytest

from oracle import adjoint as oadj
from oracle import riccati as orc
from paper_2608_01332_amd import rcr
from paper_2608_01332_amd import workloads as w

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

FACTOR_CLASSES = ("condense", "quad_contract", "quad_expand", "local_factor", "tcompose", "quad_tail")


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _instance(name, N, n, m, cross=False):
    rng = np.random.default_rng(zlib.crc32(name.encode()))
    par = w.tree_chainprob(N, 0.9, rng)
    d = w.lqr_data(par, w.DataSpec(n, m, delta_rank=n // 2, delta_scale=0.01, cross=cross), rng)
    return par, d, rng


def _rhs(rng, N, n, m, k):
    return [{"q": rng.standard_normal((N, n)), "r": rng.standard_normal((N, m)),
             "c": rng.standard_normal((N, n)) * 0.1} for _ in range(k)]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("N,n,m,cross", [(255, 4, 2, False), (3000, 8, 3, True), (4000, 12, 4, False),
                                         (1500, 16, 4, True), (700, 5, 3, False)])
def test_factor_then_rhs_fp64(N, n, m, cross):
    print(f"[gpu-factor] N={N} n={n} m={m}", flush=True)
    par, d, rng = _instance(f"fac{N}-{n}-{m}", N, n, m, cross)
    plan = rcr.Plan(par, n, m)
    dev = rcr.to_device(d)
    fac = rcr.factor(plan, dev, check=True)
    rhs = _rhs(rng, N, n, m, 4)
    res = rcr.solve_rhs(plan, dev, fac, [{k: _dev(v) for k, v in r_.items()} for r_ in rhs], check=True,
                        kkt_residual=True, kernel_ms=True)
    torch.cuda.synchronize()
    for c in FACTOR_CLASSES:
        assert res["kernel_launches"][c] == 0, (c, res["kernel_launches"])
    assert res["kkt_residual"] <= 1e-8
    for i, r_ in enumerate(rhs):
        di = dict(d)
        di.update(r_)
        ref = orc.tree_riccati(par, di)
        if i == 0:
            for k in ("K", "P"):
                assert _rel(fac[k].cpu().numpy(), ref[k]) <= 1e-9, k
        s = res["solutions"][i]
        for k in ("x", "u", "lam"):
            assert _rel(s[k].cpu().numpy(), ref[k]) <= 1e-9, (i, k)


@pytest.mark.parametrize("n,m,ex", [(4, 2, rcr.EXEC_LEVELS), (12, 4, rcr.EXEC_GRAPH), (8, 3, rcr.EXEC_GRAPH)])
def test_split_equals_solve_bitwise(n, m, ex):
    """rcr_factor + rcr_solve_rhs on the problem's own right-hand side returns
    what rcr_solve returns, bit for bit, with either executor."""
    print(f"[gpu-split] n={n} m={m} ex={ex}", flush=True)
    par, d, rng = _instance(f"split{n}", 5000, n, m, cross=True)
    plan = rcr.Plan(par, n, m)
    dev = rcr.to_device(d)
    one = rcr.solve(plan, dev, executor=ex, check=True)
    one = {k: v.clone() for k, v in one.items()}
    for rep in range(2):  # the second pass replays captured graphs
        fac = rcr.factor(plan, dev, executor=ex, check=True)
        res = rcr.solve_rhs(plan, dev, fac, [{k: dev[k] for k in ("q", "r", "c")}], executor=ex, check=True)
        torch.cuda.synchronize()
        for k in ("K", "P"):
            assert torch.equal(fac[k], one[k]), (rep, k)
        for k in ("x", "u", "lam"):
            assert torch.equal(res["solutions"][0][k], one[k]), (rep, k)


@pytest.mark.parametrize("n,m,prec", [(12, 4, rcr.FP64), (8, 3, rcr.FP64), (12, 4, rcr.MIXED32)])
def test_solve_leaves_no_factor_for_rhs(n, m, prec):
    """rcr_solve_rhs on the plan-owned workspace needs a factor from rcr_factor:
    after an rcr_solve in the same precision it is refused (RCR_BAD_OPTION; a
    float64 solve does not store A^cl), and a new rcr_factor makes it work again,
    equal bit for bit to the first factor's solve."""
    print(f"[gpu-split] refused after solve n={n} m={m} prec={prec}", flush=True)
    par, d, rng = _instance(f"refuse{n}", 3000, n, m, cross=False)
    plan = rcr.Plan(par, n, m)
    dev = rcr.to_device(d)
    rhs = [{k: _dev(v) for k, v in r_.items()} for r_ in _rhs(rng, 3000, n, m, 1)]
    fac = rcr.factor(plan, dev, precision=prec, check=True)
    first = rcr.solve_rhs(plan, dev, fac, rhs, precision=prec, check=True)["solutions"][0]
    first = {k: v.clone() for k, v in first.items()}
    rcr.solve(plan, dev, precision=prec, check=True)
    with pytest.raises(rcr.RcrError) as ei:
        rcr.solve_rhs(plan, dev, fac, rhs, precision=prec, check=True)
    assert ei.value.status == rcr.ERR_BAD_OPTION
    fac = rcr.factor(plan, dev, precision=prec, check=True)
    again = rcr.solve_rhs(plan, dev, fac, rhs, precision=prec, check=True)["solutions"][0]
    torch.cuda.synchronize()
    for k in ("x", "u", "lam"):
        assert torch.equal(again[k], first[k]), k


def test_factor_then_rhs_mixed32():
    print("[gpu-factor-mixed]", flush=True)
    par, d, rng = _instance("facmix", 20000, 8, 3, cross=True)
    N, n, m = len(par), 8, 3
    plan = rcr.Plan(par, n, m)
    dev = rcr.to_device(d)
    fac = rcr.factor(plan, dev, precision=rcr.MIXED32, check=True)
    rhs = _rhs(rng, N, n, m, 3)
    res = rcr.solve_rhs(plan, dev, fac, [{k: _dev(v) for k, v in r_.items()} for r_ in rhs],
                        precision=rcr.MIXED32, refine_steps=1, check=True, kkt_residual=True)
    torch.cuda.synchronize()
    assert res["kkt_residual"] <= 1e-8, res["kkt_residual"]
    for i, r_ in enumerate(rhs):
        di = dict(d)
        di.update(r_)
        ref = orc.tree_riccati(par, di)
        s = res["solutions"][i]
        prob_i = dict(dev)
        prob_i.update({k: _dev(v) for k, v in r_.items()})
        assert rcr.kkt_residual(plan, prob_i, s) <= 1e-8
        for k in ("x", "u", "lam"):
            assert _rel(s[k].cpu().numpy(), ref[k]) <= 1e-7, (i, k)
    ref0 = orc.tree_riccati(par, d)
    for k in ("K", "P"):
        assert _rel(fac[k].cpu().numpy(), ref0[k]) <= 1e-4, k


def test_factor_own_workspace_and_two_factors():
    """A factor lives in the workspace it was made in: two factors of two
    problems on one plan, in two caller workspaces, each serve their own
    right-hand sides."""
    print("[gpu-factor-ws]", flush=True)
    par, d1, rng = _instance("facws", 2000, 6, 2)
    d2 = w.lqr_data(par, w.DataSpec(6, 2, delta_rank=3, delta_scale=0.01), rng)
    plan = rcr.Plan(par, 6, 2)
    nb = plan.workspace_size(rcr.FP64)
    ws = [torch.empty(nb // 8 + 1, dtype=torch.float64, device="cuda:0") for _ in range(2)]
    devs = [rcr.to_device(d1), rcr.to_device(d2)]
    facs = [rcr.factor(plan, devs[i], workspace=ws[i], check=True) for i in range(2)]
    for i, d in enumerate((d1, d2)):
        res = rcr.solve_rhs(plan, devs[i], facs[i], [{k: devs[i][k] for k in ("q", "r", "c")}], workspace=ws[i],
                            check=True)
        torch.cuda.synchronize()
        ref = orc.tree_riccati(par, d)
        for k in ("x", "u", "lam"):
            assert _rel(res["solutions"][0][k].cpu().numpy(), ref[k]) <= 1e-9, (i, k)


@pytest.mark.parametrize("N,n,m,cross,prec", [(255, 4, 2, True, rcr.FP64), (4000, 12, 4, True, rcr.FP64),
                                              (3000, 8, 3, False, rcr.FP64), (600, 3, 2, True, rcr.FP64),
                                              (3000, 8, 3, True, rcr.MIXED32)])
def test_adjoint_matches_oracle(N, n, m, cross, prec):
    print(f"[gpu-adjoint] N={N} n={n} m={m} prec={prec}", flush=True)
    par, d, rng = _instance(f"adj{N}-{n}", N, n, m, cross)
    plan = rcr.Plan(par, n, m)
    dev = rcr.to_device(d)
    fwd = rcr.solve(plan, dev, check=True)
    fwd = {k: v.clone() for k, v in fwd.items()}
    seed = {"x": rng.standard_normal((N, n)), "u": rng.standard_normal((N, m)), "lam": rng.standard_normal((N, n))}
    fac = rcr.factor(plan, dev, precision=prec, check=True)
    fwd["K"], fwd["P"] = fac["K"], fac["P"]
    g = rcr.adjoint(plan, dev, fwd, {k: _dev(v) for k, v in seed.items()}, precision=prec, check=True)
    torch.cuda.synchronize()
    sol = {k: fwd[k].cpu().numpy() for k in ("x", "u", "lam")}
    ref = oadj.adjoint(par, d, sol, seed)
    tol = 1e-9 if prec == rcr.FP64 else 1e-7
    for k in rcr.GRADIENT_FIELDS:
        assert _rel(g[k].cpu().numpy(), ref[k]) <= tol, (k, _rel(g[k].cpu().numpy(), ref[k]))


def test_kkt_residual_entry_and_nan():
    """rcr_kkt_residual equals the residual rcr_solve reports for the same iterate,
    and a NaN in a single control entry gives +Inf (the max-abs fold keeps NaN)."""
    print("[gpu-residual]", flush=True)
    par, d, rng = _instance("resid", 3000, 8, 3, cross=True)
    plan = rcr.Plan(par, 8, 3)
    dev = rcr.to_device(d)
    out = rcr.solve(plan, dev, check=True, kkt_residual=True)
    r0 = rcr.kkt_residual(plan, dev, out)
    assert r0 == out["kkt_residual"]
    bad = {k: v.clone() for k, v in out.items() if k in ("x", "u", "lam")}
    child = int(np.nonzero(par >= 0)[0][5])
    bad["u"][child, 1] = float("nan")
    assert rcr.kkt_residual(plan, dev, bad) == float("inf")
    bad = {k: v.clone() for k, v in out.items() if k in ("x", "u", "lam")}
    bad["lam"][0, 0] = float("nan")
    assert rcr.kkt_residual(plan, dev, bad) == float("inf")


def test_graph_cache_stays_bounded():
    """Graph replays on fresh buffer sets: the plan keeps at most
    RCR_GRAPH_CACHE_CAP captured sequences, and every replay is correct."""
    print("[gpu-graph-cache]", flush=True)
    par, d, rng = _instance("gcache", 1000, 4, 2)
    plan = rcr.Plan(par, 4, 2)
    ref = orc.tree_riccati(par, d)
    keep = []  # live buffers: every solve sees a fresh set of addresses
    for i in range(3 * rcr.GRAPH_CACHE_CAP + 2):
        dev = rcr.to_device(d)
        out = rcr.solve(plan, dev, executor=rcr.EXEC_GRAPH, check=True)
        keep.append((dev, out))
        torch.cuda.synchronize()
        assert _rel(out["x"].cpu().numpy(), ref["x"]) <= 1e-9
        assert plan.stats()["graph_cache_entries"] <= rcr.GRAPH_CACHE_CAP
    assert plan.stats()["graph_cache_entries"] == rcr.GRAPH_CACHE_CAP


def test_factor_rhs_and_adjoint_config2_full_size():
    """The 65,536-node config-2 instance (n = 12, m = 4, rank-6 Delta): one factor,
    four right-hand sides, each against the oracle at 1e-9; then the adjoint of
    a random seed on the same factor against the oracle's adjoint at 1e-9."""
    print("[gpu-factor] config 2 full size", flush=True)
    par, d, spec = w.config_instance(2)
    N, n, m = len(par), spec.n, spec.m
    rng = np.random.default_rng(w.config_seed(2, 7, 0))
    plan = rcr.Plan(par, n, m)
    dev = rcr.to_device(d)
    fac = rcr.factor(plan, dev, check=True)
    rhs = _rhs(rng, N, n, m, 4)
    res = rcr.solve_rhs(plan, dev, fac, [{k: _dev(v) for k, v in r_.items()} for r_ in rhs], check=True,
                        kkt_residual=True)
    torch.cuda.synchronize()
    assert res["kkt_residual"] <= 1e-8
    for i, r_ in enumerate(rhs):
        di = dict(d)
        di.update(r_)
        ref = orc.tree_riccati(par, di)
        for k in ("x", "u", "lam"):
            assert _rel(res["solutions"][i][k].cpu().numpy(), ref[k]) <= 1e-9, (i, k)
    fwd = rcr.solve(plan, dev, check=True)
    fwd = {k: v.clone() for k, v in fwd.items()}
    fac = rcr.factor(plan, dev, check=True)
    fwd["K"], fwd["P"] = fac["K"], fac["P"]
    seed = {"x": rng.standard_normal((N, n)), "u": rng.standard_normal((N, m)), "lam": rng.standard_normal((N, n))}
    g = rcr.adjoint(plan, dev, fwd, {k: _dev(v) for k, v in seed.items()}, check=True)
    torch.cuda.synchronize()
    ref = oadj.adjoint(par, d, {k: fwd[k].cpu().numpy() for k in ("x", "u", "lam")}, seed)
    for k in rcr.GRADIENT_FIELDS:
        assert _rel(g[k].cpu().numpy(), ref[k]) <= 1e-9, (k, _rel(g[k].cpu().numpy(), ref[k]))
