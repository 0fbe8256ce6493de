"""GPU batched solves: many independent trees through one merged plan
(rcr_batch_plan_create) give, per tree, exactly the result of solving that
tree alone (no data is shared between trees, so every primitive sees the same
inputs and runs the same arithmetic: bitwise equality), and match the FP64
oracle."""
import numpy as np
import pytest

from oracle import riccati as orc
from paper_2608_01332_amd import rcr
from paper_2608_01332_amd import workloads as w

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _trees(count, n, m, seed):
    rng = np.random.default_rng(seed)
    pars, datas = [], []
    for t in range(count):
        N = int(round(np.exp(rng.uniform(np.log(2), np.log(3000)))))
        par = w.tree_chainprob(N, float(rng.uniform(0.8, 0.98)), rng)
        if t % 3 == 1:
            par, _ = w.permute_labels(par, rng)
        pars.append(par)
        datas.append(w.lqr_data(par, w.DataSpec(n, m, delta_rank=n // 2, delta_scale=0.01, cross=t % 2 == 0), rng))
    return pars, datas


@pytest.mark.parametrize("n,m,prec", [(4, 2, rcr.FP64), (8, 3, rcr.FP64), (12, 4, rcr.FP64), (8, 3, rcr.MIXED32)])
def test_batched_equals_alone_and_oracle(n, m, prec):
    print(f"[gpu-batch] n={n} m={m} prec={prec}", flush=True)
    pars, datas = _trees(24, n, m, 1000 + n)
    plans = [rcr.Plan(p, n, m) for p in pars]
    B = rcr.Plan.batch(plans)
    big = rcr.to_device(rcr.concat_problems(datas))
    ob = rcr.solve(B, big, precision=prec, executor=rcr.EXEC_GRAPH, check=True, kkt_residual=True)
    torch.cuda.synchronize()
    assert ob["kkt_residual"] <= 1e-8
    for t, (p, d) in enumerate(zip(plans, datas)):
        oa = rcr.solve(p, rcr.to_device(d), precision=prec, check=True)
        torch.cuda.synchronize()
        lo, hi = int(B.offsets[t]), int(B.offsets[t + 1])
        ref = orc.tree_riccati(pars[t], d)
        for k in rcr.SOLUTION_FIELDS:
            a = oa[k].cpu().numpy()
            b = ob[k][lo:hi].cpu().numpy()
            np.testing.assert_array_equal(a, b, err_msg=f"tree {t} {k}")
            tol = 1e-9 if prec == rcr.FP64 or k in ("x", "u", "lam") else 1e-4
            rel = np.abs(b - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-300)
            assert rel <= tol, (t, k, rel)


@pytest.mark.parametrize("n,m,prec,ex", [(4, 2, rcr.FP64, rcr.EXEC_LEVELS), (12, 4, rcr.FP64, rcr.EXEC_GRAPH),
                                         (8, 3, rcr.MIXED32, rcr.EXEC_GRAPH)])
def test_batch_solve_own_buffers(n, m, prec, ex):
    """rcr_batch_solve with each tree's own problem and solution buffers equals
    solving each tree alone, bit for bit; a second call with other buffers
    (replaying the captured sequence) too."""
    print(f"[gpu-batch-solve] n={n} m={m} prec={prec} ex={ex}", flush=True)
    pars, datas = _trees(20, n, m, 2000 + n)
    plans = [rcr.Plan(p, n, m) for p in pars]
    rcr.batch_prepare(plans)
    alone = []
    for p, d in zip(plans, datas):
        oa = rcr.solve(p, rcr.to_device(d), precision=prec, check=True)
        alone.append({k: v.clone() for k, v in oa.items()})
    for rep in range(2):
        probs = [rcr.to_device(d) for d in datas]
        res = rcr.batch_solve(plans, probs, precision=prec, executor=ex, check=True, kkt_residual=True)
        torch.cuda.synchronize()
        assert res["kkt_residual"] <= 1e-8
        for t in range(len(plans)):
            for k in rcr.SOLUTION_FIELDS:
                assert torch.equal(res["solutions"][t][k], alone[t][k]), (rep, t, k)
    assert rcr.batch_workspace_size(plans, prec) > plans[0].workspace_size(prec)


def test_config3_full_size():
    """The 512-tree batched workload (N log-uniform in [256, 16384], p ~ U(0.8, 0.98),
    n = 8, m = 3, MIXED32 + one refinement step) in one rcr_batch_solve, every tree
    against the FP64 oracle run on all host cores: x, u, lam <= 1e-7 and K, P <= 1e-4
    relative, KKT residual <= 1e-8."""
    import os
    print("[gpu-config3] generating 512 trees", flush=True)
    pars, datas = [], []
    for t in range(512):
        p_, d_, spec = w.config_instance(3, tree=t)
        pars.append(p_)
        datas.append(d_)
    n, m = spec.n, spec.m
    plans = [rcr.Plan(p_, n, m) for p_ in pars]
    probs = [rcr.to_device(d_) for d_ in datas]
    print(f"[gpu-config3] solving {sum(len(p_) for p_ in pars)} nodes", flush=True)
    res = rcr.batch_solve(plans, probs, precision=rcr.MIXED32, refine_steps=1, executor=rcr.EXEC_GRAPH, check=True,
                          kkt_residual=True)
    torch.cuda.synchronize()
    assert res["kkt_residual"] <= 1e-8, res["kkt_residual"]
    del probs
    nth = min(16, os.cpu_count() or 1)
    print(f"[gpu-config3] oracle on {nth} threads", flush=True)
    worst = {k: 0.0 for k in rcr.SOLUTION_FIELDS}
    for lo in range(0, 512, 64):
        refs = orc.tree_riccati_batch(list(zip(pars[lo:lo + 64], datas[lo:lo + 64])), nth)
        for t, ref in enumerate(refs, start=lo):
            g = res["solutions"][t]
            for k in rcr.SOLUTION_FIELDS:
                a = g[k].cpu().numpy()
                worst[k] = max(worst[k], float(np.abs(a - ref[k]).max() / max(np.abs(ref[k]).max(), 1e-300)))
    print(f"[gpu-config3] worst relative error {worst}", flush=True)
    for k in ("x", "u", "lam"):
        assert worst[k] <= 1e-7, worst
    for k in ("K", "P"):
        assert worst[k] <= 1e-4, worst
