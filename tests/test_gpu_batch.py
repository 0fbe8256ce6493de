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
