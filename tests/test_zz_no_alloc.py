"""rcr_solve_noalloc (the entry point that allocates nothing) against rcr_solve.

Two calls in a row through the C-ABI, the second on a smaller problem, each
equal to rcr_solve on the same inputs bit for bit (the same kernels on a
different workspace) and to the FP64 oracle within 1e-9; a MIXED32 call; a
problem whose workspace exceeds the static array is rejected; a plan without
a device copy is rejected."""
import numpy as np
import pytest

from oracle import riccati as orc
from paper_2608_01332_amd import rcr
from paper_2608_01332_amd import workloads as w

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _problem(N, n, m, seed):
    rng = np.random.default_rng(seed)
    par = w.tree_chainprob(N, 0.9, rng)
    d = w.lqr_data(par, w.DataSpec(n, m, delta_rank=n // 2, delta_scale=0.01, cross=True), rng)
    return par, d


@pytest.mark.parametrize("prec", [rcr.FP64, rcr.MIXED32])
def test_noalloc_equals_solve_on_two_calls(prec):
    print(f"[gpu-noalloc] prec={prec}", flush=True)
    for N, n, m, seed in ((9000, 8, 3, 1), (300, 4, 2, 2)):  # second call: a smaller input
        par, d = _problem(N, n, m, seed)
        plan = rcr.Plan(par, n, m)
        assert plan.workspace_size(prec) <= rcr.noalloc_scratch_bytes()
        dev = rcr.to_device(d)
        ref = rcr.solve(plan, dev, precision=prec, check=True, kkt_residual=True)
        ref = {k: (v.clone() if torch.is_tensor(v) else v) for k, v in ref.items()}
        plan.upload()
        out = rcr.alloc_solution(plan, "cuda:0")
        got = rcr.solve_noalloc(plan, dev, out, precision=prec, check=True, kkt_residual=True)
        torch.cuda.synchronize()
        for k in rcr.SOLUTION_FIELDS:
            assert torch.equal(got[k], ref[k]), (N, k)
        assert got["kkt_residual"] == ref["kkt_residual"]
        oracle = orc.tree_riccati(par, d)
        tol = 1e-9 if prec == rcr.FP64 else 1e-4
        for k in rcr.SOLUTION_FIELDS:
            assert _rel(got[k].cpu().numpy(), oracle[k]) <= (1e-7 if prec != rcr.FP64 and k in ("x", "u", "lam")
                                                            else tol), (N, k)


def test_noalloc_rejects_what_needs_allocation():
    print("[gpu-noalloc] rejections", flush=True)
    par, d = _problem(200, 4, 2, 3)
    plan = rcr.Plan(par, 4, 2)
    dev = rcr.to_device(d)
    out = rcr.alloc_solution(plan, "cuda:0")
    with pytest.raises(rcr.RcrError) as e:  # no device copy of the plan yet
        rcr.solve_noalloc(plan, dev, out)
    assert e.value.status == rcr.ERR_BAD_OPTION
    # a workspace larger than the static array: rejected before any launch
    big_par = w.tree_chainprob(200000, 0.9, np.random.default_rng(4))
    big = rcr.Plan(big_par, 12, 4)
    assert big.workspace_size(rcr.FP64) > rcr.noalloc_scratch_bytes()
    big.upload()
    sh = rcr._shapes(big.N, 12, 4)
    zeros = {k: torch.zeros(sh[k], dtype=torch.float64, device="cuda:0") for k in rcr.PROBLEM_FIELDS}
    bout = rcr.alloc_solution(big, "cuda:0")
    with pytest.raises(rcr.RcrError) as e:
        rcr.solve_noalloc(big, zeros, bout)
    assert e.value.status == rcr.ERR_SMALL_WORKSPACE
