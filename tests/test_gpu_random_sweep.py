"""GPU parity on a fixed-seed random sweep: n and m anywhere in 1..16, tree
families (chain-probability, star, caterpillar, balanced, hub-heavy), permuted
labels, both unary selections, both executors and both precisions, each
against the FP64 oracle at the bars of the other parity tests (FP64: every
result within 1e-9 relative and KKT residual <= 1e-8; MIXED32 + 1 refinement:
KKT <= 1e-8, x, u, lam within 1e-7 and K, P within 1e-4)."""
import math

import numpy as np
import pytest

from oracle import riccati as orc
from paper_2608_01332_amd import rcr
from paper_2608_01332_amd import workloads as w

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CASES = 80


def _case(k):
    rng = np.random.default_rng(4400 + k)
    n, m = int(rng.integers(1, 17)), int(rng.integers(1, 17))
    N = int(round(math.exp(rng.uniform(0, math.log(6000)))))
    kind = ["chainprob", "star", "caterpillar", "balanced", "hub"][k % 5]
    if kind == "chainprob":
        par = w.tree_chainprob(N, float(rng.uniform(0.2, 0.99)), rng)
    elif kind == "star":
        par = w.tree_star(N)
    elif kind == "caterpillar":
        par = w.tree_caterpillar(max(1, N // 4), 3)
    elif kind == "balanced":
        par = w.tree_balanced(N)
    else:
        chains = min(N, 200)
        par = w.tree_star_heavy(chains, np.full(chains, max(1, N // 200)))
    if rng.random() < 0.5 and len(par) > 2:
        par = w.permute_labels(par, rng)[0]
    sel = rcr.SELECT_LIST_RANK if rng.random() < 0.3 else rcr.SELECT_GREEDY_INDEX
    prec = rcr.MIXED32 if rng.random() < 0.3 else rcr.FP64
    ex = rcr.EXEC_GRAPH if rng.random() < 0.5 else rcr.EXEC_LEVELS
    spec = w.DataSpec(n, m, delta_rank=int(rng.integers(0, n + 1)), delta_scale=0.01, cross=bool(rng.random() < 0.5))
    return kind, par, n, m, sel, prec, ex, spec, w.lqr_data(par, spec, rng)


@pytest.mark.parametrize("k", range(CASES))
def test_random_case_against_oracle(k):
    kind, par, n, m, sel, prec, ex, spec, d = _case(k)
    print(f"[gpu-sweep] case {k}: {kind} N={len(par)} n={n} m={m} sel={sel} prec={prec} ex={ex} "
          f"rank={spec.delta_rank} cross={spec.cross}", flush=True)
    plan = rcr.Plan(par, n, m, selection=sel)
    out = rcr.solve(plan, rcr.to_device(d), precision=prec, refine_steps=1 if prec == rcr.MIXED32 else 0,
                    executor=ex, check=True, kkt_residual=True)
    torch.cuda.synchronize()
    ref = orc.tree_riccati(par, d)
    errs = {f: float(np.abs(out[f].cpu().numpy() - ref[f]).max() / max(np.abs(ref[f]).max(), 1e-300))
            for f in rcr.SOLUTION_FIELDS}
    assert out["kkt_residual"] <= 1e-8, (out["kkt_residual"], errs)
    if prec == rcr.FP64:
        assert max(errs.values()) <= 1e-9, errs
    else:
        assert max(errs[f] for f in ("x", "u", "lam")) <= 1e-7, errs
        assert max(errs["K"], errs["P"]) <= 1e-4, errs
