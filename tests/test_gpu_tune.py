"""Launch-mapping autotuner (rcr_plan_tune) and explicit mappings: the narrow
levels may run in per-level launches or in the single-workgroup tail kernels,
and the results must be bitwise the same for every mapping (each primitive
runs the same arithmetic wherever it is launched).  In the wide layout with
control size up to 4, the first level runs fused with the condensation when
it is launched on its own and after a separate condensation when the tail
covers it: the wide tails mapping below puts level 1 of these trees in the
tail, so the two paths are compared bit for bit."""
import numpy as np
import pytest

from paper_2608_01332_amd import rcr
from paper_2608_01332_amd import workloads as w

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

MAPPINGS = [
    {"quad_tail_rounds": -1, "vec_tail_rounds": -1, "vec_tail_waves": 0},   # no tails
    {"quad_tail_rounds": 1, "vec_tail_rounds": 2, "vec_tail_waves": 8},
    {"quad_tail_rounds": 64, "vec_tail_rounds": 64, "vec_tail_waves": 16},  # wide tails
]


@pytest.mark.parametrize("n,m,N,prec", [(4, 2, 255, rcr.FP64), (12, 4, 3000, rcr.FP64), (8, 3, 4000, rcr.MIXED32),
                                        (6, 2, 2000, rcr.MIXED32), (16, 4, 1500, rcr.FP64),
                                        (12, 4, 3000, rcr.MIXED32), (12, 2, 2500, rcr.FP64), (12, 8, 2000, rcr.FP64)])
def test_mappings_bitwise_equal(n, m, N, prec):
    print(f"[gpu-tune] mappings n={n} m={m} N={N} prec={prec}", flush=True)
    par = w.tree_chainprob(N, 0.9, np.random.default_rng(N))
    d = w.lqr_data(par, w.DataSpec(n, m, delta_rank=n // 2), np.random.default_rng(N + 1))
    prob = rcr.to_device(d)
    plan = rcr.Plan(par, n, m)
    ref = rcr.solve(plan, prob, precision=prec, refine_steps=1, check=True)
    ref = {k: v.clone() for k, v in ref.items()}
    for cfg in MAPPINGS:
        plan.set_launch(cfg)
        for ex in (rcr.EXEC_LEVELS, rcr.EXEC_GRAPH):
            out = rcr.solve(plan, prob, precision=prec, refine_steps=1, executor=ex, check=True)
            for k in rcr.SOLUTION_FIELDS:
                assert torch.equal(out[k], ref[k]), (cfg, ex, k)


def test_tune_keeps_fastest_and_results():
    print("[gpu-tune] tune a batched plan", flush=True)
    plans, datas = [], []
    for t in range(6):
        par = w.tree_chainprob(500 + 700 * t, 0.9, np.random.default_rng(t))
        plans.append(rcr.Plan(par, 8, 3))
        datas.append(w.lqr_data(par, w.DataSpec(8, 3), np.random.default_rng(100 + t)))
    bp = rcr.Plan.batch(plans)
    prob = rcr.to_device(rcr.concat_problems(datas))
    ref = rcr.solve(bp, prob, precision=rcr.MIXED32, refine_steps=1)
    ref = {k: v.clone() for k, v in ref.items()}
    cfg, ms = bp.tune(prob, precision=rcr.MIXED32, refine_steps=1)
    assert ms > 0
    assert cfg["quad_tail_rounds"] in (-1, 1, 2, 4, 8)
    assert cfg["vec_tail_rounds"] == -1 or (cfg["vec_tail_rounds"] in (2, 4, 8) and cfg["vec_tail_waves"] in (8, 16))
    assert bp.get_launch() == cfg
    out = rcr.solve(bp, prob, precision=rcr.MIXED32, refine_steps=1, executor=rcr.EXEC_GRAPH, kkt_residual=True)
    assert out["kkt_residual"] <= 1e-8
    for k in rcr.SOLUTION_FIELDS:
        assert torch.equal(out[k], ref[k]), k
