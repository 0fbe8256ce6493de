"""GPU parity of the node-control solve through the exact lifting (Sec. II-B,
Prop. 2): small trees against the native dense KKT solve, the 65,536-node
instance (n = 12, m = 4, lifted to state 16) against the FP64 oracle (oracle
lifting + sequential tree Riccati + projection), element by element."""
import numpy as np
import pytest

from oracle import dense_kkt  # noqa: F401  (the oracle package is importable)
from oracle import lifting as olift
from oracle import riccati as orc
from paper_2608_01332_amd import rcr
from paper_2608_01332_amd import workloads as w

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _rel(g, r):
    return float(np.abs(g - r).max() / max(np.abs(r).max(), 1e-300))


def _oracle_lifted(par, nd, n):
    lp, ld, plus = olift.lift(par, nd)
    ref = orc.tree_riccati(lp, ld)
    return olift.project(n, plus, ref["x"], ref["u"], ref["lam"])


TINY = [
    ("single", lambda rng: np.array([-1])),
    ("pair", lambda rng: np.array([-1, 0])),
    ("chain7", lambda rng: w.tree_chain(7)),
    ("star6", lambda rng: w.tree_star(6)),
    ("random25", lambda rng: w.tree_chainprob(25, 0.5, rng)),
    ("permuted30", lambda rng: w.permute_labels(w.tree_chainprob(30, 0.7, rng), rng)[0]),
]


@pytest.mark.parametrize("name,make", TINY)
@pytest.mark.parametrize("n,m,cross,rank", [(3, 2, False, 0), (4, 3, True, 2), (12, 4, True, 6)])
def test_lift_solve_tiny_against_native_kkt(name, make, n, m, cross, rank):
    print(f"[gpu-lift] tiny {name} n={n} m={m}", flush=True)
    rng = np.random.default_rng(1000 * [t[0] for t in TINY].index(name) + 10 * n + m)
    par = make(rng)
    nd = w.native_node_control_data(par, w.DataSpec(n, m, delta_rank=rank, cross=cross), rng)
    x, v, y = olift.solve_native(par, nd)
    plan = rcr.Plan.lift(par, n, m)
    out = rcr.lift_solve(plan, rcr.to_device(nd, fields=rcr.NATIVE_FIELDS), check=True)
    for k, ref in (("x", x), ("v", v), ("lam", y)):
        assert _rel(out[k].cpu().numpy(), ref) <= 1e-9, (name, k)


def test_lift_solve_config2_fp64_against_oracle():
    print("[gpu-lift] 65,536-node node-control instance, FP64", flush=True)
    par, nd = w.config2_lift_instance()
    plan = rcr.Plan.lift(par, 12, 4)
    dev = rcr.to_device(nd, fields=rcr.NATIVE_FIELDS)
    out = rcr.lift_solve(plan, dev, check=True, kkt_residual=True)
    assert out["kkt_residual"] <= 1e-9
    x, v, y = _oracle_lifted(par, nd, 12)
    for k, ref in (("x", x), ("v", v), ("lam", y)):
        assert _rel(out[k].cpu().numpy(), ref) <= 1e-9, k
    g = rcr.lift_solve(plan, dev, executor=rcr.EXEC_GRAPH)
    g = rcr.lift_solve(plan, dev, executor=rcr.EXEC_GRAPH)
    for k in rcr.NATIVE_SOLUTION_FIELDS:
        assert torch.equal(g[k], out[k]), k


def test_lift_solve_config2_mixed32():
    print("[gpu-lift] 65,536-node node-control instance, MIXED32 + 1 refinement", flush=True)
    par, nd = w.config2_lift_instance()
    plan = rcr.Plan.lift(par, 12, 4)
    dev = rcr.to_device(nd, fields=rcr.NATIVE_FIELDS)
    out = rcr.lift_solve(plan, dev, precision=rcr.MIXED32, refine_steps=1, check=True, kkt_residual=True)
    assert out["kkt_residual"] <= 1e-8
    x, v, y = _oracle_lifted(par, nd, 12)
    for k, ref in (("x", x), ("v", v), ("lam", y)):
        assert _rel(out[k].cpu().numpy(), ref) <= 1e-7, k


def test_lift_solve_caller_workspace_and_errors():
    print("[gpu-lift] caller workspace, plain plan rejected", flush=True)
    par = w.tree_chainprob(400, 0.9, np.random.default_rng(2))
    nd = w.native_node_control_data(par, w.DataSpec(6, 2, delta_rank=3), np.random.default_rng(3))
    dev = rcr.to_device(nd, fields=rcr.NATIVE_FIELDS)
    plan = rcr.Plan.lift(par, 6, 2)
    ref = rcr.lift_solve(plan, dev)
    ws = torch.empty(plan.workspace_size(rcr.FP64), dtype=torch.uint8, device="cuda")
    out = rcr.lift_solve(plan, dev, workspace=ws)
    for k in rcr.NATIVE_SOLUTION_FIELDS:
        assert torch.equal(out[k], ref[k])
    small = torch.empty(plan.workspace_size(rcr.FP64) - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(rcr.RcrError) as ei:
        rcr.lift_solve(plan, dev, workspace=small)
    assert ei.value.status == rcr.ERR_SMALL_WORKSPACE
    plain = rcr.Plan(par, 6, 2)
    plain.native_N, plain.native_n = len(par), 6
    with pytest.raises(rcr.RcrError) as ei:
        rcr.lift_solve(plain, dev)
    assert ei.value.status == rcr.ERR_BAD_OPTION
