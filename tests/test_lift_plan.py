"""Host side of the exact lifting (Sec. II-B, Prop. 2): the lifted plan built
by the library equals the plan of the lifted tree that the oracle constructs
independently, and invalid input is rejected."""
import numpy as np
import pytest

from oracle import lifting as olift
from paper_2608_01332_amd import rcr
from paper_2608_01332_amd import workloads as w


def _native(parent, n, m, seed=0):
    return w.native_node_control_data(parent, w.DataSpec(n, m), np.random.default_rng(seed))


@pytest.mark.parametrize("make", [lambda: w.tree_chain(9), lambda: w.tree_star(7),
                                  lambda: w.tree_chainprob(300, 0.8, np.random.default_rng(4)),
                                  lambda: w.permute_labels(w.tree_chainprob(120, 0.6, np.random.default_rng(5)),
                                                           np.random.default_rng(6))[0],
                                  lambda: np.array([-1])])
def test_lift_plan_matches_plan_of_oracle_lifted_tree(make):
    par = make()
    n, m = 3, 2
    lp, _, plus = olift.lift(par, _native(par, n, m))
    a = rcr.Plan.lift(par, n, m)
    b = rcr.Plan(lp, n + m, m)
    sa, sb = a.stats(), b.stats()
    assert sa["N"] == len(lp) == len(par) + int((plus >= 0).sum())
    assert (sa["n"], sa["m"]) == (n + m, m)
    for k in ("rounds", "levels", "n_rake", "n_compress", "n_combine", "n_absorb", "height"):
        assert sa[k] == sb[k], k
    assert np.array_equal(a.export_ops(), b.export_ops())


def test_lift_workspace_holds_lifted_buffers():
    par = w.tree_chainprob(500, 0.9, np.random.default_rng(1))
    n, m = 4, 2
    a = rcr.Plan.lift(par, n, m)
    lp, _, _ = olift.lift(par, _native(par, n, m))
    b = rcr.Plan(lp, n + m, m)
    d, NL = n + m, len(lp)
    words = NL * ((3 * d * d + 2 * d + m * m + 2 * d * m + m) + (d * m + d * d + 2 * d + m))
    for prec in (rcr.FP64, rcr.MIXED32):
        extra = a.workspace_size(prec) - b.workspace_size(prec)
        assert words * 8 <= extra <= words * 8 + 14 * 256


@pytest.mark.parametrize("par,n,m,status", [
    ([-1, 0, 5], 3, 2, "INVALID_TREE"),          # index out of range
    ([-1, 2, 1], 3, 2, "INVALID_TREE"),          # cycle
    ([-1, -1, 0], 3, 2, "INVALID_TREE"),         # two roots
    ([-1, 0, 0], 14, 3, "BAD_DIMS"),             # n + m above the compiled maximum
    ([-1, 0, 0], 0, 2, "BAD_DIMS"),
])
def test_lift_plan_rejects(par, n, m, status):
    with pytest.raises(rcr.RcrError) as ei:
        rcr.Plan.lift(np.array(par), n, m)
    assert ei.value.status == getattr(rcr, "ERR_" + status)


def test_lift_plans_cannot_be_merged():
    a = rcr.Plan.lift(w.tree_chain(5), 2, 1)
    b = rcr.Plan.lift(w.tree_chain(6), 2, 1)
    with pytest.raises(rcr.RcrError):
        rcr.Plan.batch([a, b])
