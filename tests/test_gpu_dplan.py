"""The device-side planner (rcr_plan_create_device): plans built on the GPU from
a device parent array are byte-identical to the host planner's with the
list-rank selection (rcr_plan_digest over every array, plus the statistics
and the exported ops), from one node to the 1,048,576-node shape-extreme
trees and the 65,536-node config-2 tree, with labels in any order (hubs
whose sibling groups the whole workgroup builds among them); invalid
trees and the greedy selection are rejected; a solve on the device-built plan
equals the solve on the host-built one bit for bit."""
import ctypes
import time

import numpy as np
import pytest

from paper_2608_01332_amd import rcr
from paper_2608_01332_amd import workloads as w

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _trees():
    rng = np.random.default_rng(w.config_seed(9, 0, 1))
    yield "single", np.array([-1], dtype=np.int64)
    yield "pair", np.array([1, -1], dtype=np.int64)
    yield "chain5000", w.tree_chain(5000)
    yield "star20000", w.tree_star(20000)
    yield "balanced", w.tree_balanced(32767)
    yield "comb", w.tree_comb(20000)
    for p in (0.5, 0.9, 0.97):
        t = w.tree_chainprob(30000, p, rng)
        yield f"chainprob{p}", t
        yield f"permuted{p}", w.permute_labels(t, rng)[0]
    # hubs: sibling groups of thousands of contributions of mixed levels, built by the whole workgroup
    yield "star_of_chains", w.tree_star_heavy(3000, rng.integers(1, 60, size=3000))
    yield "config2", w.config_instance(2)[0]
    for kind in ("caterpillar", "star_heavy", "chainprob"):
        yield f"extreme_{kind}", w.shape_extreme(kind)


@pytest.mark.parametrize("name,parent", list(_trees()), ids=lambda v: v if isinstance(v, str) else "")
def test_device_plan_equals_host_plan(name, parent):
    print(f"[gpu-dplan] {name} N={len(parent)}", flush=True)
    par_d = torch.from_numpy(parent).to("cuda:0")
    t0 = time.perf_counter()
    dev = rcr.Plan.from_device(par_d, 6, 2)
    t1 = time.perf_counter()
    host = rcr.Plan(parent, 6, 2, selection=rcr.SELECT_LIST_RANK)
    t2 = time.perf_counter()
    print(f"[gpu-dplan] {name}: device {1e3 * (t1 - t0):.2f} ms, host {1e3 * (t2 - t1):.2f} ms", flush=True)
    assert dev.digest() == host.digest()
    sd, sh = dev.stats(), host.stats()
    for k in ("N", "root", "height", "leaves", "max_degree", "rounds", "n_rake", "n_compress", "n_combine",
              "n_absorb", "levels"):
        if k in sh:
            assert sd[k] == sh[k], k
    np.testing.assert_array_equal(dev.export_ops(), host.export_ops())


@pytest.mark.parametrize("parent", [[-1, 0, -1], [1, 0], [-1, 1], [-1, 7], [-1, 0, 3, 2], [-1, -2]])
def test_device_plan_rejects_invalid_trees(parent):
    par_d = torch.tensor(parent, dtype=torch.int64, device="cuda:0")
    with pytest.raises(rcr.RcrError) as e:
        rcr.Plan.from_device(par_d, 4, 2)
    assert e.value.status == -1  # RCR_INVALID_TREE


def test_device_plan_rejects_greedy_selection():
    L = rcr.lib()
    par_d = torch.from_numpy(w.tree_chain(10)).to("cuda:0")
    h = ctypes.c_void_p()
    opt = rcr.PlanOptions(selection=rcr.SELECT_GREEDY_INDEX)
    rc = L.rcr_plan_create_device(ctypes.c_void_p(par_d.data_ptr()), 10, 4, 2, ctypes.byref(opt),
                                  ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), ctypes.byref(h))
    assert rc == -9  # RCR_BAD_OPTION


@pytest.mark.parametrize("precision", [rcr.FP64, rcr.MIXED32])
def test_solve_on_device_plan_matches_host_plan(precision):
    print(f"[gpu-dplan] solve precision={precision}", flush=True)
    parent, data, spec = w.config_instance(2)
    dev_data = rcr.to_device(data, "cuda:0")
    pd = rcr.Plan.from_device(torch.from_numpy(parent).to("cuda:0"), spec.n, spec.m)
    ph = rcr.Plan(parent, spec.n, spec.m, selection=rcr.SELECT_LIST_RANK)
    a = rcr.solve(pd, dev_data, precision=precision, kkt_residual=True)
    b = rcr.solve(ph, dev_data, precision=precision, kkt_residual=True)
    torch.cuda.synchronize()
    for k in rcr.SOLUTION_FIELDS:
        assert torch.equal(a[k], b[k]), k
    assert a["kkt_residual"] <= 1e-8


def test_device_plan_random_trees():
    """40 random trees (five families, sizes from 1 to 40,000, labels permuted or
    not), each device-built plan identical to the host planner's."""
    rng = np.random.default_rng(w.config_seed(9, 1, 0))
    for case in range(40):
        fam = case % 5
        N = int(rng.integers(1, 40000)) if case % 4 else int(rng.integers(1, 64))
        if fam == 0:
            par = w.tree_chainprob(N, float(rng.uniform(0.3, 0.999)), rng)
        elif fam == 1:
            par = w.tree_star(N)
        elif fam == 2:
            par = w.tree_balanced(N)
        elif fam == 3:
            par = w.tree_comb(max(N, 2))
        else:
            par = np.full(N, -1, dtype=np.int64)
            par[1:] = [int(rng.integers(0, i)) for i in range(1, N)]  # uniform random recursive tree
        if rng.random() < 0.5 and len(par) > 1:
            par = w.permute_labels(par, rng)[0]
        n, m = int(rng.integers(1, 17)), int(rng.integers(1, 17))
        print(f"[gpu-dplan] random case {case} family {fam} N={len(par)} n={n} m={m}", flush=True)
        dev = rcr.Plan.from_device(torch.from_numpy(np.ascontiguousarray(par, dtype=np.int64)).to("cuda:0"), n, m)
        host = rcr.Plan(par, n, m, selection=rcr.SELECT_LIST_RANK)
        assert dev.digest() == host.digest(), case
