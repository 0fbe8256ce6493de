"""GPU tests of the serving loop: each request's result is the same alone and
in the mix (bitwise: a request's arithmetic is that of the same kernels on its
own nodes whichever group it runs in), admission under a tight HBM budget
completes every request, and one plan serves concurrent solves on different
streams with distinct workspaces."""
import numpy as np
import pytest

from oracle import riccati as orc
from paper_2608_01332_amd import rcr
from paper_2608_01332_amd import serve
from paper_2608_01332_amd import workloads as w

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _requests(count, seed, n_choices=(4, 8), m_choices=(2,), N_range=(300, 6000)):
    specs = w.serve_requests(count, 1000.0, seed, n_choices=n_choices, m_choices=m_choices, N_range=N_range)
    pool = {}
    for e in specs:
        key = (e["n"], e["m"], e["variant"])
        pool[key] = max(pool.get(key, 0), e["N"])
    dev = {}
    host = {}
    for (n, m, v), Nmax in pool.items():
        d = w.serve_data_block(Nmax, n, m, v, seed=seed)
        host[(n, m, v)] = d
        dev[(n, m, v)] = rcr.to_device(d)
    reqs = []
    for e in specs:
        key = (e["n"], e["m"], e["variant"])
        reqs.append(serve.Request(rid=e["rid"], parent=w.serve_tree(e), n=e["n"], m=e["m"],
                                  prob={k: t[:e["N"]] for k, t in dev[key].items()}, topo=e["topo"]))
        reqs[-1].host = {k: a[:e["N"]] for k, a in host[key].items()}
    return reqs


def _alone(r):
    plan = rcr.Plan(r.parent, r.n, r.m)
    return rcr.solve(plan, r.prob, precision=rcr.MIXED32, refine_steps=1, kkt_residual=True)


def test_serve_results_identical_alone_and_in_mix():
    print("[gpu-serve] mix of 24 requests, 3 slots", flush=True)
    reqs = _requests(24, seed=3)
    srv = serve.Server("cuda:0", slots=3, hbm_budget=8 << 30, planner_threads=4)
    for r in reqs[:10]:
        srv.submit(r)
    for _ in range(3):
        srv.poll()
    for r in reqs[10:]:
        srv.submit(r)
    srv.drain()
    assert len(srv.done) == len(reqs) and srv.in_use == 0
    assert max(r.group_size for r in reqs) > 1, "no request was merged into a group"
    for r in reqs:
        a = _alone(r)
        assert a["kkt_residual"] <= 1e-8, (r.rid, a["kkt_residual"])
        for k in rcr.SOLUTION_FIELDS:
            assert torch.equal(a[k], r.out[k]), (r.rid, r.group_size, k)
    srv.close()


def test_serve_full_request_distribution():
    """Requests drawn from the full serving distribution (N log-uniform in [1k, 128k],
    n in {4, 8, 12, 16}, m in {2, 4}; this seed has three n = 16, m = 4 requests of
    more than 100k nodes): each served result equals the request solved alone, bit
    for bit, and merged groups occur."""
    print("[gpu-serve] 20 requests of the full distribution, 4 slots", flush=True)
    reqs = _requests(20, seed=8, n_choices=(4, 8, 12, 16), m_choices=(2, 4), N_range=(1024, 131072))
    assert max(r.N for r in reqs if (r.n, r.m) == (16, 4)) > 100000
    srv = serve.Server("cuda:0", slots=4, planner_threads=4)
    for r in reqs:  # all at once: the slots fill and the rest queue, so groups form
        srv.submit(r)
    srv.drain()
    assert len(srv.done) == len(reqs) and srv.in_use == 0
    assert max(r.group_size for r in reqs) > 1, "no request was merged into a group"
    for r in reqs:
        a = _alone(r)
        assert a["kkt_residual"] <= 1e-8, (r.rid, a["kkt_residual"])
        for k in rcr.SOLUTION_FIELDS:
            assert torch.equal(a[k], r.out[k]), (r.rid, r.group_size, k)
    srv.close()


def test_serve_mixed32_against_oracle():
    print("[gpu-serve] oracle parity of served results", flush=True)
    reqs = _requests(6, seed=5, n_choices=(4, 12), m_choices=(2, 4))
    srv = serve.Server("cuda:0", slots=2, planner_threads=2)
    for r in reqs:
        srv.submit(r)
    srv.drain()
    for r in reqs:
        ref = orc.tree_riccati(r.parent, r.host)
        for k in ("x", "u", "lam"):
            g = r.out[k].cpu().numpy()
            rel = np.abs(g - ref[k]).max() / np.abs(ref[k]).max()
            assert rel <= 1e-7, (r.rid, k, rel)
    srv.close()


def test_serve_tight_budget_stays_within_budget():
    print("[gpu-serve] tight HBM budget", flush=True)
    reqs = _requests(8, seed=7, n_choices=(8,))
    plans = [rcr.Plan(r.parent, r.n, r.m) for r in reqs]
    need = max(serve.group_footprint([r], rcr.MIXED32, p.workspace_size(rcr.MIXED32), p.stats()["plan_device_bytes"])
               for r, p in zip(reqs, plans))
    srv = serve.Server("cuda:0", slots=4, hbm_budget=need, planner_threads=2)
    for r in reqs:
        srv.submit(r)
    peak = 0
    while srv.busy():
        srv.poll()
        peak = max(peak, srv.held())
        assert srv.held() <= need
    assert peak <= need and len(srv.done) == len(reqs)
    # the largest request needs the whole budget: it ran alone
    big = max(reqs, key=lambda r: r.N)
    assert big.group_size == 1
    for r in reqs:
        a = _alone(r)
        for k in rcr.SOLUTION_FIELDS:
            assert torch.equal(a[k], r.out[k])
    srv.close()


def test_plan_shared_across_streams():
    print("[gpu-serve] one plan, two streams, two workspaces", flush=True)
    par = w.tree_chainprob(4000, 0.9, np.random.default_rng(1))
    plan = rcr.Plan(par, 8, 2)
    d0 = w.lqr_data(par, w.DataSpec(8, 2, delta_rank=4), np.random.default_rng(2))
    d1 = w.lqr_data(par, w.DataSpec(8, 2, delta_rank=4), np.random.default_rng(3))
    p0, p1 = rcr.to_device(d0), rcr.to_device(d1)
    ref0 = rcr.solve(plan, p0)
    ref1 = rcr.solve(plan, p1)
    torch.cuda.synchronize()
    s0, s1 = torch.cuda.Stream(), torch.cuda.Stream()
    nb = plan.workspace_size(rcr.FP64)
    outs = []
    for rep in range(3):
        ws0 = torch.empty(nb, dtype=torch.uint8, device="cuda")
        ws1 = torch.empty(nb, dtype=torch.uint8, device="cuda")
        torch.cuda.synchronize()
        o0 = rcr.solve(plan, p0, workspace=ws0, stream=s0)
        o1 = rcr.solve(plan, p1, workspace=ws1, stream=s1)
        torch.cuda.synchronize()
        outs.append((o0, o1))
    for o0, o1 in outs:
        for k in rcr.SOLUTION_FIELDS:
            assert torch.equal(o0[k], ref0[k]) and torch.equal(o1[k], ref1[k])
    plan.close()
    torch.cuda.synchronize()


def test_serve_with_device_planner():
    """Plan cache misses built on the GPU (rcr_plan_create_device): every served
    result equals the same request solved alone on the host's list-rank plan of
    its tree, bit for bit."""
    print("[gpu-serve] device planner", flush=True)
    reqs = _requests(60, seed=12, n_choices=(4, 8, 12), N_range=(300, 20000))
    srv = serve.Server("cuda:0", slots=4, planner_threads=4, device_planner=True)
    for r in reqs:
        srv.submit(r)
    srv.drain()
    assert len(srv.done) == len(reqs)
    for r in reqs:
        plan = rcr.Plan(r.parent, r.n, r.m, selection=rcr.SELECT_LIST_RANK)
        a = rcr.solve(plan, r.prob, precision=rcr.MIXED32, refine_steps=1, kkt_residual=True)
        for k in rcr.SOLUTION_FIELDS:
            assert torch.equal(a[k], r.out[k]), (r.rid, k)
        assert a["kkt_residual"] <= 1e-8
    srv.close()
