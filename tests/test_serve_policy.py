"""Host logic of the serving loop: HBM-footprint admission and grouping
(no GPU: requests carry a stand-in plan that only reports its workspace)."""
import numpy as np

from paper_2608_01332_amd import rcr
from paper_2608_01332_amd import serve
from paper_2608_01332_amd import workloads as w


class _FakePlan:
    def __init__(self, ws):
        self.ws = ws

    def workspace_size(self, precision):
        return self.ws


def _req(rid, N, n, m, ws=1000):
    return serve.Request(rid=rid, parent=np.arange(-1, N - 1), n=n, m=m, prob={}, arrival=float(rid),
                         plan=_FakePlan(ws))


def _ws_of(g):
    return sum(r.plan.workspace_size(rcr.MIXED32) for r in g), 0


def test_io_words_counts_problem_and_solution():
    n, m, N = 3, 2, 5
    w_in, w_out = serve.io_words(N, n, m)
    # Q, Delta, A (n^2 each), q, c (n each), R (m^2), S, B (n m each), r (m)
    assert w_in == N * (3 * n * n + 2 * n + m * m + 2 * n * m + m)
    # K (m n), P (n^2), x, lam (n each), u (m)
    assert w_out == N * (m * n + n * n + 2 * n + m)


def test_group_oldest_head_same_dims_only():
    ready = [_req(0, 100, 4, 2), _req(1, 100, 8, 2), _req(2, 100, 4, 2), _req(3, 100, 4, 4), _req(4, 50, 4, 2)]
    g, fp = serve.form_group(ready, 1 << 40, 10 ** 9, _ws_of, rcr.MIXED32)
    assert [r.rid for r in g] == [0, 2, 4]
    assert fp == serve.group_footprint(g, rcr.MIXED32, *_ws_of(g))


def test_group_node_cap_and_footprint():
    ready = [_req(0, 100, 4, 2), _req(1, 100, 4, 2), _req(2, 30, 4, 2)]
    g, fp = serve.form_group(ready, 1 << 40, 130, _ws_of, rcr.MIXED32)
    assert [r.rid for r in g] == [0, 2]
    g1, fp1 = serve.form_group(ready, 1 << 40, 100, _ws_of, rcr.MIXED32)
    assert [r.rid for r in g1] == [0]
    assert fp1 == 1000 + serve.output_layout(g1)[1]
    assert fp == 2000 + serve.output_layout(g)[1]
    assert serve.group_footprint(g, rcr.MIXED32, 2000, 77) == fp + 77


def test_output_layout_packs_aligned_fields():
    """Every output field of every request gets its own 256-byte aligned range
    of the group's block, large enough for its shape; the block is the next
    power of two at or above the packed total."""
    g = [_req(0, 100, 4, 2), _req(1, 37, 4, 2), _req(2, 1, 4, 2)]
    offs, total = serve.output_layout(g)
    spans = []
    for r, o in zip(g, offs):
        sh = rcr.solution_shapes(r.N, r.n, r.m)
        for k in rcr.SOLUTION_FIELDS:
            assert o[k] % serve.OUT_FIELD_ALIGN == 0
            spans.append((o[k], o[k] + 8 * int(np.prod(sh[k]))))
    spans.sort()
    assert all(a[1] <= b[0] for a, b in zip(spans, spans[1:]))
    packed = sum(-(-(b - a) // 256) * 256 for a, b in spans)
    assert total >= spans[-1][1] and total & (total - 1) == 0 and total < 2 * packed
    # the outputs of one request are what io_words counts
    w_in, w_out = serve.io_words(100, 4, 2)
    sh = rcr.solution_shapes(100, 4, 2)
    assert sum(int(np.prod(sh[k])) for k in rcr.SOLUTION_FIELDS) == w_out


def test_group_respects_budget_and_blocks_when_head_does_not_fit():
    ready = [_req(0, 100, 4, 2), _req(1, 100, 4, 2)]
    single = serve.group_footprint(ready[:1], rcr.MIXED32, 1000)
    g, fp = serve.form_group(ready, single, 10 ** 9, _ws_of, rcr.MIXED32)
    assert [r.rid for r in g] == [0] and fp == single
    g, fp = serve.form_group(ready, single - 1, 10 ** 9, _ws_of, rcr.MIXED32)
    assert g == [] and fp == 0
    assert serve.form_group([], 1 << 40, 10, _ws_of, rcr.MIXED32) == ([], 0)


def test_serve_stream_statistics():
    reqs = w.serve_requests(4000, 1000.0, seed=11)
    N = np.array([e["N"] for e in reqs])
    assert N.min() >= 1024 and N.max() <= 131072
    # log-uniform on [1k, 128k]: the median is near the geometric mean (~11.6k)
    assert 8000 < np.median(N) < 16000
    resend = np.mean([e["topo"] != e["rid"] for e in reqs])
    assert 0.26 < resend < 0.34
    gaps = np.diff([e["arrival"] for e in reqs])
    assert abs(gaps.mean() - 1e-3) < 1e-4 and np.all(gaps >= 0)
    for e in reqs:
        if e["topo"] != e["rid"]:
            src = reqs[e["topo"]]
            assert (e["N"], e["n"], e["m"], e["tree_seed"]) == (src["N"], src["n"], src["m"], src["tree_seed"])
            assert src["resend_of"] == -1
            assert e["variant"] != reqs[e["resend_of"]]["variant"]
            assert reqs[e["resend_of"]]["topo"] == e["topo"]
    par = w.serve_tree(reqs[0])
    assert par[0] == -1 and np.all(par[1:] < np.arange(1, len(par)))


def test_batch_workspace_bound():
    """The serving admission bounds a merged group's workspace by the sum of its
    parts' plus the staging of rcr_batch_solve; the library's exact figure is the
    merged plan's workspace plus that same staging (host only, no GPU)."""
    rng = np.random.default_rng(4)
    for n, m in ((4, 2), (8, 3), (12, 4)):
        pars = [w.tree_chainprob(int(rng.integers(300, 5000)), 0.9, rng) for _ in range(7)]
        plans = [rcr.Plan(p, n, m) for p in pars]
        merged = rcr.Plan.batch(plans)
        for prec in (rcr.FP64, rcr.MIXED32):
            stage = serve.batch_staging_bytes([len(p) for p in pars], n, m)
            exact = rcr.batch_workspace_size(plans, prec)
            assert exact == merged.workspace_size(prec) + stage
            assert exact <= sum(p.workspace_size(prec) for p in plans) + stage
        assert merged.stats()["plan_device_bytes"] <= sum(p.stats()["plan_device_bytes"] for p in plans)
        rcr.batch_release(plans)
