"""The C++ planner behind the C-ABI (host only, no GPU): bit-exact agreement
with the topology oracle for the paper's greedy index-order selection, and
structural validity (Lemma 2 maximality, Lemma 4 depth, CREW) for the
list-ranking selection, where several plans are correct."""
import os
import re

import numpy as np
import pytest

from oracle import plan as pl
from paper_2608_01332_amd import rcr
from paper_2608_01332_amd import workloads as w

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
RAKE, COMBINE, ABSORB, COMPRESS = 0, 1, 2, 3


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "rcr.h")).read()
    decl = set(re.findall(r"\b(rcr_[a-z_]+)\s*\(", hdr))
    assert decl == set(rcr.EXPORTED)
    L = rcr.lib()
    for name in decl:
        assert hasattr(L, name), name


def _canon_cpp(ops):
    removed, combines, absorbs = {}, set(), set()
    cover = {}
    for kind, rnd, lvl, a, b, c, d, e in ops.tolist():
        if kind == RAKE:
            removed[a] = ("R", rnd, lvl)
            cover[c] = (a,)
    for kind, rnd, lvl, a, b, c, d, e in ops.tolist():  # ops are level-sorted: inputs precede outputs
        if kind == COMBINE:
            cover[c] = tuple(sorted(cover[a] + cover[b]))
            combines.add((d, rnd, lvl, cover[c]))
        elif kind == ABSORB:
            absorbs.add((a, rnd, lvl))
        elif kind == COMPRESS:
            removed[a] = ("C", rnd, lvl)
    return removed, combines, absorbs


def _trees():
    rng = np.random.default_rng(77)
    out = [("chain7", np.array([-1, 0, 1, 2, 3, 4, 5])), ("comb_fig2", np.array([-1, 0, 1, 1, 2, 4, 4, 5])),
           ("chain300", w.tree_chain(300)), ("star200", w.tree_star(200)), ("balanced255", w.tree_balanced(255)),
           ("comb101", w.tree_comb(101)), ("caterpillar", w.tree_caterpillar(40, 3)),
           ("tight", w.lemma2_tight_tree(32)), ("single", np.array([-1])), ("pair", np.array([1, -1]))]
    for t in range(10):
        par = w.tree_chainprob(int(rng.integers(2, 2000)), float(rng.uniform(0.3, 0.99)), rng)
        if t % 2:
            par = w.permute_labels(par, rng)[0]
        out.append((f"random{t}", par))
    return out


@pytest.mark.parametrize("name,parent", _trees(), ids=[t[0] for t in _trees()])
def test_greedy_plan_matches_oracle_exactly(name, parent):
    P = rcr.Plan(parent, 3, 2, selection=rcr.SELECT_GREEDY_INDEX)
    st = P.stats()
    ref = pl.make_plan(parent)
    removed, combines, absorbs = _canon_cpp(P.export_ops())
    assert removed == ref["removed"]
    assert combines == set(ref["combines"])
    assert absorbs == set(ref["absorbs"])
    assert st["rounds"] == ref["rounds"]
    assert st["levels"] == ref["levels"]
    assert st["crew_ok"] == 1
    assert st["n_rake"] + st["n_compress"] == len(parent) - 1
    assert st["depth_bound"] == pl.depth_bound(len(parent))


def _replay_valid(parent, ops):
    """Replay the rounds and check: rakes = all non-root leaves at the round start;
    compressions = a maximal set of pairwise non-adjacent non-root unary nodes of the
    post-rake tree; every non-root node removed once."""
    N = len(parent)
    cur_par = list(map(int, parent))
    alive = [True] * N
    root = cur_par.index(-1)
    by_round = {}
    for kind, rnd, lvl, a, b, c, d, e in ops.tolist():
        if kind in (RAKE, COMPRESS):
            by_round.setdefault(rnd, {RAKE: [], COMPRESS: []})[kind].append((a, e))
    for rnd in sorted(by_round):
        kids = [[] for _ in range(N)]
        for v in range(N):
            if alive[v] and v != root:
                kids[cur_par[v]].append(v)
        leaves = {v for v in range(N) if alive[v] and v != root and not kids[v]}
        assert {a for a, _ in by_round[rnd][RAKE]} == leaves
        for v in leaves:
            alive[v] = False
        kids = [[] for _ in range(N)]
        for v in range(N):
            if alive[v] and v != root:
                kids[cur_par[v]].append(v)
        unary = {v for v in range(N) if alive[v] and v != root and len(kids[v]) == 1}
        sel = {a for a, _ in by_round[rnd][COMPRESS]}
        assert sel <= unary
        for j in sel:
            assert cur_par[j] not in sel and kids[j][0] not in sel
        for v in unary - sel:  # maximal
            assert cur_par[v] in sel or kids[v][0] in sel
        for j, k in by_round[rnd][COMPRESS]:
            assert kids[j] == [k]
            cur_par[k] = cur_par[j]
            alive[j] = False
    assert sum(alive) == 1 and alive[root]


@pytest.mark.parametrize("name,parent", _trees(), ids=[t[0] for t in _trees()])
@pytest.mark.parametrize("selection", [rcr.SELECT_GREEDY_INDEX, rcr.SELECT_LIST_RANK])
def test_plan_structurally_valid(name, parent, selection):
    P = rcr.Plan(parent, 2, 1, selection=selection)
    st = P.stats()
    ops = P.export_ops()
    _replay_valid(parent, ops)
    N = len(parent)
    assert st["crew_ok"] == 1
    assert st["levels"] <= st["depth_bound"]
    R = 0
    while 1.5 ** R < N:
        R += 1
    assert st["rounds"] <= R
    assert st["expand_levels"] <= st["depth_bound"] and st["sexp_levels"] <= st["depth_bound"]
    # levels are sorted and every level is nonempty
    lv = ops[:, 2]
    assert np.all(np.diff(lv) >= 0)
    if N > 1:
        assert set(lv.tolist()) == set(range(1, st["levels"] + 1))


def test_list_rank_compresses_half_of_each_unary_path():
    """On a chain with permuted labels the list-ranking selection still takes alternate
    positions along the path (ceil(L/2) of L eligible nodes), independent of the labels."""
    rng = np.random.default_rng(5)
    par, _ = w.permute_labels(w.tree_chain(1001), rng)
    ops = rcr.Plan(par, 2, 1, selection=rcr.SELECT_LIST_RANK).export_ops()
    first = ops[(ops[:, 0] == COMPRESS) & (ops[:, 1] == 1)]
    assert len(first) == 499  # after the rake, depths 1..998 are eligible: alternate positions take 499
    greedy = rcr.Plan(par, 2, 1).export_ops()
    g1 = greedy[(greedy[:, 0] == COMPRESS) & (greedy[:, 1] == 1)]
    assert len(g1) <= len(first)


@pytest.mark.parametrize("parent", [[0, 0], [-1, -1], [-1, 2, 1], [-1, 5], [-2, 0], [1, 0, -1]])
def test_invalid_trees(parent):
    with pytest.raises(rcr.RcrError) as ei:
        rcr.Plan(np.array(parent), 2, 1)
    assert ei.value.status == -1


@pytest.mark.parametrize("n,m", [(0, 1), (1, 0), (17, 2), (2, 17)])
def test_bad_dims(n, m):
    with pytest.raises(rcr.RcrError) as ei:
        rcr.Plan(np.array([-1, 0]), n, m)
    assert ei.value.status == -2


def test_workspace_size_scales_linearly():
    a = rcr.Plan(w.tree_chainprob(1000, 0.9, np.random.default_rng(0)), 8, 3)
    b = rcr.Plan(w.tree_chainprob(4000, 0.9, np.random.default_rng(0)), 8, 3)
    ra = a.workspace_size(rcr.FP64) / 1000
    rb = b.workspace_size(rcr.FP64) / 4000
    assert 0.7 < ra / rb < 1.4
    assert a.workspace_size(rcr.MIXED32) < a.workspace_size(rcr.FP64) * 1.2


@pytest.mark.parametrize("max_nodes", [300, 8000])  # 8000: the merged forest is filled on four threads
def test_batched_plan_is_union_of_remapped_trees(max_nodes):
    """rcr_batch_plan_create: level t of the forest plan is the union of every tree's
    level t with node/edge/contribution slots offset per tree."""
    rng = np.random.default_rng(31)
    pars = [w.tree_chainprob(int(rng.integers(1, max_nodes)), float(rng.uniform(0.5, 0.98)), rng) for _ in range(7)]
    plans = [rcr.Plan(p, 4, 2) for p in pars]
    B = rcr.Plan.batch(plans)
    st = B.stats()
    sts = [p.stats() for p in plans]
    assert st["n_trees"] == 7 and st["N"] == sum(len(p) for p in pars)
    assert st["levels"] == max(s["levels"] for s in sts)
    for k in ("n_rake", "n_compress", "n_combine", "n_absorb"):
        assert st[k] == sum(s[k] for s in sts)
    N = st["N"]
    vb = B.offsets
    extra = np.cumsum([0] + [s["n_compress"] for s in sts])
    cb = np.cumsum([0] + [s["n_rake"] + s["n_combine"] for s in sts])
    want = set()
    for t, p in enumerate(plans):
        Nt = len(pars[t])
        node = lambda v: int(vb[t] + v)
        slot = lambda s_: int(vb[t] + s_) if s_ < Nt else int(N + extra[t] + s_ - Nt)
        con = lambda c: int(cb[t] + c)
        for kind, rnd, lvl, a, b, c, d, e in p.export_ops().tolist():
            if kind == RAKE:
                want.add((kind, lvl, node(a), slot(b), con(c), node(d), 0))
            elif kind == COMBINE:
                want.add((kind, lvl, con(a), con(b), con(c), node(d), 0))
            elif kind == ABSORB:
                want.add((kind, lvl, node(a), con(b), 0, 0, 0))
            else:
                want.add((kind, lvl, node(a), slot(b), slot(c), slot(d), node(e)))
    got = set()
    for kind, rnd, lvl, a, b, c, d, e in B.export_ops().tolist():
        if kind == ABSORB:
            got.add((kind, lvl, a, b, 0, 0, 0))
        elif kind in (RAKE, COMBINE):
            got.add((kind, lvl, a, b, c, d, 0))
        else:
            got.add((kind, lvl, a, b, c, d, e))
    assert got == want


def test_launch_config_set_get_and_validation():
    plan = rcr.Plan(w.tree_chainprob(200, 0.9, np.random.default_rng(0)), 4, 2)
    zero = {k: 0 for k in rcr.LAUNCH_FIELDS}
    assert plan.get_launch() == zero
    cfg = {"quad_tail_rounds": 4, "vec_tail_rounds": -1, "vec_tail_waves": 8}
    plan.set_launch(cfg)
    assert plan.get_launch() == cfg
    plan.set_launch({"vec_tail_rounds": -1})  # unspecified fields reset to their defaults
    assert plan.get_launch() == dict(zero, vec_tail_rounds=-1)
    with pytest.raises(rcr.RcrError) as ei:
        plan.set_launch({"vec_tail_waves": 17})
    assert ei.value.status == rcr.ERR_BAD_OPTION
    plan.set_launch(None)
    assert plan.get_launch() == zero


def _plan_image(parent, n=6, m=2, selection=rcr.SELECT_GREEDY_INDEX, lift=False):
    p = rcr.Plan.lift(parent, n, m, selection) if lift else rcr.Plan(parent, n, m, selection)
    try:
        return p.stats(), p.export_ops()
    finally:
        p.close()


def test_plans_do_not_depend_on_earlier_plans_of_the_thread():
    """Each planner thread keeps its working arrays between plans; a plan built
    after others (smaller, larger, above the kept size, invalid, lifted) equals
    the same plan built first on a fresh thread."""
    from concurrent.futures import ThreadPoolExecutor
    rng = np.random.default_rng(2024)
    trees = [w.tree_chainprob(5000, 0.9, rng), w.tree_chainprob(100, 0.5, rng), w.tree_chainprob(20000, 0.97, rng),
             np.array([-1, 0, 0, 1, 1, 1, 2], dtype=np.int64), w.tree_chainprob(140000, 0.9, rng),
             w.tree_chainprob(3000, 0.8, rng)]

    def fresh(job):
        with ThreadPoolExecutor(1) as ex:
            return ex.submit(_plan_image, *job).result()

    jobs = [(t, 6, 2, sel, lift) for t in trees for sel in (rcr.SELECT_GREEDY_INDEX, rcr.SELECT_LIST_RANK)
            for lift in (False, True) if not (lift and len(t) > 50000)]
    alone = [fresh(j) for j in jobs]
    bad = np.array([1, 2, 0, -1], dtype=np.int64)  # a cycle: rejected part-way through validation

    def sequence():
        out = []
        for j in jobs:
            with pytest.raises(rcr.RcrError):
                rcr.Plan(bad, 6, 2)
            out.append(_plan_image(*j))
        return out

    with ThreadPoolExecutor(1) as ex:
        seq = ex.submit(sequence).result()
    for (s0, o0), (s1, o1) in zip(alone, seq):
        assert s0 == s1
        np.testing.assert_array_equal(o0, o1)


def test_single_thread_build_equals_default():
    """rcr_plan_options.single_thread builds on the calling thread only; the plan
    (statistics and every schedule) is the one the default four-thread build of
    a tree above the threading threshold gives."""
    rng = np.random.default_rng(77)
    for N, p in ((20000, 0.95), (70000, 0.8)):
        par = w.tree_chainprob(N, p, rng)
        for sel in (rcr.SELECT_GREEDY_INDEX, rcr.SELECT_LIST_RANK):
            a = rcr.Plan(par, 8, 3, selection=sel)
            b = rcr.Plan(par, 8, 3, selection=sel, single_thread=True)
            assert a.stats() == b.stats()
            np.testing.assert_array_equal(a.export_ops(), b.export_ops())
            assert a.device_bytes() == b.device_bytes()


def test_plan_digest_identifies_plans():
    """rcr_plan_digest is equal for plans built alike and differs when any
    schedule differs (another selection, another dimension, another tree)."""
    rng = np.random.default_rng(5)
    par = w.tree_chainprob(3000, 0.9, rng)
    a = rcr.Plan(par, 6, 2, selection=rcr.SELECT_LIST_RANK)
    b = rcr.Plan(par.copy(), 6, 2, selection=rcr.SELECT_LIST_RANK, single_thread=True)
    assert a.digest() == b.digest()
    assert rcr.Plan(par, 6, 2).digest() != a.digest()
    assert rcr.Plan(par, 6, 3, selection=rcr.SELECT_LIST_RANK).digest() != a.digest()
    par2 = par.copy()
    par2[-1] = 0
    assert rcr.Plan(par2, 6, 2, selection=rcr.SELECT_LIST_RANK).digest() != a.digest()
