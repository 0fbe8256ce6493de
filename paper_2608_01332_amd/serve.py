"""Continuous-batching request loop for tree-LQR solves on one GPU.

Requests -- a tree (host parent array), its dimensions (n, m) and its FP64
problem data already resident on the device -- arrive over time.  The server

  * plans each request on arrival in a pool of host threads (the planner
    releases the interpreter lock); a topology seen before reuses its cached
    plan, whose device copy stays resident;
  * admits ready requests into execution slots, one HIP stream each, when a
    slot is free and the group's HBM footprint fits the budget left after
    the device copies of the cached plans: its workspace (for a merged group
    that of rcr_batch_solve, which stages the requests' inputs and outputs),
    its outputs and the device copy of its plan;
  * merges the requests of equal (n, m) that are ready at admission time,
    oldest first, into one rcr_batch_solve over their plans (the library
    merges them into the plan of their forest, one launch sequence), so that
    requests which arrived while others were on the GPU join the next free
    slot together and their work overlaps on the device with the groups
    running in the other slots;
  * completes a group when its stream's completion event has fired.

Every request gets its own output buffers; its arithmetic is that of the same
kernels on its own nodes, so the result does not depend on the group it ran
in.  Latency runs from the request's arrival time to the host observing its
completion event (planning on a plan-cache miss included).
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import time
from dataclasses import dataclass, field

import numpy as np

from . import rcr


def io_words(N: int, n: int, m: int) -> tuple[int, int]:
    """FP64 words of one request's inputs and outputs (rcr_problem, rcr_solution)."""
    s, t, v = n * n, n * m, m * m
    return N * (2 * s + 2 * n + v + 2 * t + m + s), N * (t + s + 2 * n + m)


@dataclass
class Request:
    rid: int
    parent: np.ndarray
    n: int
    m: int
    prob: dict                 # device float64 tensors (rcr_problem layout)
    topo: object = None        # hashable topology key; None: never cached
    arrival: float = 0.0       # host clock (time.perf_counter) of arrival
    plan: object = None
    t_ready: float = 0.0
    t_admit: float = 0.0
    t_done: float = 0.0
    group_size: int = 0
    out: dict = field(default_factory=dict)
    cache_hit: bool = False

    @property
    def N(self) -> int:
        return int(self.parent.shape[0])


COPY_CHUNK = 32768  # words per copy chunk of rcr_batch_solve's gather and scatter


def batch_staging_bytes(sizes, n: int, m: int) -> int:
    """Device bytes rcr_batch_solve adds to the merged plan's solver workspace
    for trees of these sizes: the staged inputs and outputs (each field 256-byte
    aligned) and the table of copy chunks (32 bytes each)."""
    s, t, v = n * n, n * m, m * m
    words = (s, n, n, s, v, t, m, s, t, t, s, n, m, n)  # Q q c Delta R S r A B, K P x u lam
    N = sum(sizes)
    stage = sum(-(-8 * w * N // 256) * 256 for w in words)
    chunks = sum(-(-w * Nt // COPY_CHUNK) for w in words for Nt in sizes)
    return stage + -(-32 * chunks // 256) * 256


def group_footprint(reqs, precision: int, ws_bytes: int, plan_bytes: int = 0) -> int:
    """HBM bytes a group holds while it runs: its workspace (ws_bytes, staging
    included for a merged group), its outputs and the device copy of its plan
    when that is not a cached plan's (plan_bytes)."""
    n, m = reqs[0].n, reqs[0].m
    N = sum(r.N for r in reqs)
    w_in, w_out = io_words(N, n, m)
    return ws_bytes + 8 * w_out + plan_bytes


def form_group(ready, free_bytes: int, max_nodes: int, ws_of, precision: int):
    """Admission policy: the oldest ready request heads the group; later ready
    requests of the same (n, m) join in arrival order while the group stays
    within max_nodes and its footprint within free_bytes.  Returns the group
    (possibly empty when even the head does not fit) and its footprint."""
    if not ready:
        return [], 0
    head = ready[0]
    group = [head]
    fp = group_footprint(group, precision, *ws_of(group))
    if fp > free_bytes:
        return [], 0
    nodes = head.N
    for r in list(ready)[1:]:
        if (r.n, r.m) != (head.n, head.m) or nodes + r.N > max_nodes:
            continue
        cand = group + [r]
        f2 = group_footprint(cand, precision, *ws_of(cand))
        if f2 > free_bytes:
            continue
        group, fp, nodes = cand, f2, nodes + r.N
    return group, fp


class _Slot:
    def __init__(self, device):
        import torch
        self.stream = torch.cuda.Stream(device=device)
        self.prep = None    # future of the group's host preparation (merged plan, device copy)
        self.event = None   # completion event of the group's solve
        self.group = None
        self.keep = None
        self.bytes = 0


class Server:
    def __init__(self, device="cuda:0", slots: int = 4, hbm_budget: int = 64 << 30, max_group_nodes: int = 1 << 20,
                 precision: int = rcr.MIXED32, refine_steps: int = 1, planner_threads: int = 8,
                 plan_cache: int = 512, batching: bool = True):
        import torch
        self.device = torch.device(device)
        self.slots = [_Slot(self.device) for _ in range(slots)]
        self.budget = int(hbm_budget)
        self.in_use = 0
        self.max_group_nodes = max_group_nodes if batching else 1
        self.precision = precision
        self.refine_steps = refine_steps
        self.pool = cf.ThreadPoolExecutor(max_workers=planner_threads)
        self.cache = collections.OrderedDict()  # topo -> [Plan, in-flight count]
        self.cache_cap = plan_cache
        self.cached_plan_bytes = 0              # device copies held by cached plans
        self.planning = []                      # (future, request)
        self.ready = collections.deque()
        self.done = []
        self.groups = 0
        self.stats = {"plan_s": 0.0, "prep_s": 0.0, "launch_s": 0.0}

    # ---- arrival and planning -------------------------------------------------
    def _plan(self, req: Request):
        t = time.perf_counter()
        p = rcr.Plan(req.parent, req.n, req.m)
        self.stats["plan_s"] += time.perf_counter() - t
        return p

    def submit(self, req: Request):
        key = None if req.topo is None else (req.topo, req.n, req.m)
        if key is not None and key in self.cache:
            ent = self.cache[key]
            self.cache.move_to_end(key)
            req.plan, req.cache_hit = ent[0], True
            req.t_ready = time.perf_counter()
            self.ready.append(req)
            return
        self.planning.append((self.pool.submit(self._plan, req), req))

    def _collect_plans(self):
        still = []
        for fut, req in self.planning:
            if not fut.done():
                still.append((fut, req))
                continue
            req.plan = fut.result()
            req.t_ready = time.perf_counter()
            key = None if req.topo is None else (req.topo, req.n, req.m)
            if key is not None:
                if key not in self.cache:
                    self.cache[key] = [req.plan, 0]
                    self._evict()
                else:
                    req.plan = self.cache[key][0]
            self.ready.append(req)
        self.planning = still
        if len(self.ready) > 1:
            self.ready = collections.deque(sorted(self.ready, key=lambda r: r.arrival))

    def _evict(self):
        while len(self.cache) > self.cache_cap:
            for k, ent in self.cache.items():
                if ent[1] == 0:
                    if getattr(ent[0], "_uploaded", False):
                        self.cached_plan_bytes -= ent[0].device_bytes()
                    del self.cache[k]
                    break
            else:
                return

    def _is_cached(self, req) -> bool:
        key = None if req.topo is None else (req.topo, req.n, req.m)
        return key is not None and key in self.cache and self.cache[key][0] is req.plan

    def _pin(self, reqs, delta):
        for r in reqs:
            key = None if r.topo is None else (r.topo, r.n, r.m)
            if key is not None and key in self.cache:
                self.cache[key][1] += delta

    # ---- execution ------------------------------------------------------------
    def _ws_of(self, group):
        """(workspace bytes, plan device bytes not already charged) of a group.
        A merged plan's workspace and device copy are at most the sums of its
        parts' (every array is per node, per slot or per level), so the sums
        bound the footprint before the merged plan exists."""
        if len(group) == 1:
            r = group[0]
            charged = getattr(r.plan, "_uploaded", False) and self._is_cached(r)
            return r.plan.workspace_size(self.precision), 0 if charged else r.plan.device_bytes()
        ws = sum(r.plan.workspace_size(self.precision) for r in group)
        ws += batch_staging_bytes([r.N for r in group], group[0].n, group[0].m)
        return ws, sum(r.plan.device_bytes() for r in group)

    def _prepare(self, group, stream):
        """Worker thread: the group's plan (for several requests the merged plan
        of rcr_batch_solve, built and cached by the library) and its device
        copy, made in the order of the slot's idle stream."""
        t = time.perf_counter()
        if len(group) > 1:
            plans = [r.plan for r in group]
            rcr.batch_prepare(plans, stream)
            plan = plans
        else:
            plan = group[0].plan
            plan.upload(stream)
        self.stats["prep_s"] += time.perf_counter() - t
        return plan

    def _dispatch(self, slot: _Slot, group, fp: int):
        now = time.perf_counter()
        for r in group:
            r.t_admit = now
            r.group_size = len(group)
        slot.group, slot.bytes = group, fp
        self.in_use += fp
        self._pin(group, +1)
        self.groups += 1
        if len(group) == 1 and getattr(group[0].plan, "_uploaded", False):
            self._launch(slot, group[0].plan)
        else:
            slot.prep = self.pool.submit(self._prepare, group, slot.stream)

    def _launch(self, slot: _Slot, plan):
        import torch
        t = time.perf_counter()
        group = slot.group
        with torch.cuda.stream(slot.stream):
            outs = [rcr.alloc_solution(r.plan, self.device) for r in group]
            if len(group) == 1:
                ws = torch.empty(plan.workspace_size(self.precision), dtype=torch.uint8, device=self.device)
                rcr.solve(plan, group[0].prob, out=outs[0], precision=self.precision,
                          refine_steps=self.refine_steps, executor=rcr.EXEC_LEVELS, workspace=ws,
                          stream=slot.stream)
            else:
                ws = torch.empty(rcr.batch_workspace_size(plan, self.precision), dtype=torch.uint8,
                                 device=self.device)
                rcr.batch_solve(plan, [r.prob for r in group], outs, precision=self.precision,
                                refine_steps=self.refine_steps, executor=rcr.EXEC_LEVELS, workspace=ws,
                                stream=slot.stream)
            ev = torch.cuda.Event()
            ev.record(slot.stream)
        for r, o in zip(group, outs):
            r.out = o
        slot.event = ev
        slot.keep = (plan if len(group) > 1 else None, ws)
        self.stats["launch_s"] += time.perf_counter() - t

    def poll(self) -> int:
        """Advance the loop once; returns the number of requests completed."""
        finished = 0
        for slot in self.slots:
            if slot.prep is not None and slot.prep.done():
                plan = slot.prep.result()
                slot.prep = None
                if len(slot.group) == 1 and not getattr(plan, "_uploaded", False):
                    plan._uploaded = True  # its device copy stays with the plan
                    if self._is_cached(slot.group[0]):
                        self.cached_plan_bytes += plan.device_bytes()
                self._launch(slot, plan)
            if slot.event is not None and slot.event.query():
                t = time.perf_counter()
                if slot.keep[0] is not None:
                    rcr.batch_release(slot.keep[0])  # merged groups rarely repeat
                for r in slot.group:
                    r.t_done = t
                    r.plan = None  # the cache keeps reusable plans; others are released
                    self.done.append(r)
                finished += len(slot.group)
                self._pin(slot.group, -1)
                self.in_use -= slot.bytes
                slot.group, slot.event, slot.keep, slot.bytes = None, None, None, 0
        if self.planning:
            self._collect_plans()
        for slot in self.slots:
            if slot.group is not None or not self.ready:
                continue
            while True:
                group, fp = form_group(self.ready, self.budget - self.in_use - self.cached_plan_bytes,
                                       self.max_group_nodes, self._ws_of, self.precision)
                if group or not self._evict_for_room():
                    break
            if not group:
                if not any(s_.group is not None or s_.prep is not None for s_ in self.slots):
                    raise RuntimeError(f"request {self.ready[0].rid} does not fit the HBM budget of "
                                       f"{self.budget} bytes on an idle device")
                break
            ids = {id(r) for r in group}
            self.ready = collections.deque(r for r in self.ready if id(r) not in ids)
            self._dispatch(slot, group, fp)
        self._evict()
        return finished

    def _evict_for_room(self) -> bool:
        """Release the device copy of the least recently used cached plan that no
        running group uses (the head of the queue did not fit); False if none."""
        for k, ent in self.cache.items():
            if ent[1] == 0 and getattr(ent[0], "_uploaded", False):
                self.cached_plan_bytes -= ent[0].device_bytes()
                del self.cache[k]
                return True
        return False

    def busy(self) -> bool:
        return bool(self.planning or self.ready or any(s.group is not None for s in self.slots))

    def drain(self):
        while self.busy():
            self.poll()

    def close(self):
        self.drain()
        self.pool.shutdown(wait=True)
        self.cache.clear()
