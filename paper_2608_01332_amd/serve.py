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

Every request gets its own output fields (views of one device block per
group, see output_layout); its arithmetic is that of the same
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


OUT_FIELD_ALIGN = 256  # bytes; every output field of a group's block starts on this boundary


def output_layout(reqs):
    """Byte offsets of the output fields (rcr_solution order) of each request in
    the one device block that holds a group's outputs, and the block's size: the
    fields packed on 256-byte boundaries, the total rounded up to a power of two
    so that the blocks of a serving loop come in few distinct sizes and the ones
    freed are reused rather than new device memory being mapped."""
    offs, at = [], 0
    for r in reqs:
        t, s = r.m * r.n, r.n * r.n
        o = {}
        for k, w in zip(rcr.SOLUTION_FIELDS, (t, s, r.n, r.m, r.n)):
            o[k] = at
            at += -(-8 * w * r.N // OUT_FIELD_ALIGN) * OUT_FIELD_ALIGN
        offs.append(o)
    return offs, 1 << max(at - 1, 0).bit_length()


def group_footprint(reqs, precision: int, ws_bytes: int, plan_bytes: int = 0) -> int:
    """HBM bytes a group holds while it runs: its workspace (ws_bytes, staging
    included for a merged group), its output block and the device copy of its
    plan when that is not a cached plan's (plan_bytes)."""
    return ws_bytes + output_layout(reqs)[1] + plan_bytes


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
        self.ws = None      # the slot's workspace, grown when a group needs more (never shrunk)
        self.ws_target = 0  # its size as charged by admission


class Server:
    def __init__(self, device="cuda:0", slots: int = 4, hbm_budget: int = 64 << 30, max_group_nodes: int = 1 << 18,
                 precision: int = rcr.MIXED32, refine_steps: int = 1, planner_threads: int = 8,
                 plan_cache: int = 512, batching: bool = True, device_planner: bool = False):
        import threading
        import torch
        self.device = torch.device(device)
        # plan cache misses on the GPU (rcr_plan_create_device, list-rank selection),
        # one planning stream per planner thread, instead of on the host
        self.device_planner = device_planner
        self._plan_local = threading.local()
        self.slots = [_Slot(self.device) for _ in range(slots)]
        self.budget = int(hbm_budget)
        self.in_use = 0          # outputs and plan copies of the running groups
        self.ws_held = 0         # the slots' workspaces (kept between groups)
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
        self.stats = {"plan_s": 0.0, "prep_s": 0.0, "launch_s": 0.0, "launch_max_s": 0.0, "ws_grow": 0}

    # ---- arrival and planning -------------------------------------------------
    def _plan(self, req: Request):
        t = time.perf_counter()
        if self.device_planner:
            import torch
            loc = self._plan_local
            if not hasattr(loc, "stream"):
                loc.stream = torch.cuda.Stream(device=self.device)
            with torch.cuda.stream(loc.stream):
                par = torch.from_numpy(np.ascontiguousarray(req.parent, dtype=np.int64)).to(self.device)
                p = rcr.Plan.from_device(par, req.n, req.m, stream=loc.stream)
            self.stats["plan_s"] += time.perf_counter() - t
            return p
        # the pool already builds plans side by side: no helper threads per plan
        p = rcr.Plan(req.parent, req.n, req.m, single_thread=True)
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

    def _dispatch(self, slot: _Slot, group, fp: int, ws_charge: int, ws_target: int):
        """Start a group on an idle slot.  fp is its footprint with the slot's
        workspace counted at ws_charge = max(held workspace, group's need); the
        workspace is grown to ws_target (>= ws_charge) if it is smaller."""
        now = time.perf_counter()
        for r in group:
            r.t_admit = now
            r.group_size = len(group)
        cap = slot.ws.numel() if slot.ws is not None else 0
        self.ws_held += ws_target - cap
        slot.ws_target = ws_target
        slot.group, slot.bytes = group, fp - ws_charge
        self.in_use += fp - ws_charge
        self._pin(group, +1)
        self.groups += 1
        if len(group) == 1 and getattr(group[0].plan, "_uploaded", False):
            self._launch(slot, group[0].plan)
        else:
            slot.prep = self.pool.submit(self._prepare, group, slot.stream)

    def _alloc_outputs(self, group):
        """Views of one device block per group (output_layout): each request's
        fields, shaped as rcr_solution.  A request that keeps its outputs keeps
        the block alive."""
        import torch
        offs, total = output_layout(group)
        block = torch.empty(total // 8, dtype=torch.float64, device=self.device)
        outs = []
        for r, o in zip(group, offs):
            sh = rcr.solution_shapes(r.N, r.n, r.m)
            outs.append({k: block[o[k] // 8:o[k] // 8 + int(np.prod(sh[k]))].view(sh[k]) for k in rcr.SOLUTION_FIELDS})
        return outs

    def _launch(self, slot: _Slot, plan):
        import torch
        t = time.perf_counter()
        group = slot.group
        with torch.cuda.stream(slot.stream):
            outs = self._alloc_outputs(group)
            need = (plan.workspace_size(self.precision) if len(group) == 1
                    else rcr.batch_workspace_size(plan, self.precision))
            if slot.ws is None or slot.ws.numel() < slot.ws_target:  # the size admission charged
                slot.ws = None  # the slot's stream is idle here: its previous group has completed
                slot.ws = torch.empty(slot.ws_target, dtype=torch.uint8, device=self.device)
                self.stats["ws_grow"] += 1
            ws = slot.ws[:need]
            if len(group) == 1:
                rcr.solve(plan, group[0].prob, out=outs[0], precision=self.precision,
                          refine_steps=self.refine_steps, executor=rcr.EXEC_LEVELS, workspace=ws,
                          stream=slot.stream)
            else:
                rcr.batch_solve(plan, [r.prob for r in group], outs, precision=self.precision,
                                refine_steps=self.refine_steps, executor=rcr.EXEC_LEVELS, workspace=ws,
                                stream=slot.stream)
            ev = torch.cuda.Event()
            ev.record(slot.stream)
        for r, o in zip(group, outs):
            r.out = o
        slot.event = ev
        slot.keep = (plan if len(group) > 1 else None, ws)
        dt = time.perf_counter() - t
        self.stats["launch_s"] += dt
        self.stats["launch_max_s"] = max(self.stats["launch_max_s"], dt)

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
                        # the copy is charged to the cache from here on, not to the group
                        db = plan.device_bytes()
                        self.cached_plan_bytes += db
                        slot.bytes -= db
                        self.in_use -= db
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
        blocked = False
        for slot in self.slots:
            if slot.group is not None or not self.ready:
                continue
            while True:
                cap = slot.ws.numel() if slot.ws is not None else 0

                def ws_of(g, cap=cap):  # the group runs on this slot's workspace, grown if needed
                    ws, plan_bytes = self._ws_of(g)
                    return max(cap, ws), plan_bytes

                free = self.budget - self.in_use - self.cached_plan_bytes - (self.ws_held - cap)
                group, fp = form_group(self.ready, free, self.max_group_nodes, ws_of, self.precision)
                if group or not self._evict_for_room(slot):
                    break
            if not group:
                blocked = True
                continue
            ids = {id(r) for r in group}
            self.ready = collections.deque(r for r in self.ready if id(r) not in ids)
            charge = ws_of(group)[0]
            # grow to a power of two when the budget allows: few distinct sizes,
            # so the blocks a slot gives up are reused by the others
            target = max(cap, 1 << max(charge - 1, 0).bit_length())
            if fp - charge + target > free:
                target = charge
            self._dispatch(slot, group, fp, charge, target)
        if blocked and self.ready and not any(s_.group is not None for s_ in self.slots):
            raise RuntimeError(f"request {self.ready[0].rid} does not fit the HBM budget of "
                               f"{self.budget} bytes on an idle device")
        self._evict()
        return finished

    def reserve(self, ws_bytes: int, out_bytes: int):
        """Grow every idle slot's workspace to ws_bytes (charged to the budget like
        any held workspace) and let each slot's stream allocate and release one
        output block of out_bytes, so that a serving stream does not map new
        device memory when its first large group arrives (a new mapping holds up
        the other threads of the process for tens of milliseconds)."""
        import torch
        for slot in self.slots:
            if slot.group is not None:
                continue
            cap = slot.ws.numel() if slot.ws is not None else 0
            with torch.cuda.stream(slot.stream):
                if ws_bytes > cap and self.held() + ws_bytes - cap <= self.budget:
                    slot.ws = None
                    slot.ws = torch.empty(ws_bytes, dtype=torch.uint8, device=self.device)
                    self.ws_held += ws_bytes - cap
                if out_bytes > 0:
                    blk = torch.empty(out_bytes // 8, dtype=torch.float64, device=self.device)
                    del blk
        torch.cuda.synchronize(self.device)

    def _evict_for_room(self, slot) -> bool:
        """Make room for the head of the queue: release the device copy of the least
        recently used cached plan that no running group uses, else the workspace
        of another idle slot, else this slot's own; False if there is nothing
        left to release."""
        for k, ent in self.cache.items():
            if ent[1] == 0 and getattr(ent[0], "_uploaded", False):
                self.cached_plan_bytes -= ent[0].device_bytes()
                del self.cache[k]
                return True
        for other in self.slots:
            if other is not slot and other.group is None and other.ws is not None:
                self.ws_held -= other.ws.numel()
                other.ws = None
                return True
        if slot.ws is not None:  # last, the slot's own (larger than the head needs)
            self.ws_held -= slot.ws.numel()
            slot.ws = None
            return True
        return False

    def held(self) -> int:
        """HBM the server holds: running groups' outputs and plan copies, the
        slots' workspaces and the cached plans' device copies (<= hbm_budget)."""
        return self.in_use + self.ws_held + self.cached_plan_bytes

    def busy(self) -> bool:
        return bool(self.planning or self.ready or any(s.group is not None for s in self.slots))

    def drain(self):
        while self.busy():
            self.poll()

    def close(self):
        self.drain()
        self.pool.shutdown(wait=True)
        self.cache.clear()
